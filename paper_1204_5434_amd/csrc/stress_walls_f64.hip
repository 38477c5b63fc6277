// Stress passes along walled axes in complex double precision.
#define PFT_STRESS_T double
#define PFT_STRESS_WALLS 1
#include "stress.inc"
