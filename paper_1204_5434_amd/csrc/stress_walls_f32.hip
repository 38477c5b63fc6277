// Stress passes along walled axes in complex float precision.
#define PFT_STRESS_T float
#define PFT_STRESS_WALLS 1
#include "stress.inc"
