// Stress passes of the reverse-mode sweep in complex double precision.
#define PFT_STRESS_T double
#include "stress.inc"
