// Stress passes of the reverse-mode sweep in complex float precision.
#define PFT_STRESS_T float
#include "stress.inc"
