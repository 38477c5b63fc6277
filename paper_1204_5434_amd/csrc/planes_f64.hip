// Fused yz-plane kernels in complex double precision.
#define PFT_PLANE_T double
#define PFT_PLANE_LIST PFT_PLANE_SIZES_F64
#include "planes.inc"
