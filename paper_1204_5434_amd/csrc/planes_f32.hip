// Fused yz-plane kernels with complex float propagators.
#define PFT_PLANE_T float
#define PFT_PLANE_LIST PFT_PLANE_SIZES_F32
#include "planes.inc"
