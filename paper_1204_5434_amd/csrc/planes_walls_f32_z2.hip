// Walled fused yz-plane kernels, complex float, wall kind 2 along z.
#define PFT_PLANE_EZ 2
#include "planes_walls.inc"
