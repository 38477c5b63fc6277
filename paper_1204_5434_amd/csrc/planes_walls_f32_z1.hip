// Walled fused yz-plane kernels, complex float, wall kind 1 along z.
#define PFT_PLANE_EZ 1
#include "planes_walls.inc"
