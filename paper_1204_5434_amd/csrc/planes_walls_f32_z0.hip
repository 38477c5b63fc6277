// Walled fused yz-plane kernels, complex float, wall kind 0 along z.
#define PFT_PLANE_EZ 0
#include "planes_walls.inc"

namespace pft {

bool plane_walls_supported(int n) { return plane_supported<float>(n); }

int plane_walls_private_bytes(int n, int ey, int ez)
{
    if (ey < 0 || ey > 2 || (ey == 0 && ez == 0)) return -1;
    switch (ez) {
    case 0: return plane_walls_private_bytes_z<0>(n, ey);
    case 1: return plane_walls_private_bytes_z<1>(n, ey);
    case 2: return plane_walls_private_bytes_z<2>(n, ey);
    default: return -1;
    }
}

hipError_t launch_yzpass_walls(int n, int ey, int ez, const PArgs<float>& a, hipStream_t s)
{
    if (ey < 0 || ey > 2 || (ey == 0 && ez == 0)) return hipErrorInvalidValue;
    switch (ez) {
    case 0: return launch_yzpass_walls_z<0>(n, ey, a, s);
    case 1: return launch_yzpass_walls_z<1>(n, ey, a, s);
    case 2: return launch_yzpass_walls_z<2>(n, ey, a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace pft
