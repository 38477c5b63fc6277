// Walled passes in complex double precision.
#define PFT_WALLS_T double
#include "passes_walls.inc"

namespace pft {
// Physical line lengths that have walled kernels (the same for both precisions).
bool walls_supported(int n)
{
#define PFT_CASE(NP, N1, N2) \
    if (n == NP) return true;
    PFT_AXIS_SIZES(PFT_CASE)
#undef PFT_CASE
    return false;
}
}  // namespace pft
