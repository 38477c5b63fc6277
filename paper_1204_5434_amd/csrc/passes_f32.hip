// Axis-pass kernels in complex single precision.
#include "passes.inc"

namespace pft {
template hipError_t launch_zpass<float>(int, const ZArgs<float>&, hipStream_t);
template hipError_t launch_spass<float>(int, int, int64_t, SArgs<float>, int, hipStream_t);
}  // namespace pft
