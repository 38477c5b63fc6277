// Axis-pass kernels in complex double precision.
#include "passes.inc"

namespace pft {
template hipError_t launch_zpass<double>(int, const ZArgs<double>&, hipStream_t);
template hipError_t launch_spass<double>(int, int, int64_t, SArgs<double>, int, hipStream_t);
}  // namespace pft
