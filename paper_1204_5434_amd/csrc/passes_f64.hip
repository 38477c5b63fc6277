// Default axis-pass kernels in complex double precision.
#define PFT_VARIANT_LIST PFT_AXIS_VARIANTS0
#define PFT_VARIANT_NS v0
#include "passes.inc"

namespace pft {
namespace v0 {
template hipError_t launch_zpass<double>(int, int, const ZArgs<double>&, hipStream_t);
template hipError_t launch_spass<double>(int, int, int, int64_t, SArgs<double>, int, hipStream_t);
template hipError_t launch_zpass_batch<double>(int, int, int64_t, const ZArgs<double>*, int, hipStream_t);
template hipError_t launch_spass_batch<double>(int, int, int, int64_t, int, const SArgs<double>*, int, hipStream_t);
}  // namespace v0
}  // namespace pft
