// Alternative kernel variants in complex float precision.
#define PFT_VARIANT_LIST PFT_AXIS_VARIANTS_ALT
#define PFT_VARIANT_NS alt
#include "passes.inc"

namespace pft {
namespace alt {
template hipError_t launch_zpass<float>(int, int, const ZArgs<float>&, hipStream_t);
template hipError_t launch_spass<float>(int, int, int, int64_t, SArgs<float>, int, hipStream_t);
template hipError_t launch_zpass_batch<float>(int, int, int64_t, const ZArgs<float>*, int, hipStream_t);
template hipError_t launch_spass_batch<float>(int, int, int, int64_t, int, const SArgs<float>*, int, hipStream_t);
}  // namespace alt
}  // namespace pft
