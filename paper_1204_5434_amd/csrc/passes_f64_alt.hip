// Alternative kernel variants in complex double precision.
#define PFT_VARIANT_LIST PFT_AXIS_VARIANTS_ALT
#define PFT_VARIANT_NS alt
#include "passes.inc"

namespace pft {
namespace alt {
template hipError_t launch_zpass<double>(int, int, const ZArgs<double>&, hipStream_t);
template hipError_t launch_spass<double>(int, int, int, int64_t, SArgs<double>, int, hipStream_t);
template hipError_t launch_zpass_batch<double>(int, int, int64_t, const ZArgs<double>*, int, hipStream_t);
template hipError_t launch_spass_batch<double>(int, int, int, int64_t, int, const SArgs<double>*, int, hipStream_t);
}  // namespace alt
}  // namespace pft
