// Launchers of the semi-implicit step's reciprocal-space filter (complex
// double), one kernel per axis length with a pass kernel.
#include "sis.h"

namespace pft {

hipError_t launch_sis_pass(int kind, int nx, int ny, int nz, SisArgs a, hipStream_t s)
{
    const int n = (kind == 0 || kind == 4) ? nz : (kind == 2 ? nx : ny);
#define PFT_CASE(N, N1, N2)                                                                           \
    if (n == N) {                                                                                     \
        if (kind == 0 || kind == 4) {                                                                 \
            using Sh = ZShape<N1, N2, 1>;                                                             \
            a.nlines = (int64_t)nx * ny;                                                              \
            const unsigned blocks = (unsigned)((a.nlines + Sh::kLines - 1) / Sh::kLines);             \
            const unsigned lds = (unsigned)(Sh::kLds * sizeof(cx<double>));                           \
            if (kind == 0)                                                                            \
                hipLaunchKernelGGL((k_sis_z<N1, N2, kSisFwd>), dim3(blocks), dim3(Sh::kThreads), lds, s, a); \
            else                                                                                      \
                hipLaunchKernelGGL((k_sis_z<N1, N2, kSisInvSub>), dim3(blocks), dim3(Sh::kThreads), lds, s, a); \
            return hipGetLastError();                                                                 \
        }                                                                                             \
        using Sh = SShape<double, N2, 1>;                                                             \
        const int64_t nynz = (int64_t)ny * nz;                                                        \
        int nslabs = 1;                                                                               \
        if (kind == 2) {                                                                              \
            a.S = nynz;                                                                               \
            a.slab_stride = 0;                                                                        \
            a.ncols = (int)nynz;                                                                      \
        } else {                                                                                      \
            a.S = nz;                                                                                 \
            a.slab_stride = nynz;                                                                     \
            a.ncols = nz;                                                                             \
            nslabs = nx;                                                                              \
        }                                                                                             \
        a.ntiles = (a.ncols + Sh::kCols - 1) / Sh::kCols;                                             \
        const dim3 grid((unsigned)(a.ntiles * nslabs));                                               \
        const unsigned lds = (N2 == 1) ? 0u : (unsigned)(N * Sh::kCols * sizeof(cx<double>));          \
        if (kind == 1)                                                                                \
            hipLaunchKernelGGL((k_sis_s<N1, N2, kSisFwd>), grid, dim3(Sh::kThreads), lds, s, a);      \
        else if (kind == 2)                                                                           \
            hipLaunchKernelGGL((k_sis_s<N1, N2, kSisFilter>), grid, dim3(Sh::kThreads), lds, s, a);   \
        else                                                                                          \
            hipLaunchKernelGGL((k_sis_s<N1, N2, kSisInv>), grid, dim3(Sh::kThreads), lds, s, a);      \
        return hipGetLastError();                                                                     \
    }
    PFT_AXIS_SIZES(PFT_CASE)
#undef PFT_CASE
    return hipErrorInvalidValue;
}

}  // namespace pft
