// Launchers of the semi-implicit step's reciprocal-space filter (complex
// double), one kernel per axis length with a pass kernel.
#include "sis.h"

namespace pft {

bool sis_pass_layout(int kind, int nx, int ny, int nz, SisArgs* a)
{
    const int n = (kind == 0 || kind == 4) ? nz : (kind == 2 ? nx : ny);
#define PFT_CASE(N, N1, N2)                                                                           \
    if (n == N) {                                                                                     \
        if (kind == 0 || kind == 4) {                                                                 \
            a->nlines = (int64_t)nx * ny;                                                             \
            return true;                                                                              \
        }                                                                                             \
        using Sh = SShape<double, N2, 1>;                                                             \
        const int64_t nynz = (int64_t)ny * nz;                                                        \
        if (kind == 2) {                                                                              \
            a->S = nynz;                                                                              \
            a->slab_stride = 0;                                                                       \
            a->ncols = (int)nynz;                                                                     \
        } else {                                                                                      \
            a->S = nz;                                                                                \
            a->slab_stride = nynz;                                                                    \
            a->ncols = nz;                                                                            \
        }                                                                                             \
        a->ntiles = (a->ncols + Sh::kCols - 1) / Sh::kCols;                                           \
        return true;                                                                                  \
    }
    PFT_AXIS_SIZES(PFT_CASE)
#undef PFT_CASE
    return false;
}

// Launch pass kind over R arrays: tab == nullptr launches the by-value
// kernel on a (R = 1), else the batched kernel on the table.
static hipError_t sis_launch(int kind, int nx, int ny, int nz, const SisArgs& a, const SisArgs* tab, int R,
                             hipStream_t s)
{
    const int n = (kind == 0 || kind == 4) ? nz : (kind == 2 ? nx : ny);
#define PFT_SIS_GO(K, KB, GRID, BLOCK, LDS)                                                           \
    do {                                                                                              \
        if (tab)                                                                                      \
            hipLaunchKernelGGL(KB, dim3(GRID, (unsigned)R), BLOCK, LDS, s, tab);                      \
        else                                                                                          \
            hipLaunchKernelGGL(K, dim3(GRID), BLOCK, LDS, s, a);                                      \
    } while (0)
#define PFT_CASE(N, N1, N2)                                                                           \
    if (n == N) {                                                                                     \
        if (kind == 0 || kind == 4) {                                                                 \
            using Sh = ZShape<N1, N2, 1>;                                                             \
            const unsigned blocks = (unsigned)(((int64_t)nx * ny + Sh::kLines - 1) / Sh::kLines);     \
            const unsigned lds = (unsigned)(Sh::kLds * sizeof(cx<double>));                           \
            if (kind == 0)                                                                            \
                PFT_SIS_GO((k_sis_z<N1, N2, kSisFwd>), (k_sis_z_batch<N1, N2, kSisFwd>), blocks, dim3(Sh::kThreads), lds); \
            else                                                                                      \
                PFT_SIS_GO((k_sis_z<N1, N2, kSisInvSub>), (k_sis_z_batch<N1, N2, kSisInvSub>), blocks, dim3(Sh::kThreads), lds); \
            return hipGetLastError();                                                                 \
        }                                                                                             \
        using Sh = SShape<double, N2, 1>;                                                             \
        const int ncols = kind == 2 ? ny * nz : nz;                                                   \
        const int nslabs = kind == 2 ? 1 : nx;                                                        \
        const unsigned blocks = (unsigned)(((ncols + Sh::kCols - 1) / Sh::kCols) * nslabs);           \
        const unsigned lds = (N2 == 1) ? 0u : (unsigned)(N * Sh::kCols * sizeof(cx<double>));          \
        if (kind == 1)                                                                                \
            PFT_SIS_GO((k_sis_s<N1, N2, kSisFwd>), (k_sis_s_batch<N1, N2, kSisFwd>), blocks, dim3(Sh::kThreads), lds); \
        else if (kind == 2)                                                                           \
            PFT_SIS_GO((k_sis_s<N1, N2, kSisFilter>), (k_sis_s_batch<N1, N2, kSisFilter>), blocks, dim3(Sh::kThreads), lds); \
        else                                                                                          \
            PFT_SIS_GO((k_sis_s<N1, N2, kSisInv>), (k_sis_s_batch<N1, N2, kSisInv>), blocks, dim3(Sh::kThreads), lds); \
        return hipGetLastError();                                                                     \
    }
    PFT_AXIS_SIZES(PFT_CASE)
#undef PFT_CASE
#undef PFT_SIS_GO
    return hipErrorInvalidValue;
}

hipError_t launch_sis_pass(int kind, int nx, int ny, int nz, SisArgs a, hipStream_t s)
{
    if (!sis_pass_layout(kind, nx, ny, nz, &a)) return hipErrorInvalidValue;
    return sis_launch(kind, nx, ny, nz, a, nullptr, 1, s);
}

hipError_t launch_sis_pass_batch(int kind, int nx, int ny, int nz, const SisArgs* tab, int R, hipStream_t s)
{
    if (!tab || R < 1) return hipErrorInvalidValue;
    return sis_launch(kind, nx, ny, nz, SisArgs{}, tab, R, s);
}

}  // namespace pft
