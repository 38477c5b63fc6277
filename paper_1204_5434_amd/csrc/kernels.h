// HIP kernels of the propagator hot path (gfx950, 64-lane wavefronts).
//
// One contour step of the Richardson split step, Eq. (12), is
//   q' = (4/3) E4 D_{h/2} E2 D_{h/2} E4 q  -  (1/3) E2 D_h E2 q,
// with E4 = exp(-w h/4), E2 = E4^2 and D_a = Dz Dy Dx the separable
// diffusion operator.  Because the axis operators commute and act on whole
// lines, a step runs as four memory passes over two work arrays
// U (half-step path) and V (full-step path):
//
//   Z (step j-1 -> j) : U = Dz_{h/2}(E4 q_j),          V = Dz_h(E2 q_j)
//   Y1                : U = Dy_{h/2} U,                V = Dy_h V
//   X                 : U = Dx_{h/2}(E2 Dx_{h/2} U),   V = E2 Dx_h V
//   Y2                : U = Dy_{h/2} U
//   Z (step j -> j+1) : q_{j+1} = (4 E4 Dz_{h/2} U - V) / 3, stored, and the
//                       next step's U and V are started from it in the same pass.
//
// The plain split step uses V alone: Z (q_{j+1} = E2 V; V = Dz_h(E2 q)), Y, X.
// Every axis pass holds its lines on chip (registers plus one LDS exchange per
// transform direction), so each pass reads and writes each array once.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "fft.h"

namespace pft {

enum { kSchemeRQM4 = 0, kSchemeSplit2 = 1 };

// Profiling hook: when set, the next launch through PFT_LAUNCH records this
// event pair as part of its own dispatch (start and end of the kernel, no
// queue gaps) and clears it.  Host-side state, one per host thread.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchEvents g_launch_events;

#define PFT_LAUNCH(kernel, grid, block, shmem, stream, ...)                                              \
    do {                                                                                               \
        if (::pft::g_launch_events.start) {                                                            \
            const ::pft::LaunchEvents ev_ = ::pft::g_launch_events;                                    \
            ::pft::g_launch_events = ::pft::LaunchEvents{};                                            \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, ev_.start, ev_.stop, 0, __VA_ARGS__); \
        } else {                                                                                       \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                       \
        }                                                                                              \
    } while (0)

// ------------------------------------------------------------------ z pass --
template <typename T>
struct ZArgs {
    int skip;         // batched launches: this replica has no work at this position
    int64_t nlines;   // nx * ny lines of nz contiguous points
    cx<T>* U;
    cx<T>* V;
    const cx<T>* qin; // start value when there is no previous step (NULL: q = 1)
    cx<T>* qout;      // where the completed q is stored (NULL: not stored)
    int has_prev, has_next, scheme;
    const cx<T>* Ep;  // E4 table of the step being completed (NULL: E = 1)
    const T* gh_p;    // its z factor for h/2
    const cx<T>* En;  // E4 table of the step being started (NULL: E = 1)
    const T* gh_n;    // its z factors for h/2 and h
    const T* gf_n;
    cx<T>* hcap;      // if set: the completed step's last diffused value before its
                      // final field multiply (Dz U for the Richardson step, V for the
                      // plain split), for the reverse-mode sweep
};

template <int N1, int N2>
struct LayZ {
    int l;
    __device__ __forceinline__ int operator()(int k1, int n2) const { return (l * N1 + k1) * (N2 + 1) + n2; }
};

// W multiplies the lines (z pass) or columns (strided passes) per workgroup;
// the tuner picks it per axis length.
template <int N1, int N2, int W = 1>
struct ZShape {
    static constexpr int kLines = ((N2 >= 64) ? 1 : 64 / N2) * W;  // lines per workgroup
    static constexpr int kThreads = kLines * N2;
    static constexpr int kLds = (N2 == 1) ? 0 : kLines * N1 * (N2 + 1);  // elements
};

// Walls along a line (EXT = 1 reflecting, 2 absorbing): register n of the
// line holds physical point ext_index(n) (x[2n] for n < N/2, then the odd
// points backwards), times ext_sign(n) (-1 on the odd points between
// absorbing walls), the order in which pair_diffuse() applies the walled
// diffusion with one N-point transform.  Field tables are read through the
// same index without the sign.
template <int EXT, int N>
__device__ __forceinline__ int ext_index(int n)
{
    if constexpr (EXT == 0) return n;
    else return n < N / 2 ? 2 * n : 2 * (N - 1 - n) + 1;
}
template <int EXT, int N, typename T>
__device__ __forceinline__ T ext_sign(int n)
{
    return (EXT == 2 && n >= N / 2) ? T(-1) : T(1);
}

// The line diffusion of the periodic (EXT = 0) or walled line; MEAN as in
// diffuse() (tables of diffusion factors).
template <int EXT, int N1, int N2, bool MEAN = false, typename T, class Lay>
__device__ __forceinline__ void line_diffuse(cx<T> (&a)[N1], int t, cx<T>* __restrict__ sh, const Lay& lay,
                                             const T* __restrict__ g)
{
    if constexpr (EXT == 0)
        diffuse<N1, N2, MEAN>(a, t, sh, lay, g);
    else
        pair_diffuse<N1, N2>(a, t, sh, lay, g);
}

// The Richardson combination (4 u - v) / 3 of Eq. (12).  In complex float it
// is formed in double and rounded once: multiplying by 1/3 rounded to float
// would scale every node by the same factor at every step.
template <typename T>
__device__ __forceinline__ cx<T> richardson(cx<T> u, cx<T> v)
{
    if constexpr (std::is_same<T, float>::value) {
        constexpr double third = 1.0 / 3.0;
        return {float((4.0 * double(u.re) - double(v.re)) * third), float((4.0 * double(u.im) - double(v.im)) * third)};
    } else {
        constexpr T third = T(1.0 / 3.0);
        return third * (T(4) * u - v);
    }
}

template <typename T, int N1, int N2, int W, int EXT = 0>
__device__ __forceinline__ void zpass_body(const ZArgs<T>& A, unsigned bid, cx<T>* sh)
{
    constexpr int N = N1 * N2;
    constexpr int LPW = ZShape<N1, N2, W>::kLines;
    const int tid = threadIdx.x;
    const int t = tid % N2, l = tid / N2;
    const int64_t line = (int64_t)bid * LPW + l;
    const bool act = line < A.nlines;
    const int64_t base = line * N + (EXT ? 0 : t);
    const LayZ<N1, N2> lay{l};

    // Walled lines with several lanes per line: the points of the walled-order
    // register pair (i, N1-1-i) lie in one block of 2 N2 contiguous physical
    // points (the even ones of the first, the odd ones of the second), which
    // the lanes read and write as two contiguous runs of N2 points: in run A a
    // lane of the line's first half takes its point of register i and a lane
    // of the second half its point of register N1-1-i, in run B the other way
    // round, and a select per register puts each value in place.  Every load
    // and store instruction then covers whole 128-byte lines, as in the
    // periodic pass, instead of every other point of two lines.
    constexpr bool kRuns = EXT != 0 && N2 >= 2;
    static_assert(!kRuns || N1 % 2 == 0, "register pairs need an even N1");
    const bool hi_half = t >= N2 / 2;
    // walled-order index of this lane's point in run B (or A) of pair i
    auto run_n = [&](int i, bool runB) { return ((hi_half != runB) ? N1 - 1 - i : i) * N2 + t; };
    // one point of run A or B: signed (propagator-like arrays) or not (field tables)
    auto run_ld = [&](const cx<T>* p, int n, bool sign) -> cx<T> {
        const cx<T> x = p[base + ext_index<EXT, N>(n)];
        return sign ? ext_sign<EXT, N, T>(n) * x : x;
    };
    auto load_runs = [&](const cx<T>* p, cx<T>(&r)[N1], bool sign) {
        sfor<0, N1 / 2>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const cx<T> a = run_ld(p, run_n(i, false), sign), b = run_ld(p, run_n(i, true), sign);
            r[i] = hi_half ? b : a;
            r[N1 - 1 - i] = hi_half ? a : b;
        });
    };

    // propagator-like arrays (odd points sign-flipped between absorbing walls)
    auto load = [&](const cx<T>* p, cx<T>(&r)[N1]) {
        if (act) {
            if constexpr (EXT == 0) {
                sfor<0, N1>([&](auto I) { r[decltype(I)::value] = p[base + decltype(I)::value * N2]; });
            } else if constexpr (kRuns) {
                load_runs(p, r, true);
            } else {
                sfor<0, N1>([&](auto I) {
                    const int n = decltype(I)::value * N2 + t;
                    r[decltype(I)::value] = ext_sign<EXT, N, T>(n) * p[base + ext_index<EXT, N>(n)];
                });
            }
        } else {
            sfor<0, N1>([&](auto I) { r[decltype(I)::value] = cx<T>{T(0), T(0)}; });
        }
    };
    // field tables (no sign)
    auto load_e = [&](const cx<T>* p, cx<T>(&r)[N1]) {
        if constexpr (EXT == 0) {
            load(p, r);
        } else if (act) {
            if constexpr (kRuns)
                load_runs(p, r, false);
            else
                sfor<0, N1>([&](auto I) { r[decltype(I)::value] = p[base + ext_index<EXT, N>(decltype(I)::value * N2 + t)]; });
        } else {
            sfor<0, N1>([&](auto I) { r[decltype(I)::value] = cx<T>{T(0), T(0)}; });
        }
    };
    auto store = [&](cx<T>* p, const cx<T>(&r)[N1]) {
        if (!act) return;
        if constexpr (EXT == 0) {
            sfor<0, N1>([&](auto I) { p[base + decltype(I)::value * N2] = r[decltype(I)::value]; });
        } else if constexpr (kRuns) {
            sfor<0, N1 / 2>([&](auto I) {
                constexpr int i = decltype(I)::value;
                const int na = run_n(i, false), nb = run_n(i, true);
                const cx<T> a = hi_half ? r[N1 - 1 - i] : r[i];
                const cx<T> b = hi_half ? r[i] : r[N1 - 1 - i];
                p[base + ext_index<EXT, N>(na)] = ext_sign<EXT, N, T>(na) * a;
                p[base + ext_index<EXT, N>(nb)] = ext_sign<EXT, N, T>(nb) * b;
            });
        } else {
            sfor<0, N1>([&](auto I) {
                const int n = decltype(I)::value * N2 + t;
                p[base + ext_index<EXT, N>(n)] = ext_sign<EXT, N, T>(n) * r[decltype(I)::value];
            });
        }
    };
    // the stored slice: streamed past the caches where each store instruction
    // writes whole 128-byte lines (partial lines would be written twice)
    auto store_q = [&](cx<T>* p, const cx<T>(&r)[N1]) {
        if constexpr (EXT == 0 && (N2 * sizeof(cx<T>)) % 128 == 0) {
            if (act) sfor<0, N1>([&](auto I) { store_stream(p + base + decltype(I)::value * N2, r[decltype(I)::value]); });
        } else {
            store(p, r);
        }
    };
    // one value of a propagator-like array at this lane's point i
    auto at = [&](const cx<T>* p, int i) -> cx<T> {
        if constexpr (EXT == 0) {
            return p[base + i * N2];
        } else {
            const int n = i * N2 + t;
            return ext_sign<EXT, N, T>(n) * p[base + ext_index<EXT, N>(n)];
        }
    };

    cx<T> q[N1];
    cx<T> e[N1];        // field table of the completed step, reused for the next when shared
    bool have_e = false;
    if (A.has_prev) {
        if (A.scheme == kSchemeRQM4) {
            load(A.U, q);
            line_diffuse<EXT, N1, N2, true>(q, t, sh, lay, A.gh_p);
            if (A.hcap) store(A.hcap, q);
            if (A.Ep) {
                load_e(A.Ep, e);
                have_e = true;
            }
            if (act) {
                if constexpr (kRuns) {
                    // V read in contiguous runs, one register pair at a time
                    sfor<0, N1 / 2>([&](auto I) {
                        constexpr int i = decltype(I)::value, j = N1 - 1 - i;
                        const cx<T> a = run_ld(A.V, run_n(i, false), true), b = run_ld(A.V, run_n(i, true), true);
                        const cx<T> ui = A.Ep ? q[i] * e[i] : q[i];
                        const cx<T> uj = A.Ep ? q[j] * e[j] : q[j];
                        q[i] = richardson(ui, hi_half ? b : a);
                        q[j] = richardson(uj, hi_half ? a : b);
                    });
                } else {
                    sfor<0, N1>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        const cx<T> u = A.Ep ? q[i] * e[i] : q[i];
                        q[i] = richardson(u, at(A.V, i));
                    });
                }
            }
        } else {
            load(A.V, q);
            if (A.hcap) store(A.hcap, q);
            if (A.Ep) {
                load_e(A.Ep, e);
                have_e = true;
                sfor<0, N1>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    q[i] = q[i] * (e[i] * e[i]);
                });
            }
        }
    } else if (A.qin) {
        load(A.qin, q);
    } else {
        // q = 1 (odd points sign-flipped between absorbing walls)
        sfor<0, N1>([&](auto I) {
            q[decltype(I)::value] = ext_sign<EXT, N, T>(decltype(I)::value * N2 + t) * cx<T>{T(1), T(0)};
        });
    }
    if (A.qout) store_q(A.qout, q);

    if (A.has_next) {
        // q <- E4 q (half path start) and w <- E4 E4 q (full path start)
        cx<T> w[N1];
        if (A.En) {
            if (!(have_e && A.En == A.Ep)) load_e(A.En, e);
            sfor<0, N1>([&](auto I) {
                constexpr int i = decltype(I)::value;
                q[i] = q[i] * e[i];
                w[i] = q[i] * e[i];
            });
        } else {
            sfor<0, N1>([&](auto I) { w[decltype(I)::value] = q[decltype(I)::value]; });
        }
        if (A.scheme == kSchemeRQM4) {
            line_diffuse<EXT, N1, N2, true>(q, t, sh, lay, A.gh_n);
            store(A.U, q);
        }
        line_diffuse<EXT, N1, N2, true>(w, t, sh, lay, A.gf_n);
        store(A.V, w);
    }
}

// MW: minimum waves per SIMD the register allocation must allow (1 = no bound).
template <typename T, int N1, int N2, int W, int MW>
__global__ __launch_bounds__((ZShape<N1, N2, W>::kThreads), MW) void k_zpass(ZArgs<T> A)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    zpass_body<T, N1, N2, W>(A, blockIdx.x, reinterpret_cast<cx<T>*>(smem_raw));
}

// Walled z lines of N1 N2 points.
template <typename T, int N1, int N2, int EXT>
__global__ __launch_bounds__((ZShape<N1, N2, 1>::kThreads)) void k_zpass_walls(ZArgs<T> A)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    zpass_body<T, N1, N2, 1, EXT>(A, blockIdx.x, reinterpret_cast<cx<T>*>(smem_raw));
}

// Batched: blockIdx.y selects a replica whose arguments come from a table.
template <typename T, int N1, int N2, int W, int MW>
__global__ __launch_bounds__((ZShape<N1, N2, W>::kThreads), MW) void k_zpass_batch(const ZArgs<T>* __restrict__ descs)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const ZArgs<T> A = descs[blockIdx.y];
    if (A.skip) return;
    zpass_body<T, N1, N2, W>(A, blockIdx.x, reinterpret_cast<cx<T>*>(smem_raw));
}

// ------------------------------------------------------ strided (x, y) pass --
template <typename T>
struct SOps {
    const T* g1;     // first diffusion factor; NULL leaves the array untouched
    const cx<T>* e;  // E4 table: multiply by E4^2 after the first diffusion (NULL: none)
    const T* g2;     // second diffusion factor after the multiply (NULL: none)
    cx<T>* acap;     // if set: store the array after the first diffusion (before the
                     // multiply), for the reverse-mode sweep
};

template <typename T>
struct SArgs {
    int skip;             // batched launches: this replica has no work at this position
    cx<T>* U;
    cx<T>* V;
    int64_t S;            // element stride along the lines
    int64_t slab_stride;  // distance between slabs of columns
    int ncols;            // contiguous columns per slab
    int ntiles;           // column tiles per slab
    SOps<T> opU, opV;
};

template <int N2, int TC>
struct LayS {
    int c;
    __device__ __forceinline__ int operator()(int k1, int n2) const { return (k1 * N2 + n2) * TC + c; }
};

template <typename T, int N2, int W = 1>
struct SShape {
    // columns per workgroup: at least one 128-byte row segment, at least one wavefront
    static constexpr int kMinCols = 128 / int(sizeof(cx<T>));
    static constexpr int kCols = ((64 / N2 > kMinCols) ? 64 / N2 : kMinCols) * W;
    static constexpr int kThreads = kCols * N2;
};

// AXIS: 0 = x (field multiplies allowed), 1 = y.
template <typename T, int N1, int N2, int AXIS, int W, int EXT = 0>
__device__ __forceinline__ void spass_body(const SArgs<T>& A, unsigned bid, cx<T>* sh)
{
    constexpr int N = N1 * N2;
    constexpr int TC = SShape<T, N2, W>::kCols;
    const int tid = threadIdx.x;
    const int c = tid % TC, t = tid / TC;
    const int slab = bid / A.ntiles, tile = bid % A.ntiles;
    const int col = tile * TC + c;
    const bool act = col < A.ncols;
    const int64_t base = (int64_t)slab * A.slab_stride + col + (EXT ? 0 : (int64_t)t * A.S);
    const int64_t step = (int64_t)N2 * A.S;
    const LayS<N2, TC> lay{c};
    // address of this lane's point i (walls: its physical point)
    auto addr = [&](int i) -> int64_t {
        if constexpr (EXT == 0) return base + i * step;
        else return base + (int64_t)ext_index<EXT, N>(i * N2 + t) * A.S;
    };

    auto ldX = [&](const cx<T>* X, cx<T>(&a)[N1]) {
        if (act) {
            sfor<0, N1>([&](auto I) {
                constexpr int i = decltype(I)::value;
                a[i] = ext_sign<EXT, N, T>(i * N2 + t) * X[addr(i)];
            });
        } else {
            sfor<0, N1>([&](auto I) { a[decltype(I)::value] = cx<T>{T(0), T(0)}; });
        }
    };
    auto stX = [&](cx<T>* X, const cx<T>(&a)[N1]) {
        if (act)
            sfor<0, N1>([&](auto I) {
                constexpr int i = decltype(I)::value;
                X[addr(i)] = ext_sign<EXT, N, T>(i * N2 + t) * a[i];
            });
    };
    // one array: diffuse, [capture], [multiply by e2 = E4^2, diffuse again]
    auto run_on = [&](cx<T>* X, cx<T>(&a)[N1], const SOps<T>& op, const cx<T>(&e2)[N1], bool have_e2) {
        line_diffuse<EXT, N1, N2, true>(a, t, sh, lay, op.g1);
        if (op.acap) stX(op.acap, a);
        if (AXIS == 0 && op.e) {  // field multiplies happen only in the x pass
            if (have_e2) {
                sfor<0, N1>([&](auto I) { a[decltype(I)::value] = a[decltype(I)::value] * e2[decltype(I)::value]; });
            } else if (act) {
                sfor<0, N1>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    const cx<T> e = op.e[addr(i)];  // field tables: no sign
                    a[i] = a[i] * (e * e);
                });
            }
            if (op.g2) line_diffuse<EXT, N1, N2, true>(a, t, sh, lay, op.g2);
        }
        stX(X, a);
    };
    auto run = [&](cx<T>* X, const SOps<T>& op, const cx<T>(&e2)[N1], bool have_e2) {
        if (!op.g1) return;
        cx<T> a[N1];
        ldX(X, a);
        run_on(X, a, op, e2, have_e2);
    };
    cx<T> e2[N1];
    if (AXIS == 1 && N1 * sizeof(cx<T>) <= 256 && A.opU.g1 && A.opV.g1) {
        // y pass on both arrays: V's loads are issued before U's transform so
        // that their latency hides behind it (where the second array still fits
        // the registers of two waves per SIMD)
        cx<T> v[N1];
        ldX(A.V, v);
        run(A.U, A.opU, e2, false);
        run_on(A.V, v, A.opV, e2, false);
        return;
    }
    if (AXIS == 0 && A.opU.g1 && A.opV.g1 && A.opU.e && A.opU.e == A.opV.e) {
        // both arrays take the same field table: read it once
        if (act) {
            sfor<0, N1>([&](auto I) { e2[decltype(I)::value] = A.opU.e[addr(decltype(I)::value)]; });
        } else {
            sfor<0, N1>([&](auto I) { e2[decltype(I)::value] = cx<T>{T(0), T(0)}; });
        }
        sfor<0, N1>([&](auto I) { e2[decltype(I)::value] = e2[decltype(I)::value] * e2[decltype(I)::value]; });
        run(A.V, A.opV, e2, true);
        run(A.U, A.opU, e2, true);
    } else {
        run(A.U, A.opU, e2, false);
        run(A.V, A.opV, e2, false);
    }
}

// AXIS (0 = x, 1 = y) also names the kernel, so profiles tell the passes apart.
template <typename T, int N1, int N2, int AXIS, int W, int MW>
__global__ __launch_bounds__((SShape<T, N2, W>::kThreads), MW) void k_spass(SArgs<T> A)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    spass_body<T, N1, N2, AXIS, W>(A, blockIdx.x, reinterpret_cast<cx<T>*>(smem_raw));
}

// Walled x or y lines of N1 N2 points.
template <typename T, int N1, int N2, int AXIS, int EXT>
__global__ __launch_bounds__((SShape<T, N2, 1>::kThreads)) void k_spass_walls(SArgs<T> A)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    spass_body<T, N1, N2, AXIS, 1, EXT>(A, blockIdx.x, reinterpret_cast<cx<T>*>(smem_raw));
}

template <typename T, int N1, int N2, int AXIS, int W, int MW>
__global__ __launch_bounds__((SShape<T, N2, W>::kThreads), MW) void k_spass_batch(const SArgs<T>* __restrict__ descs)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const SArgs<T> A = descs[blockIdx.y];
    if (A.skip) return;
    spass_body<T, N1, N2, AXIS, W>(A, blockIdx.x, reinterpret_cast<cx<T>*>(smem_raw));
}

// ------------------------------------------------------------ launchers ----
// Axis lengths with a kernel, as (N, N1, N2): N1 points per lane, N2 lanes per line.
#define PFT_AXIS_SIZES(X) \
    X(8, 8, 1)            \
    X(12, 12, 1)          \
    X(16, 16, 1)          \
    X(20, 20, 1)          \
    X(24, 12, 2)          \
    X(32, 16, 2)          \
    X(40, 20, 2)          \
    X(48, 12, 4)          \
    X(64, 16, 4)          \
    X(80, 20, 4)          \
    X(96, 24, 4)          \
    X(128, 16, 8)         \
    X(192, 24, 8)         \
    X(256, 16, 16)

// Kernel variants per axis length, as (N, variant, N1, N2, W, MW): variant 0 is
// the default split and tile; the others widen the workgroup tile (W = 2), use
// another radix split N = N1 * N2, or bound the registers so that MW = 2 waves
// fit on each SIMD.  Variant 0 compiles with the rest of the library; the
// others sit in their own translation units.
#define PFT_AXIS_VARIANTS0(X)     \
    X(8, 0, 8, 1, 1, 1)           \
    X(12, 0, 12, 1, 1, 1)         \
    X(16, 0, 16, 1, 1, 1)         \
    X(20, 0, 20, 1, 1, 1)         \
    X(24, 0, 12, 2, 1, 1)         \
    X(32, 0, 16, 2, 1, 1)         \
    X(40, 0, 20, 2, 1, 1)         \
    X(48, 0, 12, 4, 1, 1)         \
    X(64, 0, 16, 4, 1, 1)         \
    X(80, 0, 20, 4, 1, 1)         \
    X(96, 0, 24, 4, 1, 1)         \
    X(128, 0, 16, 8, 1, 1)        \
    X(192, 0, 24, 8, 1, 1)        \
    X(256, 0, 16, 16, 1, 1)
#define PFT_AXIS_VARIANTS_ALT(X)  \
    X(16, 1, 16, 1, 2, 1)         \
    X(16, 2, 4, 4, 1, 1)          \
    X(24, 1, 12, 2, 2, 1)         \
    X(32, 1, 16, 2, 2, 1)         \
    X(32, 2, 8, 4, 1, 1)          \
    X(40, 1, 20, 2, 2, 1)         \
    X(48, 1, 12, 4, 2, 1)         \
    X(64, 1, 16, 4, 2, 1)         \
    X(64, 2, 8, 8, 1, 1)          \
    X(64, 3, 16, 4, 1, 2)         \
    X(96, 1, 24, 4, 2, 1)         \
    X(128, 1, 16, 8, 2, 1)        \
    X(128, 2, 16, 8, 1, 2)        \
    X(256, 1, 16, 16, 2, 1)
#define PFT_AXIS_VARIANTS(X) PFT_AXIS_VARIANTS0(X) PFT_AXIS_VARIANTS_ALT(X)

// Shape of variant v of axis length n; false if there is none.
inline bool axis_variant(int n, int v, int* n1, int* n2, int* w)
{
#define PFT_CASE(N, VID, A1, A2, WW, MW) \
    if (n == N && v == VID) {         \
        *n1 = A1;                     \
        *n2 = A2;                     \
        *w = WW;                      \
        return true;                  \
    }
    PFT_AXIS_VARIANTS(PFT_CASE)
#undef PFT_CASE
    return false;
}

inline bool axis_supported(int n)
{
    switch (n) {
#define PFT_CASE(N, N1, N2) case N:
        PFT_AXIS_SIZES(PFT_CASE)
#undef PFT_CASE
        return true;
    default:
        return false;
    }
}

// Launchers of one group of variants (default ones in namespace v0, the
// alternatives in namespace alt, each its own translation unit).  The
// strided launchers set ntiles from the variant's tile width.
#define PFT_DECLARE_LAUNCHERS(NS)                                                                        \
    namespace NS {                                                                                     \
    template <typename T>                                                                              \
    hipError_t launch_zpass(int nz, int var, const ZArgs<T>& a, hipStream_t s);                        \
    template <typename T>                                                                              \
    hipError_t launch_spass(int axis, int n, int var, int64_t ncols, SArgs<T> a, int nslabs, hipStream_t s); \
    template <typename T>                                                                              \
    hipError_t launch_zpass_batch(int nz, int var, int64_t nlines, const ZArgs<T>* descs, int nrep,    \
                                  hipStream_t s);                                                      \
    template <typename T>                                                                              \
    hipError_t launch_spass_batch(int axis, int n, int var, int64_t ncols, int nslabs, const SArgs<T>* descs, \
                                  int nrep, hipStream_t s);                                            \
    }
PFT_DECLARE_LAUNCHERS(v0)
PFT_DECLARE_LAUNCHERS(alt)
#undef PFT_DECLARE_LAUNCHERS

// Walled passes (EXT = 1 reflecting, 2 absorbing) over lines of n points,
// for every n of the axis list (default radix split), with the factor tables
// of pair_diffuse().
template <typename T>
hipError_t launch_zpass_walls(int nz, int ext, const ZArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_spass_walls(int axis, int n, int ext, int64_t ncols, SArgs<T> a, int nslabs, hipStream_t s);
bool walls_supported(int n);

// `var` selects the kernel variant of the axis length (0 = default).
template <typename T>
inline hipError_t launch_zpass(int nz, int var, const ZArgs<T>& a, hipStream_t s)
{
    return var == 0 ? v0::launch_zpass<T>(nz, 0, a, s) : alt::launch_zpass<T>(nz, var, a, s);
}
template <typename T>
inline hipError_t launch_spass(int axis, int n, int var, int64_t ncols, SArgs<T> a, int nslabs, hipStream_t s)
{
    return var == 0 ? v0::launch_spass<T>(axis, n, 0, ncols, a, nslabs, s)
                    : alt::launch_spass<T>(axis, n, var, ncols, a, nslabs, s);
}
// Batched launches over `nrep` replicas of one grid (descs: device table of
// nrep argument sets, whose ntiles must match spass_tiles for the variant).
template <typename T>
inline hipError_t launch_zpass_batch(int nz, int var, int64_t nlines, const ZArgs<T>* descs, int nrep, hipStream_t s)
{
    return var == 0 ? v0::launch_zpass_batch<T>(nz, 0, nlines, descs, nrep, s)
                    : alt::launch_zpass_batch<T>(nz, var, nlines, descs, nrep, s);
}
template <typename T>
inline hipError_t launch_spass_batch(int axis, int n, int var, int64_t ncols, int nslabs, const SArgs<T>* descs,
                                     int nrep, hipStream_t s)
{
    return var == 0 ? v0::launch_spass_batch<T>(axis, n, 0, ncols, nslabs, descs, nrep, s)
                    : alt::launch_spass_batch<T>(axis, n, var, ncols, nslabs, descs, nrep, s);
}

// Lanes per line (N2) of an axis length with a kernel, 0 otherwise.
inline int axis_lanes(int n)
{
    switch (n) {
#define PFT_CASE(N, N1, N2) \
    case N:                 \
        return N2;
        PFT_AXIS_SIZES(PFT_CASE)
#undef PFT_CASE
    default:
        return 0;
    }
}

// Column tiles of a strided pass over ncols columns (matches SShape), which
// the batched argument tables must carry.
template <typename T>
inline int spass_tiles(int n, int var, int64_t ncols)
{
    int n1 = 0, n2 = 0, w = 0;
    if (!axis_variant(n, var, &n1, &n2, &w)) return 0;
    const int minc = 128 / int(sizeof(cx<T>));
    const int cols = ((64 / n2 > minc) ? 64 / n2 : minc) * w;
    return (int)((ncols + cols - 1) / cols);
}

}  // namespace pft
