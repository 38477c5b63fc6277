// Fused yz-plane pass of the Richardson split step, Eq. (12).
//
// The axis-pass schedule runs one contour step as Z, Y1, X, Y2 (see
// kernels.h).  Between two x passes the work arrays go through Y2 (of the
// step being completed), Z (which completes it and starts the next) and Y1
// (of the next step).  All three act inside one x-plane (fixed x, all y and
// z), so where a whole yz-plane fits in LDS one workgroup runs the three for
// its plane with the data on chip:
//
//   U   = Dz_{h/2} Dy_{h/2} U                 (y, then z, of the completed step)
//   q'  = (4 E4 U - V) / 3                    (stored; V is the full-step path)
//   U   = Dy_{h/2} Dz_{h/2} (E4 q'),  V = Dy_h Dz_h (E2 q')   (next step)
//
// and the step becomes two memory passes (this one and X) moving 11 arrays
// per grid point instead of 17.  The plain split is the same without U:
// q' = E2 V, V = Dy_h Dz_h (E2 q').
//
// Layouts inside a plane (ny = nz = N = N1 * N2, TPB = N * N2 per plane):
//  - column layout (y transforms): lane (ty, c) holds y = n1 * N2 + ty of
//    column z = c; global accesses are 64 consecutive z per wavefront;
//  - row layout (z transforms): lane (r, tz) holds z = n1 * N2 + tz of row
//    y = r, as in the z pass.
// Between the two the plane goes through LDS (row pitch RP elements, chosen
// so that two consecutive rows start half the 32 banks apart), and the same
// buffer serves as the exchange space of every line transform.
#pragma once

#include <hip/hip_runtime.h>

#include "fft.h"
#include "kernels.h"

namespace pft {

template <typename T>
struct PArgs {
    int skip;        // batched launches: this replica has no work at this position
    int nplanes;     // nx
    cx<T>* U;
    cx<T>* V;
    const cx<T>* qin;  // start value when there is no previous step (NULL: q = 1)
    cx<T>* qout;       // where the completed q is stored (NULL: not stored)
    int has_prev, has_next, scheme;
    const cx<T>* Ep;   // E4 table of the step being completed (NULL: E = 1)
    const T* gyh_p;    // its y and z factors for h/2
    const T* gzh_p;
    const cx<T>* En;   // E4 table of the step being started (NULL: E = 1)
    const T* gzh_n;    // its z factors for h/2 and h
    const T* gzf_n;
    const T* gyh_n;    // its y factors for h/2 and h
    const T* gyf_n;
    cx<T>* hcap;       // if set: the completed step's last diffused value before its final
                       // field multiply (reverse-mode sweep), as in the z pass
};

constexpr int kPlaneMaxLds = 160 * 1024;

// Smallest pitch >= base whose dword stride is 16 modulo 32 (rows r and r + 1
// on opposite halves of the banks).
template <typename T>
constexpr int plane_pitch(int base)
{
    constexpr int dw = int(sizeof(cx<T>) / 4);
    int p = base;
    while ((p * dw) % 32 != 16) ++p;
    return p;
}

template <typename T, int N1, int N2>
struct PShape {
    static constexpr int N = N1 * N2;
    static constexpr int kPlaneThreads = N * N2;
    // padded row exchange (k1 * (N2 + 1) + n2) when the plane still fits
    static constexpr int kRPpad = plane_pitch<T>(N1 * (N2 + 1) > N ? N1 * (N2 + 1) : N);
    static constexpr bool kPad = (N2 > 1) && (int64_t)N * kRPpad * (int64_t)sizeof(cx<T>) <= kPlaneMaxLds;
    static constexpr int kRP = kPad ? kRPpad : plane_pitch<T>(N);
    static constexpr int64_t kPlaneBytes = (int64_t)N * kRP * (int64_t)sizeof(cx<T>);
    static constexpr bool kFits = kPlaneBytes <= kPlaneMaxLds;
    // several small planes per workgroup, up to 256 threads and 64 KB
    static constexpr int kPW0 = kPlaneThreads >= 256 ? 1 : 256 / kPlaneThreads;
    static constexpr int kPWlds = kPlaneBytes >= 65536 ? 1 : int(65536 / kPlaneBytes);
    static constexpr int kPW = kPW0 < kPWlds ? kPW0 : kPWlds;
    static constexpr int kThreads = kPW * kPlaneThreads;
    // Register bound of the batched kernel (minimum waves per SIMD): the
    // complex-float 40^2 pass (20 x 2 lines) runs at three waves per SIMD
    // (168 registers, a 76-byte spill) instead of two (207 registers): the
    // 256-replica field step 41.6 -> 40.8 ms (both forms timed alternately on one device).
    static constexpr int kBatchMinWaves = (std::is_same<T, float>::value && N1 == 20 && N2 == 2) ? 3 : 1;
    static constexpr int64_t kLdsBytes = kPW * kPlaneBytes;
};

template <int N2, int RP>
struct LayCol {
    int c;
    __device__ __forceinline__ int operator()(int k1, int n2) const { return (k1 * N2 + n2) * RP + c; }
};

template <int N2, int RP, int PAD>
struct LayRow {
    int r;
    __device__ __forceinline__ int operator()(int k1, int n2) const { return r * RP + k1 * (N2 + PAD) + n2; }
};

// EY, EZ: walls along y and z (0 periodic, 1 reflecting, 2 absorbing).  A
// walled line is held in the order of pair_diffuse() (register n: physical
// point ext_index(n), times ext_sign(n)); the reorder lives in the address
// maps: the column layout holds y in walled order, the row layout z, and the
// plane buffer between the two holds both axes in physical order, unsigned.
template <typename T, int N1, int N2, int EY = 0, int EZ = 0>
__device__ __forceinline__ void yzpass_body(const PArgs<T>& A, unsigned bid, cx<T>* smem)
{
    using S = PShape<T, N1, N2>;
    constexpr int N = S::N, RP = S::kRP;
    const int pw = threadIdx.x / S::kPlaneThreads;
    const int lt = threadIdx.x % S::kPlaneThreads;
    const int plane = (int)bid * S::kPW + pw;
    const bool act = plane < A.nplanes;
    cx<T>* sh = smem + pw * N * RP;
    const int64_t pbase = (int64_t)plane * N * N;
    const int c = lt % N, ty = lt / N;   // column layout
    const int r = lt / N2, tz = lt % N2;  // row layout
    // in-plane offsets stay 32-bit so that the plane base can live in scalar registers
    const int co = ty * N + c;
    const int ro = r * N + tz;
    const LayCol<N2, RP> lay_c{c};
    const LayRow<N2, RP, S::kPad ? 1 : 0> lay_r{r};
    // physical y of column register i and physical z of row register i, with
    // their signs (all identity without walls)
    auto cy = [&](int i) { return ext_index<EY, N>(i * N2 + ty); };
    auto rz = [&](int i) { return ext_index<EZ, N>(i * N2 + tz); };
    auto sy = [&](int i) { return ext_sign<EY, N, T>(i * N2 + ty); };
    auto sz = [&](int i) { return ext_sign<EZ, N, T>(i * N2 + tz); };

    auto ldc = [&](const cx<T>* p, cx<T>(&a)[N1]) {
        const cx<T>* P = p + pbase;
        if (act) {
            if constexpr (EY == 0)
                sfor<0, N1>([&](auto I) { a[decltype(I)::value] = P[co + decltype(I)::value * N2 * N]; });
            else
                sfor<0, N1>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    a[i] = sy(i) * P[cy(i) * N + c];
                });
        } else {
            sfor<0, N1>([&](auto I) { a[decltype(I)::value] = cx<T>{T(0), T(0)}; });
        }
    };
    auto stc = [&](cx<T>* p, const cx<T>(&a)[N1]) {
        cx<T>* P = p + pbase;
        if (!act) return;
        if constexpr (EY == 0)
            sfor<0, N1>([&](auto I) { P[co + decltype(I)::value * N2 * N] = a[decltype(I)::value]; });
        else
            sfor<0, N1>([&](auto I) {
                constexpr int i = decltype(I)::value;
                P[cy(i) * N + c] = sy(i) * a[i];
            });
    };
    // row layout; `sign` false for the field tables
    auto ldr = [&](const cx<T>* p, cx<T>(&a)[N1], bool sign = true) {
        const cx<T>* P = p + pbase;
        if (act) {
            if constexpr (EZ == 0)
                sfor<0, N1>([&](auto I) { a[decltype(I)::value] = P[ro + decltype(I)::value * N2]; });
            else
                sfor<0, N1>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    const cx<T> x = P[r * N + rz(i)];
                    a[i] = sign ? sz(i) * x : x;
                });
        } else {
            sfor<0, N1>([&](auto I) { a[decltype(I)::value] = cx<T>{T(0), T(0)}; });
        }
    };
    auto str = [&](cx<T>* p, const cx<T>(&a)[N1]) {
        cx<T>* P = p + pbase;
        if (!act) return;
        if constexpr (EZ == 0)
            sfor<0, N1>([&](auto I) { P[ro + decltype(I)::value * N2] = a[decltype(I)::value]; });
        else
            sfor<0, N1>([&](auto I) {
                constexpr int i = decltype(I)::value;
                P[r * N + rz(i)] = sz(i) * a[i];
            });
    };
    // column layout -> row layout through the plane buffer, and back
    auto to_rows = [&](cx<T>(&a)[N1]) {
        __syncthreads();
        sfor<0, N1>([&](auto I) {
            constexpr int i = decltype(I)::value;
            sh[cy(i) * RP + c] = sy(i) * a[i];
        });
        __syncthreads();
        sfor<0, N1>([&](auto I) {
            constexpr int i = decltype(I)::value;
            a[i] = sz(i) * sh[r * RP + rz(i)];
        });
    };
    auto to_cols = [&](cx<T>(&a)[N1]) {
        __syncthreads();
        sfor<0, N1>([&](auto I) {
            constexpr int i = decltype(I)::value;
            sh[r * RP + rz(i)] = sz(i) * a[i];
        });
        __syncthreads();
        sfor<0, N1>([&](auto I) {
            constexpr int i = decltype(I)::value;
            a[i] = sy(i) * sh[cy(i) * RP + c];
        });
    };

    cx<T> q[N1];
    cx<T> e[N1];
    bool have_e = false;
    if (A.has_prev) {
        if (A.scheme == kSchemeRQM4) {
            ldc(A.U, q);
            // Complex-float planes below 1024 lanes load V for the combine now, so
            // that it arrives during U's transforms (256-replica batch: 43.4
            // against 45.0 ms per field step); the 128^2 pass has no registers
            // to spare for it (its spill grew from 64 to 84 bytes per lane and
            // the pass slowed by 2%).
            constexpr bool kEarlyV = std::is_same<T, float>::value && S::kPlaneThreads < 1024;
            cx<T> v[N1];
            if constexpr (kEarlyV) ldr(A.V, v);
            line_diffuse<EY, N1, N2, true>(q, ty, sh, lay_c, A.gyh_p);
            to_rows(q);
            line_diffuse<EZ, N1, N2, true>(q, tz, sh, lay_r, A.gzh_p);
            if (A.hcap) str(A.hcap, q);
            const cx<T>* Vp = A.V + pbase;
            if (A.Ep) {
                ldr(A.Ep, e, false);
                have_e = true;
            }
            sfor<0, N1>([&](auto I) {
                constexpr int i = decltype(I)::value;
                cx<T> vi;
                if constexpr (kEarlyV)
                    vi = v[i];
                else if constexpr (EZ == 0)
                    vi = act ? Vp[ro + i * N2] : cx<T>{T(0), T(0)};
                else
                    vi = act ? sz(i) * Vp[r * N + rz(i)] : cx<T>{T(0), T(0)};
                const cx<T> u = A.Ep ? q[i] * e[i] : q[i];
                q[i] = richardson(u, vi);
            });
        } else {
            ldr(A.V, q);
            if (A.hcap) str(A.hcap, q);
            if (A.Ep) {
                ldr(A.Ep, e, false);
                have_e = true;
                sfor<0, N1>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    q[i] = q[i] * (e[i] * e[i]);
                });
            }
        }
    } else if (A.qin) {
        ldr(A.qin, q);
    } else {
        // q = 1, in the signed walled order of the row layout
        sfor<0, N1>([&](auto I) { q[decltype(I)::value] = sz(decltype(I)::value) * cx<T>{T(1), T(0)}; });
    }
    if (A.qout) str(A.qout, q);

    if (A.has_next) {
        cx<T> w[N1];
        if (A.En) {
            if (!(have_e && A.En == A.Ep)) ldr(A.En, e, false);
            sfor<0, N1>([&](auto I) {
                constexpr int i = decltype(I)::value;
                q[i] = q[i] * e[i];
                w[i] = q[i] * e[i];
            });
        } else {
            sfor<0, N1>([&](auto I) { w[decltype(I)::value] = q[decltype(I)::value]; });
        }
        if (A.scheme == kSchemeRQM4) {
            line_diffuse<EZ, N1, N2, true>(q, tz, sh, lay_r, A.gzh_n);
            to_cols(q);
            line_diffuse<EY, N1, N2, true>(q, ty, sh, lay_c, A.gyh_n);
            stc(A.U, q);
        }
        line_diffuse<EZ, N1, N2, true>(w, tz, sh, lay_r, A.gzf_n);
        to_cols(w);
        line_diffuse<EY, N1, N2, true>(w, ty, sh, lay_c, A.gyf_n);
        stc(A.V, w);
    }
}

template <typename T, int N1, int N2>
__global__ __launch_bounds__((PShape<T, N1, N2>::kThreads)) void k_yzpass(PArgs<T> A)
{
    __shared__ __align__(16) unsigned char smem_raw[PShape<T, N1, N2>::kLdsBytes];
    yzpass_body<T, N1, N2>(A, blockIdx.x, reinterpret_cast<cx<T>*>(smem_raw));
}

template <typename T, int N1, int N2>
__global__ __launch_bounds__((PShape<T, N1, N2>::kThreads), (PShape<T, N1, N2>::kBatchMinWaves)) void k_yzpass_batch(
    const PArgs<T>* __restrict__ descs)
{
    __shared__ __align__(16) unsigned char smem_raw[PShape<T, N1, N2>::kLdsBytes];
    const PArgs<T> A = descs[blockIdx.y];
    if (A.skip) return;
    yzpass_body<T, N1, N2>(A, blockIdx.x, reinterpret_cast<cx<T>*>(smem_raw));
}

// The fused pass between walls along y and/or z (EY, EZ not both 0).
template <typename T, int N1, int N2, int EY, int EZ>
__global__ __launch_bounds__((PShape<T, N1, N2>::kThreads)) void k_yzpass_walls(PArgs<T> A)
{
    __shared__ __align__(16) unsigned char smem_raw[PShape<T, N1, N2>::kLdsBytes];
    yzpass_body<T, N1, N2, EY, EZ>(A, blockIdx.x, reinterpret_cast<cx<T>*>(smem_raw));
}

// Plane sizes N (= ny = nz) with a fused kernel per precision, as (N, N1, N2):
// the default axis splits whose padded plane fits in LDS.
#define PFT_PLANE_SIZES_F32(X) \
    X(8, 8, 1)                 \
    X(12, 12, 1)               \
    X(16, 16, 1)               \
    X(20, 20, 1)               \
    X(24, 12, 2)               \
    X(32, 16, 2)               \
    X(40, 20, 2)               \
    X(48, 12, 4)               \
    X(64, 16, 4)               \
    X(80, 20, 4)               \
    X(96, 24, 4)               \
    X(128, 16, 8)
#define PFT_PLANE_SIZES_F64(X) \
    X(8, 8, 1)                 \
    X(12, 12, 1)               \
    X(16, 16, 1)               \
    X(20, 20, 1)               \
    X(24, 12, 2)               \
    X(32, 16, 2)               \
    X(40, 20, 2)               \
    X(48, 12, 4)               \
    X(64, 16, 4)               \
    X(80, 20, 4)               \
    X(96, 24, 4)

// True if the fused pass exists for a square yz-plane of side n.
template <typename T>
bool plane_supported(int n);

// Private (register spill) bytes per lane of the compiled fused kernel for side
// n, -1 if there is none or the runtime cannot say.
template <typename T>
int plane_private_bytes(int n);

// The walled fused pass (complex float only): whether it exists for side n,
// its spill bytes per lane (-1: none), and its launch; ey, ez in 0..2, not
// both 0.  Each wall kind along z is its own translation unit.
bool plane_walls_supported(int n);
int plane_walls_private_bytes(int n, int ey, int ez);
hipError_t launch_yzpass_walls(int n, int ey, int ez, const PArgs<float>& a, hipStream_t s);
template <int EZ>
int plane_walls_private_bytes_z(int n, int ey);
template <int EZ>
hipError_t launch_yzpass_walls_z(int n, int ey, const PArgs<float>& a, hipStream_t s);

// Launch over nx planes (a.nplanes), or over nrep replicas of one shape.
template <typename T>
hipError_t launch_yzpass(int n, const PArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_yzpass_batch(int n, int nplanes, const PArgs<T>* descs, int nrep, hipStream_t s);

}  // namespace pft
