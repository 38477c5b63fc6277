// The contour-weighted q * q-dagger reduction of the densities, Eq. (8), and
// the FP64 helpers it shares with the other reductions.  Kept apart from the
// host runtime so that the kernel's source is only this file and fft.h.
#pragma once

#include <hip/hip_runtime.h>

#include "fft.h"

namespace pft {

// Neumaier-compensated double accumulator.
struct NSum {
    double s = 0.0, c = 0.0;
    __device__ __forceinline__ void add(double x)
    {
        const double t = s + x;
        if (fabs(s) >= fabs(x))
            c += (s - t) + x;
        else
            c += (x - t) + s;
        s = t;
    }
    __device__ __forceinline__ double value() const { return s + c; }
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 cdiv(double2 a, double2 b)
{
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// Contour-weighted q * q-dagger reduction (Eq. (8) divided by rho_0):
// phi_A(x) = (1/Q) sum_{j <= J} tauA_j q_j(x) qd_{K-j}(x), phi_B over j >= J.
// Per-site compensated double sums; each lane owns one site and streams
// through the K+1 slices of both stores.
template <typename T>
__device__ __forceinline__ void density_body(const cx<T>* __restrict__ qs, const cx<T>* __restrict__ qds, int K, int J, int64_t M,
                          const double* __restrict__ tau, const double2* __restrict__ Qp,
                          double2* __restrict__ phiA, double2* __restrict__ phiB, double2* __restrict__ Qout)
{
    const double2 Q = *Qp;
    if (Qout && blockIdx.x == 0 && threadIdx.x == 0) *Qout = Q;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < M; x += (int64_t)gridDim.x * blockDim.x) {
        NSum ar, ai, br, bi;
        for (int j = 0; j <= K; ++j) {
            const cx<T> a = load_stream(qs + (int64_t)j * M + x);
            const cx<T> b = load_stream(qds + (int64_t)(K - j) * M + x);
            const double2 p = cmul(make_double2(a.re, a.im), make_double2(b.re, b.im));
            if (j <= J) {
                const double w = tau[j];
                ar.add(w * p.x);
                ai.add(w * p.y);
            }
            if (j >= J) {
                const double w = tau[K + 1 + j];
                br.add(w * p.x);
                bi.add(w * p.y);
            }
        }
        phiA[x] = cdiv(make_double2(ar.value(), ai.value()), Q);
        phiB[x] = cdiv(make_double2(br.value(), bi.value()), Q);
    }
}

template <typename T>
__global__ void k_density(const cx<T>* __restrict__ qs, const cx<T>* __restrict__ qds, int K, int J, int64_t M,
                          const double* __restrict__ tau, const double2* __restrict__ Qp,
                          double2* __restrict__ phiA, double2* __restrict__ phiB, double2* __restrict__ Qout)
{
    density_body<T>(qs, qds, K, J, M, tau, Qp, phiA, phiB, Qout);
}

}  // namespace pft
