// Reciprocal-space filter of the semi-implicit field step, Eqs. (10)-(11):
//   w <- w - IDFT[ DFT(r) / (1 + a g(|k|^2)) ],  g = g0 + gD * g_D(|k|^2),
// on complex double fields.  The multiplier is not separable over the axes,
// so the 3-D spectrum is formed: z forward, y forward, x forward * filter * x
// inverse, y inverse, z inverse with the subtraction from w.  The one-way
// passes hand the spectrum over in natural order; 1/M is applied once in the
// x pass.
#pragma once

#include <hip/hip_runtime.h>

#include "fft.h"
#include "kernels.h"

namespace pft {

enum { kSisFwd = 0, kSisInv = 1, kSisFilter = 2, kSisInvSub = 3 };

struct SisArgs {
    cx<double>* X;          // the work array, transformed in place
    cx<double>* W;          // kSisInvSub: the field receiving w -= IDFT(...)
    int64_t nlines;         // contiguous (z) passes: lines of N points
    int64_t S;              // strided passes: element stride along the lines
    int64_t slab_stride;    //                 distance between slabs of columns
    int ncols, ntiles;      //                 columns per slab, column tiles per slab
    const double* k2x;      // (2 pi m / L)^2 per axis, natural order
    const double* k2y;
    const double* k2z;
    int nz;                 // kSisFilter: columns are (y, z) pairs, col = y nz + z
    double a, g0, gD, inv_M;
};

// Debye function of the whole chain, g_D(x) = 2 (e^-x + x - 1) / x^2; its
// series 2 sum_m (-x)^m / (m+2)! below x = 0.5, where the direct form cancels.
__device__ __forceinline__ double debye_gd(double x)
{
    if (x < 0.5) {
        double term = 1.0, sum = 1.0;
#pragma unroll
        for (int m = 1; m <= 20; ++m) {
            term *= -x / (double)(m + 2);
            sum += term;
        }
        return sum;
    }
    return 2.0 * (exp(-x) + x - 1.0) / (x * x);
}

// Contiguous lines (the z axis), laid out as in the z pass.
template <int N1, int N2, int MODE>
__device__ __forceinline__ void sis_z_body(const SisArgs& A)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<double>* sh = reinterpret_cast<cx<double>*>(smem_raw);
    constexpr int N = N1 * N2;
    constexpr int LPW = ZShape<N1, N2, 1>::kLines;
    const int t = threadIdx.x % N2, l = threadIdx.x / N2;
    const int64_t line = (int64_t)blockIdx.x * LPW + l;
    const bool act = line < A.nlines;
    cx<double>* X = A.X + line * N;
    const LayZ<N1, N2> lay{l};
    cx<double> a[N1];
    if constexpr (MODE == kSisFwd) {
        sfor<0, N1>([&](auto I) {
            a[decltype(I)::value] = act ? X[decltype(I)::value * N2 + t] : cx<double>{0.0, 0.0};
        });
        line_forward<N1, N2>(a, t, sh, lay, [&](int k, cx<double> v) {
            if (act) X[k] = v;
        });
    } else {
        line_inverse<N1, N2>(a, t, sh, lay, [&](int k) { return act ? X[k] : cx<double>{0.0, 0.0}; });
        if (act) {
            cx<double>* W = A.W + line * N;
            sfor<0, N1>([&](auto I) {
                constexpr int i = decltype(I)::value;
                W[i * N2 + t] = W[i * N2 + t] - a[i];
            });
        }
    }
}

template <int N1, int N2, int MODE>
__global__ __launch_bounds__((ZShape<N1, N2, 1>::kThreads)) void k_sis_z(SisArgs A)
{
    sis_z_body<N1, N2, MODE>(A);
}

// Batched form: blockIdx.y selects the array (every array of one launch has
// the same shape).
template <int N1, int N2, int MODE>
__global__ __launch_bounds__((ZShape<N1, N2, 1>::kThreads)) void k_sis_z_batch(const SisArgs* __restrict__ tab)
{
    sis_z_body<N1, N2, MODE>(tab[blockIdx.y]);
}

// Filter factor of one x line: column (y, z) fixed, kx in natural order.
struct SisFactor {
    const double* k2x;
    double k2yz, a, g0, gD, inv_M;
    __device__ __forceinline__ double operator[](int kx) const
    {
        return inv_M / (1.0 + a * (g0 + gD * debye_gd(k2x[kx] + k2yz)));
    }
};

// Strided columns (the x and y axes), laid out as in the strided passes.
template <int N1, int N2, int MODE>
__device__ __forceinline__ void sis_s_body(const SisArgs& A)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<double>* sh = reinterpret_cast<cx<double>*>(smem_raw);
    constexpr int TC = SShape<double, N2, 1>::kCols;
    const int c = threadIdx.x % TC, t = threadIdx.x / TC;
    const int slab = blockIdx.x / A.ntiles, tile = blockIdx.x % A.ntiles;
    const int col = tile * TC + c;
    const bool act = col < A.ncols;
    cx<double>* X = A.X + (int64_t)slab * A.slab_stride + col;
    const LayS<N2, TC> lay{c};
    cx<double> a[N1];
    auto ld = [&]() {
        sfor<0, N1>([&](auto I) {
            a[decltype(I)::value] = act ? X[(int64_t)(decltype(I)::value * N2 + t) * A.S] : cx<double>{0.0, 0.0};
        });
    };
    auto st = [&]() {
        if (act) sfor<0, N1>([&](auto I) { X[(int64_t)(decltype(I)::value * N2 + t) * A.S] = a[decltype(I)::value]; });
    };
    if constexpr (MODE == kSisFwd) {
        ld();
        line_forward<N1, N2>(a, t, sh, lay, [&](int k, cx<double> v) {
            if (act) X[(int64_t)k * A.S] = v;
        });
    } else if constexpr (MODE == kSisInv) {
        line_inverse<N1, N2>(a, t, sh, lay,
                             [&](int k) { return act ? X[(int64_t)k * A.S] : cx<double>{0.0, 0.0}; });
        st();
    } else {
        ld();
        const int y = act ? col / A.nz : 0, z = act ? col % A.nz : 0;
        const SisFactor g{A.k2x, A.k2y[y] + A.k2z[z], A.a, A.g0, A.gD, A.inv_M};
        diffuse<N1, N2>(a, t, sh, lay, g);
        st();
    }
}

template <int N1, int N2, int MODE>
__global__ __launch_bounds__((SShape<double, N2, 1>::kThreads)) void k_sis_s(SisArgs A)
{
    sis_s_body<N1, N2, MODE>(A);
}

template <int N1, int N2, int MODE>
__global__ __launch_bounds__((SShape<double, N2, 1>::kThreads)) void k_sis_s_batch(const SisArgs* __restrict__ tab)
{
    sis_s_body<N1, N2, MODE>(tab[blockIdx.y]);
}

// Launch one pass of the filter on an nx x ny x nz array (FP64): kind 0 =
// z forward, 1 = y forward, 2 = x filter, 3 = y inverse, 4 = z inverse with
// W -= result.
hipError_t launch_sis_pass(int kind, int nx, int ny, int nz, SisArgs a, hipStream_t s);

// Set the line layout fields of a (nlines, S, slab_stride, ncols, ntiles) for
// pass kind on an nx x ny x nz array; false if the axis length has no kernel.
bool sis_pass_layout(int kind, int nx, int ny, int nz, SisArgs* a);

// The same pass over R arrays of one shape: tab (device) holds R argument
// sets with their layout fields set by sis_pass_layout for this kind.
hipError_t launch_sis_pass_batch(int kind, int nx, int ny, int nz, const SisArgs* tab, int R, hipStream_t s);

}  // namespace pft
