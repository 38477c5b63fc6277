// Box-derivative (stress) terms of the reverse-mode sweep in one pass per
// axis.  The L_a derivative of a diffusion factor exp(-(2 pi m / L_a)^2 h) is
// (2 h / L_a) (2 pi m / L_a)^2 times the factor, so one contour step
// contributes
//   sum_x  sum_i  coef_i  u_i(x) [-d^2/dx_a^2 X_i](x)
// where X_i are the step's captured diffused values (B, the half path after
// its second diffusion; A, after its first; C, the full path before its last
// multiply) and u_i their pointwise partners built from the adjoint vector
// lambda_{j+1}, the captured adjoint-side A and the step's E4 table:
// u_B = E4 lambda, u_A = E2 A_lambda, u_C = E2 lambda (E2 = E4^2).  Each
// kernel applies -d^2/dx_a^2 to the captures along its own lines (forward
// transform, multiply by (2 pi m / L_a)^2 / N_a, inverse) and dots the result
// with the partners at once, so no derivative array is ever written.  Each
// capture has its own row of workgroups (blockIdx.y); every workgroup adds its
// FP64 sum to a partial slot of its own, summed over the steps and reduced
// once at the end.
// Along a walled axis (EXT = 1 reflecting, 2 absorbing) the modes are
// k = pi m / L_a, which scale with 1/L_a as well, so the same sum holds with
// -d^2/dx_a^2 taken in the cosine / sine basis: the line is loaded in the
// reordered, sign-flipped order of the walled passes and transformed with
// the paired factors of (pi m / L_a)^2 / N_a; the dot with the partner runs
// over the same reordered points (the reordering is a permutation and the
// signs square to one), so nothing is reordered back.
#pragma once

#include "kernels.h"

namespace pft {

template <typename T>
struct StressPass {
    const cx<T>* X[3];  // captures B, A, C (the plain split uses X[2] = its z-pass capture only)
    double coef[3];     // their coefficients (h / L_a times 4/3, 4/3, -2/3; plain split 0, 0, 2)
    int first;          // first capture present: 0 (Richardson step) or 2 (plain split)
    const cx<T>* lam;   // lambda_{j+1}
    const cx<T>* Alam;  // the adjoint-side capture A (Richardson step only)
    const cx<T>* E4;    // the step's E4 table
    const T* d2;        // (2 pi m / L_a)^2 / N_a in natural order; walled: the pair
                        // factors (alpha, beta re, beta im) per m of (pi m / L_a)^2 / N_a
    int64_t nlines;     // z pass: lines of nz contiguous points
    int64_t S;          // strided passes: element stride along the lines
    int64_t slab_stride;
    int ncols, ntiles;
    double2* part;      // one slot per workgroup, accumulated
};

// Compensated FP64 sum (Neumaier).
struct CSum {
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

// Workgroup sum in a fixed order; n threads, n a power of two.
__device__ __forceinline__ double2 stress_block_sum(double2 v, double2* red, int n)
{
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int w = n / 2; w > 0; w >>= 1) {
        if (tid < w) {
            red[tid].x += red[tid + w].x;
            red[tid].y += red[tid + w].y;
        }
        __syncthreads();
    }
    return red[0];
}

template <typename T>
__device__ __forceinline__ double2 wide2(cx<T> a)
{
    return make_double2((double)a.re, (double)a.im);
}

__device__ __forceinline__ double2 mul2(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// The partner of capture i at element p.
template <typename T>
__device__ __forceinline__ double2 stress_partner(const StressPass<T>& A, int i, int64_t p)
{
    const double2 e4 = wide2(A.E4[p]);
    if (i == 0) return mul2(e4, wide2(A.lam[p]));
    const double2 e2 = mul2(e4, e4);
    return mul2(e2, wide2(i == 1 ? A.Alam[p] : A.lam[p]));
}

// Lines along z (contiguous), laid out as in the z pass.
template <typename T, int N1, int N2, int EXT>
__global__ __launch_bounds__((ZShape<N1, N2, 1>::kThreads)) void k_stress_z(StressPass<T> A)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double2 red[ZShape<N1, N2, 1>::kThreads];
    cx<T>* sh = reinterpret_cast<cx<T>*>(smem_raw);
    constexpr int N = N1 * N2;
    constexpr int LPW = ZShape<N1, N2, 1>::kLines;
    const int t = threadIdx.x % N2, l = threadIdx.x / N2;
    const int64_t line = (int64_t)blockIdx.x * LPW + l;
    const bool act = line < A.nlines;
    auto pos = [&](int r) { return line * N + ext_index<EXT, N>(r * N2 + t); };
    const LayZ<N1, N2> lay{l};
    const int i = A.first + (int)blockIdx.y;  // one capture per workgroup row
    CSum re, im;
    cx<T> a[N1];
    sfor<0, N1>([&](auto I) {
        constexpr int r = decltype(I)::value;
        a[r] = act ? ext_sign<EXT, N, T>(r * N2 + t) * A.X[i][pos(r)] : cx<T>{T(0), T(0)};
    });
    line_diffuse<EXT, N1, N2>(a, t, sh, lay, A.d2);
    if (act) {
        sfor<0, N1>([&](auto I) {
            constexpr int r = decltype(I)::value;
            const double2 v = mul2(stress_partner(A, i, pos(r)), wide2(ext_sign<EXT, N, T>(r * N2 + t) * a[r]));
            re.add(A.coef[i] * v.x);
            im.add(A.coef[i] * v.y);
        });
    }
    const double2 s = stress_block_sum(make_double2(re.value(), im.value()), red, ZShape<N1, N2, 1>::kThreads);
    if (threadIdx.x == 0) {
        const int64_t k = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
        const double2 o = A.part[k];
        A.part[k] = make_double2(o.x + s.x, o.y + s.y);
    }
}

// Strided lines along x or y, laid out as in the strided passes.
template <typename T, int N1, int N2, int EXT>
__global__ __launch_bounds__((SShape<T, N2, 1>::kThreads)) void k_stress_s(StressPass<T> A)
{
    constexpr int N = N1 * N2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int TC = SShape<T, N2, 1>::kCols;
    constexpr int NT = SShape<T, N2, 1>::kThreads;
    __shared__ double2 red[NT];
    cx<T>* sh = reinterpret_cast<cx<T>*>(smem_raw);
    const int c = threadIdx.x % TC, t = threadIdx.x / TC;
    const int slab = blockIdx.x / A.ntiles, tile = blockIdx.x % A.ntiles;
    const int col = tile * TC + c;
    const bool act = col < A.ncols;
    const int64_t base = (int64_t)slab * A.slab_stride + col;
    auto pos = [&](int r) { return base + (int64_t)ext_index<EXT, N>(r * N2 + t) * A.S; };
    const LayS<N2, TC> lay{c};
    const int i = A.first + (int)blockIdx.y;  // one capture per workgroup row
    CSum re, im;
    cx<T> a[N1];
    sfor<0, N1>([&](auto I) {
        constexpr int r = decltype(I)::value;
        a[r] = act ? ext_sign<EXT, N, T>(r * N2 + t) * A.X[i][pos(r)] : cx<T>{T(0), T(0)};
    });
    line_diffuse<EXT, N1, N2>(a, t, sh, lay, A.d2);
    if (act) {
        sfor<0, N1>([&](auto I) {
            constexpr int r = decltype(I)::value;
            const double2 v = mul2(stress_partner(A, i, pos(r)), wide2(ext_sign<EXT, N, T>(r * N2 + t) * a[r]));
            re.add(A.coef[i] * v.x);
            im.add(A.coef[i] * v.y);
        });
    }
    const double2 s = stress_block_sum(make_double2(re.value(), im.value()), red, NT);
    if (threadIdx.x == 0) {
        const int64_t k = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
        const double2 o = A.part[k];
        A.part[k] = make_double2(o.x + s.x, o.y + s.y);
    }
}

// Launch the stress pass along `axis` (0 x, 1 y, 2 z) on an nx x ny x nz grid
// (periodic axes of a supported length).  The launch uses at most
// stress_blocks() partial slots (workgroups per capture times three).
template <typename T>
hipError_t launch_stress(int axis, int nx, int ny, int nz, StressPass<T> a, hipStream_t s);
// The same along a walled axis (ext = 1 reflecting, 2 absorbing; d2 holds the
// pair factors).
template <typename T>
hipError_t launch_stress_walls(int axis, int ext, int nx, int ny, int nz, StressPass<T> a, hipStream_t s);
template <typename T>
int64_t stress_blocks(int axis, int nx, int ny, int nz);

}  // namespace pft
