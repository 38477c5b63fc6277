// Host runtime and C ABI of the propagator library (see include/pft.h), plus
// the elementwise and reduction kernels around the axis passes: field
// operator tables, the contour-weighted q * q-dagger reduction, Q, H, the
// Euler-Maruyama field step and its Philox4x64-10 noise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pft.h"
#include "density.h"
#include "kernels.h"
#include "planes.h"
#include "sis.h"
#include "stress.h"
#include "walls_batch.h"

using pft::cdiv;
using pft::cmul;
using pft::cx;
using pft::density_body;
using pft::k_density;
using pft::NSum;

namespace pft {
thread_local LaunchEvents g_launch_events;
}

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kPi = 3.1415926535897932384626433832795;

// ============================================================ device code ==

constexpr int kRedThreads = 256;

// Fixed-order tree sum over the block (deterministic).
__device__ __forceinline__ double2 block_sum(double2 v, double2* sh)
{
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if (tid < w) {
            sh[tid].x += sh[tid + w].x;
            sh[tid].y += sh[tid + w].y;
        }
        __syncthreads();
    }
    return sh[0];
}

// Field operator tables E = exp(-w_b a) for up to four (block, a) pairs,
// evaluated in double and rounded once to the working precision.
struct TabDesc {
    int n;
    int blk[4];
    double a[4];
};

template <typename T>
__device__ __forceinline__ void field_tables_body(const double2* __restrict__ wp, const double2* __restrict__ wm, int64_t M,
                               TabDesc d, cx<T>* __restrict__ out)
{
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < M; x += (int64_t)gridDim.x * blockDim.x) {
        const double2 p = wp[x], m = wm ? wm[x] : make_double2(0.0, 0.0);
        // w_A = i w_+ - w_-, w_B = i w_+ + w_- (no w_- array: w_- = 0, the Edwards field i omega)
        const double2 wA = make_double2(-p.y - m.x, p.x - m.y);
        const double2 wB = make_double2(-p.y + m.x, p.x + m.y);
        for (int k = 0; k < d.n; ++k) {
            const double2 w = d.blk[k] == 0 ? wA : wB;
            const double mag = exp(-w.x * d.a[k]);
            double s, c;
            sincos(-w.y * d.a[k], &s, &c);
            out[(int64_t)k * M + x] = cx<T>{T(mag * c), T(mag * s)};
        }
    }
}

template <typename T>
__global__ void k_field_tables(const double2* __restrict__ wp, const double2* __restrict__ wm, int64_t M,
                               TabDesc d, cx<T>* __restrict__ out)
{
    field_tables_body<T>(wp, wm, M, d, out);
}

template <typename T>
__global__ void k_to_work(const double2* __restrict__ in, cx<T>* __restrict__ out, int64_t M)
{
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < M; x += (int64_t)gridDim.x * blockDim.x)
        out[x] = cx<T>{T(in[x].x), T(in[x].y)};
}

template <typename T>
__global__ void k_from_work(const cx<T>* __restrict__ in, double2* __restrict__ out, int64_t M)
{
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < M; x += (int64_t)gridDim.x * blockDim.x)
        out[x] = make_double2(double(in[x].re), double(in[x].im));
}

// Partial sums (one per block) of a complex array, compensated.
template <typename T>
__device__ __forceinline__ void sum_partials_body(const cx<T>* __restrict__ x, int64_t n,
                                                              double2* __restrict__ partials)
{
    __shared__ double2 sh[kRedThreads];
    NSum re, im;
    for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads) {
        re.add(double(x[i].re));
        im.add(double(x[i].im));
    }
    const double2 s = block_sum(make_double2(re.value(), im.value()), sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_sum_partials(const cx<T>* __restrict__ x, int64_t n,
                                                              double2* __restrict__ partials)
{
    sum_partials_body<T>(x, n, partials);
}

// Per-node sums of q_j * qd_{K-j}: blockIdx.y is the node.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_nodeq_partials(const cx<T>* __restrict__ qs,
                                                                const cx<T>* __restrict__ qds, int K, int64_t M,
                                                                double2* __restrict__ partials)
{
    __shared__ double2 sh[kRedThreads];
    const int j = blockIdx.y;
    const cx<T>* a = qs + (int64_t)j * M;
    const cx<T>* b = qds + (int64_t)(K - j) * M;
    NSum re, im;
    for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < M; i += (int64_t)gridDim.x * kRedThreads) {
        const double2 p = cmul(make_double2(a[i].re, a[i].im), make_double2(b[i].re, b[i].im));
        re.add(p.x);
        im.add(p.y);
    }
    const double2 s = block_sum(make_double2(re.value(), im.value()), sh);
    if (threadIdx.x == 0) partials[(int64_t)j * gridDim.x + blockIdx.x] = s;
}

// Final reduction of nrows rows of np partials each: out[r] = scale * sum.
// Optionally flags a non-finite result (bit 0) and mirrors row 0 to out2.
__device__ __forceinline__ void final_sum_body(const double2* __restrict__ partials, int np,
                                                           double scale, double2* __restrict__ out,
                                                           double2* __restrict__ out2, uint32_t* flags)
{
    __shared__ double2 sh[kRedThreads];
    const int r = blockIdx.x;
    NSum re, im;
    for (int i = threadIdx.x; i < np; i += kRedThreads) {
        re.add(partials[(int64_t)r * np + i].x);
        im.add(partials[(int64_t)r * np + i].y);
    }
    const double2 s = block_sum(make_double2(re.value(), im.value()), sh);
    if (threadIdx.x == 0) {
        const double2 v = make_double2(s.x * scale, s.y * scale);
        out[r] = v;
        if (out2 && r == 0) *out2 = v;
        if (flags && !(isfinite(v.x) && isfinite(v.y)) ) atomicOr(flags, 1u);
    }
}

__global__ __launch_bounds__(kRedThreads) void k_final_sum(const double2* __restrict__ partials, int np,
                                                           double scale, double2* __restrict__ out,
                                                           double2* __restrict__ out2, uint32_t* flags)
{
    final_sum_body(partials, np, scale, out, out2, flags);
}

// Contour sum on the fly (stored-product storage modes): node pair (j, K-j)
// adds tau^A_j q_j qd_{K-j} and tau^B_j q_j qd_{K-j} to FP64 accumulators
// (first: overwrite).
template <typename T>
__global__ void k_accum_node(const cx<T>* __restrict__ q, const cx<T>* __restrict__ qd, int64_t M, double ta,
                             double tb, double2* __restrict__ accA, double2* __restrict__ accB, int first)
{
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < M; x += (int64_t)gridDim.x * blockDim.x) {
        const cx<T> a = q[x], b = qd[x];
        const double2 p = cmul(make_double2(a.re, a.im), make_double2(b.re, b.im));
        double2 A = make_double2(ta * p.x, ta * p.y), Bv = make_double2(tb * p.x, tb * p.y);
        if (!first) {
            const double2 a0 = accA[x], b0 = accB[x];
            A = make_double2(a0.x + A.x, a0.y + A.y);
            Bv = make_double2(b0.x + Bv.x, b0.y + Bv.y);
        }
        accA[x] = A;
        accB[x] = Bv;
    }
}

// phi = accumulated contour sum / Q.
__global__ void k_norm_density(const double2* __restrict__ accA, const double2* __restrict__ accB, int64_t M,
                               const double2* __restrict__ Qp, double2* __restrict__ phiA, double2* __restrict__ phiB,
                               double2* __restrict__ Qout)
{
    const double2 Q = *Qp;
    if (Qout && blockIdx.x == 0 && threadIdx.x == 0) *Qout = Q;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < M; x += (int64_t)gridDim.x * blockDim.x) {
        phiA[x] = cdiv(accA[x], Q);
        phiB[x] = cdiv(accB[x], Q);
    }
}

// Partial sums of w_-^2 / chiN - i w_+ (the local part of Eq. (3)).
__device__ __forceinline__ void ham_partials_body(const double2* __restrict__ wp,
                                                              const double2* __restrict__ wm, int64_t M,
                                                              double inv_chiN, double2* __restrict__ partials)
{
    __shared__ double2 sh[kRedThreads];
    NSum re, im;
    for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < M; i += (int64_t)gridDim.x * kRedThreads) {
        const double2 m = wm[i], p = wp ? wp[i] : make_double2(0.0, 0.0);
        const double2 m2 = cmul(m, m);
        re.add(m2.x * inv_chiN + p.y);
        im.add(m2.y * inv_chiN - p.x);
    }
    const double2 s = block_sum(make_double2(re.value(), im.value()), sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRedThreads) void k_ham_partials(const double2* __restrict__ wp,
                                                              const double2* __restrict__ wm, int64_t M,
                                                              double inv_chiN, double2* __restrict__ partials)
{
    ham_partials_body(wp, wm, M, inv_chiN, partials);
}

// H = C dV S - C V Log Q (principal branch), h = H / (C V).
__device__ __forceinline__ void ham_final_body(const double2* __restrict__ partials, int np, double C,
                                                           double dV, double V, const double2* __restrict__ Qp,
                                                           double2* __restrict__ H, double2* __restrict__ hint,
                                                           double2* __restrict__ Sout)
{
    __shared__ double2 sh[kRedThreads];
    NSum re, im;
    for (int i = threadIdx.x; i < np; i += kRedThreads) {
        re.add(partials[i].x);
        im.add(partials[i].y);
    }
    const double2 s = block_sum(make_double2(re.value(), im.value()), sh);
    if (threadIdx.x == 0) {
        const double2 Q = *Qp;
        const double lr = 0.5 * log(Q.x * Q.x + Q.y * Q.y);
        const double li = atan2(Q.y, Q.x);
        const double2 h = make_double2(C * dV * s.x - C * V * lr, C * dV * s.y - C * V * li);
        *H = h;
        if (hint) *hint = make_double2(h.x / (C * V), h.y / (C * V));
        if (Sout) *Sout = s;
    }
}

__global__ __launch_bounds__(kRedThreads) void k_ham_final(const double2* __restrict__ partials, int np, double C,
                                                           double dV, double V, const double2* __restrict__ Qp,
                                                           double2* __restrict__ H, double2* __restrict__ hint,
                                                           double2* __restrict__ Sout)
{
    ham_final_body(partials, np, C, dV, V, Qp, H, hint, Sout);
}

// ------------------------------------------------------------ Philox noise --
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64 -> 128-bit products with a Weyl-sequence key schedule.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// Four standard normals for sites 4g..4g+3 of one field: counter (g, field,
// step, 0), key (seed, replica); Box-Muller on (u0,u1) and (u2,u3), with
// u = ((bits >> 11) + 1/2) 2^-53 never zero.
__device__ __forceinline__ void normals4(uint64_t g, int field, uint64_t step, uint64_t seed, uint64_t rep,
                                         double z[4])
{
    uint64_t c[4] = {g, (uint64_t)field, step, 0};
    philox4x64_10(c, seed, rep);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const double a = ((double)(c[2 * p] >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        const double b = ((double)(c[2 * p + 1] >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        const double rad = sqrt(-2.0 * log(a));
        double s, co;
        sincos(kTwoPi * b, &s, &co);
        z[2 * p] = rad * co;
        z[2 * p + 1] = rad * s;
    }
}

__global__ void k_noise_words(uint64_t seed, uint64_t rep, uint64_t step, int field, int64_t ngroups,
                              uint64_t* __restrict__ out)
{
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ngroups; g += (int64_t)gridDim.x * blockDim.x) {
        uint64_t c[4] = {(uint64_t)g, (uint64_t)field, step, 0};
        philox4x64_10(c, seed, rep);
        for (int r = 0; r < 4; ++r) out[4 * g + r] = c[r];
    }
}

__global__ void k_noise_normals(uint64_t seed, uint64_t rep, uint64_t step, int field, int64_t M,
                                double* __restrict__ out)
{
    const int64_t ng = (M + 3) / 4;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += (int64_t)gridDim.x * blockDim.x) {
        double z[4];
        normals4(g, field, step, seed, rep, z);
        for (int r = 0; r < 4 && 4 * g + r < M; ++r) out[4 * g + r] = z[r];
    }
}

// Explicit Euler-Maruyama field step, Eq. (9), in place, one lane per block
// of four sites: F_+ = i (phi_A + phi_B - 1), F_- = 2 w_-/chiN + phi_B - phi_A.
struct UpdArgs {
    double2* wp;
    double2* wm;
    const double2* phiA;
    const double2* phiB;
    int64_t M;
    double two_over_chiN, dtp, dtm, sp, sm;
    int noise;
    uint64_t seed, rep, step;
    int edwards;       // Edwards model: wp holds omega, F = b_over_c omega + i phiA, wm untouched
    double b_over_c;
};

__device__ __forceinline__ void update_body(UpdArgs a)
{
    const int64_t ng = (a.M + 3) / 4;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += (int64_t)gridDim.x * blockDim.x) {
        double zp[4] = {0, 0, 0, 0}, zm[4] = {0, 0, 0, 0};
        if (a.noise) {
            normals4(g, 0, a.step, a.seed, a.rep, zp);
            if (!a.edwards) normals4(g, 1, a.step, a.seed, a.rep, zm);
        }
        for (int r = 0; r < 4; ++r) {
            const int64_t x = 4 * g + r;
            if (x >= a.M) break;
            if (a.edwards) {
                const double2 ph = a.phiA[x], om = a.wp[x];
                const double2 F = make_double2(a.b_over_c * om.x - ph.y, a.b_over_c * om.y + ph.x);
                a.wp[x] = make_double2(om.x - a.dtp * F.x + a.sp * zp[r], om.y - a.dtp * F.y);
                continue;
            }
            const double2 pa = a.phiA[x], pb = a.phiB[x], p = a.wp[x], m = a.wm[x];
            // F_+ = i (phi - 1)
            const double2 Fp = make_double2(-(pa.y + pb.y), pa.x + pb.x - 1.0);
            const double2 Fm = make_double2(a.two_over_chiN * m.x + pb.x - pa.x, a.two_over_chiN * m.y + pb.y - pa.y);
            a.wp[x] = make_double2(p.x - a.dtp * Fp.x + a.sp * zp[r], p.y - a.dtp * Fp.y);
            a.wm[x] = make_double2(m.x - a.dtm * Fm.x + a.sm * zm[r], m.y - a.dtm * Fm.y);
        }
    }
}

__global__ void k_update(UpdArgs a)
{
    update_body(a);
}

// Semi-implicit step, local part: the explicit increment r = lam dt F - s xi of
// the field filtered in reciprocal space (w_+, or the Edwards omega) goes to R;
// the diblock's w_- is updated here, its implicit linear term 2/chiN making
// the filter a constant: w_- <- w_- - (lam dt F_- - s xi) / (1 + 2 lam dt / chiN).
struct SisIncArgs {
    const double2* wp;
    double2* wm;
    const double2* phiA;
    const double2* phiB;
    double2* R;
    int64_t M;
    double two_over_chiN, ap, am, sp, sm, den_m;
    int noise;
    uint64_t seed, rep, step;
    const uint64_t* step_dev;  // if set, *step_dev is added to step (graph-replayed batches)
    int edwards;
    double b_over_c;
};

__device__ __forceinline__ void sis_increment_body(SisIncArgs a)
{
    if (a.step_dev) a.step += *a.step_dev;
    const int64_t ng = (a.M + 3) / 4;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += (int64_t)gridDim.x * blockDim.x) {
        double zp[4] = {0, 0, 0, 0}, zm[4] = {0, 0, 0, 0};
        if (a.noise) {
            normals4(g, 0, a.step, a.seed, a.rep, zp);
            if (!a.edwards) normals4(g, 1, a.step, a.seed, a.rep, zm);
        }
        for (int r = 0; r < 4; ++r) {
            const int64_t x = 4 * g + r;
            if (x >= a.M) break;
            const double2 pa = a.phiA[x], p = a.wp[x];
            if (a.edwards) {
                const double2 F = make_double2(a.b_over_c * p.x - pa.y, a.b_over_c * p.y + pa.x);
                a.R[x] = make_double2(a.ap * F.x - a.sp * zp[r], a.ap * F.y);
                continue;
            }
            const double2 pb = a.phiB[x], m = a.wm[x];
            const double2 Fp = make_double2(-(pa.y + pb.y), pa.x + pb.x - 1.0);
            const double2 Fm = make_double2(a.two_over_chiN * m.x + pb.x - pa.x, a.two_over_chiN * m.y + pb.y - pa.y);
            a.R[x] = make_double2(a.ap * Fp.x - a.sp * zp[r], a.ap * Fp.y);
            a.wm[x] = make_double2(m.x - (a.am * Fm.x - a.sm * zm[r]) / a.den_m, m.y - a.am * Fm.y / a.den_m);
        }
    }
}

__global__ void k_sis_increment(SisIncArgs a) { sis_increment_body(a); }

// Batched form: blockIdx.y is the replica.
__global__ void k_sis_increment_batch(const SisIncArgs* __restrict__ jobs) { sis_increment_body(jobs[blockIdx.y]); }

// Between reflecting walls the filter runs on the even mirror image of the
// increment, of period 2L along each walled axis (ne = 2n there), where the
// Fourier basis is the cosine basis of the walled box: X = image of R, W = 0.
struct MirrorArgs {
    const double2* R;
    double2* X;
    double2* W;
    int n[3], ne[3];
    int64_t Me;
};

__device__ __forceinline__ void sis_mirror_body(const MirrorArgs& a)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < a.Me; e += (int64_t)gridDim.x * blockDim.x) {
        const int ze = (int)(e % a.ne[2]);
        const int ye = (int)((e / a.ne[2]) % a.ne[1]);
        const int xe = (int)(e / ((int64_t)a.ne[1] * a.ne[2]));
        const int x = xe < a.n[0] ? xe : 2 * a.n[0] - 1 - xe;
        const int y = ye < a.n[1] ? ye : 2 * a.n[1] - 1 - ye;
        const int z = ze < a.n[2] ? ze : 2 * a.n[2] - 1 - ze;
        a.X[e] = a.R[((int64_t)x * a.n[1] + y) * a.n[2] + z];
        a.W[e] = make_double2(0.0, 0.0);
    }
}

__global__ void k_sis_mirror(MirrorArgs a) { sis_mirror_body(a); }

// |k|^2 = (2 pi m / Le)^2 per axis in natural order (m = j, or j - ne above
// ne / 2), Le the period the filter sees (2L along a reflecting axis): row
// blockIdx.x of k2.  The same operations, in the same order, as the host
// table of the context's semi-implicit step.
struct K2Rows {
    int ne[3];
    double Le[3];
};

__global__ void k_fill_k2(double* __restrict__ k2, int pitch, K2Rows r)
{
    const int ax = blockIdx.x;
    for (int j = threadIdx.x; j < r.ne[ax]; j += blockDim.x) {
        const int m = (j <= r.ne[ax] / 2) ? j : j - r.ne[ax];
        const double k = kTwoPi * m / r.Le[ax];
        k2[(size_t)ax * pitch + j] = k * k;
    }
}

// w += W on the physical part of the image (W holds minus the filtered increment).
__device__ __forceinline__ void sis_unmirror_body(const MirrorArgs& a, double2* __restrict__ w, int64_t M)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
        const int z = (int)(i % a.n[2]);
        const int y = (int)((i / a.n[2]) % a.n[1]);
        const int x = (int)(i / ((int64_t)a.n[1] * a.n[2]));
        const double2 d = a.W[((int64_t)x * a.ne[1] + y) * a.ne[2] + z];
        w[i] = make_double2(w[i].x + d.x, w[i].y + d.y);
    }
}

__global__ void k_sis_unmirror(MirrorArgs a, double2* __restrict__ w, int64_t M) { sis_unmirror_body(a, w, M); }

// Batched forms (blockIdx.y is the replica): the image arguments and the field
// that receives the filtered increment.
struct MirrorJob {
    MirrorArgs m;
    double2* w;
    int64_t M;
};

__global__ void k_sis_mirror_batch(const MirrorJob* __restrict__ jobs) { sis_mirror_body(jobs[blockIdx.y].m); }

__global__ void k_sis_unmirror_batch(const MirrorJob* __restrict__ jobs)
{
    const MirrorJob& j = jobs[blockIdx.y];
    sis_unmirror_body(j.m, j.w, j.M);
}

// ------------------------------------------------------------ reverse mode --
// Per-step contribution to dQ/dw_b (times M) of step j, accumulated in FP64
// with Neumaier compensation into the block's (sum, comp) arrays.  With
// lam1 = lambda_{j+1}, lam0 = lambda_j, the captures A = D_{h/2} E4 (.),
// B = D_{h/2}(E2 A) (so the half step is E4 B) and E2 = E4^2, the derivative of
// the Richardson step of Eq. (12) sums the three field factors of the half
// path and the two of the full path; eliminating the full path through
// q_{j+1} = (4 E4 Bq - Fq)/3 gives
//   g = (h/3)(lam1 E4 Bq + E4 Bl q0) - (h/2)(lam1 q1 + lam0 q0) - (2h/3) Al E2 Aq.
// The plain split step gives g = -(h/2)(lam1 q1 + lam0 q0).
template <typename T>
struct AccArgs {
    const cx<T>* lam1;
    const cx<T>* lam0;
    const cx<T>* Al;
    const cx<T>* Bl;
    const cx<T>* q0;
    const cx<T>* q1;
    const cx<T>* Aq;
    const cx<T>* Bq;
    const cx<T>* E4;
    double h;
    int rqm4;
    int64_t M;
    double2* Gs;
    double2* Gc;
};

__device__ __forceinline__ double2 d2(double re, double im) { return make_double2(re, im); }
template <typename T>
__device__ __forceinline__ double2 wide(cx<T> v) { return make_double2(double(v.re), double(v.im)); }

__device__ __forceinline__ void nacc(double& s, double& c, double x)
{
    const double t = s + x;
    if (fabs(s) >= fabs(x))
        c += (s - t) + x;
    else
        c += (x - t) + s;
    s = t;
}

template <typename T>
__global__ void k_adj_accum(AccArgs<T> a)
{
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < a.M; x += (int64_t)gridDim.x * blockDim.x) {
        const double2 l1 = wide(a.lam1[x]), l0 = wide(a.lam0[x]), q0 = wide(a.q0[x]), q1 = wide(a.q1[x]);
        const double2 tr = cmul(l1, q1), tl = cmul(l0, q0);
        double2 g = d2(-0.5 * a.h * (tr.x + tl.x), -0.5 * a.h * (tr.y + tl.y));
        if (a.rqm4) {
            const double2 e4 = wide(a.E4[x]);
            const double2 e2 = cmul(e4, e4);
            const double2 u = cmul(l1, cmul(e4, wide(a.Bq[x])));
            const double2 v = cmul(cmul(e4, wide(a.Bl[x])), q0);
            const double2 m = cmul(cmul(wide(a.Al[x]), e2), wide(a.Aq[x]));
            g.x += a.h / 3.0 * (u.x + v.x) - 2.0 * a.h / 3.0 * m.x;
            g.y += a.h / 3.0 * (u.y + v.y) - 2.0 * a.h / 3.0 * m.y;
        }
        double2 s = a.Gs[x], c = a.Gc[x];
        nacc(s.x, c.x, g.x);
        nacc(s.y, c.y, g.y);
        a.Gs[x] = s;
        a.Gc[x] = c;
    }
}

// dH/dw_+ = -i C dV [1 + (G_A + G_B)/Q],  dH/dw_- = C dV [2 w_-/chiN - (G_B - G_A)/Q],
// from dQ/dw_+ = i (G_A + G_B)/M, dQ/dw_- = (G_B - G_A)/M and dV = V/M.
__global__ void k_adj_final(const double2* __restrict__ G, int64_t M, const double2* __restrict__ wm,
                            const double2* __restrict__ Qp, double C, double dV, double chiN,
                            double2* __restrict__ dwp, double2* __restrict__ dwm)
{
    const double2 Q = *Qp;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < M; x += (int64_t)gridDim.x * blockDim.x) {
        // G layout: [A sum][A comp][B sum][B comp]
        const double2 ga = d2(G[x].x + G[M + x].x, G[x].y + G[M + x].y);
        const double2 gb = d2(G[2 * M + x].x + G[3 * M + x].x, G[2 * M + x].y + G[3 * M + x].y);
        const double2 sp = cdiv(d2(ga.x + gb.x, ga.y + gb.y), Q);
        const double2 sm = cdiv(d2(gb.x - ga.x, gb.y - ga.y), Q);
        // -i C dV (1 + sp)
        dwp[x] = d2(C * dV * sp.y, -C * dV * (1.0 + sp.x));
        const double2 w = wm[x];
        dwm[x] = d2(C * dV * (2.0 * w.x / chiN - sm.x), C * dV * (2.0 * w.y / chiN - sm.y));
    }
}

// Box-derivative terms of one step.  The L_a derivative of a diffusion D_h'
// multiplies its factor by 2 k_a^2 h'/L_a, i.e. u^T dD/dL_a v = (2h'/L_a) u^T
// (-d^2/dx_a^2) D_h' v.  The stress passes (one per axis and step) evaluate
// these with the captures X = B (= D_{h/2} E2 Aq), A (= D_{h/2} E4 q),
// C (= D_h E2 q) and the left vectors E4 lam1, E2 Al, E2 lam1, adding their
// workgroup sums to acc[a][block]; sums[a] is their total.
// dH/dL_a = C dV S / L_a - C (V/L_a) Log Q - C V (dQ/dL_a)/Q with
// dQ/dL_a = sums[a] / M and S = sum_x [w_-^2/chiN - i w_+].
__global__ void k_stress_final(const double2* __restrict__ sums, const double2* __restrict__ Sp,
                               const double2* __restrict__ Qp, double C, double lx, double ly, double lz,
                               int64_t M, double2* __restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double2 Q = *Qp, S = *Sp;
    const double V = lx * ly * lz, dV = V / (double)M;
    const double L[3] = {lx, ly, lz};
    const double2 lq = d2(0.5 * log(Q.x * Q.x + Q.y * Q.y), atan2(Q.y, Q.x));
    for (int a = 0; a < 3; ++a) {
        const double2 r = cdiv(d2(sums[a].x / (double)M, sums[a].y / (double)M), Q);
        out[a] = d2(C * dV * S.x / L[a] - C * V / L[a] * lq.x - C * V * r.x,
                    C * dV * S.y / L[a] - C * V / L[a] * lq.y - C * V * r.y);
    }
}

__global__ void k_fill_zero(double2* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_double2(0.0, 0.0);
}

// ---------------------------------------------------------------- batches --
// Job-table versions of the small kernels: blockIdx.y selects a replica,
// whose arguments are read from a device table.
template <typename T>
struct TabJob {
    const double2* wp;
    const double2* wm;
    int64_t M;
    TabDesc d;
    cx<T>* out;
};
template <typename T>
struct SumJob {
    const cx<T>* x;
    int64_t n;
    double2* partials;
};
struct FinJob {
    const double2* partials;
    int np;
    double scale;
    double2* out;
    uint32_t* flags;
};
template <typename T>
struct DensJob {
    const cx<T>* qs;
    const cx<T>* qds;
    int K, J;
    int64_t M;
    const double* tau;
    const double2* Qp;
    double2* phiA;
    double2* phiB;
    double2* Qout;
};
struct HamJob {
    const double2* wp;
    const double2* wm;
    int64_t M;
    double inv_chiN;
    double2* partials;
    int np;
    double C, dV, V;
    const double2* Qp;
    double2* H;
    double2* hint;
    double2* Sout;
};
struct LogJob {
    const double2* Q;
    const double2* H;
};

template <typename T>
__global__ void k_tables_batch(const TabJob<T>* __restrict__ jobs)
{
    const TabJob<T> a = jobs[blockIdx.y];
    field_tables_body<T>(a.wp, a.wm, a.M, a.d, a.out);
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_sum_partials_batch(const SumJob<T>* __restrict__ jobs)
{
    const SumJob<T> a = jobs[blockIdx.y];
    sum_partials_body<T>(a.x, a.n, a.partials);
}

// grid (1, replicas): final_sum_body reduces row blockIdx.x = 0 of each job
__global__ __launch_bounds__(kRedThreads) void k_final_batch(const FinJob* __restrict__ jobs)
{
    const FinJob a = jobs[blockIdx.y];
    final_sum_body(a.partials, a.np, a.scale, a.out, (double2*)nullptr, a.flags);
}

template <typename T>
__global__ void k_density_batch(const DensJob<T>* __restrict__ jobs)
{
    const DensJob<T> a = jobs[blockIdx.y];
    density_body<T>(a.qs, a.qds, a.K, a.J, a.M, a.tau, a.Qp, a.phiA, a.phiB, a.Qout);
}

__global__ __launch_bounds__(kRedThreads) void k_ham_partials_batch(const HamJob* __restrict__ jobs)
{
    const HamJob a = jobs[blockIdx.y];
    ham_partials_body(a.wp, a.wm, a.M, a.inv_chiN, a.partials);
}

__global__ __launch_bounds__(kRedThreads) void k_ham_final_batch(const HamJob* __restrict__ jobs)
{
    const HamJob a = jobs[blockIdx.y];
    ham_final_body(a.partials, a.np, a.C, a.dV, a.V, a.Qp, a.H, a.hint, a.Sout);
}

// The Langevin step index comes from device memory so one captured graph
// serves every step.
__global__ void k_update_batch(const UpdArgs* __restrict__ jobs, const uint64_t* __restrict__ step)
{
    UpdArgs a = jobs[blockIdx.y];
    a.step += *step;
    update_body(a);
}

// Q and H of every replica at log row *row (if below capacity).
__global__ void k_batch_log(const LogJob* __restrict__ jobs, int n, double2* __restrict__ log,
                            const uint64_t* __restrict__ row, uint64_t capacity)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t i = *row;
    if (r < n && i < capacity) {
        log[(i * n + r) * 2] = *jobs[r].Q;
        log[(i * n + r) * 2 + 1] = *jobs[r].H;
    }
}

__global__ void k_batch_advance(uint64_t* __restrict__ step, uint64_t* __restrict__ row)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *step += 1;
        *row += 1;
    }
}

__global__ void k_set_u64(uint64_t* __restrict__ p, uint64_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Plain streaming copy (16 bytes per lane per iteration).
__global__ void k_copy_probe(const double2* __restrict__ src, double2* __restrict__ dst, int64_t n)
{
    // four loads in flight per lane before the stores
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const double2 a0 = src[i], a1 = src[i + stride], a2 = src[i + 2 * stride], a3 = src[i + 3 * stride];
        dst[i] = a0;
        dst[i + stride] = a1;
        dst[i + 2 * stride] = a2;
        dst[i + 3 * stride] = a3;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

// ============================================================== host side ==

int grid_for(int64_t n, int threads, int cap = 8192)
{
    const int64_t b = (n + threads - 1) / threads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

int reduction_blocks(int64_t n) { return grid_for(n, kRedThreads * 8, 1024); }

// Contour plan; see pft_contour_plan in the header.
int contour_plan(int ns, double f, double* h, int* blk, int* junction)
{
    if (ns < 2 || !(f > 0.0 && f < 1.0)) return -1;
    const double ds = 1.0 / ns;
    const double fn = f * ns;
    const double r = std::floor(fn + 0.5);
    int K = 0;
    if (std::fabs(fn - r) <= 1e-9) {
        const int na = (int)r;
        for (int j = 0; j < ns; ++j) {
            h[K] = ds;
            blk[K] = j < na ? 0 : 1;
            ++K;
        }
        *junction = na;
    } else {
        const int nst = (int)std::floor(fn);
        for (int j = 0; j < nst; ++j) {
            h[K] = ds;
            blk[K++] = 0;
        }
        h[K] = f - nst * ds;
        blk[K++] = 0;
        h[K] = (nst + 1) * ds - f;
        blk[K++] = 1;
        for (int j = nst + 1; j < ns; ++j) {
            h[K] = ds;
            blk[K++] = 1;
        }
        *junction = nst + 1;
    }
    return K;
}

}  // namespace

namespace {
// Kernel variant per (precision, axis length, kind: 0 = z pass, 1 = strided
// passes), used by contexts created afterwards; filled by pft_autotune or
// pft_tune_load (also from $PFT_TUNE_CACHE on the first pft_create).
int g_tune[2][257][2] = {};
bool g_tune_env_checked = false;

int tuned_variant(int prec, int n, int kind)
{
    int n1, n2, w;
    const int v = (n >= 0 && n <= 256) ? g_tune[prec & 1][n][kind] : 0;
    return pft::axis_variant(n, v, &n1, &n2, &w) ? v : 0;
}
}  // namespace

constexpr int kRing = 4;  // device slots per direction of host staging

struct pft_ctx {
    pft_params p{};
    hipStream_t stream = nullptr;
    int device = 0;               // the device current at creation
    int64_t M = 0;
    int K = 0, J = 0;
    std::vector<double> h;
    std::vector<int> blk, kind, hid;  // per step: E table kind (0..3), step-length id (0..2)
    double hval[3] = {0, 0, 0};       // ds, A junction sub-step, B junction sub-step
    int maxN = 0;
    int var[3] = {0, 0, 0};           // kernel variant of each axis pass (x, y, z)
    bool fused = false;               // sweeps use the fused yz-plane pass (square yz-plane in LDS)
    bool fused_conj_only = false;     // ... only the conjugate sweep (the forward one runs axis passes)
    size_t elem = 0;                  // bytes per propagator value
    // device buffers
    void* qs = nullptr;
    void* qds = nullptr;   // the Edwards model's conjugate store is qs itself (symmetric chain)
    void* U = nullptr;
    void* V = nullptr;
    void* U2 = nullptr;    // work pair of the conjugate sweep when it runs on s2
    void* V2 = nullptr;
    hipStream_t s2 = nullptr;
    bool dual_off = false;        // run both sweeps on the context stream
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    void* E = nullptr;     // 4 * M field operator tables
    void* work = nullptr;  // 2 * M scratch in working precision
    void* gtab = nullptr;  // diffusion factors: [hid 3][half/full 2][axis 3][maxN]
    double* tau = nullptr; // 2 (K+1) trapezoid weights
    double2* phi = nullptr;       // internal phi_A, phi_B (2 M)
    double* k2 = nullptr;         // semi-implicit step: (2 pi m / L)^2 per axis [3][maxN], natural order
    // stored-product storage modes
    std::vector<double> tau_h;    // host copy of the trapezoid weights
    void* qh = nullptr;           // PFT_STORE_HOST: pinned host store of q, (K+1) slices
    void* ring = nullptr;         // device slots: [kRing] staging q, [kRing] prefetched q, [2] q-dagger
    hipStream_t cs = nullptr;     // copy stream
    hipEvent_t ev_st[kRing] = {}, ev_cp[kRing] = {}, ev_rd[kRing] = {}, ev_fr[kRing] = {}, ev_done = nullptr;
    double2* sisbuf = nullptr;    // semi-implicit step: the filtered increment (M)
    double2* sisext = nullptr;    // ... between reflecting walls: its even image and the result (2 Me)
    double2* partials = nullptr;  // reduction scratch
    double2* scal = nullptr;      // [0] Q, [1] H, [2] h, [3..] node Q
    uint32_t* flags = nullptr;
    int nparts = 0;
    bool propagated = false;
    std::string err;
    // reverse mode: working-precision slices and FP64 accumulators, allocated
    // on the first pft_adjoint call for its checkpoint interval
    int adj_kc = 0;
    size_t adj_slices = 0;
    void* adj = nullptr;
    hipEvent_t ev_adj[5] = {};  // segment buffer ready (2), buffer free, spare, checkpoints done
    double2* adjG = nullptr;    // [A sum][A comp][B sum][B comp], M each
    double2* adjAcc = nullptr;  // [3][nparts] box-derivative partials
    // graph replay of one evaluation (pft_evaluate_graph): captured on gs for
    // the buffers in gkey, replayed there between two events
    hipStream_t gs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t ev_g0 = nullptr, ev_g1 = nullptr;
    const void* gkey[5] = {};
    // profiling: event pairs recorded around each launch while prof is set
    bool prof = false;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    std::vector<int> ev_kind;
    std::vector<double> ev_bytes;

    pft_status fail(pft_status s, const char* fmt, ...)
    {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        return s;
    }
};

namespace {

#define PFT_HIP(ctx, call)                                                                             \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return (ctx)->fail(PFT_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));           \
    } while (0)

bool aligned16(const void* p) { return p && (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Brackets one launch with a pair of events on the context stream while
// profiling is on; records the launch's kernel kind and algorithmic bytes.
// With `single` the scope holds exactly one launch made through PFT_LAUNCH,
// which records the pair inside its own dispatch (kernel start to end);
// otherwise the pair is recorded on the stream around the scope's launches.
struct ProfScope {
    pft_ctx* c;
    size_t i = 0;
    bool on;
    hipStream_t st;
    bool single;
    ProfScope(pft_ctx* ctx, int kind, double bytes, hipStream_t s = nullptr, bool one_launch = false)
        : c(ctx), on(ctx->prof), st(s ? s : ctx->stream), single(one_launch)
    {
        if (!on) return;
        i = c->ev_used;
        while (c->ev.size() < 2 * (i + 1)) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) {
                on = false;
                return;
            }
            c->ev.push_back(e);
        }
        if (c->ev_kind.size() <= i) {
            c->ev_kind.resize(i + 1);
            c->ev_bytes.resize(i + 1);
        }
        c->ev_kind[i] = kind;
        c->ev_bytes[i] = bytes;
        c->ev_used = i + 1;
        if (single)
            pft::g_launch_events = pft::LaunchEvents{c->ev[2 * i], c->ev[2 * i + 1]};
        else
            (void)hipEventRecord(c->ev[2 * i], st);
    }
    ~ProfScope()
    {
        if (!on) return;
        if (single) {
            if (pft::g_launch_events.start) {
                // the launch did not take the pair (it failed): keep the pair valid
                pft::g_launch_events = pft::LaunchEvents{};
                (void)hipEventRecord(c->ev[2 * i], st);
                (void)hipEventRecord(c->ev[2 * i + 1], st);
            }
        } else {
            (void)hipEventRecord(c->ev[2 * i + 1], st);
        }
    }
};

template <typename T>
const T* gptr(const pft_ctx* c, int hid, int full, int axis)
{
    return static_cast<const T*>(c->gtab) + ((size_t)((hid * 2 + full) * 3 + axis)) * c->maxN;
}

template <typename T>
cx<T>* etab(const pft_ctx* c, int kind)
{
    return static_cast<cx<T>*>(c->E) + (size_t)kind * c->M;
}

template <typename T>
cx<T>* slice(void* store, const pft_ctx* c, int node)
{
    return static_cast<cx<T>*>(store) + (size_t)node * c->M;
}

// The pair of work arrays a pipeline of passes runs on (half-step path U,
// full-step path V); NULL members mean the context's own pair.
struct Work {
    void* U = nullptr;
    void* V = nullptr;
    hipStream_t stream = nullptr;  // NULL: the context's stream
};

// The z pass on the context's grid (the walled kernels on a walled z axis).
template <typename T>
hipError_t launch_z(const pft_ctx* c, const pft::ZArgs<T>& a, hipStream_t st)
{
    if (c->p.bc[2]) return pft::launch_zpass_walls<T>(c->p.nz, c->p.bc[2], a, st);
    return pft::launch_zpass<T>(c->p.nz, c->var[2], a, st);
}

// Z pass completing step `prev` (-1: none) and starting step `next` (-1: none).
template <typename T>
pft_status zpass(pft_ctx* c, int prev, int next, const cx<T>* qin, cx<T>* qout, const Work& w = Work(),
                 cx<T>* hcap = nullptr)
{
    pft::ZArgs<T> a{};
    a.nlines = (int64_t)c->p.nx * c->p.ny;
    a.U = static_cast<cx<T>*>(w.U ? w.U : c->U);
    a.V = static_cast<cx<T>*>(w.V ? w.V : c->V);
    a.hcap = hcap;
    a.qin = qin;
    a.qout = qout;
    a.scheme = c->p.scheme;
    a.has_prev = prev >= 0;
    a.has_next = next >= 0;
    if (prev >= 0) {
        a.Ep = etab<T>(c, c->kind[prev]);
        a.gh_p = gptr<T>(c, c->hid[prev], 0, 2);
    }
    if (next >= 0) {
        a.En = etab<T>(c, c->kind[next]);
        a.gh_n = gptr<T>(c, c->hid[next], 0, 2);
        a.gf_n = gptr<T>(c, c->hid[next], 1, 2);
    }
    // algorithmic bytes: each distinct array read or written once
    const double E = (double)c->elem * (double)c->M;
    const bool rqm4 = c->p.scheme == PFT_RQM4;
    double bytes = 0;
    if (prev >= 0) bytes += (rqm4 ? 3 : 2) * E;
    else if (qin) bytes += E;
    if (qout) bytes += E;
    if (next >= 0) bytes += (rqm4 ? 2 : 1) * E + ((prev < 0 || c->kind[next] != c->kind[prev]) ? E : 0);
    if (hcap) bytes += E;
    hipStream_t st = w.stream ? w.stream : c->stream;
    ProfScope ps(c, PFT_K_ZPASS, bytes, st, c->p.bc[2] == 0);
    PFT_HIP(c, launch_z<T>(c, a, st));
    return PFT_OK;
}

// Strided pass along axis 0 (x) or 1 (y).
template <typename T>
pft_status spass(pft_ctx* c, int axis, pft::SOps<T> opU, pft::SOps<T> opV, const Work& w = Work())
{
    pft::SArgs<T> a{};
    a.U = static_cast<cx<T>*>(w.U ? w.U : c->U);
    a.V = static_cast<cx<T>*>(w.V ? w.V : c->V);
    a.opU = opU;
    a.opV = opV;
    const double E = (double)c->elem * (double)c->M;
    double bytes = (opU.g1 ? 2 * E : 0) + (opV.g1 ? 2 * E : 0);
    if (opU.g1 && opU.acap) bytes += E;
    if (opV.g1 && opV.acap) bytes += E;
    if (opU.g1 && opU.e) bytes += E;
    if (opV.g1 && opV.e && !(opU.g1 && opU.e == opV.e)) bytes += E;
    hipStream_t st = w.stream ? w.stream : c->stream;
    ProfScope ps(c, axis == 0 ? PFT_K_XPASS : PFT_K_YPASS, bytes, st, c->p.bc[axis] == 0);
    const int64_t nynz = (int64_t)c->p.ny * c->p.nz;
    if (axis == 0) {
        a.S = nynz;
        a.slab_stride = 0;
        if (c->p.bc[0])
            PFT_HIP(c, pft::launch_spass_walls<T>(0, c->p.nx, c->p.bc[0], nynz, a, 1, st));
        else
            PFT_HIP(c, pft::launch_spass<T>(0, c->p.nx, c->var[0], nynz, a, 1, st));
    } else {
        a.S = c->p.nz;
        a.slab_stride = nynz;
        if (c->p.bc[1])
            PFT_HIP(c, pft::launch_spass_walls<T>(1, c->p.ny, c->p.bc[1], c->p.nz, a, c->p.nx, st));
        else
            PFT_HIP(c, pft::launch_spass<T>(1, c->p.ny, c->var[1], c->p.nz, a, c->p.nx, st));
    }
    return PFT_OK;
}

// Fused yz-plane pass completing step `prev` (-1: none: its Y2 and Z) and
// starting step `next` (-1: none: its Z and Y1).
template <typename T>
pft_status yzpass(pft_ctx* c, int prev, int next, const cx<T>* qin, cx<T>* qout, const Work& w = Work(),
                  cx<T>* hcap = nullptr)
{
    pft::PArgs<T> a{};
    a.nplanes = c->p.nx;
    a.U = static_cast<cx<T>*>(w.U ? w.U : c->U);
    a.V = static_cast<cx<T>*>(w.V ? w.V : c->V);
    a.hcap = hcap;
    a.qin = qin;
    a.qout = qout;
    a.scheme = c->p.scheme;
    a.has_prev = prev >= 0;
    a.has_next = next >= 0;
    if (prev >= 0) {
        a.Ep = etab<T>(c, c->kind[prev]);
        a.gyh_p = gptr<T>(c, c->hid[prev], 0, 1);
        a.gzh_p = gptr<T>(c, c->hid[prev], 0, 2);
    }
    if (next >= 0) {
        a.En = etab<T>(c, c->kind[next]);
        a.gzh_n = gptr<T>(c, c->hid[next], 0, 2);
        a.gzf_n = gptr<T>(c, c->hid[next], 1, 2);
        a.gyh_n = gptr<T>(c, c->hid[next], 0, 1);
        a.gyf_n = gptr<T>(c, c->hid[next], 1, 1);
    }
    // algorithmic bytes, as for the z pass
    const double E = (double)c->elem * (double)c->M;
    const bool rqm4 = c->p.scheme == PFT_RQM4;
    double bytes = 0;
    if (prev >= 0) bytes += (rqm4 ? 3 : 2) * E;
    else if (qin) bytes += E;
    if (qout) bytes += E;
    if (next >= 0) bytes += (rqm4 ? 2 : 1) * E + ((prev < 0 || c->kind[next] != c->kind[prev]) ? E : 0);
    if (hcap) bytes += E;
    hipStream_t st = w.stream ? w.stream : c->stream;
    ProfScope ps(c, PFT_K_YZPASS, bytes, st, true);
    PFT_HIP(c, pft::launch_yzpass<T>(c->p.ny, a, st));
    return PFT_OK;
}

// The x pass of step j alone (the fused schedule's other pass).
template <typename T>
pft_status xpass_step(pft_ctx* c, int j, const Work& w = Work(), cx<T>* capA = nullptr, cx<T>* capC = nullptr)
{
    const int hd = c->hid[j];
    const cx<T>* e = etab<T>(c, c->kind[j]);
    if (c->p.scheme == PFT_RQM4)
        return spass<T>(c, 0, {gptr<T>(c, hd, 0, 0), e, gptr<T>(c, hd, 0, 0), capA},
                        {gptr<T>(c, hd, 1, 0), e, nullptr, capC}, w);
    return spass<T>(c, 0, {nullptr, nullptr, nullptr}, {gptr<T>(c, hd, 1, 0), nullptr, nullptr}, w);
}

// The Y1, X, Y2 passes of step j (Y, X for the plain split).  capA / capC,
// if set, receive D_{h/2} E4 q (half path after its first diffusion) and
// D_h E2 q (full path before its last multiply) from the x pass.
template <typename T>
pft_status step_body(pft_ctx* c, int j, const Work& w = Work(), cx<T>* capA = nullptr, cx<T>* capC = nullptr)
{
    const int hd = c->hid[j];
    const cx<T>* e = etab<T>(c, c->kind[j]);
    const pft::SOps<T> none{nullptr, nullptr, nullptr};
    pft_status s;
    if (c->p.scheme == PFT_RQM4) {
        s = spass<T>(c, 1, {gptr<T>(c, hd, 0, 1), nullptr, nullptr}, {gptr<T>(c, hd, 1, 1), nullptr, nullptr}, w);
        if (s) return s;
        s = spass<T>(c, 0, {gptr<T>(c, hd, 0, 0), e, gptr<T>(c, hd, 0, 0), capA},
                     {gptr<T>(c, hd, 1, 0), e, nullptr, capC}, w);
        if (s) return s;
        return spass<T>(c, 1, {gptr<T>(c, hd, 0, 1), nullptr, nullptr}, none, w);
    }
    s = spass<T>(c, 1, none, {gptr<T>(c, hd, 1, 1), nullptr, nullptr}, w);
    if (s) return s;
    return spass<T>(c, 0, none, {gptr<T>(c, hd, 1, 0), nullptr, nullptr}, w);
}

// One sweep over the K steps, forward (q) or mirrored (q-dagger).  Node i
// (i = 0..K, in sweep order) is written to out(i), and after(i) runs once the
// pass that stores it has been enqueued.
template <typename T, class Out, class After>
pft_status sweep_nodes(pft_ctx* c, bool backward, const Work& w, const Out& out, const After& after)
{
    auto stepj = [&](int i) { return backward ? c->K - 1 - i : i; };
    const bool fused = c->fused && (backward || !c->fused_conj_only);
    pft_status s = fused ? yzpass<T>(c, -1, stepj(0), nullptr, out(0), w) : zpass<T>(c, -1, stepj(0), nullptr, out(0), w);
    if (s) return s;
    if ((s = after(0))) return s;
    for (int i = 0; i < c->K; ++i) {
        const int j = stepj(i);
        const int next = i + 1 < c->K ? stepj(i + 1) : -1;
        if (fused) {
            // two passes per step: X, then yz completing it and starting the next
            s = xpass_step<T>(c, j, w);
            if (s) return s;
            s = yzpass<T>(c, j, next, nullptr, out(i + 1), w);
        } else {
            s = step_body<T>(c, j, w);
            if (s) return s;
            s = zpass<T>(c, j, next, nullptr, out(i + 1), w);
        }
        if (s) return s;
        if ((s = after(i + 1))) return s;
    }
    return PFT_OK;
}

// Sweep storing every node into `store`.
template <typename T>
pft_status sweep(pft_ctx* c, bool backward, void* store, const Work& w = Work())
{
    return sweep_nodes<T>(c, backward, w, [&](int i) { return slice<T>(store, c, i); },
                          [](int) { return PFT_OK; });
}

template <typename T>
pft_status field_tables_t(pft_ctx* c, const double* wp, const double* wm)
{
    TabDesc d{};
    d.n = 4;
    d.blk[0] = 0; d.a[0] = c->hval[0] / 4;
    d.blk[1] = 1; d.a[1] = c->hval[0] / 4;
    d.blk[2] = 0; d.a[2] = c->hval[1] / 4;
    d.blk[3] = 1; d.a[3] = c->hval[2] / 4;
    if (c->K == c->p.ns) d.n = 2;  // no junction sub-steps
    if (c->p.model == PFT_EDWARDS) {
        d.n = 1;  // one species: E4 = exp(-i omega h/4)
        wm = nullptr;
    }
    {
        ProfScope ps(c, PFT_K_TABLES, (32.0 + d.n * (double)c->elem) * (double)c->M, nullptr, true);
        PFT_LAUNCH((k_field_tables<T>), dim3(grid_for(c->M, 256)), dim3(256), 0, c->stream,
                       reinterpret_cast<const double2*>(wp), reinterpret_cast<const double2*>(wm), c->M, d,
                       static_cast<cx<T>*>(c->E));
    }
    PFT_HIP(c, hipGetLastError());
    return PFT_OK;
}

// Q = (1/M) sum_x q_K(x) into scal[0].
template <typename T>
pft_status reduce_q(pft_ctx* c, const cx<T>* qK)
{
    ProfScope ps(c, PFT_K_REDUCE, (double)c->elem * (double)c->M);
    hipLaunchKernelGGL((k_sum_partials<T>), dim3(c->nparts), dim3(kRedThreads), 0, c->stream, qK, c->M, c->partials);
    hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(kRedThreads), 0, c->stream, c->partials, c->nparts,
                       1.0 / (double)c->M, c->scal, (double2*)nullptr, c->flags);
    PFT_HIP(c, hipGetLastError());
    return PFT_OK;
}

// Stored-product storage modes: forward sweep into the device store (or
// staged through device slots into pinned host memory on the copy stream),
// then the conjugate sweep, whose node i is paired at once with q_{K-i} and
// added to the FP64 density accumulators (c->phi: A then B).
template <typename T>
pft_status propagate_stored_product(pft_ctx* c)
{
    const int K = c->K;
    const int64_t M = c->M;
    const bool host = c->p.storage == PFT_STORE_HOST;
    const size_t bytes = (size_t)M * c->elem;
    cx<T>* ring = static_cast<cx<T>*>(c->ring);
    auto rs = [&](int k) { return ring + (size_t)k * M; };                            // staging slots
    auto rp = [&](int k) { return ring + (size_t)(kRing + k) * M; };                  // prefetch slots
    auto rd = [&](int k) { return ring + (size_t)((host ? 2 * kRing : 0) + k) * M; };  // q-dagger slots
    char* qh = static_cast<char*>(c->qh);
    pft_status s;
    if (!host) {
        s = sweep<T>(c, false, c->qs);
    } else {
        s = sweep_nodes<T>(
            c, false, Work(),
            [&](int n) {
                // the slot's previous node must have reached the host
                if (n >= kRing) (void)hipStreamWaitEvent(c->stream, c->ev_cp[n % kRing], 0);
                return rs(n % kRing);
            },
            [&](int n) -> pft_status {
                const int k = n % kRing;
                PFT_HIP(c, hipEventRecord(c->ev_st[k], c->stream));
                PFT_HIP(c, hipStreamWaitEvent(c->cs, c->ev_st[k], 0));
                PFT_HIP(c, hipMemcpyAsync(qh + (size_t)n * bytes, rs(k), bytes, hipMemcpyDeviceToHost, c->cs));
                PFT_HIP(c, hipEventRecord(c->ev_cp[k], c->cs));
                return PFT_OK;
            });
    }
    if (s) return s;
    s = reduce_q<T>(c, host ? rs(K % kRing) : slice<T>(c->qs, c, K));
    if (s) return s;
    // q_{K-i} into prefetch slot i % kRing (after its copy to the host: same stream)
    auto prefetch = [&](int i) -> pft_status {
        const int k = i % kRing;
        PFT_HIP(c, hipMemcpyAsync(rp(k), qh + (size_t)(K - i) * bytes, bytes, hipMemcpyHostToDevice, c->cs));
        PFT_HIP(c, hipEventRecord(c->ev_rd[k], c->cs));
        return PFT_OK;
    };
    if (host)
        for (int i = 0; i < kRing && i <= K; ++i)
            if ((s = prefetch(i))) return s;
    double2* accA = c->phi;
    double2* accB = c->phi + M;
    s = sweep_nodes<T>(
        c, true, Work(), [&](int i) { return rd(i & 1); },
        [&](int i) -> pft_status {
            const int j = K - i;
            const cx<T>* q = host ? rp(i % kRing) : slice<T>(c->qs, c, j);
            if (host) PFT_HIP(c, hipStreamWaitEvent(c->stream, c->ev_rd[i % kRing], 0));
            {
                ProfScope ps(c, PFT_K_DENSITY, (2.0 * c->elem + (i == 0 ? 32.0 : 64.0)) * (double)M);
                hipLaunchKernelGGL((k_accum_node<T>), dim3(grid_for(M, 256)), dim3(256), 0, c->stream, q, rd(i & 1), M,
                                   c->tau_h[j], c->tau_h[K + 1 + j], accA, accB, i == 0 ? 1 : 0);
            }
            PFT_HIP(c, hipGetLastError());
            if (host) {
                PFT_HIP(c, hipEventRecord(c->ev_fr[i % kRing], c->stream));
                if (i + kRing <= K) {
                    PFT_HIP(c, hipStreamWaitEvent(c->cs, c->ev_fr[i % kRing], 0));
                    pft_status e = prefetch(i + kRing);
                    if (e) return e;
                }
            }
            return PFT_OK;
        });
    if (s) return s;
    if (host) {
        // later calls on the context stream see every copy finished
        PFT_HIP(c, hipEventRecord(c->ev_done, c->cs));
        PFT_HIP(c, hipStreamWaitEvent(c->stream, c->ev_done, 0));
    }
    c->propagated = true;
    return PFT_OK;
}

template <typename T>
pft_status propagate_t(pft_ctx* c, const double* wp, const double* wm)
{
    pft_status s = field_tables_t<T>(c, wp, wm);
    if (s) return s;
    if (c->p.storage != PFT_STORE_BOTH) return propagate_stored_product<T>(c);
    if (c->p.model == PFT_EDWARDS) {
        // symmetric chain: q-dagger = q, one sweep
        s = sweep<T>(c, false, c->qs);
        if (s) return s;
    } else if (c->s2 && !c->dual_off) {
        // the two sweeps are independent: the conjugate one runs on a second
        // stream with its own work pair, so one sweep's memory phases overlap
        // the other's on-chip transform phases
        PFT_HIP(c, hipEventRecord(c->ev_fork, c->stream));
        PFT_HIP(c, hipStreamWaitEvent(c->s2, c->ev_fork, 0));
        s = sweep<T>(c, true, c->qds, Work{c->U2, c->V2, c->s2});
        if (s) return s;
        PFT_HIP(c, hipEventRecord(c->ev_join, c->s2));
        s = sweep<T>(c, false, c->qs);
        if (s) return s;
        PFT_HIP(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
    } else {
        s = sweep<T>(c, false, c->qs);
        if (s) return s;
        s = sweep<T>(c, true, c->qds);
        if (s) return s;
    }
    // Q = (1/M) sum_x q_K(x)
    ProfScope ps(c, PFT_K_REDUCE, (double)c->elem * (double)c->M);
    hipLaunchKernelGGL((k_sum_partials<T>), dim3(c->nparts), dim3(kRedThreads), 0, c->stream,
                       slice<T>(c->qs, c, c->K), c->M, c->partials);
    hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(kRedThreads), 0, c->stream, c->partials, c->nparts,
                       1.0 / (double)c->M, c->scal, (double2*)nullptr, c->flags);
    PFT_HIP(c, hipGetLastError());
    c->propagated = true;
    return PFT_OK;
}

// H and h of Eq. (3) into device pointers (hint may be NULL); the local sum
// S = sum_x [w_-^2/chiN - i w_+] is kept in scal[4].
pft_status hamiltonian_launch(pft_ctx* c, const double* wp, const double* wm, double* H, double* hint)
{
    const double V = c->p.lx * c->p.ly * c->p.lz;
    ProfScope ps(c, PFT_K_REDUCE, 2.0 * sizeof(double2) * (double)c->M);
    // diblock: sum w_-^2/chiN - i w_+;  Edwards (omega in wp): sum (B/(2C)) omega^2
    const bool ed = c->p.model == PFT_EDWARDS;
    hipLaunchKernelGGL(k_ham_partials, dim3(c->nparts), dim3(kRedThreads), 0, c->stream,
                       ed ? nullptr : reinterpret_cast<const double2*>(wp),
                       reinterpret_cast<const double2*>(ed ? wp : wm), c->M,
                       ed ? c->p.B / (2.0 * c->p.C) : 1.0 / c->p.chiN, c->partials);
    hipLaunchKernelGGL(k_ham_final, dim3(1), dim3(kRedThreads), 0, c->stream, c->partials, c->nparts, c->p.C,
                       V / (double)c->M, V, c->scal, reinterpret_cast<double2*>(H), reinterpret_cast<double2*>(hint),
                       c->scal + 4);
    PFT_HIP(c, hipGetLastError());
    return PFT_OK;
}

template <typename T>
pft_status densities_t(pft_ctx* c, double* phi_a, double* phi_b, double* Q)
{
    if (c->p.storage != PFT_STORE_BOTH) {
        // the contour sums were accumulated during the conjugate sweep
        hipLaunchKernelGGL(k_norm_density, dim3(grid_for(c->M, 256)), dim3(256), 0, c->stream, c->phi, c->phi + c->M,
                           c->M, c->scal, reinterpret_cast<double2*>(phi_a), reinterpret_cast<double2*>(phi_b),
                           reinterpret_cast<double2*>(Q));
        PFT_HIP(c, hipGetLastError());
        return PFT_OK;
    }
    ProfScope ps(c, PFT_K_DENSITY, (2.0 * (c->K + 1) * (double)c->elem + 2.0 * sizeof(double2)) * (double)c->M,
                 nullptr, true);
    PFT_LAUNCH((k_density<T>), dim3(grid_for(c->M, 256)), dim3(256), 0, c->stream,
                       static_cast<const cx<T>*>(c->qs), static_cast<const cx<T>*>(c->qds), c->K, c->J, c->M,
                       c->tau, c->scal, reinterpret_cast<double2*>(phi_a), reinterpret_cast<double2*>(phi_b),
                       reinterpret_cast<double2*>(Q));
    PFT_HIP(c, hipGetLastError());
    return PFT_OK;
}

template <typename T>
pft_status nodeq_t(pft_ctx* c, double* out)
{
    const int nb = std::min(c->nparts, 64);
    dim3 grid(nb, c->K + 1);
    hipLaunchKernelGGL((k_nodeq_partials<T>), grid, dim3(kRedThreads), 0, c->stream, static_cast<const cx<T>*>(c->qs),
                       static_cast<const cx<T>*>(c->qds), c->K, c->M, c->partials);
    hipLaunchKernelGGL(k_final_sum, dim3(c->K + 1), dim3(kRedThreads), 0, c->stream, c->partials, nb,
                       1.0 / (double)c->M, reinterpret_cast<double2*>(out), (double2*)nullptr, (uint32_t*)nullptr);
    PFT_HIP(c, hipGetLastError());
    return PFT_OK;
}

template <typename T>
pft_status get_slice_t(pft_ctx* c, int which, int node, double* out)
{
    const cx<T>* src;
    if (c->p.storage == PFT_STORE_HOST) {
        // bring the host slice into the first staging slot (ordered on the stream)
        cx<T>* slot = static_cast<cx<T>*>(c->ring);
        PFT_HIP(c, hipMemcpyAsync(slot, static_cast<const char*>(c->qh) + (size_t)node * c->M * c->elem,
                                  (size_t)c->M * c->elem, hipMemcpyHostToDevice, c->stream));
        src = slot;
    } else {
        src = slice<T>(which ? c->qds : c->qs, c, node);
    }
    hipLaunchKernelGGL((k_from_work<T>), dim3(grid_for(c->M, 256)), dim3(256), 0, c->stream, src,
                       reinterpret_cast<double2*>(out), c->M);
    PFT_HIP(c, hipGetLastError());
    return PFT_OK;
}

template <typename T>
pft_status apply_step_t(pft_ctx* c, int j, const double* qin, double* qout)
{
    cx<T>* w0 = static_cast<cx<T>*>(c->work);
    cx<T>* w1 = w0 + c->M;
    hipLaunchKernelGGL((k_to_work<T>), dim3(grid_for(c->M, 256)), dim3(256), 0, c->stream,
                       reinterpret_cast<const double2*>(qin), w0, c->M);
    PFT_HIP(c, hipGetLastError());
    pft_status s;
    if (c->fused) {
        s = yzpass<T>(c, -1, j, w0, nullptr);
        if (s) return s;
        s = xpass_step<T>(c, j);
        if (s) return s;
        s = yzpass<T>(c, j, -1, nullptr, w1);
    } else {
        s = zpass<T>(c, -1, j, w0, nullptr);
        if (s) return s;
        s = step_body<T>(c, j);
        if (s) return s;
        s = zpass<T>(c, j, -1, nullptr, w1);
    }
    if (s) return s;
    hipLaunchKernelGGL((k_from_work<T>), dim3(grid_for(c->M, 256)), dim3(256), 0, c->stream, w1,
                       reinterpret_cast<double2*>(qout), c->M);
    PFT_HIP(c, hipGetLastError());
    return PFT_OK;
}

template <typename T>
std::vector<T> axis_factors(int n, double L, double h)
{
    std::vector<T> g(n);
    for (int j = 0; j < n; ++j) {
        const int m = (j <= n / 2) ? j : j - n;
        const double k = kTwoPi * m / L;
        g[j] = T(std::exp(-k * k * h) / n);
    }
    return g;
}

// Tables of the walled line diffusion (pair_diffuse): for each frequency m of
// the reordered line, alpha_m = (g_m + g_{n-m}) / 2 and
// beta_m = (g_m - g_{n-m}) exp(i pi m / n) / 2, with g_m = exp(-(pi m / L)^2 h)
// for the cosine modes of reflecting walls and g_m = exp(-(pi (n - m) / L)^2 h)
// for the sine modes of absorbing walls (alpha_0 = g_0, beta_0 = 0), all / n.
// lap: g_m = k^2 of the same modes instead (-d^2/dx^2, for the box derivative).
template <typename T>
std::vector<T> wall_factors(int n, double L, double h, int bc, bool lap = false)
{
    auto g = [&](int m) {
        const double mode = bc == PFT_ABSORBING ? (double)(n - m) : (double)m;
        const double k = kPi * mode / L;
        return (lap ? k * k : std::exp(-k * k * h)) / n;
    };
    std::vector<T> ab(3 * (size_t)n);
    for (int m = 0; m < n; ++m) {
        double al = g(m), br = 0.0, bi = 0.0;
        if (m > 0) {
            const double gp = g(m), gq = g(n - m);
            al = 0.5 * (gp + gq);
            const double d = 0.5 * (gp - gq), th = kPi * m / n;
            br = d * std::cos(th);
            bi = d * std::sin(th);
        }
        ab[3 * m] = T(al);
        ab[3 * m + 1] = T(br);
        ab[3 * m + 2] = T(bi);
    }
    return ab;
}

template <typename T>
pft_status upload_factors(pft_ctx* c, int hid, double h)
{
    const int n[3] = {c->p.nx, c->p.ny, c->p.nz};
    const double L[3] = {c->p.lx, c->p.ly, c->p.lz};
    for (int full = 0; full < 2; ++full)
        for (int ax = 0; ax < 3; ++ax) {
            const double hh = full ? h : h / 2;
            const std::vector<T> g = c->p.bc[ax] ? wall_factors<T>(n[ax], L[ax], hh, c->p.bc[ax])
                                                 : axis_factors<T>(n[ax], L[ax], hh);
            PFT_HIP(c, hipMemcpy(const_cast<T*>(gptr<T>(c, hid, full, ax)), g.data(), g.size() * sizeof(T),
                                 hipMemcpyHostToDevice));
        }
    return PFT_OK;
}

// Spectral -d^2/dx_a^2 per axis, (2 pi m / L_a)^2 / N_a, in table slot 4
// (walled axes: the pair factors of (pi m / L_a)^2 / N_a).
template <typename T>
pft_status upload_second_derivative(pft_ctx* c)
{
    const int n[3] = {c->p.nx, c->p.ny, c->p.nz};
    const double L[3] = {c->p.lx, c->p.ly, c->p.lz};
    for (int ax = 0; ax < 3; ++ax) {
        if (c->p.bc[ax]) {
            const std::vector<T> g = wall_factors<T>(n[ax], L[ax], 0.0, c->p.bc[ax], true);
            PFT_HIP(c, hipMemcpy(const_cast<T*>(gptr<T>(c, 4, 0, ax)), g.data(), g.size() * sizeof(T),
                                 hipMemcpyHostToDevice));
            continue;
        }
        std::vector<T> g(n[ax]);
        for (int j = 0; j < n[ax]; ++j) {
            const int m = (j <= n[ax] / 2) ? j : j - n[ax];
            const double k = kTwoPi * m / L[ax];
            g[j] = T(k * k / n[ax]);
        }
        PFT_HIP(c, hipMemcpy(const_cast<T*>(gptr<T>(c, 4, 0, ax)), g.data(), g.size() * sizeof(T),
                             hipMemcpyHostToDevice));
    }
    return PFT_OK;
}

// D_h through the axis passes: u is staged in the working precision, run
// through the z, y and x passes with the full-step factors for h (kept in a
// spare table slot so the step tables stay intact) and read back from V.
// The work arrays are overwritten; the propagator stores are not touched.
template <typename T>
pft_status diffuse_t(pft_ctx* c, double* u, double h)
{
    PFT_HIP(c, hipStreamSynchronize(c->stream));  // earlier work may still read the spare slot
    pft_status s = upload_factors<T>(c, 3, h);
    if (s) return s;
    cx<T>* w0 = static_cast<cx<T>*>(c->work);
    hipLaunchKernelGGL((k_to_work<T>), dim3(grid_for(c->M, 256)), dim3(256), 0, c->stream,
                       reinterpret_cast<const double2*>(u), w0, c->M);
    PFT_HIP(c, hipGetLastError());
    pft::ZArgs<T> a{};
    a.nlines = (int64_t)c->p.nx * c->p.ny;
    a.U = static_cast<cx<T>*>(c->U);
    a.V = static_cast<cx<T>*>(c->V);
    a.qin = w0;
    a.scheme = PFT_SPLIT2;
    a.has_next = 1;
    a.gh_n = gptr<T>(c, 3, 0, 2);
    a.gf_n = gptr<T>(c, 3, 1, 2);
    PFT_HIP(c, launch_z<T>(c, a, c->stream));
    const pft::SOps<T> none{nullptr, nullptr, nullptr};
    s = spass<T>(c, 1, none, {gptr<T>(c, 3, 1, 1), nullptr, nullptr});
    if (s) return s;
    s = spass<T>(c, 0, none, {gptr<T>(c, 3, 1, 0), nullptr, nullptr});
    if (s) return s;
    hipLaunchKernelGGL((k_from_work<T>), dim3(grid_for(c->M, 256)), dim3(256), 0, c->stream,
                       static_cast<const cx<T>*>(c->V), reinterpret_cast<double2*>(u), c->M);
    PFT_HIP(c, hipGetLastError());
    return PFT_OK;
}

// ---------------------------------------------------------------- adjoint --
// Reverse mode through the K split steps.  The forward sweep keeps q only at
// the checkpoint nodes 0, Kc, 2Kc, ... and q_K.  The adjoint vector of step j
// is lambda_{j+1} = qd_{K-j-1} (each step operator is complex-symmetric), so
// the lambda sweep is the q-dagger sweep run on its own work pair.  Segments
// [a, b) are visited from the end; before the first of its steps is needed,
// each segment is recomputed forward from its checkpoint on the context's
// work pair, storing q_{a+1..b} and the captures A, B, C of every step.
template <typename T>
pft_status adjoint_t(pft_ctx* c, const double* wp, const double* wm, int Kc, double* dwp, double* dwm, double* dL,
                     double* H)
{
    const int K = c->K;
    const int64_t M = c->M;
    const bool rqm4 = c->p.scheme == PFT_RQM4;
    const int nck = (K + Kc - 1) / Kc;  // checkpoint nodes a = 0, Kc, ... < K
    // the segment buffers are doubled when the next segment's recomputation
    // runs on the second stream beside the current segment's adjoint steps
    const bool conc = c->s2 && !c->dual_off && nck > 1;
    const int nbuf = conc ? 2 : 1;
    const size_t nslices = (size_t)nck + 1 + 4 * (size_t)nbuf * Kc + 4 + 2;
    if (!c->adj || c->adj_kc != Kc || c->adj_slices != nslices) {
        if (c->adj) (void)hipFree(c->adj);
        c->adj = nullptr;
        if (hipMalloc(&c->adj, nslices * M * c->elem) != hipSuccess) {
            (void)hipGetLastError();
            c->adj_kc = 0;
            c->adj_slices = 0;
            return c->fail(PFT_E_NOMEM, "pft_adjoint: cannot allocate %zu slices", nslices);
        }
        c->adj_kc = Kc;
        c->adj_slices = nslices;
    }
    for (hipEvent_t* e : {&c->ev_adj[0], &c->ev_adj[1], &c->ev_adj[2], &c->ev_adj[3], &c->ev_adj[4]})
        if (!*e && hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            *e = nullptr;
            return c->fail(PFT_E_DEVICE, "pft_adjoint: cannot create events");
        }
    if (!c->adjG && hipMalloc((void**)&c->adjG, 4 * M * sizeof(double2)) != hipSuccess) {
        (void)hipGetLastError();
        c->adjG = nullptr;
        return c->fail(PFT_E_NOMEM, "pft_adjoint: cannot allocate accumulators");
    }
    // stress partials: one slot per workgroup of each axis's stress pass
    int64_t np = 1;
    for (int ax = 0; ax < 3; ++ax)
        np = std::max<int64_t>(np, pft::stress_blocks<T>(ax, c->p.nx, c->p.ny, c->p.nz));
    if (!c->adjAcc && hipMalloc((void**)&c->adjAcc, 3 * (size_t)np * sizeof(double2)) != hipSuccess) {
        (void)hipGetLastError();
        c->adjAcc = nullptr;
        return c->fail(PFT_E_NOMEM, "pft_adjoint: cannot allocate stress partials");
    }
    cx<T>* base = static_cast<cx<T>*>(c->adj);
    auto sl = [&](size_t i) { return base + i * (size_t)M; };
    auto ckpt = [&](int node) { return sl((size_t)(node / Kc)); };
    cx<T>* qK = sl(nck);
    size_t o = nck + 1;
    cx<T>* segQ[2];  // segQ[buf][i] = q_{a+1+i}
    cx<T>* segA[2];
    cx<T>* segB[2];
    cx<T>* segC[2];
    for (int bf = 0; bf < nbuf; ++bf) {
        segQ[bf] = sl(o); o += Kc;
        segA[bf] = sl(o); o += Kc;
        segB[bf] = sl(o); o += Kc;
        segC[bf] = sl(o); o += Kc;
    }
    if (nbuf == 1) {
        segQ[1] = segQ[0];
        segA[1] = segA[0];
        segB[1] = segB[0];
        segC[1] = segC[0];
    }
    cx<T>* lam[2] = {sl(o), sl(o + 1)}; o += 2;
    cx<T>* Al = sl(o++);
    cx<T>* Bl = sl(o++);
    const Work wl{sl(o), sl(o + 1)}; o += 2;
    auto seg = [&](cx<T>* buf, int i) { return buf + (size_t)i * M; };

    pft_status s = field_tables_t<T>(c, wp, wm);
    if (s) return s;
    // forward sweep keeping checkpoints
    s = zpass<T>(c, -1, 0, nullptr, ckpt(0));
    if (s) return s;
    for (int i = 0; i < K; ++i) {
        s = step_body<T>(c, i);
        if (s) return s;
        const int node = i + 1;
        cx<T>* out = node == K ? qK : (node % Kc == 0 ? ckpt(node) : nullptr);
        s = zpass<T>(c, i, i + 1 < K ? i + 1 : -1, nullptr, out);
        if (s) return s;
    }
    hipLaunchKernelGGL((k_sum_partials<T>), dim3(c->nparts), dim3(kRedThreads), 0, c->stream, qK, M, c->partials);
    hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(kRedThreads), 0, c->stream, c->partials, c->nparts,
                       1.0 / (double)M, c->scal, (double2*)nullptr, c->flags);
    PFT_HIP(c, hipGetLastError());
    s = hamiltonian_launch(c, wp, wm, H ? H : reinterpret_cast<double*>(c->scal + 1), nullptr);
    if (s) return s;
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(4 * M, 256)), dim3(256), 0, c->stream, c->adjG, 4 * M);
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(3 * np, 256)), dim3(256), 0, c->stream, c->adjAcc, (int64_t)3 * np);
    PFT_HIP(c, hipGetLastError());

    auto dtab = [&](int ax) { return gptr<T>(c, 4, 0, ax); };
    const double L[3] = {c->p.lx, c->p.ly, c->p.lz};

    // Segment sg covers steps [sg Kc, min(sg Kc + Kc, K)) and uses buffer
    // sg % 2.  Its recomputation (forward from its checkpoint, storing q and
    // the captures of each step) runs on the recompute stream rs, the next
    // lower segment's while this one's adjoint steps run on the context stream.
    const hipStream_t rs = conc ? c->s2 : c->stream;
    const Work wr{c->U, c->V, rs};
    auto recompute = [&](int sg) -> pft_status {
        const int a0 = sg * Kc, b0 = std::min(a0 + Kc, K), bf = sg % 2;
        pft_status e = zpass<T>(c, -1, a0, ckpt(a0), nullptr, wr);
        if (e) return e;
        for (int jj = a0; jj < b0; ++jj) {
            e = step_body<T>(c, jj, wr, rqm4 ? seg(segA[bf], jj - a0) : nullptr, rqm4 ? seg(segC[bf], jj - a0) : nullptr);
            if (e) return e;
            e = zpass<T>(c, jj, jj + 1 < b0 ? jj + 1 : -1, nullptr, seg(segQ[bf], jj - a0), wr, seg(segB[bf], jj - a0));
            if (e) return e;
        }
        PFT_HIP(c, hipEventRecord(c->ev_adj[bf], rs));  // ready
        return PFT_OK;
    };
    if (conc) {
        // the checkpoints are complete: start the last segment's recomputation
        PFT_HIP(c, hipEventRecord(c->ev_adj[4], c->stream));
        PFT_HIP(c, hipStreamWaitEvent(rs, c->ev_adj[4], 0));
        if ((s = recompute(nck - 1))) return s;
    }

    // lambda_K = 1, then the steps in reverse order
    s = zpass<T>(c, -1, K - 1, nullptr, lam[0], wl);
    if (s) return s;
    int cur = 0;
    for (int j = K - 1; j >= 0; --j) {
        const int a = (j / Kc) * Kc, b = std::min(a + Kc, K);
        const int sg = j / Kc, bf = sg % 2;
        if (j == b - 1) {
            if (!conc) {
                // one buffer on one stream: recompute this segment in place
                if ((s = recompute(sg))) return s;
            } else {
                PFT_HIP(c, hipStreamWaitEvent(c->stream, c->ev_adj[bf], 0));
                if (sg > 0) {
                    // the next lower segment reuses the buffer of the segment
                    // above this one, whose adjoint steps are all enqueued
                    PFT_HIP(c, hipEventRecord(c->ev_adj[2], c->stream));
                    PFT_HIP(c, hipStreamWaitEvent(rs, c->ev_adj[2], 0));
                    if ((s = recompute(sg - 1))) return s;
                }
            }
        }
        cx<T>* const sQ = segQ[bf];
        cx<T>* const sA = segA[bf];
        cx<T>* const sB = segB[bf];
        cx<T>* const sC = segC[bf];
        s = step_body<T>(c, j, wl, rqm4 ? Al : nullptr, nullptr);
        if (s) return s;
        s = zpass<T>(c, j, j > 0 ? j - 1 : -1, nullptr, lam[1 - cur], wl, rqm4 ? Bl : nullptr);
        if (s) return s;
        const cx<T>* q0 = (j == a) ? ckpt(a) : seg(sQ, j - a - 1);
        AccArgs<T> ac{lam[cur], lam[1 - cur], Al, Bl, q0, seg(sQ, j - a), seg(sA, j - a), seg(sB, j - a),
                      etab<T>(c, c->kind[j]), c->h[j], rqm4 ? 1 : 0, M,
                      c->adjG + (c->blk[j] == 0 ? 0 : 2 * M), c->adjG + (c->blk[j] == 0 ? M : 3 * M)};
        {
            ProfScope ps(c, PFT_K_REDUCE, (9.0 * c->elem + 64.0) * (double)M);
            hipLaunchKernelGGL((k_adj_accum<T>), dim3(grid_for(M, 256)), dim3(256), 0, c->stream, ac);
        }
        PFT_HIP(c, hipGetLastError());
        if (dL) {
            // -d^2/dx_a^2 of each capture along each axis, dotted with its partner
            pft::StressPass<T> sp{};
            sp.X[0] = seg(sB, j - a);
            sp.X[1] = seg(sA, j - a);
            sp.X[2] = rqm4 ? seg(sC, j - a) : seg(sB, j - a);  // plain split: D_h E2 q
            sp.first = rqm4 ? 0 : 2;
            sp.lam = lam[cur];
            sp.Alam = Al;
            sp.E4 = etab<T>(c, c->kind[j]);
            for (int ax = 0; ax < 3; ++ax) {
                const double r = c->h[j] / L[ax];
                sp.coef[0] = rqm4 ? 4.0 / 3.0 * r : 0.0;
                sp.coef[1] = rqm4 ? 4.0 / 3.0 * r : 0.0;
                sp.coef[2] = rqm4 ? -2.0 / 3.0 * r : 2.0 * r;
                sp.d2 = dtab(ax);
                sp.part = c->adjAcc + (size_t)ax * np;
                if (c->p.bc[ax])
                    PFT_HIP(c, pft::launch_stress_walls<T>(ax, c->p.bc[ax], c->p.nx, c->p.ny, c->p.nz, sp, c->stream));
                else
                    PFT_HIP(c, pft::launch_stress<T>(ax, c->p.nx, c->p.ny, c->p.nz, sp, c->stream));
            }
        }
        cur = 1 - cur;
    }
    const double dV = c->p.lx * c->p.ly * c->p.lz / (double)M;
    hipLaunchKernelGGL(k_adj_final, dim3(grid_for(M, 256)), dim3(256), 0, c->stream, c->adjG, M,
                       reinterpret_cast<const double2*>(wm), c->scal, c->p.C, dV, c->p.chiN,
                       reinterpret_cast<double2*>(dwp), reinterpret_cast<double2*>(dwm));
    PFT_HIP(c, hipGetLastError());
    if (dL) {
        hipLaunchKernelGGL(k_final_sum, dim3(3), dim3(kRedThreads), 0, c->stream, c->adjAcc, (int)np, 1.0,
                           c->scal + 5, (double2*)nullptr, (uint32_t*)nullptr);
        hipLaunchKernelGGL(k_stress_final, dim3(1), dim3(64), 0, c->stream, c->scal + 5, c->scal + 4, c->scal,
                           c->p.C, c->p.lx, c->p.ly, c->p.lz, M, reinterpret_cast<double2*>(dL));
        PFT_HIP(c, hipGetLastError());
    }
    return PFT_OK;
}

// Argument sets of the passes, built without launching (the batched tables
// hold one per replica and sweep position).
template <typename T>
pft::ZArgs<T> zargs(const pft_ctx* c, int prev, int next, const cx<T>* qin, cx<T>* qout)
{
    pft::ZArgs<T> a{};
    a.nlines = (int64_t)c->p.nx * c->p.ny;
    a.U = static_cast<cx<T>*>(c->U);
    a.V = static_cast<cx<T>*>(c->V);
    a.qin = qin;
    a.qout = qout;
    a.scheme = c->p.scheme;
    a.has_prev = prev >= 0;
    a.has_next = next >= 0;
    if (prev >= 0) {
        a.Ep = etab<T>(c, c->kind[prev]);
        a.gh_p = gptr<T>(c, c->hid[prev], 0, 2);
    }
    if (next >= 0) {
        a.En = etab<T>(c, c->kind[next]);
        a.gh_n = gptr<T>(c, c->hid[next], 0, 2);
        a.gf_n = gptr<T>(c, c->hid[next], 1, 2);
    }
    return a;
}

template <typename T>
pft::PArgs<T> pargs(const pft_ctx* c, int prev, int next, const cx<T>* qin, cx<T>* qout)
{
    pft::PArgs<T> a{};
    a.nplanes = c->p.nx;
    a.U = static_cast<cx<T>*>(c->U);
    a.V = static_cast<cx<T>*>(c->V);
    a.qin = qin;
    a.qout = qout;
    a.scheme = c->p.scheme;
    a.has_prev = prev >= 0;
    a.has_next = next >= 0;
    if (prev >= 0) {
        a.Ep = etab<T>(c, c->kind[prev]);
        a.gyh_p = gptr<T>(c, c->hid[prev], 0, 1);
        a.gzh_p = gptr<T>(c, c->hid[prev], 0, 2);
    }
    if (next >= 0) {
        a.En = etab<T>(c, c->kind[next]);
        a.gzh_n = gptr<T>(c, c->hid[next], 0, 2);
        a.gzf_n = gptr<T>(c, c->hid[next], 1, 2);
        a.gyh_n = gptr<T>(c, c->hid[next], 0, 1);
        a.gyf_n = gptr<T>(c, c->hid[next], 1, 1);
    }
    return a;
}

template <typename T>
pft::SArgs<T> sargs(const pft_ctx* c, int axis, pft::SOps<T> opU, pft::SOps<T> opV)
{
    pft::SArgs<T> a{};
    a.U = static_cast<cx<T>*>(c->U);
    a.V = static_cast<cx<T>*>(c->V);
    a.opU = opU;
    a.opV = opV;
    const int64_t nynz = (int64_t)c->p.ny * c->p.nz;
    if (axis == 0) {
        a.S = nynz;
        a.slab_stride = 0;
        a.ncols = (int)nynz;
        a.ntiles = pft::spass_tiles<T>(c->p.nx, c->var[0], nynz);
    } else {
        a.S = c->p.nz;
        a.slab_stride = nynz;
        a.ncols = c->p.nz;
        a.ntiles = pft::spass_tiles<T>(c->p.ny, c->var[1], c->p.nz);
    }
    return a;
}

// The strided passes of step j, in order (three for the Richardson step,
// two for the plain split), as in step_body.
template <typename T>
int body_passes(const pft_ctx* c, int j, int axis[3], pft::SArgs<T> out[3])
{
    const int hd = c->hid[j];
    const cx<T>* e = etab<T>(c, c->kind[j]);
    const pft::SOps<T> none{nullptr, nullptr, nullptr};
    if (c->p.scheme == PFT_RQM4) {
        axis[0] = 1;
        out[0] = sargs<T>(c, 1, {gptr<T>(c, hd, 0, 1), nullptr, nullptr}, {gptr<T>(c, hd, 1, 1), nullptr, nullptr});
        axis[1] = 0;
        out[1] = sargs<T>(c, 0, {gptr<T>(c, hd, 0, 0), e, gptr<T>(c, hd, 0, 0)}, {gptr<T>(c, hd, 1, 0), e, nullptr});
        axis[2] = 1;
        out[2] = sargs<T>(c, 1, {gptr<T>(c, hd, 0, 1), nullptr, nullptr}, none);
        return 3;
    }
    axis[0] = 1;
    out[0] = sargs<T>(c, 1, none, {gptr<T>(c, hd, 1, 1), nullptr, nullptr});
    axis[1] = 0;
    out[1] = sargs<T>(c, 0, none, {gptr<T>(c, hd, 1, 0), nullptr, nullptr});
    return 2;
}

void free_all(pft_ctx* c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    if (c->gs) {
        (void)hipStreamSynchronize(c->gs);
        (void)hipStreamDestroy(c->gs);
        c->gs = nullptr;
    }
    for (hipEvent_t* e : {&c->ev_g0, &c->ev_g1})
        if (*e) {
            (void)hipEventDestroy(*e);
            *e = nullptr;
        }
    for (hipEvent_t& e : c->ev_adj)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    c->ev.clear();
    if (c->s2) (void)hipStreamDestroy(c->s2);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    c->s2 = nullptr;
    if (c->qds == c->qs) c->qds = nullptr;
    if (c->cs) {
        (void)hipStreamSynchronize(c->cs);
        (void)hipStreamDestroy(c->cs);
        c->cs = nullptr;
    }
    for (int k = 0; k < kRing; ++k)
        for (hipEvent_t* e : {&c->ev_st[k], &c->ev_cp[k], &c->ev_rd[k], &c->ev_fr[k]})
            if (*e) {
                (void)hipEventDestroy(*e);
                *e = nullptr;
            }
    if (c->ev_done) (void)hipEventDestroy(c->ev_done);
    c->ev_done = nullptr;
    if (c->qh) (void)hipHostFree(c->qh);
    c->qh = nullptr;
    void* bufs[] = {c->qs,  c->qds,  c->U,        c->V,    c->U2,    c->V2,  c->E,   c->work,
                    c->gtab, c->tau, c->phi,      c->partials, c->scal, c->flags, c->adj, c->adjG,
                    c->adjAcc, c->k2, c->sisbuf, c->sisext, c->ring};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
}

}  // namespace


// The semi-implicit step (defined with the field steps below).
static pft_status sis_prepare(pft_ctx* c);
static pft_status sis_upload_k2(pft_ctx* c);
// Work memory of one semi-implicit step: the increment R (M sites), between
// reflecting walls its even image X and the image's update W (Me sites each),
// and |k|^2 per axis (3 rows of `pitch` doubles, natural order).
struct SisBufs {
    double2* R = nullptr;
    double2* X = nullptr;
    double2* W = nullptr;
    const double* k2 = nullptr;
    int pitch = 0;
};
static SisBufs ctx_sis_bufs(const pft_ctx* c);
static SisIncArgs sis_inc_args(const pft_ctx* c, const SisBufs& sb, const UpdArgs& u, const uint64_t* step_dev);
static pft::SisArgs sis_filter_args(const SisBufs& sb, const UpdArgs& u, double2* X, double2* W, int ne_z,
                                    int64_t Me);
static MirrorArgs sis_image(const pft_ctx* c, const SisBufs& sb);
static const char* sis_walls_unsupported(const pft_params& p);

// ================================================================ batches ==
// Many independent replicas (uneven grids, contour step counts, f, chi N) run
// together: replicas are grouped by grid shape; every pass of a group is one
// launch over all its replicas, whose arguments for each sweep position come
// from device tables built once; groups run on their own streams; one field
// step of the whole batch is captured into a HIP graph and replayed.
namespace {

struct BatchGroup {
    int nx = 0, ny = 0, nz = 0;
    int bc[3] = {0, 0, 0};       // walls of the group's replicas (fused groups have none on y and z)
    int ndir = 2;                // sweeps per evaluation: 2, or 1 for the Edwards model (q-dagger = q)
    std::vector<int> reps;
    int maxK = 0;
    int64_t maxM = 0;
    int npass = 0;               // strided passes per step (3 or 2)
    int sp_axis[3] = {0, 0, 0};
    int var[3] = {0, 0, 0};      // kernel variants (x, y, z) of the group's grid
    bool fused = false;          // fused yz-plane schedule: zd holds PArgs, sd the x passes only
    hipStream_t s = nullptr;
    hipEvent_t done = nullptr;
    void* zd = nullptr;          // [dir 2][pos maxK+1][R] ZArgs (PArgs when fused)
    void* sd = nullptr;          // [dir 2][pos maxK][npass][R] SArgs
    void* jobs[2] = {nullptr, nullptr};  // job tables of the small kernels: [0] evaluations, [1] the captured field step
    size_t off_sisinc = 0, off_sis = 0;  // semi-implicit step: [R] SisIncArgs, [5 passes][R] SisArgs,
    size_t off_mirror = 0;               //   [R] MirrorJob (walled groups: the filter runs on the even image)
    size_t off_tab = 0, off_sum = 0, off_fin = 0, off_dens = 0, off_ham = 0, off_upd = 0;
};

}  // namespace

struct pft_batch {
    int n = 0;
    int precision = 0, scheme = 0, model = 0;
    hipStream_t stream = nullptr;  // the caller's stream
    hipStream_t own = nullptr;     // the batch's stream: work is captured and replayed here
    std::vector<pft_ctx*> ctx;
    std::vector<BatchGroup> groups;
    hipEvent_t fork = nullptr;
    hipEvent_t in = nullptr, out = nullptr;  // joins with the caller's stream
    uint64_t* counters = nullptr;  // [0] Langevin step, [1] log row
    LogJob* logj = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const double*> gwp, gwm;  // field pointers baked into the graph
    std::vector<const void*> ekey;        // pointers held by the evaluation job tables
    pft_step gst{};
    double* glog = nullptr;
    int64_t gcap = 0;
    std::string err;

    pft_status fail(pft_status s, const char* fmt, ...)
    {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        return s;
    }
};

namespace {

#define PFT_BHIP(b, call)                                                                              \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return (b)->fail(PFT_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));             \
    } while (0)

void batch_free(pft_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (BatchGroup& g : b->groups) {
        if (g.s) (void)hipStreamDestroy(g.s);
        if (g.done) (void)hipEventDestroy(g.done);
        if (g.zd) (void)hipFree(g.zd);
        if (g.sd) (void)hipFree(g.sd);
        for (void* j : g.jobs)
            if (j) (void)hipFree(j);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->in) (void)hipEventDestroy(b->in);
    if (b->out) (void)hipEventDestroy(b->out);
    if (b->own) (void)hipStreamDestroy(b->own);
    if (b->counters) (void)hipFree(b->counters);
    if (b->logj) (void)hipFree(b->logj);
    for (pft_ctx* c : b->ctx) pft_destroy(c);
}

// Argument tables of the passes of one group, for both sweeps and every
// sweep position; a replica whose K is exhausted is marked skip.
template <typename T>
pft_status batch_build_pass_tables(pft_batch* b, BatchGroup& g)
{
    const int R = (int)g.reps.size();
    const int D = g.ndir;
    std::vector<pft::ZArgs<T>> zd(g.fused ? 0 : (size_t)D * (g.maxK + 1) * R);
    std::vector<pft::PArgs<T>> pd(g.fused ? (size_t)D * (g.maxK + 1) * R : 0);
    std::vector<pft::SArgs<T>> sd((size_t)D * g.maxK * g.npass * R);
    for (int dir = 0; dir < g.ndir; ++dir)
        for (int ri = 0; ri < R; ++ri) {
            pft_ctx* c = b->ctx[g.reps[ri]];
            const int K = c->K;
            auto stepj = [&](int i) { return dir ? K - 1 - i : i; };
            void* store = dir ? c->qds : c->qs;
            // the two sweeps advance in the same launches, so each has its own work pair
            cx<T>* wU = static_cast<cx<T>*>(dir ? c->U2 : c->U);
            cx<T>* wV = static_cast<cx<T>*>(dir ? c->V2 : c->V);
            for (int p = 0; p <= g.maxK; ++p) {
                const int i = p - 1;  // Z (or yz) at position p completes step i and starts step i + 1
                const size_t at = ((size_t)p * D + dir) * R + ri;
                const int prev = i >= 0 ? stepj(i) : -1, next = i + 1 < K ? stepj(i + 1) : -1;
                if (g.fused) {
                    if (i >= K) {
                        pd[at].skip = 1;
                    } else {
                        pd[at] = pargs<T>(c, prev, next, nullptr, slice<T>(store, c, i + 1));
                        pd[at].U = wU;
                        pd[at].V = wV;
                    }
                } else {
                    if (i >= K) {
                        zd[at].skip = 1;
                    } else {
                        zd[at] = zargs<T>(c, prev, next, nullptr, slice<T>(store, c, i + 1));
                        zd[at].U = wU;
                        zd[at].V = wV;
                    }
                }
            }
            for (int p = 0; p < g.maxK; ++p) {
                int ax[3];
                pft::SArgs<T> sa[3];
                if (p < K) body_passes<T>(c, stepj(p), ax, sa);
                for (int k = 0; k < g.npass; ++k) {
                    pft::SArgs<T>& d = sd[(((size_t)p * g.npass + k) * D + dir) * R + ri];
                    if (p >= K) {
                        d.skip = 1;
                        continue;
                    }
                    d = g.fused ? sa[1] : sa[k];  // fused: the x pass alone
                    d.U = wU;
                    d.V = wV;
                    const int axk = g.sp_axis[k];
                    if (g.bc[axk])  // walled kernels take the default tile
                        d.ntiles = pft::spass_tiles<T>(axk == 0 ? g.nx : g.ny, 0, d.ncols);
                }
            }
        }
    const size_t zbytes = g.fused ? pd.size() * sizeof(pd[0]) : zd.size() * sizeof(zd[0]);
    PFT_BHIP(b, hipMalloc(&g.zd, zbytes));
    PFT_BHIP(b, hipMalloc(&g.sd, std::max<size_t>(1, sd.size()) * sizeof(pft::SArgs<T>)));
    PFT_BHIP(b, hipMemcpy(g.zd, g.fused ? (const void*)pd.data() : (const void*)zd.data(), zbytes,
                          hipMemcpyHostToDevice));
    if (!sd.empty()) PFT_BHIP(b, hipMemcpy(g.sd, sd.data(), sd.size() * sizeof(sd[0]), hipMemcpyHostToDevice));
    return PFT_OK;
}

// Job tables of the small kernels of one group for the given field pointers
// and outputs (phi / Q / H default to each context's internal buffers).
template <typename T>
pft_status batch_build_jobs(pft_batch* b, BatchGroup& g, int slot, const double* const* wp, const double* const* wm,
                            double* const* phia, double* const* phib, double* Qout, double* Hout, const pft_step* st)
{
    const int R = (int)g.reps.size();
    std::vector<TabJob<T>> tab(R);
    std::vector<SumJob<T>> sum(R);
    std::vector<FinJob> fin(R);
    std::vector<DensJob<T>> dens(R);
    std::vector<HamJob> ham(R);
    std::vector<UpdArgs> upd(R);
    constexpr int kQParts = 64;
    for (int ri = 0; ri < R; ++ri) {
        const int r = g.reps[ri];
        pft_ctx* c = b->ctx[r];
        const bool ed = c->p.model == PFT_EDWARDS;  // one field omega (in wp), q-dagger = q
        const double* wmr = ed ? nullptr : wm[r];
        TabDesc d{};
        d.n = ed ? 1 : c->K == c->p.ns ? 2 : 4;
        d.blk[0] = 0; d.a[0] = c->hval[0] / 4;
        d.blk[1] = 1; d.a[1] = c->hval[0] / 4;
        d.blk[2] = 0; d.a[2] = c->hval[1] / 4;
        d.blk[3] = 1; d.a[3] = c->hval[2] / 4;
        tab[ri] = {reinterpret_cast<const double2*>(wp[r]), reinterpret_cast<const double2*>(wmr), c->M, d,
                   static_cast<cx<T>*>(c->E)};
        sum[ri] = {slice<T>(c->qs, c, c->K), c->M, c->partials};
        fin[ri] = {c->partials, kQParts, 1.0 / (double)c->M, c->scal, c->flags};
        double2* pa = phia ? reinterpret_cast<double2*>(phia[r]) : c->phi;
        double2* pb = phib ? reinterpret_cast<double2*>(phib[r]) : c->phi + c->M;
        dens[ri] = {static_cast<const cx<T>*>(c->qs), static_cast<const cx<T>*>(c->qds), c->K, c->J, c->M, c->tau,
                    c->scal, pa, pb, Qout ? reinterpret_cast<double2*>(Qout) + r : nullptr};
        const double V = c->p.lx * c->p.ly * c->p.lz;
        // diblock: sum w_-^2/chiN - i w_+;  Edwards: sum (B/(2C)) omega^2
        ham[ri] = {ed ? nullptr : reinterpret_cast<const double2*>(wp[r]),
                   reinterpret_cast<const double2*>(ed ? wp[r] : wmr), c->M,
                   ed ? c->p.B / (2.0 * c->p.C) : 1.0 / c->p.chiN, c->partials + kQParts, kQParts, c->p.C,
                   V / (double)c->M, V, c->scal, Hout ? reinterpret_cast<double2*>(Hout) + r : c->scal + 1,
                   c->scal + 2, c->scal + 4};
        UpdArgs a{};
        if (st) {
            const double dV = V / (double)c->M;
            a.wp = reinterpret_cast<double2*>(const_cast<double*>(wp[r]));
            a.wm = reinterpret_cast<double2*>(const_cast<double*>(wmr));
            a.phiA = pa;
            a.phiB = pb;
            a.M = c->M;
            a.two_over_chiN = 2.0 / c->p.chiN;
            a.dtp = st->lambda_plus * st->dt;
            a.dtm = st->lambda_minus * st->dt;
            a.noise = st->noise != 0;
            a.sp = a.noise ? std::sqrt(2.0 * st->lambda_plus * st->dt / (c->p.C * dV)) : 0.0;
            a.sm = a.noise ? std::sqrt(2.0 * st->lambda_minus * st->dt / (c->p.C * dV)) : 0.0;
            a.seed = st->seed;
            a.rep = st->replica + (uint64_t)r;
            a.step = 0;  // the device step counter is added at run time
            if (ed) {
                a.edwards = 1;
                a.b_over_c = c->p.B / c->p.C;
            }
        }
        upd[ri] = a;
    }
    size_t o = 0;
    auto place = [&](size_t bytes) {
        const size_t at = o;
        o += (bytes + 255) & ~size_t(255);
        return at;
    };
    g.off_tab = place(R * sizeof(TabJob<T>));
    g.off_sum = place(R * sizeof(SumJob<T>));
    g.off_fin = place(R * sizeof(FinJob));
    g.off_dens = place(R * sizeof(DensJob<T>));
    g.off_ham = place(R * sizeof(HamJob));
    g.off_upd = place(R * sizeof(UpdArgs));
    g.off_sisinc = place(R * sizeof(SisIncArgs));
    g.off_sis = place(5 * R * sizeof(pft::SisArgs));
    g.off_mirror = place(R * sizeof(MirrorJob));
    if (!g.jobs[slot]) PFT_BHIP(b, hipMalloc(&g.jobs[slot], o));
    char* base = static_cast<char*>(g.jobs[slot]);
    PFT_BHIP(b, hipMemcpy(base + g.off_tab, tab.data(), R * sizeof(tab[0]), hipMemcpyHostToDevice));
    PFT_BHIP(b, hipMemcpy(base + g.off_sum, sum.data(), R * sizeof(sum[0]), hipMemcpyHostToDevice));
    PFT_BHIP(b, hipMemcpy(base + g.off_fin, fin.data(), R * sizeof(fin[0]), hipMemcpyHostToDevice));
    PFT_BHIP(b, hipMemcpy(base + g.off_dens, dens.data(), R * sizeof(dens[0]), hipMemcpyHostToDevice));
    PFT_BHIP(b, hipMemcpy(base + g.off_ham, ham.data(), R * sizeof(ham[0]), hipMemcpyHostToDevice));
    PFT_BHIP(b, hipMemcpy(base + g.off_upd, upd.data(), R * sizeof(upd[0]), hipMemcpyHostToDevice));
    if (st && st->update == 1) {
        // the filter buffers exist (sis_prepare ran for every replica); the
        // noise step is read from the batch's device counter
        std::vector<SisIncArgs> inc(R);
        std::vector<pft::SisArgs> fil(5 * (size_t)R);
        std::vector<MirrorJob> mir(R);
        const bool walls = g.bc[0] || g.bc[1] || g.bc[2];
        for (int ri = 0; ri < R; ++ri) {
            const pft_ctx* c = b->ctx[g.reps[ri]];
            const SisBufs sb = ctx_sis_bufs(c);
            inc[ri] = sis_inc_args(c, sb, upd[ri], b->counters);
            const MirrorArgs ma = sis_image(c, sb);
            mir[ri] = {ma, upd[ri].wp, c->M};
            const pft::SisArgs f = walls ? sis_filter_args(sb, upd[ri], ma.X, ma.W, ma.ne[2], ma.Me)
                                         : sis_filter_args(sb, upd[ri], sb.R, upd[ri].wp, g.nz, c->M);
            for (int kind = 0; kind < 5; ++kind) {
                pft::SisArgs& e = fil[(size_t)kind * R + ri];
                e = f;
                if (!pft::sis_pass_layout(kind, ma.ne[0], ma.ne[1], ma.ne[2], &e))
                    return b->fail(PFT_E_UNSUPPORTED, "semi-implicit step: no kernel for this grid");
            }
        }
        PFT_BHIP(b, hipMemcpy(base + g.off_sisinc, inc.data(), R * sizeof(inc[0]), hipMemcpyHostToDevice));
        PFT_BHIP(b, hipMemcpy(base + g.off_sis, fil.data(), fil.size() * sizeof(fil[0]), hipMemcpyHostToDevice));
        PFT_BHIP(b, hipMemcpy(base + g.off_mirror, mir.data(), R * sizeof(mir[0]), hipMemcpyHostToDevice));
    }
    return PFT_OK;
}

// Enqueue one evaluation (and, if update, the field step: explicit, or
// semi-implicit when sis) of one group on its stream.
template <typename T>
pft_status batch_enqueue_group(pft_batch* b, BatchGroup& g, int slot, bool update, bool sis)
{
    const int R = (int)g.reps.size();
    hipStream_t s = g.s;
    char* jb = static_cast<char*>(g.jobs[slot]);
    const int64_t nlines = (int64_t)g.nx * g.ny;
    hipLaunchKernelGGL((k_tables_batch<T>), dim3(grid_for(g.maxM, 256), R), dim3(256), 0, s,
                       reinterpret_cast<const TabJob<T>*>(jb + g.off_tab));
    PFT_BHIP(b, hipGetLastError());
    const pft::ZArgs<T>* zd = static_cast<const pft::ZArgs<T>*>(g.zd);
    const pft::SArgs<T>* sd = static_cast<const pft::SArgs<T>*>(g.sd);
    const int n_ax[2] = {g.nx, g.ny};
    const int64_t ncols[2] = {(int64_t)g.ny * g.nz, g.nz};
    const int nslabs[2] = {1, g.nx};
    const pft::PArgs<T>* pd = static_cast<const pft::PArgs<T>*>(g.zd);
    // Both sweeps advance together: every launch at sweep position p covers
    // the q and the q-dagger work of all replicas of the group (D R table
    // entries, laid out [position][pass][sweep][replica]).
    const int DR = g.ndir * R;
    // the z pass, or the fused yz pass, at sweep position p
    auto zlaunch = [&](int p) -> hipError_t {
        const size_t at = (size_t)p * DR;
        if (g.fused) return pft::launch_yzpass_batch<T>(g.ny, g.nx, pd + at, DR, s);
        if (g.bc[2]) return pft::launch_zpass_walls_batch<T>(g.nz, g.bc[2], nlines, zd + at, DR, s);
        return pft::launch_zpass_batch<T>(g.nz, g.var[2], nlines, zd + at, DR, s);
    };
    PFT_BHIP(b, zlaunch(0));
    for (int p = 0; p < g.maxK; ++p) {
        for (int k = 0; k < g.npass; ++k) {
            const int ax = g.sp_axis[k];
            const pft::SArgs<T>* at = sd + ((size_t)p * g.npass + k) * DR;
            if (g.bc[ax])
                PFT_BHIP(b, pft::launch_spass_walls_batch<T>(ax, n_ax[ax], g.bc[ax], ncols[ax], nslabs[ax], at, DR, s));
            else
                PFT_BHIP(b, pft::launch_spass_batch<T>(ax, n_ax[ax], g.var[ax], ncols[ax], nslabs[ax], at, DR, s));
        }
        PFT_BHIP(b, zlaunch(p + 1));
    }
    hipLaunchKernelGGL((k_sum_partials_batch<T>), dim3(64, R), dim3(kRedThreads), 0, s,
                       reinterpret_cast<const SumJob<T>*>(jb + g.off_sum));
    hipLaunchKernelGGL(k_final_batch, dim3(1, R), dim3(kRedThreads), 0, s, reinterpret_cast<const FinJob*>(jb + g.off_fin));
    hipLaunchKernelGGL((k_density_batch<T>), dim3(grid_for(g.maxM, 256), R), dim3(256), 0, s,
                       reinterpret_cast<const DensJob<T>*>(jb + g.off_dens));
    hipLaunchKernelGGL(k_ham_partials_batch, dim3(64, R), dim3(kRedThreads), 0, s,
                       reinterpret_cast<const HamJob*>(jb + g.off_ham));
    hipLaunchKernelGGL(k_ham_final_batch, dim3(1, R), dim3(kRedThreads), 0, s,
                       reinterpret_cast<const HamJob*>(jb + g.off_ham));
    if (update && !sis)
        hipLaunchKernelGGL(k_update_batch, dim3(grid_for((g.maxM + 3) / 4, 256), R), dim3(256), 0, s,
                           reinterpret_cast<const UpdArgs*>(jb + g.off_upd), b->counters);
    PFT_BHIP(b, hipGetLastError());
    if (update && sis) {
        // the local increment, then the five filter passes, each one launch
        // over the group's replicas
        hipLaunchKernelGGL(k_sis_increment_batch, dim3(grid_for((g.maxM + 3) / 4, 256), R), dim3(256), 0, s,
                           reinterpret_cast<const SisIncArgs*>(jb + g.off_sisinc));
        PFT_BHIP(b, hipGetLastError());
        // reflecting walls: the filter runs on the even image of the increment
        const int ne[3] = {g.bc[0] ? 2 * g.nx : g.nx, g.bc[1] ? 2 * g.ny : g.ny, g.bc[2] ? 2 * g.nz : g.nz};
        const int64_t Me = (int64_t)ne[0] * ne[1] * ne[2];
        const bool walls = g.bc[0] || g.bc[1] || g.bc[2];
        const MirrorJob* mir = reinterpret_cast<const MirrorJob*>(jb + g.off_mirror);
        if (walls) hipLaunchKernelGGL(k_sis_mirror_batch, dim3(grid_for(Me, 256), R), dim3(256), 0, s, mir);
        PFT_BHIP(b, hipGetLastError());
        const pft::SisArgs* fil = reinterpret_cast<const pft::SisArgs*>(jb + g.off_sis);
        for (int kind = 0; kind < 5; ++kind)
            PFT_BHIP(b, pft::launch_sis_pass_batch(kind, ne[0], ne[1], ne[2], fil + (size_t)kind * R, R, s));
        if (walls) hipLaunchKernelGGL(k_sis_unmirror_batch, dim3(grid_for(g.maxM, 256), R), dim3(256), 0, s, mir);
        PFT_BHIP(b, hipGetLastError());
    }
    return PFT_OK;
}

// Fork the group streams off the batch stream, enqueue every group, join.
template <typename T>
pft_status batch_enqueue(pft_batch* b, int slot, bool update, bool sis, const double2* logbuf, int64_t cap)
{
    PFT_BHIP(b, hipEventRecord(b->fork, b->own));
    for (BatchGroup& g : b->groups) {
        PFT_BHIP(b, hipStreamWaitEvent(g.s, b->fork, 0));
        pft_status st = batch_enqueue_group<T>(b, g, slot, update, sis);
        if (st) return st;
        PFT_BHIP(b, hipEventRecord(g.done, g.s));
        PFT_BHIP(b, hipStreamWaitEvent(b->own, g.done, 0));
    }
    if (update) {
        if (logbuf)
            hipLaunchKernelGGL(k_batch_log, dim3((b->n + 255) / 256), dim3(256), 0, b->own, b->logj, b->n,
                               const_cast<double2*>(logbuf), b->counters + 1, (uint64_t)cap);
        hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, b->own, b->counters, b->counters + 1);
        PFT_BHIP(b, hipGetLastError());
    }
    return PFT_OK;
}

template <typename T>
pft_status batch_setup_t(pft_batch* b)
{
    for (BatchGroup& g : b->groups) {
        pft_status s = batch_build_pass_tables<T>(b, g);
        if (s) return s;
    }
    return PFT_OK;
}

// Wait until nothing queued on the batch's own and group streams remains:
// the job tables are rewritten with host copies, which are not ordered after
// that work, and a graph still replaying must not be destroyed.
pft_status batch_quiesce(pft_batch* b)
{
    PFT_BHIP(b, hipStreamSynchronize(b->own));
    for (BatchGroup& g : b->groups) PFT_BHIP(b, hipStreamSynchronize(g.s));
    return PFT_OK;
}

template <typename T>
pft_status batch_evaluate_t(pft_batch* b, const double* const* wp, const double* const* wm, double* const* pa,
                            double* const* pb, double* Q, double* H)
{
    // the evaluation tables (slot 0) are rebuilt only when a pointer changes;
    // the captured field step keeps its own tables (slot 1)
    std::vector<const void*> key;
    key.reserve(4 * (size_t)b->n + 2);
    for (int r = 0; r < b->n; ++r) {
        key.push_back(wp[r]);
        key.push_back(wm ? wm[r] : nullptr);
        key.push_back(pa[r]);
        key.push_back(pb[r]);
    }
    key.push_back(Q);
    key.push_back(H);
    if (key != b->ekey) {
        b->ekey.clear();
        pft_status s = batch_quiesce(b);
        if (s) return s;
        for (BatchGroup& g : b->groups) {
            s = batch_build_jobs<T>(b, g, 0, wp, wm, pa, pb, Q, H, nullptr);
            if (s) return s;
        }
        b->ekey = std::move(key);
    }
    PFT_BHIP(b, hipEventRecord(b->in, b->stream));
    PFT_BHIP(b, hipStreamWaitEvent(b->own, b->in, 0));
    pft_status s = batch_enqueue<T>(b, 0, false, false, nullptr, 0);
    if (s) return s;
    PFT_BHIP(b, hipEventRecord(b->out, b->own));
    PFT_BHIP(b, hipStreamWaitEvent(b->stream, b->out, 0));
    return PFT_OK;
}

template <typename T>
pft_status batch_steps_t(pft_batch* b, const double* const* wp, const double* const* wm, const pft_step* st,
                         int nsteps, double* log, int64_t cap)
{
    const bool same = b->exec && b->gwp.size() == (size_t)b->n &&
                      std::equal(b->gwp.begin(), b->gwp.end(), wp) &&
                      (wm ? std::equal(b->gwm.begin(), b->gwm.end(), wm) : b->gwm.empty()) &&
                      b->glog == log && b->gcap == cap && b->gst.dt == st->dt &&
                      b->gst.lambda_plus == st->lambda_plus && b->gst.lambda_minus == st->lambda_minus &&
                      b->gst.seed == st->seed && b->gst.replica == st->replica && b->gst.noise == st->noise &&
                      b->gst.update == st->update;
    if (!same) {
        b->gwp.clear();
        pft_status qs = batch_quiesce(b);  // a replay may still read the tables
        if (qs) return qs;
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        if (st->update == 1)  // the filter buffers must exist before the tables and the capture
            for (int r = 0; r < b->n; ++r) {
                const pft_status ps = sis_prepare(b->ctx[r]);
                if (ps) return b->fail(ps, "replica %d: %s", r, b->ctx[r]->err.c_str());
            }
        for (BatchGroup& g : b->groups) {
            pft_status s = batch_build_jobs<T>(b, g, 1, wp, wm, nullptr, nullptr, nullptr, nullptr, st);
            if (s) return s;
        }
        std::vector<LogJob> lj(b->n);
        for (int r = 0; r < b->n; ++r) lj[r] = {b->ctx[r]->scal, b->ctx[r]->scal + 1};
        PFT_BHIP(b, hipMemcpy(b->logj, lj.data(), lj.size() * sizeof(LogJob), hipMemcpyHostToDevice));
        PFT_BHIP(b, hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal));
        pft_status s = batch_enqueue<T>(b, 1, true, st->update == 1, reinterpret_cast<const double2*>(log), cap);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(b->own, &graph);
        if (s) {
            if (graph) (void)hipGraphDestroy(graph);
            return s;
        }
        if (ec != hipSuccess) return b->fail(PFT_E_DEVICE, "graph capture failed: %s", hipGetErrorString(ec));
        b->graph = graph;
        PFT_BHIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->gwp.assign(wp, wp + b->n);
        if (wm)
            b->gwm.assign(wm, wm + b->n);
        else
            b->gwm.clear();
        b->glog = log;
        b->gcap = cap;
        b->gst = *st;
    }
    PFT_BHIP(b, hipEventRecord(b->in, b->stream));
    PFT_BHIP(b, hipStreamWaitEvent(b->own, b->in, 0));
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, b->own, b->counters, st->step);
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, b->own, b->counters + 1, (uint64_t)0);
    PFT_BHIP(b, hipGetLastError());
    for (int i = 0; i < nsteps; ++i) PFT_BHIP(b, hipGraphLaunch(b->exec, b->own));
    PFT_BHIP(b, hipEventRecord(b->out, b->own));
    PFT_BHIP(b, hipStreamWaitEvent(b->stream, b->out, 0));
    return PFT_OK;
}

}  // namespace


// ============================================================== autotuner ==
namespace {

std::string device_arch()
{
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// Side length A of the two other axes of the timing grid (A * A * N <= 4 Mi sites).
int tune_side(int N)
{
    const int sides[] = {256, 192, 128, 96, 64, 48, 32, 24, 16, 8};
    for (int a : sides)
        if ((int64_t)a * a * N <= (int64_t)4 << 20) return a;
    return 8;
}

// Average duration (ms) of `reps` launches of one pass kind with variant v.
template <typename T>
double time_variant(pft_ctx* c, int kind, int v, int reps)
{
    cx<T>* w0 = static_cast<cx<T>*>(c->work);
    const cx<T>* e = etab<T>(c, 0);
    // the passes in their Richardson-step form, as the sweeps run them
    auto launch = [&]() -> hipError_t {
        if (kind == 0) {
            // z pass completing one step and starting the next
            pft::ZArgs<T> a{};
            a.nlines = (int64_t)c->p.nx * c->p.ny;
            a.U = static_cast<cx<T>*>(c->U);
            a.V = static_cast<cx<T>*>(c->V);
            a.qout = w0;
            a.scheme = PFT_RQM4;
            a.has_prev = 1;
            a.has_next = 1;
            a.Ep = e;
            a.En = e;
            a.gh_p = gptr<T>(c, 0, 0, 2);
            a.gh_n = gptr<T>(c, 0, 0, 2);
            a.gf_n = gptr<T>(c, 0, 1, 2);
            return pft::launch_zpass<T>(c->p.nz, v, a, c->stream);
        }
        // x pass on both arrays with the field multiply (the strided pass with
        // the most work on chip)
        const int64_t nynz = (int64_t)c->p.ny * c->p.nz;
        pft::SArgs<T> a{};
        a.U = static_cast<cx<T>*>(c->U);
        a.V = static_cast<cx<T>*>(c->V);
        a.opU = {gptr<T>(c, 0, 0, 0), e, gptr<T>(c, 0, 0, 0), nullptr};
        a.opV = {gptr<T>(c, 0, 1, 0), e, nullptr, nullptr};
        a.S = nynz;
        return pft::launch_spass<T>(0, c->p.nx, v, nynz, a, 1, c->stream);
    };
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1;
    }
    double ms = -1;
    bool ok = launch() == hipSuccess && launch() == hipSuccess;  // warm-up
    if (ok) ok = hipEventRecord(e0, c->stream) == hipSuccess;
    for (int i = 0; ok && i < reps; ++i) ok = launch() == hipSuccess;
    if (ok) ok = hipEventRecord(e1, c->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float t = 0.f;
    if (ok && hipEventElapsedTime(&t, e0, e1) == hipSuccess) ms = t / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

}  // namespace

// ================================================================ C ABI ====
extern "C" {

const char* pft_status_string(pft_status s)
{
    switch (s) {
    case PFT_OK: return "PFT_OK";
    case PFT_E_INVALID: return "PFT_E_INVALID";
    case PFT_E_UNSUPPORTED: return "PFT_E_UNSUPPORTED";
    case PFT_E_NOMEM: return "PFT_E_NOMEM";
    case PFT_E_DEVICE: return "PFT_E_DEVICE";
    case PFT_E_NONFINITE: return "PFT_E_NONFINITE";
    case PFT_E_STATE: return "PFT_E_STATE";
    }
    return "PFT_E_UNKNOWN";
}

int32_t pft_contour_plan(int32_t ns, double f, double* h, int32_t* blk, int32_t* junction)
{
    if (!h || !blk || !junction) return -1;
    std::vector<int> b(ns > 0 ? ns + 1 : 1);
    int J = 0;
    const int K = contour_plan(ns, f, h, b.data(), &J);
    if (K < 0) return -1;
    for (int j = 0; j < K; ++j) blk[j] = b[j];
    *junction = J;
    return K;
}

static pft_status create_ctx(const pft_params* params, void* hip_stream, bool dual, pft_ctx** out);

pft_status pft_create(const pft_params* params, void* hip_stream, pft_ctx** out)
{
    return create_ctx(params, hip_stream, true, out);
}

pft_status pft_set_concurrent_sweeps(pft_ctx* c, int32_t on)
{
    if (!c) return PFT_E_INVALID;
    if (!on) {
        (void)hipStreamSynchronize(c->stream);
        if (c->s2) (void)hipStreamSynchronize(c->s2);
        c->dual_off = true;
    } else {
        if (!c->s2) return c->fail(PFT_E_UNSUPPORTED, "this context was created without a second stream");
        c->dual_off = false;
    }
    return PFT_OK;
}

static bool fused_supported(const pft_params& p)
{
    if (p.ny != p.nz || p.bc[1] || p.bc[2]) return false;
    return p.precision == PFT_C128 ? pft::plane_supported<double>(p.ny) : pft::plane_supported<float>(p.ny);
}

// The fused schedule is the default where its kernel keeps (nearly) everything
// in registers: beyond this many spilled bytes per lane the spill traffic and
// latency outweigh the saved passes (measured: complex double 80^2 with 244 B
// still gains, 96^2 with 720 B loses to the axis schedule).
constexpr int kFusedMaxSpill = 256;

static bool fused_default(const pft_params& p)
{
    if (!fused_supported(p)) return false;
    const int b = p.precision == PFT_C128 ? pft::plane_private_bytes<double>(p.ny) : pft::plane_private_bytes<float>(p.ny);
    return b >= 0 && b <= kFusedMaxSpill;
}

pft_status pft_set_fused_planes(pft_ctx* c, int32_t on)
{
    if (!c) return PFT_E_INVALID;
    if (on < 0 || on > 2) return c->fail(PFT_E_INVALID, "schedule %d is not 0, 1 or 2", on);
    if (on && !fused_supported(c->p))
        return c->fail(PFT_E_UNSUPPORTED, "no fused yz-plane pass for a %d x %d plane in this precision", c->p.ny, c->p.nz);
    c->fused = on != 0;
    c->fused_conj_only = on == 2;
    return PFT_OK;
}

int32_t pft_fused_planes(const pft_ctx* c) { return c ? (c->fused ? (c->fused_conj_only ? 2 : 1) : 0) : -1; }

static pft_status create_ctx(const pft_params* params, void* hip_stream, bool dual, pft_ctx** out)
{
    if (!out) return PFT_E_INVALID;
    *out = nullptr;
    if (!params) return PFT_E_INVALID;
    const pft_params& p = *params;
    const bool ed = p.model == PFT_EDWARDS;
    if (p.nx < 1 || p.ny < 1 || p.nz < 1 || !(p.lx > 0) || !(p.ly > 0) || !(p.lz > 0) || p.ns < 2 || !(p.C > 0) ||
        (p.precision != PFT_C128 && p.precision != PFT_C64) || (p.scheme != PFT_RQM4 && p.scheme != PFT_SPLIT2) ||
        (p.model != PFT_DIBLOCK && p.model != PFT_EDWARDS))
        return PFT_E_INVALID;
    if (ed ? !(p.B > 0) : (!(p.f > 0.0 && p.f < 1.0) || !(p.chiN > 0))) return PFT_E_INVALID;
    if (p.storage < PFT_STORE_BOTH || p.storage > PFT_STORE_HOST) return PFT_E_INVALID;
    for (int a = 0; a < 3; ++a) {
        if (p.bc[a] < PFT_PERIODIC || p.bc[a] > PFT_ABSORBING) return PFT_E_INVALID;
        if (p.bc[a] && !pft::walls_supported(a == 0 ? p.nx : a == 1 ? p.ny : p.nz)) return PFT_E_UNSUPPORTED;
    }
    if (p.storage != PFT_STORE_BOTH && ed) return PFT_E_UNSUPPORTED;
    if (ed || p.storage != PFT_STORE_BOTH) dual = false;  // one sweep, or sweeps in sequence
    if (!pft::axis_supported(p.nx) || !pft::axis_supported(p.ny) || !pft::axis_supported(p.nz))
        return PFT_E_UNSUPPORTED;

    if (!g_tune_env_checked) {
        g_tune_env_checked = true;
        if (const char* path = std::getenv("PFT_TUNE_CACHE")) (void)pft_tune_load(path);
    }
    pft_ctx* c = new (std::nothrow) pft_ctx();
    if (!c) return PFT_E_NOMEM;
    c->p = p;
    if (hipGetDevice(&c->device) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return PFT_E_DEVICE;
    }
    c->var[0] = tuned_variant(p.precision, p.nx, 1);
    c->var[1] = tuned_variant(p.precision, p.ny, 1);
    c->var[2] = tuned_variant(p.precision, p.nz, 0);
    c->fused = fused_default(p);
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->M = (int64_t)p.nx * p.ny * p.nz;
    // table slot length: n factors per periodic axis, 3n per walled axis
    c->maxN = std::max((p.bc[0] ? 3 : 1) * p.nx, std::max((p.bc[1] ? 3 : 1) * p.ny, (p.bc[2] ? 3 : 1) * p.nz));
    c->elem = p.precision == PFT_C128 ? sizeof(cx<double>) : sizeof(cx<float>);
    c->h.resize(p.ns + 1);
    c->blk.resize(p.ns + 1);
    if (ed) {
        // one species along the whole chain: K = ns equal steps, no junction
        c->K = p.ns;
        for (int j = 0; j < p.ns; ++j) {
            c->h[j] = 1.0 / p.ns;
            c->blk[j] = 0;
        }
        c->J = c->K;
    } else {
        c->K = contour_plan(p.ns, p.f, c->h.data(), c->blk.data(), &c->J);
    }
    const double ds = 1.0 / p.ns;
    c->hval[0] = ds;
    c->kind.resize(c->K);
    c->hid.resize(c->K);
    for (int j = 0; j < c->K; ++j) {
        const bool regular = (c->K == p.ns) || !(j == c->J - 1 || j == c->J);
        if (regular) {
            c->kind[j] = c->blk[j];
            c->hid[j] = 0;
        } else {
            c->kind[j] = 2 + c->blk[j];
            c->hid[j] = 1 + c->blk[j];
            c->hval[1 + c->blk[j]] = c->h[j];
        }
    }
    // trapezoid weights per block: tau[0..K] for A, tau[K+1..2K+1] for B
    std::vector<double> tau(2 * (c->K + 1), 0.0);
    for (int j = 0; j < c->K; ++j) {
        double* t = tau.data() + (c->blk[j] == 0 ? 0 : c->K + 1);
        t[j] += 0.5 * c->h[j];
        t[j + 1] += 0.5 * c->h[j];
    }
    c->nparts = reduction_blocks(c->M);

    auto alloc = [&](void** ptr, size_t bytes) -> bool { return hipMalloc(ptr, std::max<size_t>(bytes, 16)) == hipSuccess; };
    const size_t store = (size_t)(c->K + 1) * c->M * c->elem;
    const bool both = p.storage == PFT_STORE_BOTH, host = p.storage == PFT_STORE_HOST;
    const size_t slots = host ? 2 * kRing + 2 : (both ? 0 : 2);
    bool ok = (host || alloc(&c->qs, store)) && (ed || !both || alloc(&c->qds, store)) &&
              (slots == 0 || alloc(&c->ring, slots * c->M * c->elem)) && alloc(&c->U, c->M * c->elem) &&
              alloc(&c->V, c->M * c->elem) && (!dual || (alloc(&c->U2, c->M * c->elem) && alloc(&c->V2, c->M * c->elem))) &&
              alloc(&c->E, 4 * c->M * c->elem) && alloc(&c->work, 2 * c->M * c->elem) &&
              alloc(&c->gtab, (size_t)5 * 2 * 3 * c->maxN * (c->elem / 2)) &&
              alloc((void**)&c->tau, tau.size() * sizeof(double)) && alloc((void**)&c->phi, 2 * c->M * sizeof(double2)) &&
              alloc((void**)&c->partials, (size_t)std::max(c->nparts, 64 * (c->K + 1)) * sizeof(double2)) &&
              alloc((void**)&c->scal, (size_t)(8 + c->K + 1) * sizeof(double2)) && alloc((void**)&c->flags, sizeof(uint32_t));
    if (!ok) {
        (void)hipGetLastError();
        free_all(c);
        delete c;
        return PFT_E_NOMEM;
    }
    if (ed) c->qds = c->qs;  // symmetric chain: the conjugate propagator is q
    pft_status s = PFT_OK;
    c->tau_h = tau;
    if (host) {
        if (hipHostMalloc(&c->qh, store, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            c->qh = nullptr;
            s = PFT_E_NOMEM;
        }
        if (s == PFT_OK && hipStreamCreateWithFlags(&c->cs, hipStreamNonBlocking) != hipSuccess) s = PFT_E_DEVICE;
        for (int k = 0; k < kRing && s == PFT_OK; ++k)
            if (hipEventCreateWithFlags(&c->ev_st[k], hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&c->ev_cp[k], hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&c->ev_rd[k], hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&c->ev_fr[k], hipEventDisableTiming) != hipSuccess)
                s = PFT_E_DEVICE;
        if (s == PFT_OK && hipEventCreateWithFlags(&c->ev_done, hipEventDisableTiming) != hipSuccess) s = PFT_E_DEVICE;
    }
    if (dual && (hipStreamCreateWithFlags(&c->s2, hipStreamNonBlocking) != hipSuccess ||
                 hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
                 hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess))
        s = PFT_E_DEVICE;
    if (hipMemcpy(c->tau, tau.data(), tau.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(c->flags, 0, sizeof(uint32_t)) != hipSuccess || hipMemset(c->scal, 0, (8 + c->K + 1) * sizeof(double2)) != hipSuccess)
        s = PFT_E_DEVICE;
    for (int hd = 0; hd < 3 && s == PFT_OK; ++hd) {
        const double hv = c->hval[hd] > 0 ? c->hval[hd] : ds;
        s = p.precision == PFT_C128 ? upload_factors<double>(c, hd, hv) : upload_factors<float>(c, hd, hv);
    }
    if (s == PFT_OK) s = p.precision == PFT_C128 ? upload_second_derivative<double>(c) : upload_second_derivative<float>(c);
    if (s != PFT_OK) {
        free_all(c);
        delete c;
        return s;
    }
    *out = c;
    return PFT_OK;
}

void pft_destroy(pft_ctx* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    if (c->s2) (void)hipStreamSynchronize(c->s2);
    free_all(c);
    delete c;
}

const char* pft_last_error(const pft_ctx* c) { return c ? c->err.c_str() : "null context"; }

int32_t pft_num_steps(const pft_ctx* c) { return c ? c->K : -1; }

pft_status pft_propagate(pft_ctx* c, const double* wp, const double* wm)
{
    if (!c) return PFT_E_INVALID;
    const bool need_wm = c->p.model != PFT_EDWARDS;
    if (!aligned16(wp) || (need_wm && !aligned16(wm)))
        return c->fail(PFT_E_INVALID, "w_plus/w_minus must be non-null and 16-byte aligned");
    c->propagated = false;
    return c->p.precision == PFT_C128 ? propagate_t<double>(c, wp, wm) : propagate_t<float>(c, wp, wm);
}

pft_status pft_densities(pft_ctx* c, double* phi_a, double* phi_b, double* Q)
{
    if (!c) return PFT_E_INVALID;
    if (!aligned16(phi_a) || !aligned16(phi_b) || (Q && !aligned16(Q)))
        return c->fail(PFT_E_INVALID, "phi_a/phi_b must be non-null and 16-byte aligned (Q aligned if given)");
    if (!c->propagated) return c->fail(PFT_E_STATE, "pft_densities needs a prior pft_propagate");
    return c->p.precision == PFT_C128 ? densities_t<double>(c, phi_a, phi_b, Q) : densities_t<float>(c, phi_a, phi_b, Q);
}

pft_status pft_evaluate_graph(pft_ctx* c, const double* wp, const double* wm, double* phi_a, double* phi_b, double* Q,
                              int32_t nreps)
{
    if (!c) return PFT_E_INVALID;
    if (nreps < 0) return c->fail(PFT_E_INVALID, "nreps must be >= 0");
    if (c->p.storage != PFT_STORE_BOTH)
        return c->fail(PFT_E_UNSUPPORTED, "graph replay needs both stores in device memory (storage 0)");
    if (c->prof) return c->fail(PFT_E_STATE, "graph replay is not available while profiling");
    const bool need_wm = c->p.model != PFT_EDWARDS;
    if (!aligned16(wp) || (need_wm && !aligned16(wm)) || !aligned16(phi_a) || !aligned16(phi_b) || (Q && !aligned16(Q)))
        return c->fail(PFT_E_INVALID, "w_plus/w_minus/phi_a/phi_b must be non-null and 16-byte aligned (Q aligned if given)");
    const void* key[5] = {wp, need_wm ? wm : nullptr, phi_a, phi_b, Q};
    if (!c->gexec || std::memcmp(key, c->gkey, sizeof key) != 0) {
        if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
        if (c->graph) (void)hipGraphDestroy(c->graph);
        c->gexec = nullptr;
        c->graph = nullptr;
        if (!c->gs) {
            if (hipStreamCreateWithFlags(&c->gs, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&c->ev_g0, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&c->ev_g1, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                return c->fail(PFT_E_DEVICE, "graph replay: cannot create its stream and events");
            }
        }
        // capture one evaluation with the capture stream standing in for the
        // context stream (the conjugate sweep's stream joins through its events)
        PFT_HIP(c, hipStreamBeginCapture(c->gs, hipStreamCaptureModeThreadLocal));
        const hipStream_t saved = c->stream;
        c->stream = c->gs;
        pft_status s = pft_propagate(c, wp, wm);
        if (s == PFT_OK) s = pft_densities(c, phi_a, phi_b, Q);
        c->stream = saved;
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(c->gs, &g);
        c->propagated = false;
        if (s != PFT_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            return s != PFT_OK ? s : c->fail(PFT_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        }
        if (hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            c->gexec = nullptr;
            return c->fail(PFT_E_DEVICE, "graph instantiation failed");
        }
        c->graph = g;
        std::memcpy(c->gkey, key, sizeof key);
    }
    if (nreps == 0) return PFT_OK;
    PFT_HIP(c, hipEventRecord(c->ev_g0, c->stream));
    PFT_HIP(c, hipStreamWaitEvent(c->gs, c->ev_g0, 0));
    for (int r = 0; r < nreps; ++r) PFT_HIP(c, hipGraphLaunch(c->gexec, c->gs));
    PFT_HIP(c, hipEventRecord(c->ev_g1, c->gs));
    PFT_HIP(c, hipStreamWaitEvent(c->stream, c->ev_g1, 0));
    c->propagated = true;
    return PFT_OK;
}

pft_status pft_set_box(pft_ctx* c, double lx, double ly, double lz)
{
    if (!c) return PFT_E_INVALID;
    if (!(lx > 0) || !(ly > 0) || !(lz > 0) || !std::isfinite(lx) || !std::isfinite(ly) || !std::isfinite(lz))
        return c->fail(PFT_E_INVALID, "box edges must be finite and > 0");
    // queued work may still read the tables rewritten below
    PFT_HIP(c, hipStreamSynchronize(c->stream));
    if (c->s2) PFT_HIP(c, hipStreamSynchronize(c->s2));
    if (c->gs) PFT_HIP(c, hipStreamSynchronize(c->gs));
    if (c->cs) PFT_HIP(c, hipStreamSynchronize(c->cs));
    c->p.lx = lx;
    c->p.ly = ly;
    c->p.lz = lz;
    c->propagated = false;
    const bool dbl = c->p.precision == PFT_C128;
    for (int hd = 0; hd < 3; ++hd) {
        const double hv = c->hval[hd] > 0 ? c->hval[hd] : c->hval[0];
        const pft_status s = dbl ? upload_factors<double>(c, hd, hv) : upload_factors<float>(c, hd, hv);
        if (s) return s;
    }
    const pft_status s = dbl ? upload_second_derivative<double>(c) : upload_second_derivative<float>(c);
    if (s) return s;
    if (c->k2) return sis_upload_k2(c);
    return PFT_OK;
}

pft_status pft_hamiltonian(pft_ctx* c, const double* wp, const double* wm, double* H, double* hint)
{
    if (!c) return PFT_E_INVALID;
    if (!aligned16(wp) || (c->p.model != PFT_EDWARDS && !aligned16(wm)) || !aligned16(H) || (hint && !aligned16(hint)))
        return c->fail(PFT_E_INVALID, "w_plus/w_minus/H must be non-null and 16-byte aligned");
    if (!c->propagated) return c->fail(PFT_E_STATE, "pft_hamiltonian needs a prior pft_propagate");
    return hamiltonian_launch(c, wp, wm, H, hint);
}

// Semi-implicit step (Eqs. (10)-(11)) from the explicit step's arguments: the
// local increment kernel, then the reciprocal-space filter of the w_+ (or
// omega) increment in five axis passes over a work array.
// |k|^2 per axis for the semi-implicit filter (walled axes: the modes of the
// even image, period 2L), written into the allocated c->k2.
static pft_status sis_upload_k2(pft_ctx* c)
{
    const pft_params& p = c->p;
    const int n[3] = {p.nx, p.ny, p.nz};
    const double L[3] = {p.lx, p.ly, p.lz};
    std::vector<double> k2(3 * (size_t)c->maxN, 0.0);
    for (int ax = 0; ax < 3; ++ax) {
        const int ne = p.bc[ax] ? 2 * n[ax] : n[ax];
        for (int j = 0; j < ne; ++j) {
            const int m = (j <= ne / 2) ? j : j - ne;
            const double k = kTwoPi * m / ((double)ne / n[ax] * L[ax]);
            k2[(size_t)ax * c->maxN + j] = k * k;
        }
    }
    PFT_HIP(c, hipMemcpy(c->k2, k2.data(), k2.size() * sizeof(double), hipMemcpyHostToDevice));
    return PFT_OK;
}

// Buffers of the semi-implicit step (allocated on first use; batches allocate
// them before capturing their graphs).
static pft_status sis_prepare(pft_ctx* c)
{
    const pft_params& p = c->p;
    if (!c->sisbuf) {
        if (hipMalloc((void**)&c->sisbuf, (size_t)c->M * sizeof(double2)) != hipSuccess) {
            (void)hipGetLastError();
            c->sisbuf = nullptr;
            return c->fail(PFT_E_NOMEM, "semi-implicit step: cannot allocate the work array");
        }
    }
    // reflecting walls: the filter runs on the even image (2n points, period 2L)
    const bool walls = p.bc[0] || p.bc[1] || p.bc[2];
    const int n[3] = {p.nx, p.ny, p.nz};
    int ne[3];
    for (int ax = 0; ax < 3; ++ax) ne[ax] = p.bc[ax] ? 2 * n[ax] : n[ax];
    const int64_t Me = (int64_t)ne[0] * ne[1] * ne[2];
    if (walls && !c->sisext) {
        if (hipMalloc((void**)&c->sisext, 2 * (size_t)Me * sizeof(double2)) != hipSuccess) {
            (void)hipGetLastError();
            c->sisext = nullptr;
            return c->fail(PFT_E_NOMEM, "semi-implicit step: cannot allocate the mirror image");
        }
    }
    if (!c->k2) {
        if (hipMalloc((void**)&c->k2, 3 * (size_t)c->maxN * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            c->k2 = nullptr;
            return c->fail(PFT_E_NOMEM, "semi-implicit step: cannot allocate the k tables");
        }
        return sis_upload_k2(c);
    }
    return PFT_OK;
}

// Arguments of the local increment kernel of one context; step_dev: device
// step counter added to the noise step (batches), or NULL.
static SisBufs ctx_sis_bufs(const pft_ctx* c)
{
    SisBufs sb;
    sb.R = c->sisbuf;
    sb.X = c->sisext;
    if (c->sisext) {
        const int n[3] = {c->p.nx, c->p.ny, c->p.nz};
        int64_t Me = 1;
        for (int ax = 0; ax < 3; ++ax) Me *= c->p.bc[ax] ? 2 * n[ax] : n[ax];
        sb.W = c->sisext + Me;
    }
    sb.k2 = c->k2;
    sb.pitch = c->maxN;
    return sb;
}

static SisIncArgs sis_inc_args(const pft_ctx* c, const SisBufs& sb, const UpdArgs& u, const uint64_t* step_dev)
{
    SisIncArgs a{};
    a.wp = u.wp;
    a.wm = u.wm;
    a.phiA = u.phiA;
    a.phiB = u.phiB;
    a.R = sb.R;
    a.M = c->M;
    a.two_over_chiN = u.two_over_chiN;
    a.ap = u.dtp;
    a.am = u.dtm;
    a.sp = u.sp;
    a.sm = u.sm;
    a.den_m = 1.0 + u.dtm * u.two_over_chiN;
    a.noise = u.noise;
    a.seed = u.seed;
    a.rep = u.rep;
    a.step = u.step;
    a.step_dev = step_dev;
    a.edwards = u.edwards;
    a.b_over_c = u.b_over_c;
    return a;
}

// Arguments of the reciprocal-space filter passes over X (Me sites, last
// axis ne_z long), subtracting from W.
static pft::SisArgs sis_filter_args(const SisBufs& sb, const UpdArgs& u, double2* X, double2* W, int ne_z,
                                    int64_t Me)
{
    pft::SisArgs f{};
    f.X = reinterpret_cast<cx<double>*>(X);
    f.W = reinterpret_cast<cx<double>*>(W);
    f.k2x = sb.k2;
    f.k2y = sb.k2 + sb.pitch;
    f.k2z = sb.k2 + 2 * (size_t)sb.pitch;
    f.nz = ne_z;
    f.a = u.dtp;
    f.g0 = u.edwards ? u.b_over_c : 0.0;
    f.gD = 1.0;
    f.inv_M = 1.0 / (double)Me;
    return f;
}

// Why the semi-implicit step cannot run on this machine, or NULL: absorbing walls
// have no diagonal linear response, and a reflecting axis of n points needs a
// kernel for its image of 2n.
static const char* sis_walls_unsupported(const pft_params& p)
{
    const int n[3] = {p.nx, p.ny, p.nz};
    for (int ax = 0; ax < 3; ++ax) {
        int n1, n2, w;
        if (p.bc[ax] == PFT_ABSORBING) return "the semi-implicit step has no linear response between absorbing walls";
        if (p.bc[ax] == PFT_REFLECTING && !pft::axis_variant(2 * n[ax], 0, &n1, &n2, &w))
            return "semi-implicit step between walls: no kernel for the image length of a walled axis";
    }
    return nullptr;
}

// The grid the filter runs on (the even image, 2n points along a reflecting
// axis) and the image arguments over the context's buffers (sis_prepare ran).
static MirrorArgs sis_image(const pft_ctx* c, const SisBufs& sb)
{
    const pft_params& p = c->p;
    MirrorArgs ma{};
    const int n[3] = {p.nx, p.ny, p.nz};
    for (int ax = 0; ax < 3; ++ax) {
        ma.n[ax] = n[ax];
        ma.ne[ax] = p.bc[ax] ? 2 * n[ax] : n[ax];
    }
    ma.Me = (int64_t)ma.ne[0] * ma.ne[1] * ma.ne[2];
    ma.R = sb.R;
    ma.X = sb.X;
    ma.W = sb.W;
    return ma;
}

// ext: work memory in place of the context's (whose buffers are allocated on
// first use when ext is NULL); its |k|^2 rows are filled here, on the stream.
static pft_status sis_step(pft_ctx* c, const UpdArgs& u, const SisBufs* ext = nullptr)
{
    const pft_params& p = c->p;
    if (!ext) {
        pft_status ps0 = sis_prepare(c);
        if (ps0) return ps0;
    }
    const SisBufs sb = ext ? *ext : ctx_sis_bufs(c);
    const bool walls = p.bc[0] || p.bc[1] || p.bc[2];
    const MirrorArgs ma = sis_image(c, sb);
    const int* ne = ma.ne;
    const int64_t Me = ma.Me;
    if (ext) {
        const int n[3] = {p.nx, p.ny, p.nz};
        const double L[3] = {p.lx, p.ly, p.lz};
        K2Rows kr{};
        for (int ax = 0; ax < 3; ++ax) {
            kr.ne[ax] = ne[ax];
            kr.Le[ax] = (double)ne[ax] / n[ax] * L[ax];
        }
        hipLaunchKernelGGL(k_fill_k2, dim3(3), dim3(256), 0, c->stream, const_cast<double*>(sb.k2), sb.pitch, kr);
        PFT_HIP(c, hipGetLastError());
    }
    const SisIncArgs a = sis_inc_args(c, sb, u, nullptr);
    {
        ProfScope ps(c, PFT_K_REDUCE, 6.0 * sizeof(double2) * (double)c->M);
        hipLaunchKernelGGL(k_sis_increment, dim3(grid_for((c->M + 3) / 4, 256)), dim3(256), 0, c->stream, a);
    }
    PFT_HIP(c, hipGetLastError());
    if (walls) {
        hipLaunchKernelGGL(k_sis_mirror, dim3(grid_for(Me, 256)), dim3(256), 0, c->stream, ma);
        PFT_HIP(c, hipGetLastError());
    }
    const pft::SisArgs f = sis_filter_args(sb, u, walls ? ma.X : sb.R, walls ? ma.W : u.wp, ne[2], Me);
    for (int kind = 0; kind < 5; ++kind) {
        ProfScope ps(c, PFT_K_REDUCE, (kind == 4 ? 3.0 : 2.0) * sizeof(double2) * (double)Me);
        PFT_HIP(c, pft::launch_sis_pass(kind, ne[0], ne[1], ne[2], f, c->stream));
    }
    if (walls) {
        hipLaunchKernelGGL(k_sis_unmirror, dim3(grid_for(c->M, 256)), dim3(256), 0, c->stream, ma, u.wp, c->M);
        PFT_HIP(c, hipGetLastError());
    }
    return PFT_OK;
}

// The field step of pft_cl_step; sb: the semi-implicit step's work memory, or
// NULL for the context's own buffers.
static pft_status cl_step(pft_ctx* c, double* wp, double* wm, const pft_step* st, double* phi_a, double* phi_b,
                          double* Q, double* H, const SisBufs* sb)
{
    if (!st) return c->fail(PFT_E_INVALID, "step parameters are NULL");
    if (!(st->dt >= 0) || !(st->lambda_plus >= 0) || !(st->lambda_minus >= 0))
        return c->fail(PFT_E_INVALID, "dt and mobilities must be non-negative");
    if (st->update != 0 && st->update != 1) return c->fail(PFT_E_INVALID, "update must be 0 or 1");
    if (st->update == 1) {
        const char* why = sis_walls_unsupported(c->p);
        if (why) return c->fail(PFT_E_UNSUPPORTED, "%s", why);
    }
    if ((phi_a && !aligned16(phi_a)) || (phi_b && !aligned16(phi_b)) || (Q && !aligned16(Q)) || (H && !aligned16(H)))
        return c->fail(PFT_E_INVALID, "optional outputs must be 16-byte aligned");
    double* pa = phi_a ? phi_a : reinterpret_cast<double*>(c->phi);
    double* pb = phi_b ? phi_b : reinterpret_cast<double*>(c->phi + c->M);
    pft_status s = pft_propagate(c, wp, wm);
    if (s) return s;
    s = pft_densities(c, pa, pb, Q);
    if (s) return s;
    s = pft_hamiltonian(c, wp, wm, H ? H : reinterpret_cast<double*>(c->scal + 1), nullptr);
    if (s) return s;
    const double dV = c->p.lx * c->p.ly * c->p.lz / (double)c->M;
    UpdArgs a{};
    a.wp = reinterpret_cast<double2*>(wp);
    a.wm = reinterpret_cast<double2*>(wm);
    a.phiA = reinterpret_cast<const double2*>(pa);
    a.phiB = reinterpret_cast<const double2*>(pb);
    a.M = c->M;
    a.two_over_chiN = 2.0 / c->p.chiN;
    a.dtp = st->lambda_plus * st->dt;
    a.dtm = st->lambda_minus * st->dt;
    a.noise = st->noise != 0;
    a.sp = a.noise ? std::sqrt(2.0 * st->lambda_plus * st->dt / (c->p.C * dV)) : 0.0;
    a.sm = a.noise ? std::sqrt(2.0 * st->lambda_minus * st->dt / (c->p.C * dV)) : 0.0;
    a.seed = st->seed;
    a.rep = st->replica;
    a.step = st->step;
    if (c->p.model == PFT_EDWARDS) {
        a.edwards = 1;
        a.b_over_c = c->p.B / c->p.C;
        a.wm = nullptr;
    }
    if (st->update == 1) return sis_step(c, a, sb);
    ProfScope ps(c, PFT_K_REDUCE, 6.0 * sizeof(double2) * (double)c->M);
    hipLaunchKernelGGL(k_update, dim3(grid_for((c->M + 3) / 4, 256)), dim3(256), 0, c->stream, a);
    PFT_HIP(c, hipGetLastError());
    return PFT_OK;
}

pft_status pft_cl_step(pft_ctx* c, double* wp, double* wm, const pft_step* st, double* phi_a, double* phi_b,
                       double* Q, double* H)
{
    if (!c) return PFT_E_INVALID;
    return cl_step(c, wp, wm, st, phi_a, phi_b, Q, H, nullptr);
}

pft_status pft_node_q(pft_ctx* c, double* qnode)
{
    if (!c) return PFT_E_INVALID;
    if (!aligned16(qnode)) return c->fail(PFT_E_INVALID, "qnode must be non-null and 16-byte aligned");
    if (!c->propagated) return c->fail(PFT_E_STATE, "pft_node_q needs a prior pft_propagate");
    if (c->p.storage != PFT_STORE_BOTH) return c->fail(PFT_E_UNSUPPORTED, "pft_node_q needs the q-dagger store");
    return c->p.precision == PFT_C128 ? nodeq_t<double>(c, qnode) : nodeq_t<float>(c, qnode);
}

pft_status pft_get_slice(pft_ctx* c, int32_t which, int32_t node, double* out)
{
    if (!c) return PFT_E_INVALID;
    if (!aligned16(out) || (which != 0 && which != 1) || node < 0 || node > c->K)
        return c->fail(PFT_E_INVALID, "bad slice request (which %d, node %d of %d)", which, node, c->K);
    if (!c->propagated) return c->fail(PFT_E_STATE, "pft_get_slice needs a prior pft_propagate");
    if (which == 1 && c->p.storage != PFT_STORE_BOTH)
        return c->fail(PFT_E_UNSUPPORTED, "q-dagger slices are not stored in this storage mode");
    return c->p.precision == PFT_C128 ? get_slice_t<double>(c, which, node, out) : get_slice_t<float>(c, which, node, out);
}

pft_status pft_apply_step(pft_ctx* c, int32_t j, const double* qin, double* qout)
{
    if (!c) return PFT_E_INVALID;
    if (!aligned16(qin) || !aligned16(qout) || j < 0 || j >= c->K)
        return c->fail(PFT_E_INVALID, "bad step request (step %d of %d)", j, c->K);
    if (!c->propagated) return c->fail(PFT_E_STATE, "pft_apply_step needs the field tables of a prior pft_propagate");
    return c->p.precision == PFT_C128 ? apply_step_t<double>(c, j, qin, qout) : apply_step_t<float>(c, j, qin, qout);
}

pft_status pft_diffuse(pft_ctx* c, double* u, double h)
{
    if (!c) return PFT_E_INVALID;
    if (!aligned16(u) || !(h >= 0)) return c->fail(PFT_E_INVALID, "u must be aligned and h >= 0");
    return c->p.precision == PFT_C128 ? diffuse_t<double>(c, u, h) : diffuse_t<float>(c, u, h);
}

pft_status pft_debug_kgrid(const pft_ctx* c, int32_t* m2)
{
    if (!c || !m2) return PFT_E_INVALID;
    if (c->p.bc[0] || c->p.bc[1] || c->p.bc[2]) return PFT_E_UNSUPPORTED;  // Fourier modes of a periodic box
    const int nx = c->p.nx, ny = c->p.ny, nz = c->p.nz;
    auto mode = [](int j, int n) { return j <= n / 2 ? j : j - n; };
    for (int x = 0; x < nx; ++x)
        for (int y = 0; y < ny; ++y)
            for (int z = 0; z < nz; ++z) {
                const int a = mode(x, nx), b = mode(y, ny), d = mode(z, nz);
                m2[((int64_t)x * ny + y) * nz + z] = a * a + b * b + d * d;
            }
    return PFT_OK;
}

pft_status pft_status_flags(pft_ctx* c, uint32_t* flags)
{
    if (!c || !flags) return PFT_E_INVALID;
    PFT_HIP(c, hipMemcpyAsync(flags, c->flags, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    PFT_HIP(c, hipStreamSynchronize(c->stream));
    return (*flags & 1u) ? PFT_E_NONFINITE : PFT_OK;
}

pft_status pft_adjoint(pft_ctx* c, const double* wp, const double* wm, int32_t ckpt_every, double* dwp, double* dwm,
                       double* dL, double* H)
{
    if (!c) return PFT_E_INVALID;
    if (!aligned16(wp) || !aligned16(wm) || !aligned16(dwp) || !aligned16(dwm) || (dL && !aligned16(dL)) ||
        (H && !aligned16(H)))
        return c->fail(PFT_E_INVALID, "pft_adjoint: pointers must be non-null (dH_dL, H optional) and 16-byte aligned");
    if (ckpt_every < 0) return c->fail(PFT_E_INVALID, "pft_adjoint: ckpt_every must be >= 0");
    if (c->p.model != PFT_DIBLOCK) return c->fail(PFT_E_UNSUPPORTED, "pft_adjoint: diblock model only");
    if (c->p.storage != PFT_STORE_BOTH) return c->fail(PFT_E_UNSUPPORTED, "pft_adjoint: needs both stores");
    int Kc = ckpt_every;
    if (Kc == 0) Kc = (int)std::ceil(std::sqrt((double)c->K));
    Kc = std::max(1, std::min(Kc, c->K));
    c->propagated = false;  // the field tables and Q now belong to these fields
    return c->p.precision == PFT_C128 ? adjoint_t<double>(c, wp, wm, Kc, dwp, dwm, dL, H)
                                      : adjoint_t<float>(c, wp, wm, Kc, dwp, dwm, dL, H);
}

pft_status pft_profile_begin(pft_ctx* c)
{
    if (!c) return PFT_E_INVALID;
    c->prof = true;
    c->ev_used = 0;
    return PFT_OK;
}

pft_status pft_profile_end(pft_ctx* c, double* ms, int64_t* launches, double* bytes)
{
    if (!c) return PFT_E_INVALID;
    if (!c->prof) return c->fail(PFT_E_STATE, "pft_profile_end without pft_profile_begin");
    c->prof = false;
    PFT_HIP(c, hipStreamSynchronize(c->stream));
    double m[PFT_K_COUNT] = {}, b[PFT_K_COUNT] = {};
    int64_t n[PFT_K_COUNT] = {};
    for (size_t i = 0; i < c->ev_used; ++i) {
        float t = 0.f;
        PFT_HIP(c, hipEventElapsedTime(&t, c->ev[2 * i], c->ev[2 * i + 1]));
        const int k = c->ev_kind[i];
        m[k] += t;
        b[k] += c->ev_bytes[i];
        n[k] += 1;
    }
    for (int k = 0; k < PFT_K_COUNT; ++k) {
        if (ms) ms[k] = m[k];
        if (launches) launches[k] = n[k];
        if (bytes) bytes[k] = b[k];
    }
    c->ev_used = 0;
    return PFT_OK;
}

pft_status pft_copy_probe(const void* src, void* dst, int64_t bytes, void* stream)
{
    if (!aligned16(src) || !aligned16(dst) || bytes <= 0 || bytes % 16 != 0) return PFT_E_INVALID;
    const int64_t n = bytes / 16;
    hipLaunchKernelGGL(k_copy_probe, dim3(grid_for(n, 256, 2048)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const double2*>(src), static_cast<double2*>(dst), n);
    return hipGetLastError() == hipSuccess ? PFT_OK : PFT_E_DEVICE;
}

pft_status pft_batch_create(const pft_params* params, int32_t n, void* hip_stream, pft_batch** out)
{
    if (!out) return PFT_E_INVALID;
    *out = nullptr;
    if (!params || n < 1) return PFT_E_INVALID;
    for (int r = 1; r < n; ++r)
        if (params[r].precision != params[0].precision || params[r].scheme != params[0].scheme ||
            params[r].model != params[0].model)
            return PFT_E_INVALID;
    for (int r = 0; r < n; ++r)
        if (params[r].storage != PFT_STORE_BOTH) return PFT_E_UNSUPPORTED;
    pft_batch* b = new (std::nothrow) pft_batch();
    if (!b) return PFT_E_NOMEM;
    b->n = n;
    b->precision = params[0].precision;
    b->scheme = params[0].scheme;
    b->model = params[0].model;
    b->stream = static_cast<hipStream_t>(hip_stream);
    pft_status s = PFT_OK;
    for (int r = 0; r < n && s == PFT_OK; ++r) {
        pft_ctx* c = nullptr;
        s = create_ctx(&params[r], hip_stream, false, &c);
        if (s == PFT_OK) {
            b->ctx.push_back(c);
            // the conjugate sweep's work pair (both sweeps share every launch)
            if (params[r].model != PFT_EDWARDS && !c->U2 &&
                (hipMalloc(&c->U2, (size_t)c->M * c->elem) != hipSuccess ||
                 hipMalloc(&c->V2, (size_t)c->M * c->elem) != hipSuccess)) {
                (void)hipGetLastError();
                s = PFT_E_NOMEM;
            }
        }
    }
    // group by grid shape, in order of first appearance
    for (int r = 0; r < n && s == PFT_OK; ++r) {
        const pft_params& p = params[r];
        BatchGroup* g = nullptr;
        for (BatchGroup& x : b->groups)
            if (x.nx == p.nx && x.ny == p.ny && x.nz == p.nz && x.bc[0] == p.bc[0] && x.bc[1] == p.bc[1] &&
                x.bc[2] == p.bc[2] && x.fused == b->ctx[r]->fused)
                g = &x;
        if (!g) {
            b->groups.emplace_back();
            g = &b->groups.back();
            g->nx = p.nx;
            g->ny = p.ny;
            g->nz = p.nz;
            for (int a = 0; a < 3; ++a) g->bc[a] = p.bc[a];
            g->ndir = p.model == PFT_EDWARDS ? 1 : 2;
            g->fused = b->ctx[r]->fused;
            if (g->fused) {
                g->npass = 1;  // the x pass; the y and z work runs in the yz pass
                g->sp_axis[0] = 0;
            } else {
                g->npass = p.scheme == PFT_RQM4 ? 3 : 2;
                const int ax3[3] = {1, 0, 1};
                for (int k = 0; k < 3; ++k) g->sp_axis[k] = ax3[k];
            }
        }
        g->reps.push_back(r);
        for (int a = 0; a < 3; ++a) g->var[a] = b->ctx[g->reps[0]]->var[a];
        g->maxK = std::max(g->maxK, b->ctx[r]->K);
        g->maxM = std::max<int64_t>(g->maxM, b->ctx[r]->M);
    }
    if (s == PFT_OK) {
        for (BatchGroup& g : b->groups) {
            if (hipStreamCreateWithFlags(&g.s, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess) {
                s = PFT_E_DEVICE;
                break;
            }
        }
    }
    if (s == PFT_OK && (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
                        hipEventCreateWithFlags(&b->in, hipEventDisableTiming) != hipSuccess ||
                        hipEventCreateWithFlags(&b->out, hipEventDisableTiming) != hipSuccess ||
                        hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking) != hipSuccess ||
                        hipMalloc((void**)&b->counters, 2 * sizeof(uint64_t)) != hipSuccess ||
                        hipMalloc((void**)&b->logj, (size_t)n * sizeof(LogJob)) != hipSuccess))
        s = PFT_E_NOMEM;
    if (s == PFT_OK) s = b->precision == PFT_C128 ? batch_setup_t<double>(b) : batch_setup_t<float>(b);
    if (s != PFT_OK) {
        (void)hipGetLastError();
        batch_free(b);
        delete b;
        return s;
    }
    *out = b;
    return PFT_OK;
}

void pft_batch_destroy(pft_batch* b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    if (b->own) (void)hipStreamSynchronize(b->own);
    for (BatchGroup& g : b->groups) (void)hipStreamSynchronize(g.s);
    batch_free(b);
    delete b;
}

const char* pft_batch_last_error(const pft_batch* b) { return b ? b->err.c_str() : "null batch"; }

static bool batch_ptrs_ok(const pft_batch* b, const double* const* p, bool optional)
{
    if (!p) return optional;
    for (int r = 0; r < b->n; ++r)
        if (!aligned16(p[r])) return false;
    return true;
}

pft_status pft_batch_evaluate(pft_batch* b, const double* const* w_plus, const double* const* w_minus,
                              double* const* phi_a, double* const* phi_b, double* Q, double* H)
{
    if (!b) return PFT_E_INVALID;
    const bool ed = b->model == PFT_EDWARDS;  // one field: w_minus is ignored and may be NULL
    if (!batch_ptrs_ok(b, w_plus, false) || (!ed && !batch_ptrs_ok(b, w_minus, false)) ||
        !batch_ptrs_ok(b, phi_a, false) || !batch_ptrs_ok(b, phi_b, false) || !aligned16(Q) || !aligned16(H))
        return b->fail(PFT_E_INVALID, "pft_batch_evaluate: every pointer must be non-null and 16-byte aligned");
    return b->precision == PFT_C128 ? batch_evaluate_t<double>(b, w_plus, w_minus, phi_a, phi_b, Q, H)
                                    : batch_evaluate_t<float>(b, w_plus, w_minus, phi_a, phi_b, Q, H);
}

pft_status pft_batch_cl_steps(pft_batch* b, double* const* w_plus, double* const* w_minus, const pft_step* step,
                              int32_t nsteps, double* QH_log, int64_t log_rows)
{
    if (!b) return PFT_E_INVALID;
    const bool ed = b->model == PFT_EDWARDS;  // one field: w_minus is ignored and may be NULL
    if (!step || nsteps < 0 || !batch_ptrs_ok(b, const_cast<const double* const*>(w_plus), false) ||
        (!ed && !batch_ptrs_ok(b, const_cast<const double* const*>(w_minus), false)) || (QH_log && !aligned16(QH_log)) ||
        log_rows < 0)
        return b->fail(PFT_E_INVALID, "pft_batch_cl_steps: bad arguments");
    if (!(step->dt >= 0) || !(step->lambda_plus >= 0) || !(step->lambda_minus >= 0))
        return b->fail(PFT_E_INVALID, "dt and mobilities must be non-negative");
    if (step->update != 0 && step->update != 1) return b->fail(PFT_E_INVALID, "update must be 0 or 1");
    if (step->update == 1)
        for (int r = 0; r < b->n; ++r) {
            const char* why = sis_walls_unsupported(b->ctx[r]->p);
            if (why) return b->fail(PFT_E_UNSUPPORTED, "replica %d: %s", r, why);
        }
    const double* const* wp = const_cast<const double* const*>(w_plus);
    const double* const* wm = ed ? nullptr : const_cast<const double* const*>(w_minus);
    return b->precision == PFT_C128 ? batch_steps_t<double>(b, wp, wm, step, nsteps, QH_log, QH_log ? log_rows : 0)
                                    : batch_steps_t<float>(b, wp, wm, step, nsteps, QH_log, QH_log ? log_rows : 0);
}

pft_status pft_batch_sync(pft_batch* b)
{
    if (!b) return PFT_E_INVALID;
    PFT_BHIP(b, hipStreamSynchronize(b->stream));
    return PFT_OK;
}

pft_status pft_autotune(int32_t precision, const int32_t* sizes, int32_t nsizes, void* hip_stream, int32_t* choices,
                        double* timings)
{
    if ((precision != PFT_C128 && precision != PFT_C64) || !sizes || nsizes < 1) return PFT_E_INVALID;
    for (int i = 0; i < nsizes; ++i)
        if (!pft::axis_supported(sizes[i])) return PFT_E_UNSUPPORTED;
    for (int i = 0; i < nsizes; ++i) {
        const int N = sizes[i];
        const int A = tune_side(N);
        for (int kind = 0; kind < 2; ++kind) {
            pft_params p{};
            p.nx = kind == 0 ? A : N;
            p.ny = A;
            p.nz = kind == 0 ? N : A;
            p.lx = p.ly = p.lz = 0.1 * A;
            if (kind == 0) p.lz = 0.1 * N; else p.lx = 0.1 * N;
            p.ns = 2;
            p.f = 0.5;
            p.chiN = 10;
            p.C = 1;
            p.precision = precision;
            p.scheme = PFT_SPLIT2;
            pft_ctx* c = nullptr;
            pft_status st = pft_create(&p, hip_stream, &c);
            if (st) return st;
            // the timed inputs: zeros are fine for timing (no data-dependent work)
            hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(c->M * c->elem / 16, 256)), dim3(256), 0, c->stream,
                               static_cast<double2*>(c->work), (int64_t)(c->M * c->elem / 16));
            hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(c->M * c->elem / 4, 256)), dim3(256), 0, c->stream,
                               static_cast<double2*>(c->E), (int64_t)(c->M * c->elem / 4));
            hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(c->M * c->elem / 16, 256)), dim3(256), 0, c->stream,
                               static_cast<double2*>(c->U), (int64_t)(c->M * c->elem / 16));
            hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(c->M * c->elem / 16, 256)), dim3(256), 0, c->stream,
                               static_cast<double2*>(c->V), (int64_t)(c->M * c->elem / 16));
            int best = 0;
            double best_ms = -1;
            for (int v = 0; v < PFT_MAX_VARIANTS; ++v) {
                int n1, n2, w;
                double ms = -1;
                if (pft::axis_variant(N, v, &n1, &n2, &w))
                    ms = precision == PFT_C128 ? time_variant<double>(c, kind, v, 10) : time_variant<float>(c, kind, v, 10);
                if (timings) timings[(i * 2 + kind) * PFT_MAX_VARIANTS + v] = ms;
                if (ms > 0 && (best_ms < 0 || ms < best_ms)) {
                    best_ms = ms;
                    best = v;
                }
            }
            pft_destroy(c);
            if (best_ms < 0) return PFT_E_DEVICE;
            g_tune[precision][N][kind] = best;
            if (choices) choices[i * 2 + kind] = best;
        }
    }
    return PFT_OK;
}

pft_status pft_tune_save(const char* path)
{
    if (!path) return PFT_E_INVALID;
    FILE* f = std::fopen(path, "w");
    if (!f) return PFT_E_INVALID;
    const std::string arch = device_arch();
    for (int prec = 0; prec < 2; ++prec)
        for (int n = 0; n <= 256; ++n)
            for (int kind = 0; kind < 2; ++kind)
                if (pft::axis_supported(n))
                    std::fprintf(f, "%s %d %d %d %d\n", arch.c_str(), prec, n, kind, g_tune[prec][n][kind]);
    std::fclose(f);
    return PFT_OK;
}

pft_status pft_tune_load(const char* path)
{
    if (!path) return PFT_E_INVALID;
    FILE* f = std::fopen(path, "r");
    if (!f) return PFT_E_INVALID;
    const std::string arch = device_arch();
    char a[64];
    int prec, n, kind, v;
    while (std::fscanf(f, "%63s %d %d %d %d", a, &prec, &n, &kind, &v) == 5) {
        int n1, n2, w;
        if (arch == a && (prec == 0 || prec == 1) && (kind == 0 || kind == 1) && n >= 0 && n <= 256 &&
            pft::axis_variant(n, v, &n1, &n2, &w))
            g_tune[prec][n][kind] = v;
    }
    std::fclose(f);
    return PFT_OK;
}

pft_status pft_set_variant(pft_ctx* c, int32_t axis, int32_t variant)
{
    if (!c || axis < 0 || axis > 2) return PFT_E_INVALID;
    const int n = axis == 0 ? c->p.nx : axis == 1 ? c->p.ny : c->p.nz;
    int n1, n2, w;
    if (!pft::axis_variant(n, variant, &n1, &n2, &w)) return c->fail(PFT_E_UNSUPPORTED, "no variant %d for %d", variant, n);
    c->var[axis] = variant;
    return PFT_OK;
}

pft_status pft_noise_words(uint64_t seed, uint64_t rep, uint64_t step, int32_t field, int64_t M, uint64_t* out,
                           void* stream)
{
    if (!out || M < 1 || (field != 0 && field != 1)) return PFT_E_INVALID;
    const int64_t ng = (M + 3) / 4;
    hipLaunchKernelGGL(k_noise_words, dim3(grid_for(ng, 256)), dim3(256), 0, static_cast<hipStream_t>(stream), seed, rep,
                       step, field, ng, out);
    return hipGetLastError() == hipSuccess ? PFT_OK : PFT_E_DEVICE;
}

pft_status pft_noise_normals(uint64_t seed, uint64_t rep, uint64_t step, int32_t field, int64_t M, double* out,
                             void* stream)
{
    if (!out || M < 1 || (field != 0 && field != 1)) return PFT_E_INVALID;
    hipLaunchKernelGGL(k_noise_normals, dim3(grid_for((M + 3) / 4, 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), seed, rep, step, field, M, out);
    return hipGetLastError() == hipSuccess ? PFT_OK : PFT_E_DEVICE;
}

}  // extern "C"
