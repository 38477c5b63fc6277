// Elementwise and reduction kernels of the propagator runtime (everything
// around the axis and plane passes): field operator tables, the compensated
// sums behind Q, node Q and H, the Euler-Maruyama field step with its
// Philox4x64-10 noise, the local part of the semi-implicit step and its
// mirror images, the reverse-mode accumulation and box stress, and job-table
// forms of these for batches.  Host code includes this once per translation
// unit (internal linkage).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "density.h"
#include "fft.h"

using pft::cdiv;
using pft::cmul;
using pft::cx;
using pft::density_body;
using pft::k_density;
using pft::NSum;

namespace pft::ops {

// Field operator tables E = exp(-w_b a) for up to four (block, a) pairs,
// evaluated in double and rounded once to the working precision.
struct TabDesc {
    int n;
    int blk[4];
    double a[4];
};

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

// |k|^2 = (2 pi m / Le)^2 per axis in natural order (m = j, or j - ne above
// ne / 2), Le the period the filter sees (2L along a reflecting axis): row
// blockIdx.x of k2.  The same operations, in the same order, as the host
// table of the context's semi-implicit step.
struct K2Rows {
    int ne[3];
    double Le[3];
};

// Batched forms (blockIdx.y is the replica): the image arguments and the field
// that receives the filtered increment.
struct MirrorJob {
    MirrorArgs m;
    double2* w;
    int64_t M;
};

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

}  // namespace pft::ops

using namespace pft::ops;

// Every translation unit of the runtime includes this file and launches a
// subset of its kernels.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wunused-function"

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


__global__ void k_sis_mirror_batch(const MirrorJob* __restrict__ jobs) { sis_mirror_body(jobs[blockIdx.y].m); }

__global__ void k_sis_unmirror_batch(const MirrorJob* __restrict__ jobs)
{
    const MirrorJob& j = jobs[blockIdx.y];
    sis_unmirror_body(j.m, j.w, j.M);
}


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

}  // namespace

#pragma clang diagnostic pop
