/*
 * pft_oracle.c -- plain FP64 CPU oracle for the propagator hot path of
 * K. T. Delaney and G. H. Fredrickson, "Polymer Field-Theory Simulations on
 * Graphics Processing Units" (arXiv:1204.5434).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct reference the
 * GPU library is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header, table
 * or constant with the GPU library and the GPU library never calls it.
 *
 * Everything is IEEE double precision (C99 double complex).  Fields are
 * stored in C order [nx][ny][nz] (z fastest).  No FFT library is used: the
 * discrete Fourier transform is either the O(M^2) definition written out
 * (or_dft3_naive) or a plain recursive Cooley-Tukey FFT (or_fft3).
 *
 * Readings of points the paper leaves open (the q-dagger convention, the
 * contour quadrature, the A/B junction, the update sign, the noise stream)
 * are stated next to the function that takes them.
 *
 * Parity status: every function here is pinned by the CPU test suite
 * (closed forms, invariants, Debye response, convergence order, brute-force
 * DFT, numpy's Philox, finite differences); none is "parity unpinned".
 */
#include <complex.h>
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define OR_TWO_PI 6.283185307179586476925286766559

/* Model and discretisation parameters.  Lengths in units of R_g, the contour
 * normalised to [0, 1] (Sec. II, Eqs. (3)-(5)). */
typedef struct {
    int32_t nx, ny, nz;    /* grid points per axis                               */
    double lx, ly, lz;     /* periodic box edges                                 */
    int32_t ns;            /* contour steps, ds = 1/ns                           */
    double f;              /* A-block fraction f_A (Eq. (8))                     */
    double chiN;           /* chi_AB N (Eq. (3))                                 */
    double C;              /* chain number density parameter (Eq. (3))           */
    int32_t scheme;        /* 0 = Richardson split step (Eq. (12)), 1 = plain split */
    int32_t naive_dft;     /* 1: use the O(M^2) DFT definition, 0: recursive FFT */
    int32_t bc[3];         /* per axis: 0 periodic (DFT), 1 reflecting walls (Neumann,
                              cosine transform), 2 absorbing walls (Dirichlet, sine
                              transform) -- Sec. III, boundary conditions of Eq. (5) */
} or_params;

enum { OR_PERIODIC = 0, OR_NEUMANN = 1, OR_DIRICHLET = 2 };

enum { OR_RQM4 = 0, OR_SPLIT2 = 1 };

static int64_t grid_m(const or_params *p) { return (int64_t)p->nx * p->ny * p->nz; }

void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Contour discretisation.                                                   */
/*                                                                           */
/* Reading of Eq. (8): the A block occupies s in [0, f], the B block [f, 1]. */
/* The contour is cut into ns steps of ds = 1/ns.  When f*ns is not an       */
/* integer, a node is inserted at s = f and the step that straddles it is    */
/* split into an A sub-step of length f - n*ds and a B sub-step of length    */
/* (n+1)*ds - f, so each step sees a single field and the block integrals of */
/* Eq. (8) end exactly on a node.                                            */
/*                                                                           */
/* Outputs: h[j], blk[j] (0 = A, 1 = B) for steps j = 0..K-1; *junction = the */
/* node index J with s_J = f.  Returns K.                                    */
/* ------------------------------------------------------------------------ */
int or_contour(int32_t ns, double f, double *h, int32_t *blk, int32_t *junction)
{
    const double ds = 1.0 / ns;
    const double fn = f * ns;
    const double r = floor(fn + 0.5);
    int K = 0;
    if (fabs(fn - r) <= 1e-9) {
        const int na = (int)r;
        for (int j = 0; j < ns; j++) {
            h[K] = ds;
            blk[K] = (j < na) ? 0 : 1;
            K++;
        }
        *junction = na;
    } else {
        const int nstar = (int)floor(fn);
        for (int j = 0; j < nstar; j++) { h[K] = ds; blk[K] = 0; K++; }
        h[K] = f - nstar * ds; blk[K] = 0; K++;
        h[K] = (nstar + 1) * ds - f; blk[K] = 1; K++;
        for (int j = nstar + 1; j < ns; j++) { h[K] = ds; blk[K] = 1; K++; }
        *junction = nstar + 1;
    }
    return K;
}

/* Composite trapezoid weights of each block on its own nodes (reading of the */
/* contour integrals in Eq. (8)): an end node of a block gets half its one     */
/* adjacent step, an interior node half of each of its two adjacent steps.    */
/* tauA, tauB have K+1 entries (one per node); tauA is zero on B-only nodes.  */
void or_trapezoid(int K, const double *h, const int32_t *blk, double *tauA, double *tauB)
{
    for (int j = 0; j <= K; j++) { tauA[j] = 0.0; tauB[j] = 0.0; }
    for (int j = 0; j < K; j++) {
        double *tau = (blk[j] == 0) ? tauA : tauB;
        tau[j] += 0.5 * h[j];
        tau[j + 1] += 0.5 * h[j];
    }
}

/* Integer wave number of DFT index j on an axis of n points: j for j <= n/2, */
/* j - n above.  Only its square enters the diffusion operator.               */
int32_t or_mode(int32_t j, int32_t n) { return (j <= n / 2) ? j : j - n; }

/* ------------------------------------------------------------------------ */
/* Discrete Fourier transform.                                               */
/* Forward: U[k] = sum_x u[x] exp(-2 pi i k.x / n) (sign = -1), unnormalised. */
/* Inverse: sign = +1, also unnormalised (the 1/M lives in or_diffuse).      */
/* ------------------------------------------------------------------------ */

/* e^{sign 2 pi i a / n} with the angle reduced exactly in integers. */
static cplx unit_root(int64_t a, int64_t n, int sign)
{
    int64_t r = a % n;
    if (r < 0) r += n;
    const double t = OR_TWO_PI * (double)r / (double)n;
    return cos(t) + sign * sin(t) * I;
}

/* The definition written out: O(M^2) three-dimensional DFT. */
void or_dft3_naive(const cplx *in, cplx *out, int32_t nx, int32_t ny, int32_t nz, int32_t sign)
{
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < (int64_t)nx * ny * nz; k++) {
        const int64_t kx = k / ((int64_t)ny * nz), ky = (k / nz) % ny, kz = k % nz;
        cplx acc = 0.0;
        for (int64_t x = 0; x < nx; x++)
            for (int64_t y = 0; y < ny; y++)
                for (int64_t z = 0; z < nz; z++) {
                    /* phase = kx x/nx + ky y/ny + kz z/nz, summed over a common denominator */
                    const int64_t den = (int64_t)nx * ny * nz;
                    const int64_t num = kx * x * ny * nz + ky * y * nx * nz + kz * z * nx * ny;
                    acc += in[(x * ny + y) * nz + z] * unit_root(num, den, sign);
                }
        out[k] = acc;
    }
}

static int smallest_factor(int n)
{
    for (int p = 2; p * p <= n; p++)
        if (n % p == 0) return p;
    return n;
}

/*
 * Recursive decimation-in-time Cooley-Tukey FFT of length n.
 * x: input with element stride s; X: contiguous output of length n.
 * tw[t] = e^{sign 2 pi i t / ntop}; W_n^a = tw[a * (ntop / n)].
 * With p the smallest factor of n and m = n/p:
 *   Y_r[k] = DFT_m of x[(i p + r) s] over i,
 *   X[k + m q] = sum_r W_n^{r (k + m q)} Y_r[k].
 */
static void fft_rec(const cplx *x, ptrdiff_t s, cplx *X, int n, const cplx *tw, int ntop)
{
    if (n == 1) { X[0] = x[0]; return; }
    const int p = smallest_factor(n);
    const int m = n / p;
    const int step = ntop / n;
    if (p == n) {               /* prime length: the definition */
        for (int k = 0; k < n; k++) {
            cplx acc = 0.0;
            for (int j = 0; j < n; j++) acc += x[j * s] * tw[(int64_t)((j * k) % n) * step];
            X[k] = acc;
        }
        return;
    }
    for (int r = 0; r < p; r++) fft_rec(x + r * s, s * p, X + r * m, m, tw, ntop);
    cplx t[64];
    cplx *tmp = (p <= 64) ? t : (cplx *)malloc(sizeof(cplx) * p);
    for (int k = 0; k < m; k++) {
        for (int r = 0; r < p; r++) tmp[r] = X[r * m + k] * tw[(int64_t)((r * k) % n) * step];
        for (int q = 0; q < p; q++) {
            cplx acc = 0.0;
            for (int r = 0; r < p; r++) acc += tmp[r] * tw[(int64_t)((r * q) % p) * m * step];
            X[k + m * q] = acc;
        }
    }
    if (tmp != t) free(tmp);
}

/* 1-D FFT along one axis of a [nx][ny][nz] array, in place, all lines. */
static void fft_axis(cplx *a, int32_t nx, int32_t ny, int32_t nz, int axis, int sign)
{
    const int n = (axis == 0) ? nx : (axis == 1) ? ny : nz;
    const ptrdiff_t stride = (axis == 0) ? (ptrdiff_t)ny * nz : (axis == 1) ? nz : 1;
    const int64_t nlines = (int64_t)nx * ny * nz / n;
    cplx *tw = (cplx *)malloc(sizeof(cplx) * n);
    for (int t = 0; t < n; t++) tw[t] = unit_root(t, n, sign);
    #pragma omp parallel
    {
        cplx *in = (cplx *)malloc(sizeof(cplx) * n);
        cplx *out = (cplx *)malloc(sizeof(cplx) * n);
        #pragma omp for schedule(static)
        for (int64_t l = 0; l < nlines; l++) {
            ptrdiff_t base;
            if (axis == 2) base = l * nz;
            else if (axis == 1) base = (l / nz) * (ptrdiff_t)ny * nz + (l % nz);
            else base = l;
            for (int i = 0; i < n; i++) in[i] = a[base + i * stride];
            fft_rec(in, 1, out, n, tw, n);
            for (int i = 0; i < n; i++) a[base + i * stride] = out[i];
        }
        free(in);
        free(out);
    }
    free(tw);
}

/* Three-dimensional FFT in place: the 1-D transform along z, y and x. */
void or_fft3(cplx *a, int32_t nx, int32_t ny, int32_t nz, int32_t sign)
{
    fft_axis(a, nx, ny, nz, 2, sign);
    fft_axis(a, nx, ny, nz, 1, sign);
    fft_axis(a, nx, ny, nz, 0, sign);
}

static void dft3(const or_params *p, cplx *u, int sign)
{
    if (p->naive_dft) {
        const int64_t M = grid_m(p);
        cplx *t = (cplx *)malloc(sizeof(cplx) * M);
        or_dft3_naive(u, t, p->nx, p->ny, p->nz, sign);
        memcpy(u, t, sizeof(cplx) * M);
        free(t);
    } else {
        or_fft3(u, p->nx, p->ny, p->nz, sign);
    }
}

/* |k|^2 of DFT index (jx, jy, jz): sum over axes of (2 pi m / L)^2. */
static double ksq(const or_params *p, int64_t jx, int64_t jy, int64_t jz)
{
    const double kx = OR_TWO_PI * or_mode((int32_t)jx, p->nx) / p->lx;
    const double ky = OR_TWO_PI * or_mode((int32_t)jy, p->ny) / p->ly;
    const double kz = OR_TWO_PI * or_mode((int32_t)jz, p->nz) / p->lz;
    return kx * kx + ky * ky + kz * kz;
}

/* |k|^2 on the whole grid, natural DFT order (a test hook for the k-grid). */
void or_ksq_grid(const or_params *p, double *out)
{
    for (int64_t jx = 0; jx < p->nx; jx++)
        for (int64_t jy = 0; jy < p->ny; jy++)
            for (int64_t jz = 0; jz < p->nz; jz++)
                out[(jx * p->ny + jy) * p->nz + jz] = ksq(p, jx, jy, jz);
}

/*
 * One-dimensional diffusion exp(h d^2/dx^2) along one axis with walls, exact
 * on the eigenbasis of the walled Laplacian on the cell-centred grid
 * x_n = (n + 1/2) L / N:
 *   reflecting (Neumann): cos(pi m x / L), m = 0..N-1, the DCT-II pair
 *     X_m = sum_n u_n cos(pi m (n+1/2)/N),
 *     u_n = X_0 / N + (2/N) sum_{m>=1} X_m cos(pi m (n+1/2)/N);
 *   absorbing (Dirichlet): sin(pi m x / L), m = 1..N, the DST-II pair
 *     X_m = sum_n u_n sin(pi m (n+1/2)/N),
 *     u_n = (2/N) sum_{m<N} X_m sin(pi m (n+1/2)/N) + (1/N) X_N sin(pi N (n+1/2)/N);
 * each mode decays by exp(-(pi m / L)^2 h) (lap = 1: is multiplied by
 * (pi m / L)^2 instead, which applies -d^2/dx^2).  Written out as the
 * definitions, O(N^2) per line.
 */
static void walls_axis_modes(const or_params *p, double h, cplx *u, int axis, int lap)
{
    const int n = (axis == 0) ? p->nx : (axis == 1) ? p->ny : p->nz;
    const double L = (axis == 0) ? p->lx : (axis == 1) ? p->ly : p->lz;
    const ptrdiff_t stride = (axis == 0) ? (ptrdiff_t)p->ny * p->nz : (axis == 1) ? p->nz : 1;
    const int64_t nlines = grid_m(p) / n;
    const int dir = p->bc[axis] == OR_DIRICHLET;
    const double pi = OR_TWO_PI / 2.0;
    #pragma omp parallel
    {
        cplx *in = (cplx *)malloc(sizeof(cplx) * n);
        cplx *X = (cplx *)malloc(sizeof(cplx) * (n + 1));
        #pragma omp for schedule(static)
        for (int64_t l = 0; l < nlines; l++) {
            ptrdiff_t base;
            if (axis == 2) base = l * p->nz;
            else if (axis == 1) base = (l / p->nz) * (ptrdiff_t)p->ny * p->nz + (l % p->nz);
            else base = l;
            for (int i = 0; i < n; i++) in[i] = u[base + i * stride];
            for (int m = dir ? 1 : 0; m <= (dir ? n : n - 1); m++) {
                cplx acc = 0.0;
                for (int i = 0; i < n; i++) {
                    const double arg = pi * m * (i + 0.5) / n;
                    acc += in[i] * (dir ? sin(arg) : cos(arg));
                }
                const double k = pi * m / L;
                X[m] = acc * (lap ? k * k : exp(-k * k * h));
            }
            for (int i = 0; i < n; i++) {
                cplx acc = 0.0;
                if (dir) {
                    for (int m = 1; m < n; m++) acc += 2.0 * X[m] * sin(pi * m * (i + 0.5) / n);
                    acc += X[n] * sin(pi * n * (i + 0.5) / n);
                } else {
                    acc = X[0];
                    for (int m = 1; m < n; m++) acc += 2.0 * X[m] * cos(pi * m * (i + 0.5) / n);
                }
                u[base + i * stride] = acc / (double)n;
            }
        }
        free(in);
        free(X);
    }
}

static void diffuse_walls_axis(const or_params *p, double h, cplx *u, int axis)
{
    walls_axis_modes(p, h, u, axis, 0);
}

/* The diffusion operator exp(h Laplacian) of Eq. (5), exact on the Fourier */
/* basis: u <- IDFT( e^{-|k|^2 h} DFT(u) ) / M.  With walls on some axes the */
/* operator factorises over the axes: the periodic ones diffuse through the  */
/* 1-D DFT, the walled ones through their sine or cosine basis.              */
void or_diffuse(const or_params *p, double h, cplx *u)
{
    const int64_t M = grid_m(p);
    if (p->bc[0] || p->bc[1] || p->bc[2]) {
        for (int axis = 0; axis < 3; axis++) {
            if (p->bc[axis]) {
                diffuse_walls_axis(p, h, u, axis);
                continue;
            }
            const int n = (axis == 0) ? p->nx : (axis == 1) ? p->ny : p->nz;
            const double L = (axis == 0) ? p->lx : (axis == 1) ? p->ly : p->lz;
            fft_axis(u, p->nx, p->ny, p->nz, axis, -1);
            #pragma omp parallel for schedule(static)
            for (int64_t x = 0; x < M; x++) {
                const int64_t j = (axis == 0) ? x / ((int64_t)p->ny * p->nz) : (axis == 1) ? (x / p->nz) % p->ny : x % p->nz;
                const double k = OR_TWO_PI * or_mode((int32_t)j, n) / L;
                u[x] *= exp(-k * k * h) / (double)n;
            }
            fft_axis(u, p->nx, p->ny, p->nz, axis, +1);
        }
        return;
    }
    dft3(p, u, -1);
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < M; k++) {
        const int64_t jx = k / ((int64_t)p->ny * p->nz), jy = (k / p->nz) % p->ny, jz = k % p->nz;
        u[k] *= exp(-ksq(p, jx, jy, jz) * h) / (double)M;
    }
    dft3(p, u, +1);
}

/* u <- e^{-w a} u, the field operator of the split step, pointwise. */
static void mul_field_exp(cplx *u, const cplx *w, double a, int64_t M)
{
    #pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < M; x++) u[x] *= cexp(-w[x] * a);
}

/*
 * One contour step of length h in the field w, q_out = T_h(q_in; w).
 * Plain split (second order):  T = E_{h/2} D_h E_{h/2}.
 * Richardson split step, Eq. (12):
 *   T = -(1/3) [ E_{h/2} D_h E_{h/2} - 4 E_{h/4} D_{h/2} E_{h/2} D_{h/2} E_{h/4} ],
 * with E_a = e^{-w a} and D_a the diffusion operator; operators act right to left.
 * work must hold 2*M values.
 */
void or_step(const or_params *p, int32_t scheme, double h, const cplx *w,
             const cplx *qin, cplx *qout, cplx *work)
{
    const int64_t M = grid_m(p);
    cplx *full = work, *half = work + M;
    /* one full step: E_{h/2} D_h E_{h/2} q */
    memcpy(full, qin, sizeof(cplx) * M);
    mul_field_exp(full, w, h / 2, M);
    or_diffuse(p, h, full);
    mul_field_exp(full, w, h / 2, M);
    if (scheme == OR_SPLIT2) {
        memcpy(qout, full, sizeof(cplx) * M);
        return;
    }
    /* two half steps: E_{h/4} D_{h/2} E_{h/2} D_{h/2} E_{h/4} q */
    memcpy(half, qin, sizeof(cplx) * M);
    mul_field_exp(half, w, h / 4, M);
    or_diffuse(p, h / 2, half);
    mul_field_exp(half, w, h / 2, M);
    or_diffuse(p, h / 2, half);
    mul_field_exp(half, w, h / 4, M);
    for (int64_t x = 0; x < M; x++) qout[x] = -(1.0 / 3.0) * (full[x] - 4.0 * half[x]);
}

/* Block fields w_A = i w_+ - w_-, w_B = i w_+ + w_- (Sec. II, after Eq. (3)). */
void or_block_fields(const or_params *p, const cplx *wp, const cplx *wm, cplx *wA, cplx *wB)
{
    const int64_t M = grid_m(p);
    for (int64_t x = 0; x < M; x++) {
        wA[x] = I * wp[x] - wm[x];
        wB[x] = I * wp[x] + wm[x];
    }
}

/*
 * Forward and conjugate propagators (Eq. (5) with the initial conditions that
 * follow it).  Reading of the q-dagger convention of Eq. (8): q-dagger runs on
 * its own contour s' = 1 - s from q-dagger(s'=0) = 1 at the B end, so node j
 * of q pairs with node K-j of q-dagger.
 *   q_0 = 1,  q_{j+1} = T_{h_j}(q_j; w_{blk(j)}),
 *   qd_0 = 1, qd_{i+1} = T_{h_{K-1-i}}(qd_i; w_{blk(K-1-i)}).
 * qs and qds hold (K+1)*M values each (slice j at offset j*M); either may be
 * NULL to skip that sweep.  Returns K.
 */
int or_propagate(const or_params *p, const cplx *wp, const cplx *wm, cplx *qs, cplx *qds)
{
    const int64_t M = grid_m(p);
    double *h = (double *)malloc(sizeof(double) * (p->ns + 2));
    int32_t *blk = (int32_t *)malloc(sizeof(int32_t) * (p->ns + 2));
    int32_t J;
    const int K = or_contour(p->ns, p->f, h, blk, &J);
    cplx *wA = (cplx *)malloc(sizeof(cplx) * M);
    cplx *wB = (cplx *)malloc(sizeof(cplx) * M);
    cplx *work = (cplx *)malloc(sizeof(cplx) * 2 * M);
    or_block_fields(p, wp, wm, wA, wB);
    if (qs) {
        for (int64_t x = 0; x < M; x++) qs[x] = 1.0;
        for (int j = 0; j < K; j++)
            or_step(p, p->scheme, h[j], blk[j] == 0 ? wA : wB, qs + (int64_t)j * M,
                    qs + (int64_t)(j + 1) * M, work);
    }
    if (qds) {
        for (int64_t x = 0; x < M; x++) qds[x] = 1.0;
        for (int i = 0; i < K; i++) {
            const int j = K - 1 - i;
            or_step(p, p->scheme, h[j], blk[j] == 0 ? wA : wB, qds + (int64_t)i * M,
                    qds + (int64_t)(i + 1) * M, work);
        }
    }
    free(h); free(blk); free(wA); free(wB); free(work);
    return K;
}

/*
 * Partition function and segment densities from stored propagators.
 * Q = (1/M) sum_x q_K(x)   (Eq. (4), the integral as the grid mean).
 * Qnode[j] = (1/M) sum_x q_j(x) qd_{K-j}(x) for every node (equal to Q in
 * exact arithmetic; a diagnostic of the sweeps).
 * phi_A = (1/Q) sum_j tauA_j q_j qd_{K-j},  phi_B likewise (Eq. (8) divided by
 * rho_0, with the trapezoid weights of or_trapezoid).
 */
void or_densities(const or_params *p, const cplx *qs, const cplx *qds,
                  cplx *phiA, cplx *phiB, cplx *Q, cplx *Qnode)
{
    const int64_t M = grid_m(p);
    double *h = (double *)malloc(sizeof(double) * (p->ns + 2));
    int32_t *blk = (int32_t *)malloc(sizeof(int32_t) * (p->ns + 2));
    int32_t J;
    const int K = or_contour(p->ns, p->f, h, blk, &J);
    double *tauA = (double *)malloc(sizeof(double) * (K + 1));
    double *tauB = (double *)malloc(sizeof(double) * (K + 1));
    or_trapezoid(K, h, blk, tauA, tauB);

    cplx sum = 0.0;
    for (int64_t x = 0; x < M; x++) sum += qs[(int64_t)K * M + x];
    *Q = sum / (double)M;
    if (Qnode) {
        for (int j = 0; j <= K; j++) {
            cplx s = 0.0;
            for (int64_t x = 0; x < M; x++) s += qs[(int64_t)j * M + x] * qds[(int64_t)(K - j) * M + x];
            Qnode[j] = s / (double)M;
        }
    }
    #pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < M; x++) {
        cplx a = 0.0, b = 0.0;
        for (int j = 0; j <= K; j++) {
            const cplx prod = qs[(int64_t)j * M + x] * qds[(int64_t)(K - j) * M + x];
            a += tauA[j] * prod;
            b += tauB[j] * prod;
        }
        phiA[x] = a / *Q;
        phiB[x] = b / *Q;
    }
    free(h); free(blk); free(tauA); free(tauB);
}

/*
 * Diblock Hamiltonian, Eq. (3), on the grid (integral -> dV * sum):
 *   H = C dV sum_x [ w_-^2 / chiN - i w_+ ] - C V log Q,
 * with dV = V/M, V = lx ly lz and the principal branch of the complex log.
 * Also returns the intensive h = H / (C V).
 */
void or_hamiltonian(const or_params *p, const cplx *wp, const cplx *wm, double Qre, double Qim,
                    cplx *H, cplx *hint)
{
    const cplx Q = Qre + Qim * I;
    const int64_t M = grid_m(p);
    const double V = p->lx * p->ly * p->lz;
    const double dV = V / (double)M;
    cplx s = 0.0;
    for (int64_t x = 0; x < M; x++) s += wm[x] * wm[x] / p->chiN - I * wp[x];
    *H = p->C * dV * s - p->C * V * clog(Q);
    *hint = *H / (p->C * V);
}

/*
 * Mean-field forces (the functional derivatives of Eq. (3) per unit C dV,
 * written in terms of phi = rho/rho_0; the unnumbered mean-field equations
 * of Sec. II):
 *   F_+ = i (phi_A + phi_B - 1),   F_- = 2 w_- / chiN + phi_B - phi_A.
 */
void or_forces(const or_params *p, const cplx *wm, const cplx *phiA, const cplx *phiB,
               cplx *Fp, cplx *Fm)
{
    const int64_t M = grid_m(p);
    for (int64_t x = 0; x < M; x++) {
        Fp[x] = I * (phiA[x] + phiB[x] - 1.0);
        Fm[x] = 2.0 * wm[x] / p->chiN + phiB[x] - phiA[x];
    }
}

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random       */
/* numbers: as easy as 1, 2, 3"): ten rounds of two 64x64->128 multiplies   */
/* with a Weyl-sequence key schedule.                                       */
/* ------------------------------------------------------------------------ */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    const unsigned __int128 prod = (unsigned __int128)a * b;
    *hi = (uint64_t)(prod >> 64);
    *lo = (uint64_t)prod;
}

void or_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, c0, &hi0, &lo0);
        mulhilo64(M1, c2, &hi1, &lo1);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0, 1), never 0: the top 53 bits plus one half, times 2^-53. */
static double u01(uint64_t x) { return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

/*
 * Standard normal deviates for one field at one Langevin step.
 * Stream layout: key = (seed, replica); the block of four sites 4g..4g+3 of
 * field `field` at step `step` uses counter (g, field, step, 0); its four
 * 64-bit words become two Box-Muller pairs (u0,u1) -> (z0,z1), (u2,u3) -> (z2,z3),
 * and site 4g+r takes z_r.
 */
void or_gaussian(uint64_t seed, uint64_t replica, uint64_t step, int32_t field, int64_t M, double *xi)
{
    const uint64_t key[2] = {seed, replica};
    for (int64_t g = 0; 4 * g < M; g++) {
        const uint64_t ctr[4] = {(uint64_t)g, (uint64_t)field, step, 0};
        uint64_t r[4];
        or_philox4x64_10(ctr, key, r);
        double z[4];
        for (int pair = 0; pair < 2; pair++) {
            const double a = u01(r[2 * pair]), b = u01(r[2 * pair + 1]);
            const double rad = sqrt(-2.0 * log(a));
            z[2 * pair] = rad * cos(OR_TWO_PI * b);
            z[2 * pair + 1] = rad * sin(OR_TWO_PI * b);
        }
        for (int rr = 0; rr < 4 && 4 * g + rr < M; rr++) xi[4 * g + rr] = z[rr];
    }
}

/*
 * Explicit Euler-Maruyama step of the field equation of motion, Eq. (9), for
 * both fields at once from the forces of the current fields:
 *   w_+ <- w_+ - lam_+ dt F_+ + s_+ xi_+,   w_- <- w_- - lam_- dt F_- + s_- xi_-,
 * with xi real standard normals and s^2 = 2 lam dt / (C dV), the discrete noise
 * variance given after Eq. (10) for forces taken per unit C dV.  Reading: the
 * fields are not Wick rotated (Sec. III), so the drift is -lam F for both;
 * noise = 0 gives the deterministic (SCFT) relaxation.
 */
void or_em_update(const or_params *p, cplx *wp, cplx *wm, const cplx *phiA, const cplx *phiB,
                  double dt, double lam_p, double lam_m, int32_t noise,
                  uint64_t seed, uint64_t replica, uint64_t step)
{
    const int64_t M = grid_m(p);
    const double dV = p->lx * p->ly * p->lz / (double)M;
    cplx *Fp = (cplx *)malloc(sizeof(cplx) * M);
    cplx *Fm = (cplx *)malloc(sizeof(cplx) * M);
    double *xp = (double *)calloc(M, sizeof(double));
    double *xm = (double *)calloc(M, sizeof(double));
    or_forces(p, wm, phiA, phiB, Fp, Fm);
    if (noise) {
        or_gaussian(seed, replica, step, 0, M, xp);
        or_gaussian(seed, replica, step, 1, M, xm);
    }
    const double sp = noise ? sqrt(2.0 * lam_p * dt / (p->C * dV)) : 0.0;
    const double sm = noise ? sqrt(2.0 * lam_m * dt / (p->C * dV)) : 0.0;
    for (int64_t x = 0; x < M; x++) {
        wp[x] = wp[x] - lam_p * dt * Fp[x] + sp * xp[x];
        wm[x] = wm[x] - lam_m * dt * Fm[x] + sm * xm[x];
    }
    free(Fp); free(Fm); free(xp); free(xm);
}

/*
 * One full field evaluation: propagators, Q, per-node Q, densities and H.
 * Convenience wrapper over the functions above.  Qnode may be NULL.
 */
int or_evaluate(const or_params *p, const cplx *wp, const cplx *wm,
                cplx *phiA, cplx *phiB, cplx *Q, cplx *Qnode, cplx *H, cplx *hint)
{
    const int64_t M = grid_m(p);
    const int64_t K = p->ns + 1; /* upper bound on the step count */
    cplx *qs = (cplx *)malloc(sizeof(cplx) * (K + 1) * M);
    cplx *qds = (cplx *)malloc(sizeof(cplx) * (K + 1) * M);
    if (!qs || !qds) { free(qs); free(qds); return -1; }
    const int k = or_propagate(p, wp, wm, qs, qds);
    or_densities(p, qs, qds, phiA, phiB, Q, Qnode);
    or_hamiltonian(p, wp, wm, creal(*Q), cimag(*Q), H, hint);
    free(qs); free(qds);
    return k;
}

/* ------------------------------------------------------------------------ */
/* First-order semi-implicit field step (Eq. (10) and the effective step of  */
/* Eq. (11)).  The linear part L of the force is taken implicitly, mode by   */
/* mode in reciprocal space:                                                 */
/*   w^(t+dt)(k) = w^t(k) - [lam dt F^t(k) - eta(k)] / (1 + lam dt g(k)).     */
/* Readings: the noise is divided by the same factor (solving Eq. (10) for   */
/* w^(t+dt) gives it so; Eq. (11) writes the transformed noise as one term); */
/* g is the linear response per unit C dV of the force to its own field:    */
/*   diblock w_+ : g = g_D(|k|^2), the Debye function of the whole chain     */
/*                 (delta(phi_A + phi_B) = -g_D delta(i w_+) in the weak-   */
/*                 field limit), g_D(0) = 1;                                  */
/*   diblock w_- : g = 2 / chiN, the explicitly linear term of F_- (the      */
/*                 density part of F_- stays explicit), so this update is    */
/*                 local in real space;                                      */
/*   Edwards     : g = B / C + g_D(|k|^2).                                    */
/* Lengths are in units of R_g, so the Debye argument is |k|^2 R_g^2 = |k|^2. */
/* ------------------------------------------------------------------------ */

/* Debye function of a whole Gaussian chain, g_D(x) = 2 (e^-x + x - 1) / x^2.
 * Below x = 0.5 the direct form loses digits to cancellation; there the
 * series 2 sum_m (-x)^m / (m+2)!, m = 0..20, is used (truncation < 1e-25). */
double or_debye(double x)
{
    if (x < 0.5) {
        double term = 1.0, sum = 1.0; /* m = 0: 2 / 2! */
        for (int m = 1; m <= 20; m++) {
            term *= -x / (double)(m + 2);
            sum += term;
        }
        return sum;
    }
    return 2.0 * (exp(-x) + x - 1.0) / (x * x);
}

/* Cosine transform along one reflecting axis, in place, as the definitions
 * (the DCT-II / DCT-III pair of the walled diffusion above):
 *   forward  X_m = sum_n u_n cos(pi m (n+1/2)/N),
 *   inverse  u_n = X_0 / N + (2/N) sum_{m>=1} X_m cos(pi m (n+1/2)/N). */
static void dct_axis(const or_params *p, cplx *u, int axis, int inverse)
{
    const int n = (axis == 0) ? p->nx : (axis == 1) ? p->ny : p->nz;
    const ptrdiff_t stride = (axis == 0) ? (ptrdiff_t)p->ny * p->nz : (axis == 1) ? p->nz : 1;
    const int64_t nlines = grid_m(p) / n;
    const double pi = OR_TWO_PI / 2.0;
    #pragma omp parallel
    {
        cplx *in = (cplx *)malloc(sizeof(cplx) * n);
        #pragma omp for schedule(static)
        for (int64_t l = 0; l < nlines; l++) {
            ptrdiff_t base;
            if (axis == 2) base = l * p->nz;
            else if (axis == 1) base = (l / p->nz) * (ptrdiff_t)p->ny * p->nz + (l % p->nz);
            else base = l;
            for (int i = 0; i < n; i++) in[i] = u[base + i * stride];
            for (int o = 0; o < n; o++) {
                cplx acc = 0.0;
                if (!inverse) {
                    for (int i = 0; i < n; i++) acc += in[i] * cos(pi * o * (i + 0.5) / n);
                } else {
                    acc = in[0];
                    for (int m = 1; m < n; m++) acc += 2.0 * in[m] * cos(pi * m * (o + 0.5) / n);
                    acc /= (double)n;
                }
                u[base + o * stride] = acc;
            }
        }
        free(in);
    }
}

/* u <- u - T^-1[ T(r) / (1 + a g(k)) ] with g(k) = g0 + gD * g_D(|k|^2): T is
 * the 3-D DFT in a periodic box; with reflecting walls (Sec. III) it is the
 * cosine transform along the walled axes (k = pi m / L there, m = 0..N-1)
 * and the DFT along the others (k = 2 pi m / L).  Absorbing walls have no
 * diagonal linear response and are not handled here. */
static void sis_apply_walls(const or_params *p, cplx *u, const cplx *r, double a, double g0, double gD)
{
    const int64_t M = grid_m(p);
    const int32_t n[3] = {p->nx, p->ny, p->nz};
    const double L[3] = {p->lx, p->ly, p->lz};
    cplx *t = (cplx *)malloc(sizeof(cplx) * M);
    memcpy(t, r, sizeof(cplx) * M);
    for (int axis = 0; axis < 3; axis++) {
        if (p->bc[axis]) dct_axis(p, t, axis, 0);
        else fft_axis(t, p->nx, p->ny, p->nz, axis, -1);
    }
    for (int64_t jx = 0; jx < p->nx; jx++)
        for (int64_t jy = 0; jy < p->ny; jy++)
            for (int64_t jz = 0; jz < p->nz; jz++) {
                const int64_t j[3] = {jx, jy, jz};
                double k2 = 0.0;
                for (int axis = 0; axis < 3; axis++) {
                    const double k = p->bc[axis] ? (OR_TWO_PI / 2.0) * j[axis] / L[axis]
                                                 : OR_TWO_PI * or_mode((int32_t)j[axis], n[axis]) / L[axis];
                    k2 += k * k;
                }
                const int64_t x = (jx * p->ny + jy) * p->nz + jz;
                t[x] = t[x] / (1.0 + a * (g0 + gD * or_debye(k2)));
            }
    for (int axis = 0; axis < 3; axis++) {
        if (p->bc[axis]) {
            dct_axis(p, t, axis, 1);
        } else {
            fft_axis(t, p->nx, p->ny, p->nz, axis, +1);
            for (int64_t x = 0; x < M; x++) t[x] /= (double)n[axis];
        }
    }
    for (int64_t x = 0; x < M; x++) u[x] -= t[x];
    free(t);
}

/* u <- u - IDFT[ DFT(r) / (1 + a g(k)) ] with g(k) = g0 + gD * g_D(|k|^2). */
static void sis_apply(const or_params *p, cplx *u, const cplx *r, double a, double g0, double gD)
{
    if (p->bc[0] || p->bc[1] || p->bc[2]) {
        sis_apply_walls(p, u, r, a, g0, gD);
        return;
    }
    const int64_t M = grid_m(p);
    cplx *t = (cplx *)malloc(sizeof(cplx) * M);
    memcpy(t, r, sizeof(cplx) * M);
    dft3(p, t, -1);
    for (int64_t jx = 0; jx < p->nx; jx++)
        for (int64_t jy = 0; jy < p->ny; jy++)
            for (int64_t jz = 0; jz < p->nz; jz++) {
                const int64_t x = (jx * p->ny + jy) * p->nz + jz;
                const double g = g0 + gD * or_debye(ksq(p, jx, jy, jz));
                t[x] = t[x] / (1.0 + a * g);
            }
    dft3(p, t, +1);
    for (int64_t x = 0; x < M; x++) u[x] -= t[x] / (double)M;
    free(t);
}

/* Diblock: both fields at once from the forces of the current fields. */
void or_sis_update(const or_params *p, cplx *wp, cplx *wm, const cplx *phiA, const cplx *phiB,
                   double dt, double lam_p, double lam_m, int32_t noise,
                   uint64_t seed, uint64_t replica, uint64_t step)
{
    const int64_t M = grid_m(p);
    const double dV = p->lx * p->ly * p->lz / (double)M;
    cplx *Fp = (cplx *)malloc(sizeof(cplx) * M);
    cplx *Fm = (cplx *)malloc(sizeof(cplx) * M);
    double *xp = (double *)calloc(M, sizeof(double));
    double *xm = (double *)calloc(M, sizeof(double));
    or_forces(p, wm, phiA, phiB, Fp, Fm);
    if (noise) {
        or_gaussian(seed, replica, step, 0, M, xp);
        or_gaussian(seed, replica, step, 1, M, xm);
    }
    const double sp = noise ? sqrt(2.0 * lam_p * dt / (p->C * dV)) : 0.0;
    const double sm = noise ? sqrt(2.0 * lam_m * dt / (p->C * dV)) : 0.0;
    /* r = lam dt F - s xi, the explicit increment with its sign flipped */
    for (int64_t x = 0; x < M; x++) Fp[x] = lam_p * dt * Fp[x] - sp * xp[x];
    sis_apply(p, wp, Fp, lam_p * dt, 0.0, 1.0);
    const double den = 1.0 + lam_m * dt * 2.0 / p->chiN;
    for (int64_t x = 0; x < M; x++) wm[x] -= (lam_m * dt * Fm[x] - sm * xm[x]) / den;
    free(Fp); free(Fm); free(xp); free(xm);
}

/* ------------------------------------------------------------------------ */
/* Edwards model of homopolymers in an implicit solvent, Eq. (2):           */
/*   H[omega] = (B/2) int dx omega^2 - C V ln Q[i omega].                     */
/* One chain species feels w = i omega along the whole contour; the chain is */
/* symmetric, so the conjugate propagator is q itself (qd_i = q_i) and the   */
/* density pairs node j with node K - j of the same sweep.  The contour is   */
/* K = ns equal steps (no junction).  p->f and p->chiN are not used.          */
/* ------------------------------------------------------------------------ */

/* q_0 = 1, q_{j+1} = T_ds(q_j; i omega) (Eq. (5) with w = i omega); qs holds
 * (ns+1)*M values.  Returns K = ns. */
int or_edwards_propagate(const or_params *p, const cplx *omega, cplx *qs)
{
    const int64_t M = grid_m(p);
    const double ds = 1.0 / p->ns;
    cplx *w = (cplx *)malloc(sizeof(cplx) * M);
    cplx *work = (cplx *)malloc(sizeof(cplx) * 2 * M);
    for (int64_t x = 0; x < M; x++) w[x] = I * omega[x];
    for (int64_t x = 0; x < M; x++) qs[x] = 1.0;
    for (int j = 0; j < p->ns; j++)
        or_step(p, p->scheme, ds, w, qs + (int64_t)j * M, qs + (int64_t)(j + 1) * M, work);
    free(w); free(work);
    return p->ns;
}

/* Q = (1/M) sum_x q_K(x) (Eq. (4)) and phi = (1/Q) sum_j tau_j q_j q_{K-j}
 * with the composite trapezoid weights on [0, 1] (tau_0 = tau_K = ds/2,
 * ds elsewhere), the one-species form of Eq. (8) divided by rho_0. */
void or_edwards_densities(const or_params *p, const cplx *qs, cplx *phi, cplx *Q)
{
    const int64_t M = grid_m(p);
    const int K = p->ns;
    const double ds = 1.0 / K;
    cplx sum = 0.0;
    for (int64_t x = 0; x < M; x++) sum += qs[(int64_t)K * M + x];
    *Q = sum / (double)M;
    #pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < M; x++) {
        cplx a = 0.0;
        for (int j = 0; j <= K; j++) {
            const double tau = (j == 0 || j == K) ? 0.5 * ds : ds;
            a += tau * qs[(int64_t)j * M + x] * qs[(int64_t)(K - j) * M + x];
        }
        phi[x] = a / *Q;
    }
}

/* H = (B/2) dV sum_x omega^2 - C V log Q (Eq. (2) on the grid, principal
 * branch); hint = H / (C V). */
void or_edwards_hamiltonian(const or_params *p, double B, const cplx *omega, double Qre, double Qim,
                            cplx *H, cplx *hint)
{
    const cplx Q = Qre + Qim * I;
    const int64_t M = grid_m(p);
    const double V = p->lx * p->ly * p->lz;
    const double dV = V / (double)M;
    cplx s = 0.0;
    for (int64_t x = 0; x < M; x++) s += omega[x] * omega[x];
    *H = 0.5 * B * dV * s - p->C * V * clog(Q);
    *hint = *H / (p->C * V);
}

/* Force per unit C dV: dH/domega(x) = dV [B omega(x) + i C phi(x)], since
 * d(-C V ln Q)/dw(x) = C dV phi(x) and dw/domega = i.  So
 *   F = (B / C) omega + i phi. */
void or_edwards_force(const or_params *p, double B, const cplx *omega, const cplx *phi, cplx *F)
{
    const int64_t M = grid_m(p);
    for (int64_t x = 0; x < M; x++) F[x] = (B / p->C) * omega[x] + I * phi[x];
}

/* Euler-Maruyama step of Eq. (9) for omega (field 0 of the noise stream):
 * omega <- omega - lam dt F + s xi, s^2 = 2 lam dt / (C dV). */
void or_edwards_em_update(const or_params *p, double B, cplx *omega, const cplx *phi, double dt, double lam,
                          int32_t noise, uint64_t seed, uint64_t replica, uint64_t step)
{
    const int64_t M = grid_m(p);
    const double dV = p->lx * p->ly * p->lz / (double)M;
    cplx *F = (cplx *)malloc(sizeof(cplx) * M);
    double *xi = (double *)calloc(M, sizeof(double));
    or_edwards_force(p, B, omega, phi, F);
    if (noise) or_gaussian(seed, replica, step, 0, M, xi);
    const double sg = noise ? sqrt(2.0 * lam * dt / (p->C * dV)) : 0.0;
    for (int64_t x = 0; x < M; x++) omega[x] = omega[x] - lam * dt * F[x] + sg * xi[x];
    free(F); free(xi);
}

/* Semi-implicit step for omega with g = B/C + g_D(|k|^2) (see or_sis_update). */
void or_edwards_sis_update(const or_params *p, double B, cplx *omega, const cplx *phi, double dt, double lam,
                           int32_t noise, uint64_t seed, uint64_t replica, uint64_t step)
{
    const int64_t M = grid_m(p);
    const double dV = p->lx * p->ly * p->lz / (double)M;
    cplx *F = (cplx *)malloc(sizeof(cplx) * M);
    double *xi = (double *)calloc(M, sizeof(double));
    or_edwards_force(p, B, omega, phi, F);
    if (noise) or_gaussian(seed, replica, step, 0, M, xi);
    const double sg = noise ? sqrt(2.0 * lam * dt / (p->C * dV)) : 0.0;
    for (int64_t x = 0; x < M; x++) F[x] = lam * dt * F[x] - sg * xi[x];
    sis_apply(p, omega, F, lam * dt, B / p->C, 1.0);
    free(F); free(xi);
}

/* One evaluation: q, Q, phi, H.  Returns K (-1 if out of memory). */
int or_edwards_evaluate(const or_params *p, double B, const cplx *omega, cplx *phi, cplx *Q, cplx *H, cplx *hint)
{
    const int64_t M = grid_m(p);
    cplx *qs = (cplx *)malloc(sizeof(cplx) * (int64_t)(p->ns + 1) * M);
    if (!qs) return -1;
    const int K = or_edwards_propagate(p, omega, qs);
    or_edwards_densities(p, qs, phi, Q);
    or_edwards_hamiltonian(p, B, omega, creal(*Q), cimag(*Q), H, hint);
    free(qs);
    return K;
}

/* ------------------------------------------------------------------------ */
/* Reverse-mode derivatives of H (Eq. (3)) through the discrete split steps. */
/*                                                                           */
/* Q = (1/M) 1^T q_K with q_{j+1} = T_j q_j.  Every step operator is complex- */
/* symmetric (E diagonal, D symmetric because its multiplier is even in k),  */
/* so the adjoint vector of step j is lambda_{j+1} = qd_{K-j-1}, the stored  */
/* conjugate propagator, and                                                 */
/*   dQ/dw_b(x) = (1/M) sum_{j in block b} lambda_{j+1}^T (dT_j/dw(x)) q_j.   */
/* Each factor E_a = exp(-w a) contributes -a times the product of what      */
/* stands to its left (transposed, acting on lambda) and to its right (acting */
/* on q) at site x.  The box derivative replaces the axis factor of D_h by   */
/* d/dL_a exp(-(2 pi m / L_a)^2 h) = exp(...) * 2 k_a^2 h / L_a.              */
/* ------------------------------------------------------------------------ */

/* u^T (dD_h/dL_a) v = (1/M) sum_k (2 k_a^2 h / L_a) e^{-|k|^2 h} U(-k) V(k),  */
/* with U, V the unnormalised DFTs of u and v.                               */
static cplx dbilinear(const or_params *p, double h, int axis, const cplx *u, const cplx *v)
{
    const int64_t M = grid_m(p);
    cplx *U = (cplx *)malloc(sizeof(cplx) * M), *Vv = (cplx *)malloc(sizeof(cplx) * M);
    memcpy(U, u, sizeof(cplx) * M);
    memcpy(Vv, v, sizeof(cplx) * M);
    dft3(p, U, -1);
    dft3(p, Vv, -1);
    const int n[3] = {p->nx, p->ny, p->nz};
    const double L[3] = {p->lx, p->ly, p->lz};
    cplx acc = 0.0;
    for (int64_t jx = 0; jx < n[0]; jx++)
        for (int64_t jy = 0; jy < n[1]; jy++)
            for (int64_t jz = 0; jz < n[2]; jz++) {
                const int64_t j[3] = {jx, jy, jz};
                const double ka = OR_TWO_PI * or_mode((int32_t)j[axis], n[axis]) / L[axis];
                const double d = 2.0 * ka * ka * h / L[axis] * exp(-ksq(p, jx, jy, jz) * h);
                const int64_t mx = (n[0] - jx) % n[0], my = (n[1] - jy) % n[1], mz = (n[2] - jz) % n[2];
                acc += d * U[(mx * n[1] + my) * n[2] + mz] * Vv[(jx * n[1] + jy) * n[2] + jz];
            }
    free(U);
    free(Vv);
    return acc / (double)M;
}

/* The same with walls on some axes.  On a walled axis the modes are
 * k = pi m / L_a (sine or cosine), so again dk^2/dL_a = -2 k^2 / L_a and
 *   dD_h/dL_a = (2 h / L_a) (-d^2/dx_a^2) D_h,
 * the axis Laplacian taken in that axis's own mode basis (1-D DFT on a
 * periodic axis, cosine / sine modes on a walled one):
 *   u^T (dD_h/dL_a) v = (2 h / L_a) sum_x u(x) [(-d^2/dx_a^2) D_h v](x). */
static cplx dbilinear_walls(const or_params *p, double h, int axis, const cplx *u, const cplx *v)
{
    const int64_t M = grid_m(p);
    const int n = (axis == 0) ? p->nx : (axis == 1) ? p->ny : p->nz;
    const double L = (axis == 0) ? p->lx : (axis == 1) ? p->ly : p->lz;
    cplx *t = (cplx *)malloc(sizeof(cplx) * M);
    memcpy(t, v, sizeof(cplx) * M);
    or_diffuse(p, h, t);
    if (p->bc[axis]) {
        walls_axis_modes(p, 0.0, t, axis, 1);
    } else {
        fft_axis(t, p->nx, p->ny, p->nz, axis, -1);
        for (int64_t x = 0; x < M; x++) {
            const int64_t j = (axis == 0) ? x / ((int64_t)p->ny * p->nz) : (axis == 1) ? (x / p->nz) % p->ny : x % p->nz;
            const double k = OR_TWO_PI * or_mode((int32_t)j, n) / L;
            t[x] *= k * k / (double)n;
        }
        fft_axis(t, p->nx, p->ny, p->nz, axis, +1);
    }
    cplx acc = 0.0;
    for (int64_t x = 0; x < M; x++) acc += u[x] * t[x];
    free(t);
    return 2.0 * h / L * acc;
}

static cplx dbil(const or_params *p, double h, int axis, const cplx *u, const cplx *v)
{
    if (p->bc[0] || p->bc[1] || p->bc[2]) return dbilinear_walls(p, h, axis, u, v);
    return dbilinear(p, h, axis, u, v);
}

static void copy_mul(cplx *dst, const cplx *src, const cplx *w, double a, int64_t M)
{
    for (int64_t x = 0; x < M; x++) dst[x] = src[x] * cexp(-w[x] * a);
}

/*
 * dH/dw_+(x), dH/dw_-(x) (holomorphic derivatives, per site, not per unit
 * volume) and dH/dL_a for a = x, y, z (each edge varied alone, the grid and
 * the fields' values on it held fixed).  Returns K.
 */
int or_adjoint(const or_params *p, const cplx *wp, const cplx *wm, cplx *dHdwp, cplx *dHdwm, cplx *dHdL)
{
    const int64_t M = grid_m(p);
    double *h = (double *)malloc(sizeof(double) * (p->ns + 2));
    int32_t *blk = (int32_t *)malloc(sizeof(int32_t) * (p->ns + 2));
    int32_t J;
    const int K = or_contour(p->ns, p->f, h, blk, &J);
    cplx *qs = (cplx *)malloc(sizeof(cplx) * (K + 1) * M);
    cplx *qds = (cplx *)malloc(sizeof(cplx) * (K + 1) * M);
    cplx *wA = (cplx *)malloc(sizeof(cplx) * M), *wB = (cplx *)malloc(sizeof(cplx) * M);
    cplx *G[2] = {(cplx *)calloc(M, sizeof(cplx)), (cplx *)calloc(M, sizeof(cplx))};
    cplx *t[12];
    for (int i = 0; i < 12; i++) t[i] = (cplx *)malloc(sizeof(cplx) * M);
    or_block_fields(p, wp, wm, wA, wB);
    or_propagate(p, wp, wm, qs, qds);
    cplx Q = 0.0;
    for (int64_t x = 0; x < M; x++) Q += qs[(int64_t)K * M + x];
    Q /= (double)M;
    cplx dQdL[3] = {0.0, 0.0, 0.0};

    for (int j = 0; j < K; j++) {
        const double hj = h[j];
        const cplx *w = blk[j] == 0 ? wA : wB;
        const cplx *q = qs + (int64_t)j * M;
        const cplx *lam = qds + (int64_t)(K - j - 1) * M;   /* lambda_{j+1} */
        cplx *g = G[blk[j]];
        /* full path: F = E_{h/2} D_h E_{h/2} applied to q and to lambda */
        cplx *e2q = t[0], *e2l = t[1], *Fq = t[2], *Fl = t[3];
        copy_mul(e2q, q, w, hj / 2, M);
        copy_mul(e2l, lam, w, hj / 2, M);
        memcpy(Fq, e2q, sizeof(cplx) * M); or_diffuse(p, hj, Fq); copy_mul(Fq, Fq, w, hj / 2, M);
        memcpy(Fl, e2l, sizeof(cplx) * M); or_diffuse(p, hj, Fl); copy_mul(Fl, Fl, w, hj / 2, M);
        if (p->scheme == OR_SPLIT2) {
            for (int64_t x = 0; x < M; x++)
                g[x] += -(hj / 2) * lam[x] * Fq[x] - (hj / 2) * Fl[x] * q[x];
            for (int a = 0; a < 3; a++) dQdL[a] += dbil(p, hj, a, e2l, e2q);
            continue;
        }
        /* half path: A = D_{h/2} E_{h/4} (.), H = E_{h/4} D_{h/2} E_{h/2} A */
        cplx *e4q = t[4], *e4l = t[5], *Aq = t[6], *Al = t[7], *Hq = t[8], *Hl = t[9];
        copy_mul(e4q, q, w, hj / 4, M);
        copy_mul(e4l, lam, w, hj / 4, M);
        memcpy(Aq, e4q, sizeof(cplx) * M); or_diffuse(p, hj / 2, Aq);
        memcpy(Al, e4l, sizeof(cplx) * M); or_diffuse(p, hj / 2, Al);
        cplx *e2Aq = t[10], *e2Al = t[11];
        copy_mul(e2Aq, Aq, w, hj / 2, M);
        copy_mul(e2Al, Al, w, hj / 2, M);
        memcpy(Hq, e2Aq, sizeof(cplx) * M); or_diffuse(p, hj / 2, Hq); copy_mul(Hq, Hq, w, hj / 4, M);
        memcpy(Hl, e2Al, sizeof(cplx) * M); or_diffuse(p, hj / 2, Hl); copy_mul(Hl, Hl, w, hj / 4, M);
        for (int64_t x = 0; x < M; x++) {
            const cplx E2 = cexp(-w[x] * (hj / 2));
            const cplx half = -(hj / 4) * lam[x] * Hq[x] - (hj / 2) * Al[x] * E2 * Aq[x] - (hj / 4) * Hl[x] * q[x];
            const cplx full = -(hj / 2) * lam[x] * Fq[x] - (hj / 2) * Fl[x] * q[x];
            g[x] += (4.0 / 3.0) * half - (1.0 / 3.0) * full;
        }
        for (int a = 0; a < 3; a++)
            dQdL[a] += (4.0 / 3.0) * (dbil(p, hj / 2, a, e4l, e2Aq) + dbil(p, hj / 2, a, e2Al, e4q))
                       - (1.0 / 3.0) * dbil(p, hj, a, e2l, e2q);
    }
    const double V = p->lx * p->ly * p->lz, dV = V / (double)M;
    cplx S = 0.0;
    for (int64_t x = 0; x < M; x++) {
        /* dQ/dw_+ = i (dQ/dw_A + dQ/dw_B), dQ/dw_- = dQ/dw_B - dQ/dw_A, dQ/dw_b = G_b / M */
        const cplx dQp = I * (G[0][x] + G[1][x]) / (double)M;
        const cplx dQm = (G[1][x] - G[0][x]) / (double)M;
        dHdwp[x] = -I * p->C * dV - p->C * V * dQp / Q;
        dHdwm[x] = 2.0 * p->C * dV * wm[x] / p->chiN - p->C * V * dQm / Q;
        S += wm[x] * wm[x] / p->chiN - I * wp[x];
    }
    const double L[3] = {p->lx, p->ly, p->lz};
    for (int a = 0; a < 3; a++)
        dHdL[a] = p->C * S * dV / L[a] - p->C * (V / L[a]) * clog(Q) - p->C * V * (dQdL[a] / (double)M) / Q;
    for (int i = 0; i < 12; i++) free(t[i]);
    free(G[0]); free(G[1]); free(wA); free(wB); free(qs); free(qds); free(h); free(blk);
    return K;
}
