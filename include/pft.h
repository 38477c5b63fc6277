/*
 * pft.h -- C ABI of the MI355X (gfx950) propagator library for polymer
 * field theory: the pseudo-spectral operator-split solution of the modified
 * diffusion equation for the chain propagators q and q-dagger of an
 * incompressible AB diblock melt in a periodic box, the contour-integrated
 * segment densities, the single-chain partition function Q, the Hamiltonian,
 * and one explicit field (SCFT / complex-Langevin) step.
 *
 * Paper: K. T. Delaney and G. H. Fredrickson, "Polymer Field-Theory
 * Simulations on Graphics Processing Units", arXiv:1204.5434.
 *
 * Conventions that hold for every entry point:
 *  - Fields, densities and debug arrays are HIP DEVICE memory owned by the
 *    caller: complex128, interleaved (re, im) doubles, C order [nx][ny][nz]
 *    (z fastest), 16-byte aligned.  Scalar results (Q, H, ...) are written to
 *    caller-owned DEVICE memory as complex128 (two doubles), so no call needs
 *    a host synchronisation.
 *  - The context owns every internal buffer (propagator slice stores, field
 *    operator tables, diffusion factors, work arrays, reduction scratch).
 *  - Work is enqueued asynchronously on the HIP stream given to pft_create.
 *    Device pointers passed in must stay valid until that work completes.
 *  - No call throws or aborts.  Each returns a pft_status; on failure
 *    pft_last_error(ctx) holds a message (owned by the context).  Invalid
 *    arguments are rejected before anything is enqueued.
 *  - Propagator precision: PFT_C128 runs the propagators and FFTs in complex
 *    double; PFT_C64 in complex float.  Field operator tables, twiddles and
 *    diffusion factors are computed in double and rounded once.  Q, log Q,
 *    the contour sums, H and the field update are always double precision
 *    with compensated (Neumaier) summation.
 */
#ifndef PFT_H
#define PFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pft_ctx pft_ctx;

typedef enum {
    PFT_OK = 0,
    PFT_E_INVALID = 1,     /* bad argument (null/misaligned pointer, bad parameter) */
    PFT_E_UNSUPPORTED = 2, /* grid size without a kernel, or an unsupported mode      */
    PFT_E_NOMEM = 3,       /* device allocation failed; nothing is leaked             */
    PFT_E_DEVICE = 4,      /* a HIP runtime call failed (the message names it)        */
    PFT_E_NONFINITE = 5,   /* a non-finite Q was produced (reported by status_flags)  */
    PFT_E_STATE = 6        /* call order violated, e.g. densities before propagate     */
} pft_status;

typedef enum { PFT_C128 = 0, PFT_C64 = 1 } pft_precision;

/* PFT_RQM4: the Richardson-extrapolated split step of Eq. (12) (Sec. III),
 *   T_h = (4/3) E_{h/4} D_{h/2} E_{h/2} D_{h/2} E_{h/4} - (1/3) E_{h/2} D_h E_{h/2},
 * globally fourth order in the contour step.  PFT_SPLIT2: the plain
 * second-order split step E_{h/2} D_h E_{h/2}.  E_a = exp(-w a), D_h =
 * exp(h Laplacian) applied in Fourier space. */
typedef enum { PFT_RQM4 = 0, PFT_SPLIT2 = 1 } pft_scheme;

/* Model and discretisation.  Lengths in units of R_g; the contour is
 * normalised to [0, 1] and cut into ns steps (Sec. II, Eqs. (3)-(5)). */
typedef struct {
    int32_t nx, ny, nz; /* grid points per axis; each must be one of
                           8 12 16 20 24 32 40 48 64 80 96 128 192 256        */
    double lx, ly, lz;  /* periodic box edges, > 0                            */
    int32_t ns;         /* contour steps, >= 2                                */
    double f;           /* A-block fraction, 0 < f < 1 (Eq. (8))              */
    double chiN;        /* Flory parameter times N, > 0 (Eq. (3))             */
    double C;           /* chain number density parameter, > 0 (Eq. (3))      */
    int32_t precision;  /* pft_precision                                      */
    int32_t scheme;     /* pft_scheme                                         */
    int32_t model;      /* pft_model (0 = the AB diblock melt of Eq. (3))     */
    double B;           /* Edwards model: excluded-volume parameter, > 0       */
    int32_t storage;    /* pft_storage (0 = both propagators in device memory) */
    int32_t bc[3];      /* per axis x, y, z: pft_boundary (0 = periodic)       */
} pft_params;

/* Boundary conditions of Eq. (5) per axis (Sec. III: Fourier, cosine and sine
 * transforms for periodic, Neumann and Dirichlet boundaries).  Walls sit half a
 * cell outside the grid points x_n = (n + 1/2) L / N.  PFT_REFLECTING: zero
 * normal derivative (cosine modes, decay exp(-(pi m / L)^2 h), m = 0..N-1);
 * PFT_ABSORBING: q = 0 on the walls (sine modes, m = 1..N).  A walled line of
 * N points is diffused with one N-point transform of its even/odd-reordered
 * points and a pairing of frequencies m and N - m, for every N of the axis
 * list (else PFT_E_UNSUPPORTED).  Walled contexts run the axis
 * schedule on walled y or z axes; the semi-implicit step takes reflecting
 * walls (modes of the cosine basis) when 2N is in the axis list, not
 * absorbing ones; pft_adjoint gives dH/dw and dH/dL with walls (walled
 * modes k = pi m / L); batches take walls (their semi-implicit step as the
 * single one); pft_debug_kgrid accepts periodic boxes only
 * (PFT_E_UNSUPPORTED). */
typedef enum { PFT_PERIODIC = 0, PFT_REFLECTING = 1, PFT_ABSORBING = 2 } pft_boundary;

/* Where the propagators live (diblock model).
 * PFT_STORE_BOTH: q and q-dagger, (K+1) slices each, in device memory (needed
 *   by pft_node_q, pft_get_slice of q-dagger, pft_adjoint; the default).
 * PFT_STORE_Q: q only in device memory; the conjugate sweep runs after the
 *   forward one and accumulates tau_j q_j q-dagger_{K-j} into FP64 density
 *   accumulators as it goes (the stored-product scheme of Sec. IV.C), halving
 *   the slice memory.
 * PFT_STORE_HOST: q is staged into pinned host memory during the forward sweep
 *   (device-to-host copies on a second stream overlapping the passes) and
 *   fetched back ahead of use during the conjugate sweep (Sec. V's host-memory
 *   option): device memory is O(M), the host holds (K+1) slices.
 * With PFT_STORE_Q / PFT_STORE_HOST, pft_node_q, pft_get_slice(which = 1) and
 * pft_adjoint return PFT_E_UNSUPPORTED, and the sweeps run one after the other. */
typedef enum { PFT_STORE_BOTH = 0, PFT_STORE_Q = 1, PFT_STORE_HOST = 2 } pft_storage;

/* Models.  PFT_DIBLOCK: the incompressible AB diblock melt, Eq. (3), fields
 * (w_+, w_-).  PFT_EDWARDS: homopolymers in implicit solvent, Eq. (2),
 *   H[omega] = (B/2) int dx omega^2 - C V ln Q[i omega],
 * one field omega passed as w_plus (w_minus is ignored and may be NULL); f and
 * chiN are ignored.  The chain is symmetric, so q-dagger = q: pft_propagate
 * runs the forward sweep only (half the diblock work) over K = ns equal steps,
 * pft_densities writes phi to phi_a and zeros to phi_b, and pft_cl_step uses
 * the force per unit C dV  F = (B/C) omega + i phi  (omega <- omega -
 * lambda_plus dt F + s xi, noise field 0).  pft_adjoint and batches accept the
 * diblock model only (PFT_E_UNSUPPORTED). */
typedef enum { PFT_DIBLOCK = 0, PFT_EDWARDS = 1 } pft_model;

/* One explicit Euler-Maruyama step of the field equation of motion, Eq. (9):
 *   w_+ <- w_+ - lambda_+ dt F_+ + s_+ xi_+,  w_- <- w_- - lambda_- dt F_- + s_- xi_-,
 * F_+ = i (phi_A + phi_B - 1), F_- = 2 w_- / chiN + phi_B - phi_A, s^2 =
 * 2 lambda dt / (C dV) (the discrete noise variance stated after Eq. (10)),
 * xi real standard normals from Philox4x64-10 keyed by (seed, replica) with
 * counter (site / 4, field, step, 0).  noise = 0 gives SCFT relaxation. */
typedef struct {
    double dt, lambda_plus, lambda_minus;
    uint64_t seed, replica, step;
    int32_t noise;
    int32_t update;  /* 0: the explicit step above; 1: first-order semi-implicit,
                        Eqs. (10)-(11): every Fourier mode of the increment
                        lambda dt F - s xi is divided by 1 + lambda dt g(k), with
                        g = g_D(|k|^2) (Debye function of the whole chain,
                        lengths in R_g) for w_+, g = 2/chiN for w_- (its
                        explicitly linear term; local in real space), and
                        g = B/C + g_D(|k|^2) for the Edwards field; between
                        reflecting walls the modes of a walled axis are the
                        cosine modes, k = pi m / L (the filter runs on the
                        even image of period 2L).  Batches accept both. */
} pft_step;

/* Create a context for one parameter set on the current HIP device.
 * hip_stream: a hipStream_t (NULL = the default stream).  Allocates the two
 * propagator slice stores ((K+1) * M values each, K = ns or ns+1) and all
 * tables.  Errors: PFT_E_INVALID (bad parameter; *out = NULL),
 * PFT_E_UNSUPPORTED (axis length without a kernel), PFT_E_NOMEM, PFT_E_DEVICE.
 * On failure *out is NULL and nothing stays allocated. */
pft_status pft_create(const pft_params* params, void* hip_stream, pft_ctx** out);

/* The q and q-dagger sweeps are independent; by default the q-dagger sweep of
 * pft_propagate runs on a second (default-priority) stream with its own work
 * arrays, forked from and joined back to the context stream, so the memory
 * phases of one overlap the on-chip transform phases of the other (and
 * pft_adjoint recomputes its next segment there).  on = 0 runs everything on
 * the context stream.  Errors: PFT_E_INVALID. */
pft_status pft_set_concurrent_sweeps(pft_ctx* ctx, int32_t on);

/* Schedule of the sweeps (Eq. (12) either way; results agree to rounding).
 * The axis schedule runs a step as four memory passes (z, y, x, y).  When
 * ny == nz and one yz-plane fits in the 160 KB LDS of a compute unit (complex
 * float: up to 128 x 128; complex double: up to 96 x 96) the y, z, y passes
 * between two x passes fuse into one pass per x-plane, and a step moves 11
 * instead of 17 arrays.  New contexts use the fused schedule where it exists
 * and its compiled kernel spills at most 256 bytes per lane (on gfx950 every
 * such plane except complex double 96 x 96, measured slower than the axis
 * schedule); pft_set_fused_planes overrides the choice.
 * The schedule applies to pft_propagate, pft_cl_step and pft_apply_step, and
 * batches use the fused one for every replica group whose shape has it; the
 * reverse mode (pft_adjoint) always uses the axis schedule.
 * on = 2 fuses only the conjugate (q-dagger) sweep of pft_propagate, whose
 * on-chip-bound plane passes then share the device with the forward sweep's
 * memory-bound axis passes when the two sweeps run concurrently.
 * on = 1 or 2 without a fused kernel for the shape: PFT_E_UNSUPPORTED
 * (schedule unchanged); other values: PFT_E_INVALID.  pft_fused_planes returns
 * the current setting (0, 1, 2), -1 for NULL. */
pft_status pft_set_fused_planes(pft_ctx* ctx, int32_t on);
int32_t pft_fused_planes(const pft_ctx* ctx);

/* Release everything the context owns (synchronises its stream). NULL is a no-op. */
void pft_destroy(pft_ctx* ctx);

/* Last error message of the context ("" if none); valid until the next call. */
const char* pft_last_error(const pft_ctx* ctx);

/* Static name of a status code. */
const char* pft_status_string(pft_status status);

/* Host-only contour plan (no GPU needed).  Reading of Eq. (8): ns steps of
 * 1/ns; when f*ns is not an integer the step straddling s = f is split into
 * an A sub-step f - n*ds and a B sub-step (n+1)*ds - f.  Writes the step
 * lengths h[K] and blocks blk[K] (0 = A, 1 = B; arrays of ns+1 entries) and
 * the junction node index *junction (s_J = f).  Returns K, or -1 on invalid
 * arguments. */
int32_t pft_contour_plan(int32_t ns, double f, double* h, int32_t* blk, int32_t* junction);

/* Number of contour steps K of the context (ns or ns+1). */
int32_t pft_num_steps(const pft_ctx* ctx);

/* Solve the modified diffusion equation, Eq. (5), for q (from q = 1 at s = 0)
 * and q-dagger (from 1 at s = 1) in the fields w_A = i w_+ - w_-,
 * w_B = i w_+ + w_- (Sec. II), storing every contour node, and reduce
 * Q = (1/M) sum_x q(x, 1) (Eq. (4)).  w_plus, w_minus: [nx][ny][nz]
 * complex128, read during the call's GPU work only.  Errors: PFT_E_INVALID. */
pft_status pft_propagate(pft_ctx* ctx, const double* w_plus, const double* w_minus);

/* Segment densities of Eq. (8) divided by rho_0, from the stored
 * propagators of the last pft_propagate: phi_A = (1/Q) sum_j tauA_j q_j qd_{K-j}
 * (trapezoid weights per block, compensated FP64 sums), phi_B likewise.
 * phi_a, phi_b: [nx][ny][nz] complex128 out.  Q: 2 doubles out (may be NULL).
 * Errors: PFT_E_INVALID, PFT_E_STATE (no propagate yet). */
pft_status pft_densities(pft_ctx* ctx, double* phi_a, double* phi_b, double* Q);

/* pft_propagate followed by pft_densities on these buffers, replayed from a
 * HIP graph: the first call (and any call with other buffers) captures one
 * evaluation, both sweeps' streams included, into a graph the context owns;
 * every call then enqueues nreps replays (0: capture only) after the work
 * already on the context stream, and later work on that stream waits for them.
 * The graph reads w_plus / w_minus and writes phi_a / phi_b / Q at the
 * addresses it was captured with, so their contents may change between
 * calls.  Replays of one context run one after another; the state afterwards
 * is that of a plain pft_propagate + pft_densities.  Arguments and layouts as
 * for those two calls.  Errors: PFT_E_INVALID; PFT_E_UNSUPPORTED unless both
 * stores are in device memory (storage 0); PFT_E_STATE while profiling;
 * PFT_E_DEVICE if capture or instantiation fails. */
pft_status pft_evaluate_graph(pft_ctx* ctx, const double* w_plus, const double* w_minus, double* phi_a, double* phi_b,
                              double* Q, int32_t nreps);

/* Change the box edges (lengths in R_g, each finite and > 0) of an existing
 * context, keeping its grid, contour and buffers: the diffusion factors of
 * Eq. (5) (k = 2 pi m / L, or pi m / L along a walled axis), the spectral
 * second derivatives of the box derivative and, once built, the |k|^2 tables
 * of the semi-implicit step are recomputed, and V, dV follow the new edges.
 * This is the move a variable-cell calculation makes along dH/dL (the box
 * derivative that pft_adjoint returns).  Blocks until the context's queued work
 * has finished (that work reads the tables rewritten here); a pft_propagate
 * is needed before pft_densities / pft_hamiltonian see the new box.
 * Errors: PFT_E_INVALID, PFT_E_DEVICE. */
pft_status pft_set_box(pft_ctx* ctx, double lx, double ly, double lz);

/* Hamiltonian of Eq. (3) on the grid, H = C dV sum_x [w_-^2/chiN - i w_+]
 * - C V Log Q (principal branch), with Q from the last pft_propagate (which
 * must have used these fields).  H, h_intensive (= H / (C V)): 2 doubles out
 * each (h_intensive may be NULL).  Errors: PFT_E_INVALID, PFT_E_STATE. */
pft_status pft_hamiltonian(pft_ctx* ctx, const double* w_plus, const double* w_minus, double* H,
                           double* h_intensive);

/* One field step: propagate, densities, H (all of the INPUT fields), then the
 * update of pft_step in place on w_plus, w_minus.  phi_a, phi_b, Q, H may be
 * NULL (internal buffers are used).  Errors: PFT_E_INVALID. */
pft_status pft_cl_step(pft_ctx* ctx, double* w_plus, double* w_minus, const pft_step* step,
                       double* phi_a, double* phi_b, double* Q, double* H);

/* Reverse-mode derivatives of H (Eq. (3)) through the K discrete split steps
 * of the context's scheme, with q checkpointed every ckpt_every nodes
 * (0: ceil(sqrt(K))) and each segment recomputed once: memory ~(9 sqrt(K) + 6)
 * extra fields instead of K (~(5 sqrt(K) + 6) with concurrent sweeps off).  The
 * adjoint vector of step j is the conjugate propagator (every split step is
 * complex-symmetric), so this is one checkpointed forward sweep, one segment
 * recompute (on the second stream, one segment ahead, while concurrent sweeps
 * are on) and one q-dagger sweep with per-step accumulation in FP64 (Neumaier).
 * The box derivatives take one stress pass per axis and step.
 * Outputs (device): dH_dwplus, dH_dwminus -- [nx][ny][nz] complex128, the
 * holomorphic derivative dH/dw at each grid point (not per unit volume);
 * dH_dL -- 3 complex128 (may be NULL): dH/dL_x, dH/dL_y, dH/dL_z with each box
 * edge varied alone and the field values on the grid held fixed (the diagonal
 * box stress times the volume over the edge); H -- complex128 (may be NULL),
 * the Hamiltonian of these fields.  With walls both hold: the walled
 * diffusion is symmetric too, and a walled axis's modes k = pi m / L scale
 * with 1/L as the periodic ones do, so its stress pass applies -d^2/dx^2 in
 * the cosine / sine basis (the edge varied between fixed walls, the
 * cell-centred grid scaling with it).  Overwrites the context's field tables and
 * Q, so pft_densities / pft_hamiltonian need a new pft_propagate afterwards.
 * Errors: PFT_E_INVALID, PFT_E_NOMEM, PFT_E_DEVICE. */
pft_status pft_adjoint(pft_ctx* ctx, const double* w_plus, const double* w_minus, int32_t ckpt_every,
                       double* dH_dwplus, double* dH_dwminus, double* dH_dL, double* H);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * field step as pft_cl_step (same arguments, same kernels, same results), but
 * the semi-implicit step (step->update = 1) takes its work memory -- the
 * increment (M complex doubles), between reflecting walls the even image and
 * its update (2 Me complex doubles, Me the image's sites) and the |k|^2 rows
 * (3 x the longest image axis doubles), each block 256-byte aligned -- from a
 * device array of PFT_STATIC_SCRATCH_BYTES inside the library instead of
 * buffers the context allocates on first use, and fills the |k|^2 rows with a
 * kernel instead of a host copy.  The call allocates and frees nothing (no
 * hipMalloc, hipFree or allocating library routine).  Each GPU that the
 * library runs on holds one copy of the array until the process ends; its
 * address is looked up once per device (hipGetSymbolAddress), so the
 * context's device must be current (else PFT_E_INVALID).  Limit: a step whose
 * work memory exceeds the array is refused with PFT_E_UNSUPPORTED before
 * anything is enqueued (periodic boxes up to 2,097,152 sites, e.g. 128^3).
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind: calls on one stream, in order, are safe; calls that overlap in
 * time on one GPU (other streams or other contexts without ordering between
 * them) race on the array and give wrong fields.  The explicit step
 * (update = 0) uses no work memory and equals pft_cl_step.  Errors: those of
 * pft_cl_step, PFT_E_UNSUPPORTED, PFT_E_DEVICE. */
#define PFT_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
pft_status pft_cl_step_static(pft_ctx* ctx, double* w_plus, double* w_minus, const pft_step* step,
                              double* phi_a, double* phi_b, double* Q, double* H);

/* Per-node diagnostic Qnode[j] = (1/M) sum_x q_j(x) qd_{K-j}(x), j = 0..K,
 * from the last propagate; equal to Q in exact arithmetic for every node
 * because each split step is complex-symmetric.  qnode: 2*(K+1) doubles of
 * device memory.  Errors: PFT_E_INVALID, PFT_E_STATE. */
pft_status pft_node_q(pft_ctx* ctx, double* qnode);

/* Copy node `node` (0..K) of q (which = 0) or q-dagger (which = 1) from the
 * last propagate into out ([nx][ny][nz] complex128, device), widening c64.
 * Errors: PFT_E_INVALID, PFT_E_STATE. */
pft_status pft_get_slice(pft_ctx* ctx, int32_t which, int32_t node, double* out);

/* Apply contour step `step_index` (0..K-1, forward numbering) of the current
 * fields to an arbitrary q: q_out = T_{h_j}(q_in; w_{blk(j)}), with the same
 * kernels the sweeps use.  q_in, q_out: [nx][ny][nz] complex128 device (may
 * alias).  Needs a prior pft_propagate.  Errors: PFT_E_INVALID, PFT_E_STATE. */
pft_status pft_apply_step(pft_ctx* ctx, int32_t step_index, const double* q_in, double* q_out);

/* Diffusion operator D_h = exp(h Laplacian) of Eq. (5) applied in place to
 * u ([nx][ny][nz] complex128, device), through the same axis passes the
 * sweeps use (in the context's precision).  Errors: PFT_E_INVALID. */
pft_status pft_diffuse(pft_ctx* ctx, double* u, double h);

/* Squared integer wave numbers m_x^2 + m_y^2 + m_z^2 of every grid point in
 * natural DFT order, m(j) = j for j <= n/2 else j - n.  m2_out: M int32 of
 * HOST memory.  Host-only; needs no GPU work.  Errors: PFT_E_INVALID. */
pft_status pft_debug_kgrid(const pft_ctx* ctx, int32_t* m2_out);

/* Status flags accumulated on the device since creation (bit 0: a non-finite
 * Q).  Synchronises the stream.  Returns PFT_E_NONFINITE if bit 0 is set. */
pft_status pft_status_flags(pft_ctx* ctx, uint32_t* flags);

/* Noise stream test hooks (no context): the raw Philox4x64-10 words
 * (4 per block of 4 sites, 4*ceil(M/4) uint64 out) and the standard normals
 * (M doubles out) the field update draws for one field at one step.  Device
 * output, enqueued on hip_stream.  Errors: PFT_E_INVALID, PFT_E_DEVICE. */
pft_status pft_noise_words(uint64_t seed, uint64_t replica, uint64_t step, int32_t field, int64_t M,
                           uint64_t* out, void* hip_stream);
pft_status pft_noise_normals(uint64_t seed, uint64_t replica, uint64_t step, int32_t field,
                             int64_t M, double* out, void* hip_stream);

/* ---- batches of independent replicas --------------------------------------
 * Many independent systems (SCFT candidates or complex-Langevin replicas,
 * each its own pft_params: grid, box, ns, f, chiN, C) advanced together.
 * Replicas with the same grid shape and walls form a group; every axis pass of a group
 * is one launch over all its replicas (per-replica arguments come from device
 * tables, uneven contour step counts are masked); groups run on their own
 * streams; one field step of the whole batch is captured in a HIP graph and
 * replayed.  All replicas must share precision, scheme and model (Edwards
 * replicas run one sweep each and take w_minus = NULL).  This fills the
 * GPU with small grids, which on their own cannot hide memory latency
 * (Sec. VI notes the GPU only pays off above 512-2048 plane waves). */
typedef struct pft_batch pft_batch;

/* params: n parameter sets (host memory): both stores, periodic or walled.
 * Errors: PFT_E_INVALID (n < 1, mixed precision/scheme/model, or a bad
 * parameter set), PFT_E_UNSUPPORTED,
 * PFT_E_NOMEM, PFT_E_DEVICE; on failure *out = NULL and nothing is kept. */
pft_status pft_batch_create(const pft_params* params, int32_t n, void* hip_stream, pft_batch** out);
void pft_batch_destroy(pft_batch* batch);
const char* pft_batch_last_error(const pft_batch* batch);

/* One evaluation of every replica (tables, both sweeps or the Edwards model's
 * one, Q, densities, H).
 * w_plus, w_minus, phi_a, phi_b: host arrays of n device pointers (each a
 * [nx][ny][nz] complex128 field of that replica; Edwards batches: omega in
 * w_plus, w_minus NULL, phi in phi_a); Q, H: device arrays of n
 * complex128.  Errors: PFT_E_INVALID, PFT_E_DEVICE. */
pft_status pft_batch_evaluate(pft_batch* batch, const double* const* w_plus, const double* const* w_minus,
                              double* const* phi_a, double* const* phi_b, double* Q, double* H);

/* nsteps field steps of every replica (pft_cl_step semantics, explicit or
 * semi-implicit by step->update, in place on the fields), replica r drawing
 * noise with key (seed, replica + r) and step numbers step, step+1, ....  The
 * step is captured in a HIP graph on first use and replayed; a call with
 * other field pointers, log buffer or step parameters re-captures.  The
 * semi-implicit step allocates each replica's filter buffers (one complex128
 * field and the k tables) before its first capture.  QH_log (device, may be
 * NULL): rows of n (Q, H) complex128 pairs, row i for the i-th step of this
 * call, up to log_rows rows.  Asynchronous; pft_batch_sync waits.  Errors:
 * PFT_E_INVALID (also update other than 0 or 1), PFT_E_UNSUPPORTED (the
 * semi-implicit step with a replica it does not take: absorbing walls, or a
 * reflecting axis whose image length has no kernel), PFT_E_NOMEM,
 * PFT_E_DEVICE. */
pft_status pft_batch_cl_steps(pft_batch* batch, double* const* w_plus, double* const* w_minus,
                              const pft_step* step, int32_t nsteps, double* QH_log, int64_t log_rows);
pft_status pft_batch_sync(pft_batch* batch);

#define PFT_MAX_VARIANTS 4

/* ---- autotuner ---------------------------------------------------------------
 * Every axis length has up to PFT_MAX_VARIANTS kernel variants of its passes
 * (workgroup tile width, radix split N = N1 * N2, register bound for two waves
 * per SIMD; all give the same results to rounding).  pft_autotune times every
 * variant of the z, x and y passes for each listed axis length on the current
 * device (grids of ~4 Mi sites with lines of that length along the pass's
 * axis; the z pass completing and starting a Richardson step, the x pass on
 * both arrays with its field multiply, the y pass on both arrays) and makes
 * the fastest of each the default for contexts and batches created afterwards.
 * choices (may be NULL): 3 ints per size (z, x, y variant);
 * timings (may be NULL): 3 * PFT_MAX_VARIANTS doubles per size (ms per launch,
 * z then x then y, variants 0.., -1 where a variant does not exist).
 * Synchronous.
 * Errors: PFT_E_INVALID, PFT_E_UNSUPPORTED, PFT_E_NOMEM, PFT_E_DEVICE. */
pft_status pft_autotune(int32_t precision, const int32_t* sizes, int32_t nsizes, void* hip_stream,
                        int32_t* choices, double* timings);
/* Save / load the table (text: "arch precision N kind variant" per line;
 * entries for another GPU architecture are ignored).  pft_create also loads
 * the file named by $PFT_TUNE_CACHE once per process.  Errors: PFT_E_INVALID
 * (NULL path or file not writable / readable). */
pft_status pft_tune_save(const char* path);
pft_status pft_tune_load(const char* path);
/* Force kernel variant `variant` on one axis (0 = x, 1 = y, 2 = z) of a
 * context (checking every variant against the oracle).  Errors:
 * PFT_E_INVALID, PFT_E_UNSUPPORTED (no such variant). */
pft_status pft_set_variant(pft_ctx* ctx, int32_t axis, int32_t variant);

/* Kernel kinds reported by the profiling calls below. */
typedef enum {
    PFT_K_TABLES = 0,  /* field operator tables exp(-w h/4)                     */
    PFT_K_ZPASS = 1,   /* z-axis pass: completes one step and starts the next    */
    PFT_K_YPASS = 2,   /* y-axis passes                                          */
    PFT_K_XPASS = 3,   /* x-axis pass                                            */
    PFT_K_DENSITY = 4, /* contour-weighted q * q-dagger reduction               */
    PFT_K_REDUCE = 5,  /* spatial reductions (Q, H, per-node Q) and the update   */
    PFT_K_YZPASS = 6,  /* fused yz-plane pass (y, z, y of two steps)             */
    PFT_K_COUNT = 7
} pft_kernel_kind;

/* Per-kernel timing for roofline measurement.  Between pft_profile_begin and
 * pft_profile_end, every kernel the context launches is bracketed by a pair
 * of HIP events recorded on the context's stream.  pft_profile_end
 * synchronises the stream and writes, per pft_kernel_kind (arrays of
 * PFT_K_COUNT entries, host memory): the summed event-measured duration in
 * milliseconds, the number of launches, and the summed algorithmic bytes
 * (the bytes each launch must read and write given its inputs and outputs,
 * each array counted once).  Any output pointer may be NULL.
 * Errors: PFT_E_INVALID, PFT_E_STATE (end without begin), PFT_E_DEVICE. */
pft_status pft_profile_begin(pft_ctx* ctx);
/* Measurement hook (no context): a plain streaming copy of `bytes` bytes
 * (a multiple of 16) from src to dst, both device memory, 16-byte aligned, not
 * overlapping, enqueued on hip_stream.  Its hardware-counter readings give the
 * scale that converts other kernels' counter readings into bytes.
 * Errors: PFT_E_INVALID, PFT_E_DEVICE. */
pft_status pft_copy_probe(const void* src, void* dst, int64_t bytes, void* hip_stream);
pft_status pft_profile_end(pft_ctx* ctx, double* ms, int64_t* launches, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* PFT_H */
