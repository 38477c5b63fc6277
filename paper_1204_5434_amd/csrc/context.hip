// Host runtime of one context (include/pft.h): creation and teardown, the
// field tables and both sweeps, Q, the densities, H, the explicit and the
// semi-implicit field step, box changes, graph replay of an evaluation,
// diagnostics, noise-stream hooks and per-launch profiling.
#include <hip/hip_runtime.h>

#include "runtime.h"

namespace pft {
thread_local LaunchEvents g_launch_events;
}

namespace pft::rt {

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

}  // namespace pft::rt

namespace {

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

}  // namespace

namespace pft::rt {

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

}  // namespace pft::rt

namespace {

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

}  // namespace

namespace pft::rt {

// The fused schedule is the default where its kernel keeps (nearly) everything
// in registers: beyond this many spilled bytes per lane the spill traffic and
// latency outweigh the saved passes (measured: complex double 80^2 with 244 B
// still gains, 96^2 with 720 B loses to the axis schedule).
constexpr int kFusedMaxSpill = 256;
// Between walls along y or z the fused pass also holds the paired spectra of
// its walled transforms; measured at 128^2 (complex float): with 128 spilled
// bytes per lane (reflecting walls normal to z) it gains (10.55 against 11.00
// ms), with 248 (absorbing walls on y and z) it loses (12.39 against 11.85).
constexpr int kFusedMaxSpillWalls = 128;

// Walls along y or z have a fused pass in complex float only.
static bool fused_supported(const pft_params& p)
{
    if (p.ny != p.nz) return false;
    if (p.bc[1] || p.bc[2]) return p.precision == PFT_C64 && pft::plane_walls_supported(p.ny);
    return p.precision == PFT_C128 ? pft::plane_supported<double>(p.ny) : pft::plane_supported<float>(p.ny);
}

static bool fused_default(const pft_params& p)
{
    if (!fused_supported(p)) return false;
    if (p.bc[1] || p.bc[2]) {
        const int b = pft::plane_walls_private_bytes(p.ny, p.bc[1], p.bc[2]);
        return b >= 0 && b <= kFusedMaxSpillWalls;
    }
    const int b = p.precision == PFT_C128 ? pft::plane_private_bytes<double>(p.ny) : pft::plane_private_bytes<float>(p.ny);
    return b >= 0 && b <= kFusedMaxSpill;
}

pft_status create_ctx(const pft_params* params, void* hip_stream, bool dual, pft_ctx** out)
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

    tune_env_once();
    pft_ctx* c = new (std::nothrow) pft_ctx();
    if (!c) return PFT_E_NOMEM;
    c->p = p;
    if (hipGetDevice(&c->device) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return PFT_E_DEVICE;
    }
    c->var[0] = tuned_variant(p.precision, p.nx, 1);
    c->var[1] = tuned_variant(p.precision, p.ny, 2);
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
pft_status sis_prepare(pft_ctx* c)
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
SisBufs ctx_sis_bufs(const pft_ctx* c)
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

SisIncArgs sis_inc_args(const pft_ctx* c, const SisBufs& sb, const UpdArgs& u, const uint64_t* step_dev)
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
pft::SisArgs sis_filter_args(const SisBufs& sb, const UpdArgs& u, double2* X, double2* W, int ne_z,
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
const char* sis_walls_unsupported(const pft_params& p)
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
MirrorArgs sis_image(const pft_ctx* c, const SisBufs& sb)
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
pft_status cl_step(pft_ctx* c, double* wp, double* wm, const pft_step* st, double* phi_a, double* phi_b,
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

}  // namespace pft::rt

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

pft_status pft_cl_step(pft_ctx* c, double* wp, double* wm, const pft_step* st, double* phi_a, double* phi_b,
                       double* Q, double* H)
{
    if (!c) return PFT_E_INVALID;
    return cl_step(c, wp, wm, st, phi_a, phi_b, Q, H, nullptr);
}

}  // extern "C"

extern "C" {

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
