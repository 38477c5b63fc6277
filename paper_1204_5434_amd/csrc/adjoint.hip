// Reverse mode through the split steps (pft_adjoint): dH/dw and the box
// derivative dH/dL with checkpointed propagators.
#include <hip/hip_runtime.h>

#include "runtime.h"

namespace {

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

}  // namespace

extern "C" {

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

}  // extern "C"
