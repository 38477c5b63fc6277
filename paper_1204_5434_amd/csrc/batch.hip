// Batches of independent replicas (pft_batch_*): uneven grids and contours,
// one launch per pass over all replicas of a grid group, the field step
// captured in a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include "runtime.h"

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

extern "C" {

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
        // the batched fused pass has no walls along y or z
        const bool fused = b->ctx[r]->fused && !p.bc[1] && !p.bc[2];
        BatchGroup* g = nullptr;
        for (BatchGroup& x : b->groups)
            if (x.nx == p.nx && x.ny == p.ny && x.nz == p.nz && x.bc[0] == p.bc[0] && x.bc[1] == p.bc[1] &&
                x.bc[2] == p.bc[2] && x.fused == fused)
                g = &x;
        if (!g) {
            b->groups.emplace_back();
            g = &b->groups.back();
            g->nx = p.nx;
            g->ny = p.ny;
            g->nz = p.nz;
            for (int a = 0; a < 3; ++a) g->bc[a] = p.bc[a];
            g->ndir = p.model == PFT_EDWARDS ? 1 : 2;
            g->fused = fused;
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

}  // extern "C"
