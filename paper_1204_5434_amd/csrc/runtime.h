// Host runtime of the propagator library, shared by its translation units:
// the context, the pass drivers every sweep, reverse mode and batch is built
// from, and the declarations of what one unit defines for another.
#pragma once

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
#include "kernels.h"
#include "ops.h"
#include "planes.h"
#include "sis.h"
#include "stress.h"
#include "walls_batch.h"

namespace {

inline int grid_for(int64_t n, int threads, int cap = 8192)
{
    const int64_t b = (n + threads - 1) / threads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

inline int reduction_blocks(int64_t n) { return grid_for(n, kRedThreads * 8, 1024); }

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

inline bool aligned16(const void* p) { return p && (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

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
    if (c->p.bc[1] || c->p.bc[2]) {
        if constexpr (std::is_same<T, float>::value)
            PFT_HIP(c, pft::launch_yzpass_walls(c->p.ny, c->p.bc[1], c->p.bc[2], a, st));
        else
            return c->fail(PFT_E_UNSUPPORTED, "no complex-double fused pass between walls");
        return PFT_OK;
    }
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

}  // namespace

// Defined by one translation unit, used by others.
namespace pft::rt {

// Contour plan (see pft_contour_plan): step lengths, blocks and the junction node.
int contour_plan(int ns, double f, double* h, int* blk, int* junction);
// Kernel variant of an axis pass per (precision, axis length, kind: 0 = z
// pass, 1 = x pass, 2 = y pass) for contexts created from now on (autotuner).
int tuned_variant(int prec, int n, int kind);
void tune_env_once();
pft_status create_ctx(const pft_params* params, void* hip_stream, bool dual, pft_ctx** out);
void free_all(pft_ctx* c);
pft_status hamiltonian_launch(pft_ctx* c, const double* wp, const double* wm, double* H, double* hint);

// The semi-implicit step (Eqs. (10)-(11)).
pft_status sis_prepare(pft_ctx* c);
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
SisBufs ctx_sis_bufs(const pft_ctx* c);
SisIncArgs sis_inc_args(const pft_ctx* c, const SisBufs& sb, const UpdArgs& u, const uint64_t* step_dev);
pft::SisArgs sis_filter_args(const SisBufs& sb, const UpdArgs& u, double2* X, double2* W, int ne_z,
                                    int64_t Me);
MirrorArgs sis_image(const pft_ctx* c, const SisBufs& sb);
const char* sis_walls_unsupported(const pft_params& p);
pft_status cl_step(pft_ctx* c, double* wp, double* wm, const pft_step* st, double* phi_a, double* phi_b,
                   double* Q, double* H, const SisBufs* sb);

}  // namespace pft::rt

using namespace pft::rt;
