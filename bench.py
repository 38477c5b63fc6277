#!/usr/bin/env python
"""Benchmark of the propagator hot path on one MI355X.

A step is one full field evaluation of the hot path -- field operator
tables, the q sweep and the q-dagger sweep over all contour steps (Richardson
split step, Eq. (12)), Q, and the contour-weighted densities -- i.e.
pft_propagate + pft_densities, on the paper's lamellar benchmark workload at
its largest grid (128^3, f = 0.5, chi N = 14, L = 10.89 R_g) with Ns = 100.
Throughput is grid points x contour steps per second over both propagators
(2 M Ns per evaluation), inputs resident in HBM.

Both precisions are measured in the same run: the main line is the complex128
path, ``fp32`` holds the complex64-propagator path (FP64 sums).  The roofline
object reports the dominant kernel's algorithmic bytes over its HIP-event
duration against 8 TB/s; ``cpu_baseline`` times the FP64 CPU oracle on a
bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "propagator grid-pts×steps/s + %HBM peak, FP32 vs FP64 plain at 128³ Ns=100"
HBM_PEAK_GBS = 8000.0
PROFILE_KIND = {"zpass": "k_zpass", "ypass": "k_spass<..,1>", "xpass": "k_spass<..,0>",
                "yzpass": "k_yzpass", "density": "k_density", "tables": "k_field_tables",
                "reduce": "reductions"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def traffic_for(kind: str, precision: str):
    """HBM bytes per launch of a kernel kind from the committed counter summary
    (profiles/lam128_hbm_traffic.txt), if it was taken on the current sources
    of that kernel; else None."""
    path = os.path.join(ROOT, "profiles", "lam128_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    try:
        from paper_1204_5434_amd import build
        lines = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
        rec = {ln[0]: ln[1:] for ln in lines}
        entry = rec.get(f"{kind}:{precision}")
        if entry is None or len(entry) < 3 or entry[2] != build.kernel_hash(kind):
            return None
        return float(entry[0])
    except Exception:
        return None


def run_precision(binding, w, wp, wm, precision, steps, warmup, scheme):
    import torch
    prec = binding.PFT_C128 if precision == "f64" else binding.PFT_C64
    ctx = binding.Context(binding.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, prec, scheme))
    phiA = torch.empty(w.n, dtype=torch.complex128, device="cuda")
    phiB = torch.empty_like(phiA)
    Q = torch.empty(1, dtype=torch.complex128, device="cuda")

    def evaluate():
        ctx.pft_propagate(wp, wm)
        ctx.pft_densities(phiA, phiB, Q)

    def timed(n):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(n):
            evaluate()
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / n

    fused = ctx.pft_fused_planes()
    for _ in range(warmup):
        evaluate()
    torch.cuda.synchronize()
    # timed region: exactly `steps` evaluations between two events, both sweeps
    # running concurrently on two streams (the library's default)
    ms = timed(steps)
    # the same evaluations one by one (an event pair each): median and IQR
    per = []
    for _ in range(steps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        evaluate()
        b.record()
        per.append((a, b))
    torch.cuda.synchronize()
    import numpy as np
    each = np.array([a.elapsed_time(b) for a, b in per])
    spread = {"median": float(np.median(each)), "q25": float(np.percentile(each, 25)),
              "q75": float(np.percentile(each, 75))}
    by_schedule = None
    if fused:
        # the same with the other schedules, for comparison: axis passes only
        # (four per step), and fused yz passes in the conjugate sweep only
        by_schedule = {{1: "fused", 2: "fused-conjugate-sweep"}[fused]: ms}
        for mode, name in ((0, "axis"), (3 - fused, {1: "fused", 2: "fused-conjugate-sweep"}[3 - fused])):
            ctx.pft_set_fused_planes(mode)
            evaluate()
            by_schedule[name] = timed(steps)
        ctx.pft_set_fused_planes(fused)
        evaluate()
    # the same evaluations replayed from a HIP graph (captured once)
    ctx.pft_evaluate_graph(wp, wm, phiA, phiB, Q, 0)
    ctx.pft_evaluate_graph(wp, wm, phiA, phiB, Q, 1)
    torch.cuda.synchronize()
    g0 = torch.cuda.Event(enable_timing=True)
    g1 = torch.cuda.Event(enable_timing=True)
    g0.record()
    ctx.pft_evaluate_graph(wp, wm, phiA, phiB, Q, steps)
    g1.record()
    torch.cuda.synchronize()
    ms_graph = g0.elapsed_time(g1) / steps
    # the same with both sweeps on one stream, for comparison
    ctx.pft_set_concurrent_sweeps(False)
    evaluate()
    ms_single = timed(steps)
    # per-kernel HIP-event timing on one stream (kernels isolated, so each
    # launch's duration is its own)
    ctx.pft_profile_begin()
    for _ in range(steps):
        evaluate()
    prof = ctx.pft_profile_end()
    ctx.pft_set_concurrent_sweeps(True)
    flags = ctx.pft_status_flags()
    if flags:
        raise RuntimeError(f"device status flags {flags:#x}")
    # the results of one evaluation (outside every timed region), for the
    # error report against the oracle
    Hd = torch.empty(1, dtype=torch.complex128, device="cuda")
    evaluate()
    ctx.pft_hamiltonian(wp, wm, Hd)
    torch.cuda.synchronize()
    Qv = complex(Q.cpu()[0])
    results = {"phiA": phiA.cpu().numpy(), "phiB": phiB.cpu().numpy(), "Q": Qv, "H": complex(Hd.cpu()[0])}
    ctx.close()
    site_steps = 2.0 * w.M * w.ns
    rate = site_steps / (ms * 1e-3)
    # dominant kernel by measured time among the memory-pass kernels
    kinds = [k for k in ("zpass", "ypass", "xpass", "yzpass", "density") if prof[k][1] > 0]
    dom = max(kinds, key=lambda k: prof[k][0])
    kms, kn, kbytes = prof[dom]
    per_launch_ms = kms / kn
    achieved = (kbytes / kn) / (per_launch_ms * 1e-3) / 1e9
    traffic = traffic_for(dom, precision)
    roof = {"bound": "hbm", "kernel": PROFILE_KIND[dom], "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "bytes_per_launch": kbytes / kn,
            "avg_launch_us": round(per_launch_ms * 1e3, 2), "launches": kn}
    breakdown = {k: {"ms_per_step": round(v[0] / steps, 4), "launches_per_step": v[1] / steps,
                     "GB_s": round(v[2] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 else None}
                 for k, v in prof.items() if v[1] > 0}
    bytes_eval = sum(v[2] for v in prof.values()) / steps
    roof["aggregate_GB_s"] = round(bytes_eval / (ms * 1e-3) / 1e9, 1)
    # frac above is the dominant kernel's own (its bytes per launch over its
    # duration, launches timed one at a time on one stream); beside it, the
    # whole evaluation against the method's minimum traffic: per site-step
    # the forward step reads q_j and the block's two field tables and writes
    # q_{j+1} (4c), the conjugate step also reads the stored q slice and
    # updates an FP64 complex density accumulator (5c + 32): (9c + 32) / 2
    c_bytes = 16 if precision == "f64" else 8
    floor = (9 * c_bytes + 32) / 2
    roof["frac_of"] = "dominant kernel per launch (one-stream repeat, launches isolated)"
    roof["bytes_per_site_step"] = round(bytes_eval / site_steps, 1)
    roof["floor_bytes_per_site_step"] = floor
    roof["floor_GB_s"] = round(floor * rate / 1e9, 1)
    roof["floor_frac"] = round(floor * rate / 1e9 / HBM_PEAK_GBS, 4)
    out = {"value": rate, "results": results, "ms_per_step": ms, "ms_per_evaluation_spread": spread, "ms_per_step_graph": ms_graph,
           "ms_per_step_one_stream": ms_single, "roofline": roof,
           "kernels": breakdown, "Q": [Qv.real, Qv.imag],
           "schedule": {0: "axis", 1: "fused", 2: "fused-conjugate-sweep"}[fused]}
    if by_schedule is not None:
        out["ms_per_step_by_schedule"] = by_schedule
    return out


def update_cost(binding, w, wp0, wm0, steps: int):
    """Field steps (pft_cl_step: evaluation + update) at the workload, FP64,
    with the explicit and the semi-implicit update (Eqs. (10)-(11))."""
    import torch
    ctx = binding.Context(binding.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, binding.PFT_C128, binding.PFT_RQM4))
    out = {}
    for name, upd in (("explicit", 0), ("semi_implicit", 1)):
        wp, wm = wp0.clone(), wm0.clone()
        st = binding.pft_step(0.01, 1.0, 1.0, 1204, 0, 0, 1, upd)
        ctx.pft_cl_step(wp, wm, st)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for k in range(steps):
            st = binding.pft_step(0.01, 1.0, 1.0, 1204, 0, 1 + k, 1, upd)
            ctx.pft_cl_step(wp, wm, st)
        t1.record()
        torch.cuda.synchronize()
        out[name + "_ms_per_field_step"] = t0.elapsed_time(t1) / steps
    out["semi_implicit_extra_ms"] = out["semi_implicit_ms_per_field_step"] - out["explicit_ms_per_field_step"]
    ctx.close()
    return out


def storage_run(binding, w, wp, wm, steps: int, warmup: int):
    """The benchmark evaluation with the stored-product storage modes: q only
    in device memory (contour sums during the conjugate sweep), and q staged
    through pinned host memory."""
    import torch
    out = {}
    for pname, prec in (("f64", binding.PFT_C128), ("f32", binding.PFT_C64)):
        for sname, st in (("q_only", binding.PFT_STORE_Q), ("host", binding.PFT_STORE_HOST)):
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            ctx = binding.Context(binding.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, prec, binding.PFT_RQM4,
                                                 binding.PFT_DIBLOCK, 0.0, st))
            dev_bytes = free0 - torch.cuda.mem_get_info()[0]
            pa = torch.empty(w.n, dtype=torch.complex128, device="cuda")
            pb = torch.empty_like(pa)

            def evaluate():
                ctx.pft_propagate(wp, wm)
                ctx.pft_densities(pa, pb)

            for _ in range(warmup):
                evaluate()
            torch.cuda.synchronize()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record()
            for _ in range(steps):
                evaluate()
            t1.record()
            torch.cuda.synchronize()
            ms = t0.elapsed_time(t1) / steps
            out[f"{pname}_{sname}"] = {"ms_per_step": ms, "value": 2.0 * w.M * w.ns / (ms * 1e-3),
                                       "device_GB": round(dev_bytes / 1e9, 3)}
            ctx.close()
    return out


def edwards_run(binding, inputs, steps: int, warmup: int):
    """Edwards homopolymer model at 128^3, Ns = 100: one forward sweep per
    evaluation (q-dagger = q), in both working precisions."""
    import torch
    w = inputs.EDW128
    om = torch.from_numpy(inputs.fields(w)[0]).to("cuda")
    out = {"workload": w.name, "grid": list(w.n), "ns": w.ns, "B": w.extra["B"], "C": w.C,
           "site_steps_per_evaluation": w.M * w.ns}
    for name, prec in (("f64", binding.PFT_C128), ("f32", binding.PFT_C64)):
        ctx = binding.Context(binding.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, prec, binding.PFT_RQM4,
                                             binding.PFT_EDWARDS, w.extra["B"]))
        phi = torch.empty(w.n, dtype=torch.complex128, device="cuda")
        phib = torch.empty_like(phi)

        def evaluate():
            ctx.pft_propagate(om, None)
            ctx.pft_densities(phi, phib)

        for _ in range(warmup):
            evaluate()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(steps):
            evaluate()
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / steps
        out[name] = {"ms_per_evaluation": ms, "value": w.M * w.ns / (ms * 1e-3),
                     "schedule": {0: "axis", 1: "fused", 2: "fused"}[ctx.pft_fused_planes()]}
        ctx.close()
    return out


def walls_run(binding, w, wp, wm, steps: int, warmup: int):
    """The benchmark evaluation in walled boxes (Sec. III: cosine modes between
    reflecting walls, sine modes between absorbing ones): a film with
    reflecting walls normal to z, and absorbing walls on every axis; both
    working precisions, with the per-kernel breakdown on one stream."""
    import torch
    out = {}
    for gname, bc in (("film_z_reflecting", (0, 0, 1)), ("box_absorbing", (2, 2, 2))):
        for pname, prec in (("f64", binding.PFT_C128), ("f32", binding.PFT_C64)):
            ctx = binding.Context(binding.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, prec, binding.PFT_RQM4,
                                                 binding.PFT_DIBLOCK, 0.0, binding.PFT_STORE_BOTH, bc))
            pa = torch.empty(w.n, dtype=torch.complex128, device="cuda")
            pb = torch.empty_like(pa)

            def evaluate():
                ctx.pft_propagate(wp, wm)
                ctx.pft_densities(pa, pb)

            for _ in range(warmup):
                evaluate()
            torch.cuda.synchronize()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record()
            for _ in range(steps):
                evaluate()
            t1.record()
            torch.cuda.synchronize()
            ms = t0.elapsed_time(t1) / steps
            ctx.pft_set_concurrent_sweeps(False)
            ctx.pft_profile_begin()
            for _ in range(steps):
                evaluate()
            prof = ctx.pft_profile_end()
            if ctx.pft_status_flags():
                raise RuntimeError("device status flags set in the walled evaluation")
            kernels = {k: {"ms_per_step": round(v[0] / steps, 4),
                           "GB_s": round(v[2] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 else None}
                       for k, v in prof.items() if v[1] > 0}
            out[f"{gname}_{pname}"] = {"bc": list(bc), "ms_per_step": ms,
                                       "value": 2.0 * w.M * w.ns / (ms * 1e-3),
                                       "schedule": {0: "axis", 1: "fused", 2: "fused"}[ctx.pft_fused_planes()],
                                       "kernels": kernels}
            ctx.close()
    return out


def adjoint_run(binding, inputs, steps: int):
    """The gradient workload (96^3, Ns = 128, f = 0.3, checkpoints every 11
    steps): one reverse-mode pass (dH/dw+-, dH/dL and H) against one plain
    evaluation (propagate + densities) of the same state, both precisions,
    and in complex double between reflecting walls normal to z."""
    import torch
    w = inputs.GRAD96
    wp, wm = (torch.from_numpy(a).to("cuda") for a in inputs.fields(w))
    out = {"workload": w.name, "grid": list(w.n), "ns": w.ns, "f": w.f, "ckpt_every": 11}
    for name, prec, bc in (("f64", binding.PFT_C128, (0, 0, 0)), ("f32", binding.PFT_C64, (0, 0, 0)),
                           ("f64_film_z_reflecting", binding.PFT_C128, (0, 0, 1))):
        ctx = binding.Context(binding.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, prec, binding.PFT_RQM4,
                                             binding.PFT_DIBLOCK, 0.0, binding.PFT_STORE_BOTH, bc))
        gp = torch.empty(w.n, dtype=torch.complex128, device="cuda")
        gm = torch.empty_like(gp)
        dL = torch.empty(3, dtype=torch.complex128, device="cuda")
        H = torch.empty(1, dtype=torch.complex128, device="cuda")
        pa = torch.empty_like(gp)
        pb = torch.empty_like(gp)

        def grad():
            ctx.pft_adjoint(wp, wm, gp, gm, dL, H, 11)

        def evaluate():
            ctx.pft_propagate(wp, wm)
            ctx.pft_densities(pa, pb)

        res = {}
        for label, fn in (("adjoint", grad), ("evaluation", evaluate)):
            fn()
            torch.cuda.synchronize()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record()
            for _ in range(steps):
                fn()
            t1.record()
            torch.cuda.synchronize()
            res[f"{label}_ms"] = t0.elapsed_time(t1) / steps
        res["adjoint_over_evaluation"] = res["adjoint_ms"] / res["evaluation_ms"]
        if ctx.pft_status_flags():
            raise RuntimeError("device status flags set in the adjoint run")
        out[name] = res
        ctx.close()
    return out


def batched_gain(binding, inputs, count: int, steps: int, run_steps: int):
    """Uneven replicas (grids 24-48^3, Ns 40-80): complex64 propagators, all
    replicas per launch, field steps replayed from a HIP graph -- against the
    same replicas advanced one at a time in the plain complex128 form.  The
    explicit batched step is timed over a run of `run_steps` field steps (with
    the per-step Q and H log), the other forms over `steps`."""
    import torch
    reps = inputs.batch_replicas(count, 1208)
    site_steps = sum(2.0 * w.M * w.ns for w in reps)  # per field step of the whole set
    fields = [inputs.fields(w) for w in reps]
    out = {"replicas": count, "site_steps_per_field_step": site_steps}
    # batched, complex64, graph
    params = [binding.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, binding.PFT_C64, binding.PFT_RQM4) for w in reps]
    bat = binding.Batch(params)
    wp = [torch.from_numpy(f[0]).to("cuda") for f in fields]
    wm = [torch.from_numpy(f[1]).to("cuda") for f in fields]
    log = torch.empty((run_steps, count, 2), dtype=torch.complex128, device="cuda")
    st = binding.pft_step(0.01, 1.0, 1.0, 1208, 0, 0, 1)
    bat.pft_batch_cl_steps(wp, wm, st, 2, log)  # capture + warm-up
    bat.pft_batch_sync()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    bat.pft_batch_cl_steps(wp, wm, binding.pft_step(0.01, 1.0, 1.0, 1208, 0, 2, 1), run_steps, log)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / run_steps
    H = log[:, :, 1]
    out["batched_c64_graph"] = {"ms_per_field_step": ms, "value": site_steps / (ms * 1e-3),
                                "field_steps": run_steps,
                                "replicas_finite_throughout": int(torch.isfinite(H).all(dim=0).sum())}
    del log
    k0 = 2 + run_steps
    # the same batch with the semi-implicit field step (one filter per replica in the graph)
    bat.pft_batch_cl_steps(wp, wm, binding.pft_step(0.01, 1.0, 1.0, 1208, 0, k0, 1, 1), 1)  # capture
    t0.record()
    bat.pft_batch_cl_steps(wp, wm, binding.pft_step(0.01, 1.0, 1.0, 1208, 0, k0 + 1, 1, 1), steps)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    out["batched_c64_graph_semi_implicit"] = {"ms_per_field_step": ms, "value": site_steps / (ms * 1e-3)}
    bat.close()
    # Edwards replicas on the same grids and chain lengths (B = 1): one sweep each
    ed_params = [binding.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, binding.PFT_C64, binding.PFT_RQM4,
                                binding.PFT_EDWARDS, 1.0) for w in reps]
    bat = binding.Batch(ed_params)
    bat.pft_batch_cl_steps(wp, None, binding.pft_step(0.01, 1.0, 1.0, 1208, 0, 0, 1), 1)  # capture
    torch.cuda.synchronize()
    t0.record()
    bat.pft_batch_cl_steps(wp, None, binding.pft_step(0.01, 1.0, 1.0, 1208, 0, 1, 1), steps)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    out["batched_edwards_c64_graph"] = {"ms_per_field_step": ms, "site_steps_per_field_step": site_steps / 2,
                                        "value": site_steps / 2 / (ms * 1e-3)}
    bat.close()
    del wp, wm
    # one at a time, complex128, plain launches
    wp = [torch.from_numpy(f[0]).to("cuda") for f in fields]
    wm = [torch.from_numpy(f[1]).to("cuda") for f in fields]
    ctxs = [binding.Context(binding.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, binding.PFT_C128,
                                           binding.PFT_RQM4)) for w in reps]
    for r, c in enumerate(ctxs):  # warm-up
        c.pft_cl_step(wp[r], wm[r], binding.pft_step(0.01, 1.0, 1.0, 1208, r, 0, 1))
    torch.cuda.synchronize()
    plain_steps = min(steps, 5)  # ~0.65 s per field step one replica at a time
    t0.record()
    for k in range(plain_steps):
        for r, c in enumerate(ctxs):
            c.pft_cl_step(wp[r], wm[r], binding.pft_step(0.01, 1.0, 1.0, 1208, r, 1 + k, 1))
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / plain_steps
    out["single_c128_plain"] = {"ms_per_field_step": ms, "value": site_steps / (ms * 1e-3)}
    for c in ctxs:
        c.close()
    out["gain"] = out["batched_c64_graph"]["value"] / out["single_c128_plain"]["value"]
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def langevin_run(binding, inputs, steps: int):
    """The 64^3 complex-Langevin workload (Ns = 100, f = 0.4, chi N = 20,
    C = 50, dt = 0.01, real Gaussian noise): Langevin steps (evaluation, H and
    the update) per second with complex128 and with complex64 propagators."""
    import torch
    w = inputs.CL64
    wp0, wm0 = (torch.from_numpy(a).to("cuda") for a in inputs.fields(w))
    out = {"workload": w.name, "grid": list(w.n), "ns": w.ns, "site_steps_per_cl_step": 2 * w.M * w.ns}
    for name, prec in (("f64", binding.PFT_C128), ("f32", binding.PFT_C64)):
        ctx = binding.Context(binding.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, prec, binding.PFT_RQM4))
        a, b = wp0.clone(), wm0.clone()
        ctx.pft_cl_step(a, b, binding.pft_step(w.dt, 1.0, 1.0, w.seed, 0, 0, 1))
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for k in range(steps):
            ctx.pft_cl_step(a, b, binding.pft_step(w.dt, 1.0, 1.0, w.seed, 0, 1 + k, 1))
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / steps
        if ctx.pft_status_flags():
            raise RuntimeError("device status flags set in the 64^3 Langevin run")
        out[name] = {"ms_per_cl_step": ms, "cl_steps_per_s": 1e3 / ms,
                     "value": 2 * w.M * w.ns / (ms * 1e-3),
                     "schedule": {0: "axis", 1: "fused", 2: "fused"}[ctx.pft_fused_planes()]}
        ctx.close()
    return out


def large_grid_run(binding, inputs, steps: int, cl_steps: int):
    """The large single-GPU workload (256^3, Ns = 200, f = 0.35, chi N = 22,
    L = 16, C = 100): evaluations in both working precisions, its Langevin run
    (`cl_steps` steps of dt = 0.005) in complex64 against a few complex128
    steps, per-pass bandwidth from a profiled evaluation on one stream, and
    one checkpointed reverse-mode pass in complex64.  One 256^3
    array is 268 MB in complex128 and 134 MB in complex64, so the passes'
    arrays no longer fit the 256 MB Infinity Cache together."""
    import torch
    w = inputs.CL256
    wp, wm = (torch.from_numpy(a).to("cuda") for a in inputs.fields(w))
    out = {"workload": w.name, "grid": list(w.n), "box": list(w.L), "ns": w.ns, "f": w.f, "chiN": w.chiN,
           "C": w.C, "site_steps_per_evaluation": 2 * w.M * w.ns}
    for name, prec in (("f64", binding.PFT_C128), ("f32", binding.PFT_C64)):
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        ctx = binding.Context(binding.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, prec, binding.PFT_RQM4))
        dev_gb = (free0 - torch.cuda.mem_get_info()[0]) / 1e9
        pa = torch.empty(w.n, dtype=torch.complex128, device="cuda")
        pb = torch.empty_like(pa)

        def evaluate():
            ctx.pft_propagate(wp, wm)
            ctx.pft_densities(pa, pb)

        evaluate()
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(steps):
            evaluate()
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / steps
        # Langevin steps: the workload's whole run in complex64 (its stored form),
        # a few steps in complex128 for the comparison; H logged per step
        ncl = cl_steps if prec == binding.PFT_C64 else steps
        a, b = wp.clone(), wm.clone()
        Hs = torch.empty(ncl, dtype=torch.complex128, device="cuda")
        ctx.pft_cl_step(a, b, binding.pft_step(w.dt, 1.0, 1.0, w.seed, 0, 0, 1))
        torch.cuda.synchronize()
        t0.record()
        for k in range(ncl):
            ctx.pft_cl_step(a, b, binding.pft_step(w.dt, 1.0, 1.0, w.seed, 0, 1 + k, 1), H=Hs[k:k + 1])
        t1.record()
        torch.cuda.synchronize()
        ms_cl = t0.elapsed_time(t1) / ncl
        h_finite = bool(torch.isfinite(Hs).all())
        del a, b, Hs
        ctx.pft_set_concurrent_sweeps(False)
        ctx.pft_profile_begin()
        evaluate()
        prof = ctx.pft_profile_end()
        ctx.pft_set_concurrent_sweeps(True)
        res = {"ms_per_evaluation": ms, "value": 2 * w.M * w.ns / (ms * 1e-3), "ms_per_cl_step": ms_cl,
               "cl_steps": ncl, "cl_H_finite": h_finite, "device_GB": round(dev_gb, 1),
               "kernels": {k: {"ms_per_evaluation": round(v[0], 3), "launches": int(v[1]),
                               "GB_s": round(v[2] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 else None}
                           for k, v in prof.items() if v[1] > 0}}
        if prec == binding.PFT_C64:
            gp = torch.empty(w.n, dtype=torch.complex128, device="cuda")
            gm = torch.empty_like(gp)
            dL = torch.empty(3, dtype=torch.complex128, device="cuda")
            torch.cuda.synchronize()
            t0.record()
            ctx.pft_adjoint(wp, wm, gp, gm, dL, None, 0)
            t1.record()
            torch.cuda.synchronize()
            res["adjoint_ms"] = t0.elapsed_time(t1)
            del gp, gm, dL
        if ctx.pft_status_flags():
            raise RuntimeError("device status flags set in the 256^3 run")
        ctx.close()
        del pa, pb
        out[name] = res
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _errors(gpu, ref, w):
    """Per-result error of one GPU evaluation against the oracle's: phi
    relative to max|phi|, Q relative, H on |H| + C V and relative to |H|."""
    import numpy as np
    scale = max(np.abs(ref["phiA"]).max(), np.abs(ref["phiB"]).max())
    dH = abs(gpu["H"] - ref["H"])
    return {"phiA": float(np.abs(gpu["phiA"] - ref["phiA"]).max() / scale),
            "phiB": float(np.abs(gpu["phiB"] - ref["phiB"]).max() / scale),
            "Q": abs(gpu["Q"] - ref["Q"]) / abs(ref["Q"]),
            "H": dH / (abs(ref["H"]) + w.C * w.L[0] * w.L[1] * w.L[2]),
            "H_relative_to_H": dH / abs(ref["H"])}


def cpu_baseline(binding, inputs, w, wp, wm, gpu_results, seconds_one_thread: float):
    """The FP64 oracle as it stands, on the host cores.

    On all visible cores (at most 16): one full evaluation of the workload
    (both sweeps, densities, Q, H), whose results also give the per-result
    error of the GPU evaluations in both precisions; the 16^3 relaxation in
    full (100 iterations); one 64^3 Langevin step.  On one thread: a bounded
    sample of forward-sweep steps of the workload.  Also the reverse-mode
    error (dH/dw, dH/dL) of both precisions on the gradient state at 48^3,
    Ns = 64 (a reduced copy of the 96^3 state the oracle would take minutes
    on)."""
    import numpy as np
    import torch
    from oracle import oracle
    threads = min(len(os.sched_getaffinity(0)), 16)
    oracle.set_threads(threads)
    p = oracle.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, 0)
    t = time.perf_counter()
    ref = oracle.evaluate(p, wp, wm)
    el = time.perf_counter() - t
    base = {"value": 2.0 * w.M * w.ns / el, "unit": "grid-pts×steps/s", "cores": threads, "kind": "oracle",
            "cpu": cpu_model(), "host_cores_visible": len(os.sched_getaffinity(0)),
            "sample": f"one full evaluation of the {w.name} workload ({2 * ref['K']} Richardson steps over "
                      f"both sweeps, densities, Q and H): {el:.1f} s"}
    errors = {name: _errors(g, ref, w) for name, g in gpu_results.items()}
    del ref
    legs = {}
    s16 = inputs.SCFT16
    p16 = oracle.Params(*s16.n, *s16.L, s16.ns, s16.f, s16.chiN, s16.C, 0)
    a, b = inputs.fields(s16)
    t = time.perf_counter()
    for _ in range(s16.steps):
        r = oracle.evaluate(p16, a, b)
        a, b = oracle.em_update(p16, a, b, r["phiA"], r["phiB"], s16.dt)
    legs["scft16_full_100_iterations_s"] = round(time.perf_counter() - t, 3)
    c64 = inputs.CL64
    p64 = oracle.Params(*c64.n, *c64.L, c64.ns, c64.f, c64.chiN, c64.C, 0)
    a, b = inputs.fields(c64)
    t = time.perf_counter()
    r = oracle.evaluate(p64, a, b)
    oracle.em_update(p64, a, b, r["phiA"], r["phiB"], c64.dt, noise=True, seed=c64.seed, replica=0, step_=0)
    legs["cl64_one_step_s"] = round(time.perf_counter() - t, 3)
    legs["cores"] = threads
    # reverse mode at 48^3, Ns = 64: oracle against both GPU precisions
    g = inputs.GRAD96.scaled((48, 48, 48), ns=64)
    ga, gb = inputs.fields(g)
    rp, rm, rL = oracle.adjoint(oracle.Params(*g.n, *g.L, g.ns, g.f, g.chiN, g.C, 0), ga, gb)
    adj = {"workload": f"{g.name} at 48^3, Ns = 64 (f = {g.f}, junction inside a step)"}
    V = g.L[0] * g.L[1] * g.L[2]
    for name, prec in (("f64", binding.PFT_C128), ("f32", binding.PFT_C64)):
        ctx = binding.Context(binding.Params(*g.n, *g.L, g.ns, g.f, g.chiN, g.C, prec, binding.PFT_RQM4))
        gp = torch.empty(g.n, dtype=torch.complex128, device="cuda")
        gm = torch.empty_like(gp)
        dL = torch.empty(3, dtype=torch.complex128, device="cuda")
        ctx.pft_adjoint(torch.from_numpy(ga).to("cuda"), torch.from_numpy(gb).to("cuda"), gp, gm, dL, None, 8)
        gp, gm, dL = gp.cpu().numpy(), gm.cpu().numpy(), dL.cpu().numpy()
        ctx.close()
        adj[name] = {"dH_dwplus": float(np.abs(gp - rp).max() / np.abs(rp).max()),
                     "dH_dwminus": float(np.abs(gm - rm).max() / np.abs(rm).max()),
                     "dH_dL": max(abs(dL[k] - rL[k]) / (abs(rL[k]) + g.C * V / g.L[k]) for k in range(3)),
                     "dH_dL_relative_to_dL": max(abs(dL[k] - rL[k]) / abs(rL[k]) for k in range(3))}
    errors["adjoint"] = adj
    # one thread, bounded sample of forward-sweep steps
    oracle.set_threads(1)
    wA, _ = oracle.block_fields(p, wp, wm)
    h, _, _ = oracle.contour(w.ns, w.f)
    q = np.ones(w.n, complex)
    n = 0
    t = time.perf_counter()
    while True:
        q = oracle.step(p, h[n % len(h)], wA, q)
        n += 1
        el = time.perf_counter() - t
        if el >= seconds_one_thread:
            break
    one = {"value": n * w.M / el, "unit": "grid-pts×steps/s", "cores": oracle.get_threads(), "kind": "oracle",
           "cpu": cpu_model(), "sample": f"{n} forward-sweep Richardson steps of the {w.n[0]}^3 workload "
                                         f"({el:.1f} s); the density reduction is not in the sample"}
    return base, one, legs, errors


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lam128")
    ap.add_argument("--scheme", default="rqm4", choices=["rqm4", "split2"])
    ap.add_argument("--cpu-seconds", type=float, default=5.0,
                    help="length of the one-thread oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", default="both", choices=["both", "f64", "f32"])
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default kernel variants instead of timing them first")
    ap.add_argument("--tune-file", default=None,
                    help="load the variant table from this file if it exists, else tune and save it there")
    ap.add_argument("--batch-replicas", type=int, default=256,
                    help="replicas in the batched-vs-plain comparison (0 skips it)")
    ap.add_argument("--batch-steps", type=int, default=20,
                    help="field steps timed for the semi-implicit, Edwards and one-at-a-time batch forms")
    ap.add_argument("--batch-run-steps", type=int, default=500,
                    help="field steps of the timed explicit batched run (the run length of the workload)")
    ap.add_argument("--no-edwards", action="store_true",
                    help="skip the side measurements (other scheme, storage modes, field update, walls, adjoint, Edwards)")
    ap.add_argument("--no-large", action="store_true", help="skip the 256^3 measurement")
    ap.add_argument("--large-cl-steps", type=int, default=200,
                    help="Langevin steps of the complex64 256^3 run (the run length of that workload)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run the library's plain copy kernel on this many MiB (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the sharded path "
              "is a design, not a build -- run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1204_5434_amd import binding, inputs

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    binding.load()
    w = inputs.WORKLOADS[args.workload]
    wp_np, wm_np = inputs.fields(w)
    wp = torch.from_numpy(wp_np).to("cuda")
    wm = torch.from_numpy(wm_np).to("cuda")
    scheme = binding.PFT_RQM4 if args.scheme == "rqm4" else binding.PFT_SPLIT2
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 16
        a = torch.zeros(n, dtype=torch.complex128, device="cuda")
        b = torch.empty_like(a)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        binding.pft_copy_probe(a, b)
        ev[0].record()
        for _ in range(2):
            binding.pft_copy_probe(a, b)
        ev[1].record()
        torch.cuda.synchronize()
        copy_gbs = 2 * 2 * a.numel() * 16 / (ev[0].elapsed_time(ev[1]) * 1e-3) / 1e9
        log(f"[bench] copy probe: 3 x {args.copy_probe_mib} MiB, {copy_gbs:.0f} GB/s (read + write)")
        del a, b
    tuned = None
    if args.tune_file and os.path.exists(args.tune_file):
        binding.pft_tune_load(args.tune_file)
        tuned = {"loaded": args.tune_file}
        log(f"[bench] kernel variants loaded from {args.tune_file}")
    elif not args.no_autotune:
        sizes = set(w.n) | ({24, 32, 40, 48} if args.batch_replicas > 0 else set())
        if not args.no_edwards:  # the side legs' grids: 64^3 Langevin, 96^3 reverse mode, 256^3
            sizes |= {64, 96} | (set() if args.no_large else {256})
        sizes = sorted(sizes)
        tuned = {}
        for name, prec in (("f64", binding.PFT_C128), ("f32", binding.PFT_C64)):
            choice, times = binding.pft_autotune(prec, sizes)
            tuned[name] = {str(n): {"z": c[0], "x": c[1], "y": c[2]} for n, c in choice.items()}
        log(f"[bench] autotuned kernel variants: {tuned}")
        if args.tune_file:
            binding.pft_tune_save(args.tune_file)
    res = {}
    precisions = ("f64", "f32") if args.precision == "both" else (args.precision,)
    for precision in precisions:
        log(f"[bench] {w.name} {precision} {args.scheme}: warmup {args.warmup}, steps {args.steps}")
        res[precision] = run_precision(binding, w, wp, wm, precision, args.steps, args.warmup, scheme)
        log(f"[bench] {precision}: {res[precision]['ms_per_step']:.3f} ms/eval, "
            f"{res[precision]['value']:.3e} site-steps/s, roofline {res[precision]['roofline']}")
    other = None
    if not args.no_edwards:
        oname = "split2" if args.scheme == "rqm4" else "rqm4"
        osch = binding.PFT_SPLIT2 if oname == "split2" else binding.PFT_RQM4
        other = {"scheme": oname}
        for precision in precisions:
            r = run_precision(binding, w, wp, wm, precision, args.steps, args.warmup, osch)
            other[precision] = {"ms_per_step": r["ms_per_step"], "value": r["value"], "schedule": r["schedule"],
                                "roofline_frac": r["roofline"]["frac"], "kernel": r["roofline"]["kernel"]}
        log(f"[bench] other scheme: {other}")
    storage = None
    if not args.no_edwards:
        log("[bench] storage modes: q only in HBM, q staged in host memory")
        storage = storage_run(binding, w, wp, wm, max(2, args.steps // 4), 1)
        log(f"[bench] storage: {storage}")
    upd = None
    if not args.no_edwards:
        log("[bench] field step cost: explicit vs semi-implicit update (FP64)")
        upd = update_cost(binding, w, wp, wm, max(2, args.steps // 4))
        log(f"[bench] field update: {upd}")
    walls = None
    if not args.no_edwards:
        log("[bench] walled boxes: reflecting film, absorbing box")
        walls = walls_run(binding, w, wp, wm, max(2, args.steps // 4), 1)
        log(f"[bench] walls: {walls}")
    adjoint = None
    if not args.no_edwards:
        log("[bench] reverse mode at 96^3, Ns = 128")
        adjoint = adjoint_run(binding, inputs, max(2, args.steps // 4))
        log(f"[bench] adjoint: {adjoint}")
    edwards = None
    if not args.no_edwards:
        log("[bench] Edwards homopolymer model, 128^3, Ns = 100")
        edwards = edwards_run(binding, inputs, args.steps, args.warmup)
        log(f"[bench] edwards: {edwards}")
    langevin = None
    if not args.no_edwards:
        log("[bench] Langevin steps at 64^3, Ns = 100")
        langevin = langevin_run(binding, inputs, max(10, args.steps))
        log(f"[bench] langevin: {langevin}")
    large = None
    if not args.no_edwards and not args.no_large:
        log("[bench] large grid: 256^3, Ns = 200")
        large = large_grid_run(binding, inputs, max(2, args.steps // 4), args.large_cl_steps)
        log(f"[bench] large grid: {large}")
    batched = None
    if args.batch_replicas > 0:
        log(f"[bench] batched replicas: {args.batch_replicas}, {args.batch_steps} field steps")
        batched = batched_gain(binding, inputs, args.batch_replicas, args.batch_steps, args.batch_run_steps)
        log(f"[bench] batched: {batched}")
    cpu = cpu1 = legs = errors = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline: one full oracle evaluation, the 16^3 relaxation, one 64^3 step, "
            "the 48^3 reverse mode, a one-thread sample")
        gpu_results = {k: v["results"] for k, v in res.items()}
        cpu, cpu1, legs, errors = cpu_baseline(binding, inputs, w, wp_np, wm_np, gpu_results, args.cpu_seconds)
        log(f"[bench] cpu baseline: {cpu} {cpu1} {legs}")
        log(f"[bench] errors against the oracle: {errors}")
    main_ = res["f64"] if "f64" in res else res["f32"]
    line = {
        "metric": METRIC,
        "value": main_["value"],
        "unit": "grid-pts×steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_["ms_per_step"],
        "ms_per_step_one_stream": main_["ms_per_step_one_stream"],
        "ms_per_step_graph": main_["ms_per_step_graph"],
        "ms_per_evaluation_spread": main_["ms_per_evaluation_spread"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if "f64" in res else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": list(w.n), "box": list(w.L), "ns": w.ns, "f": w.f,
                   "chiN": w.chiN, "scheme": args.scheme, "site_steps_per_step": 2 * w.M * w.ns},
        "roofline": main_["roofline"],
        "cpu_baseline": cpu,
        "cpu_baseline_one_thread": cpu1,
        "cpu_legs": legs,
        "kernels": main_["kernels"],
        "schedule": main_["schedule"],
    }
    if "ms_per_step_by_schedule" in main_:
        line["ms_per_step_by_schedule"] = main_["ms_per_step_by_schedule"]
    if tuned is not None:
        line["kernel_variants"] = tuned
    if batched is not None:
        line["batched"] = batched
    if edwards is not None:
        line["edwards"] = edwards
    if upd is not None:
        line["field_update"] = upd
    if storage is not None:
        line["storage_modes"] = storage
    if walls is not None:
        line["walls"] = walls
    if other is not None:
        line["other_scheme"] = other
    if adjoint is not None:
        line["adjoint"] = adjoint
    if langevin is not None:
        line["langevin_64"] = langevin
    if large is not None:
        line["large_grid"] = large
    if errors is not None:
        line["error"] = {"vs": "FP64 oracle; one full evaluation of the workload (phi relative to max|phi|, "
                               "Q relative, H on |H| + C V); reverse mode on the reduced gradient state",
                         "f64": errors.get("f64"), "adjoint": errors.get("adjoint")}
    if "f64" in res and "f32" in res:
        line["fp32"] = {"value": res["f32"]["value"], "ms_per_step": res["f32"]["ms_per_step"],
                        "ms_per_step_one_stream": res["f32"]["ms_per_step_one_stream"],
                        "dtype": "f32 propagators, f64 sums", "roofline": res["f32"]["roofline"],
                        "kernels": res["f32"]["kernels"], "schedule": res["f32"]["schedule"],
                        "ms_per_step_graph": res["f32"]["ms_per_step_graph"],
                        "ms_per_evaluation_spread": res["f32"]["ms_per_evaluation_spread"]}
        if "ms_per_step_by_schedule" in res["f32"]:
            line["fp32"]["ms_per_step_by_schedule"] = res["f32"]["ms_per_step_by_schedule"]
        if errors is not None:
            line["fp32"]["error"] = dict(errors["f32"], adjoint=errors["adjoint"]["f32"])
    print(json.dumps(line))


if __name__ == "__main__":
    main()
