"""Batched replicas: one launch per pass over replicas of uneven grid, contour
step count, f and chi N, with the field step captured in a HIP graph.  Checked
against independent single contexts (same kernels, one replica at a time), the
oracle, and the single-context Langevin step with the same noise stream."""
import numpy as np
import pytest
import torch

from paper_1204_5434_amd import binding as B
from paper_1204_5434_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def replica_set(count, seed, prec):
    reps = inputs.batch_replicas(count, seed)
    params = [B.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, prec, B.PFT_RQM4) for w in reps]
    fields = [inputs.fields(w) for w in reps]
    return reps, params, fields


@pytest.mark.parametrize("prec", [B.PFT_C128, B.PFT_C64])
def test_batch_evaluate_matches_single_and_oracle(orc, prec):
    reps, params, fields = replica_set(10, 77, prec)
    n = len(reps)
    bat = B.Batch(params)
    wp = [dev(f[0]) for f in fields]
    wm = [dev(f[1]) for f in fields]
    pa = [torch.empty(w.n, dtype=torch.complex128, device=DEV) for w in reps]
    pb = [torch.empty_like(t) for t in pa]
    Q = torch.empty(n, dtype=torch.complex128, device=DEV)
    H = torch.empty_like(Q)
    bat.pft_batch_evaluate(wp, wm, pa, pb, Q, H)
    bat.pft_batch_sync()
    for r, w in enumerate(reps):
        print("replica", r, w.n, w.ns, round(w.f, 3), flush=True)
        ctx = B.Context(params[r])
        out = ctx.evaluate(wp[r], wm[r])
        assert np.abs(host(pa[r]) - host(out["phiA"])).max() <= 1e-13
        assert abs(host(Q)[r] - host(out["Q"])[0]) <= 1e-13 * abs(host(out["Q"])[0])
        ctx.close()
        if r < 4:  # the oracle on a subset (it is slow at 48^3)
            ref = orc.evaluate(orc.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, 0, False), *fields[r])
            tol = 1e-10 if prec == B.PFT_C128 else 2e-5
            assert np.abs(host(pa[r]) - ref["phiA"]).max() <= tol * np.abs(ref["phiA"]).max()
            assert abs(host(Q)[r] - ref["Q"]) <= tol * abs(ref["Q"])
            V = np.prod(w.L)
            assert abs(host(H)[r] - ref["H"]) <= tol * (abs(ref["H"]) + w.C * V)


def test_batch_graph_steps_match_single_steps():
    reps, params, fields = replica_set(6, 78, B.PFT_C128)
    n = len(reps)
    bat = B.Batch(params)
    wp = [dev(f[0]) for f in fields]
    wm = [dev(f[1]) for f in fields]
    log = torch.zeros((5, n, 2), dtype=torch.complex128, device=DEV)
    st = B.pft_step(0.01, 1.0, 1.0, 1208, 100, 7, 1)
    bat.pft_batch_cl_steps(wp, wm, st, 2, log)   # captures the graph, replays twice
    st2 = B.pft_step(0.01, 1.0, 1.0, 1208, 100, 9, 1)
    bat.pft_batch_cl_steps(wp, wm, st2, 2, None)  # re-capture (no log), steps 9 and 10
    bat.pft_batch_sync()
    for r, w in enumerate(reps):
        ctx = B.Context(params[r])
        a, b = dev(fields[r][0]), dev(fields[r][1])
        Qs, Hs = [], []
        Qt = torch.empty(1, dtype=torch.complex128, device=DEV)
        Ht = torch.empty_like(Qt)
        for k, stepno in enumerate((7, 8, 9, 10)):
            ctx.pft_cl_step(a, b, B.pft_step(0.01, 1.0, 1.0, 1208, 100 + r, stepno, 1), None, None, Qt, Ht)
            Qs.append(complex(host(Qt)[0]))
            Hs.append(complex(host(Ht)[0]))
        assert np.abs(host(wp[r]) - host(a)).max() <= 1e-12 * np.abs(host(a)).max()
        assert np.abs(host(wm[r]) - host(b)).max() <= 1e-12 * np.abs(host(b)).max()
        lg = host(log)
        for k in range(2):
            assert abs(lg[k, r, 0] - Qs[k]) <= 1e-12 * abs(Qs[k])
            assert abs(lg[k, r, 1] - Hs[k]) <= 1e-12 * (abs(Hs[k]) + w.C * np.prod(w.L))
        assert np.all(lg[2:] == 0)
        ctx.close()


@pytest.mark.parametrize("prec", [B.PFT_C128, B.PFT_C64])
def test_batch_semi_implicit_steps_match_single_steps(prec):
    """Semi-implicit steps (Eqs. (10)-(11)) in a batch graph, then an explicit
    step (a new capture), against the single-context sequence with the same
    noise stream."""
    reps, params, fields = replica_set(5, 79, prec)
    n = len(reps)
    bat = B.Batch(params)
    wp = [dev(f[0]) for f in fields]
    wm = [dev(f[1]) for f in fields]
    log = torch.zeros((3, n, 2), dtype=torch.complex128, device=DEV)
    bat.pft_batch_cl_steps(wp, wm, B.pft_step(0.05, 1.0, 0.8, 31, 200, 4, 1, 1), 2, log)
    bat.pft_batch_cl_steps(wp, wm, B.pft_step(0.05, 1.0, 0.8, 31, 200, 6, 1, 0), 1, None)
    bat.pft_batch_sync()
    for r, w in enumerate(reps):
        print("replica", r, w.n, w.ns, flush=True)
        ctx = B.Context(params[r])
        a, b = dev(fields[r][0]), dev(fields[r][1])
        Qt = torch.empty(1, dtype=torch.complex128, device=DEV)
        Ht = torch.empty_like(Qt)
        Qs, Hs = [], []
        for stepno, upd in ((4, 1), (5, 1), (6, 0)):
            ctx.pft_cl_step(a, b, B.pft_step(0.05, 1.0, 0.8, 31, 200 + r, stepno, 1, upd), None, None, Qt, Ht)
            Qs.append(complex(host(Qt)[0]))
            Hs.append(complex(host(Ht)[0]))
        assert np.abs(host(wp[r]) - host(a)).max() <= 1e-12 * np.abs(host(a)).max()
        assert np.abs(host(wm[r]) - host(b)).max() <= 1e-12 * np.abs(host(b)).max()
        lg = host(log)
        for k in range(2):
            assert abs(lg[k, r, 0] - Qs[k]) <= 1e-12 * abs(Qs[k])
            assert abs(lg[k, r, 1] - Hs[k]) <= 1e-12 * (abs(Hs[k]) + w.C * np.prod(w.L))
        ctx.close()


def test_batch_rejects_unknown_update():
    reps, params, fields = replica_set(2, 80, B.PFT_C128)
    bat = B.Batch(params)
    wp = [dev(f[0]) for f in fields]
    wm = [dev(f[1]) for f in fields]
    with pytest.raises(B.PftError):
        bat.pft_batch_cl_steps(wp, wm, B.pft_step(0.05, 1.0, 0.8, 31, 200, 4, 1, 2), 1, None)


def test_batch_semi_implicit_per_replica_boxes():
    """Replicas that share a grid (one launch group) but not a box: each takes
    the filter of its own k grid (and the Debye function at its own |k|^2)."""
    W = inputs.Workload
    reps = [W("a", (32, 24, 40), (3.0, 2.5, 5.0), 30, 0.4, 15.0, C=20.0, seed=5),
            W("b", (32, 24, 40), (4.5, 3.0, 3.5), 44, 0.35, 18.0, C=20.0, seed=6),
            W("c", (24, 24, 24), (3.0, 3.0, 3.0), 36, 0.45, 13.0, C=20.0, seed=7),
            W("d", (32, 24, 40), (2.0, 6.0, 4.0), 25, 0.5, 20.0, C=20.0, seed=8)]
    params = [B.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, B.PFT_C128, B.PFT_RQM4) for w in reps]
    fields = [inputs.fields(w) for w in reps]
    bat = B.Batch(params)
    wp = [dev(f[0]) for f in fields]
    wm = [dev(f[1]) for f in fields]
    bat.pft_batch_cl_steps(wp, wm, B.pft_step(0.2, 1.0, 0.5, 9, 40, 0, 1, 1), 3, None)
    bat.pft_batch_sync()
    for r, w in enumerate(reps):
        print("replica", r, w.n, w.L, flush=True)
        ctx = B.Context(params[r])
        a, b = dev(fields[r][0]), dev(fields[r][1])
        for stepno in range(3):
            ctx.pft_cl_step(a, b, B.pft_step(0.2, 1.0, 0.5, 9, 40 + r, stepno, 1, 1))
        assert np.abs(host(wp[r]) - host(a)).max() <= 1e-12 * np.abs(host(a)).max()
        assert np.abs(host(wm[r]) - host(b)).max() <= 1e-12 * np.abs(host(b)).max()
        ctx.close()


def single_like_batch(params, bc):
    """A single context on the schedule its replica runs in a batch: batched
    groups with walls along y or z run the axis schedule, where a single
    complex-float context may take the fused one (equal to rounding)."""
    ctx = B.Context(params)
    if (bc[1] or bc[2]) and ctx.pft_fused_planes():
        ctx.pft_set_fused_planes(0)
    return ctx


@pytest.mark.parametrize("prec", [B.PFT_C128, B.PFT_C64])
def test_batch_walls_match_single_and_oracle(orc, prec):
    """Walled replicas in a batch (grouped by grid and walls; a fused group
    with a walled x axis among them): evaluations and graph-replayed explicit
    steps equal those of single walled contexts, and the oracle on a subset."""
    W = inputs.Workload
    reps = [W("a", (24, 24, 24), (3.0, 3.0, 3.5), 30, 0.4, 15.0, C=20.0, seed=11),
            W("b", (24, 24, 24), (3.0, 3.0, 3.5), 30, 0.4, 15.0, C=20.0, seed=12),
            W("c", (32, 24, 40), (4.0, 3.0, 5.0), 41, 0.35, 18.0, C=20.0, seed=13),
            W("d", (24, 24, 24), (2.5, 3.5, 3.0), 44, 0.45, 13.0, C=20.0, seed=14),
            W("e", (16, 16, 16), (2.0, 2.0, 2.0), 25, 0.5, 14.0, C=20.0, seed=15)]
    bcs = [(0, 0, 1), (0, 0, 0), (2, 1, 0), (0, 0, 1), (1, 0, 0)]
    params = [B.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, prec, B.PFT_RQM4, B.PFT_DIBLOCK, 0.0,
                       B.PFT_STORE_BOTH, bc) for w, bc in zip(reps, bcs)]
    fields = [inputs.fields(w) for w in reps]
    n = len(reps)
    bat = B.Batch(params)
    wp = [dev(f[0]) for f in fields]
    wm = [dev(f[1]) for f in fields]
    pa = [torch.empty(w.n, dtype=torch.complex128, device=DEV) for w in reps]
    pb = [torch.empty_like(t) for t in pa]
    Q = torch.empty(n, dtype=torch.complex128, device=DEV)
    H = torch.empty_like(Q)
    bat.pft_batch_evaluate(wp, wm, pa, pb, Q, H)
    log = torch.zeros((2, n, 2), dtype=torch.complex128, device=DEV)
    bat.pft_batch_cl_steps(wp, wm, B.pft_step(0.01, 1.0, 1.0, 5, 300, 0, 1), 2, log)
    bat.pft_batch_sync()
    tol = 1e-10 if prec == B.PFT_C128 else 2e-5
    for r, w in enumerate(reps):
        print("replica", r, w.n, bcs[r], flush=True)
        ctx = single_like_batch(params[r], bcs[r])
        out = ctx.evaluate(dev(fields[r][0]), dev(fields[r][1]))
        assert np.abs(host(pa[r]) - host(out["phiA"])).max() <= 1e-13
        assert np.abs(host(pb[r]) - host(out["phiB"])).max() <= 1e-13
        assert abs(host(Q)[r] - host(out["Q"])[0]) <= 1e-13 * abs(host(out["Q"])[0])
        if r in (0, 2, 4):
            ref = orc.evaluate(orc.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, 0, False, bcs[r]), *fields[r])
            assert np.abs(host(pa[r]) - ref["phiA"]).max() <= tol * np.abs(ref["phiA"]).max()
            assert abs(host(Q)[r] - ref["Q"]) <= tol * abs(ref["Q"])
            assert abs(host(H)[r] - ref["H"]) <= tol * (abs(ref["H"]) + w.C * np.prod(w.L))
        a, b = dev(fields[r][0]), dev(fields[r][1])
        Qt = torch.empty(1, dtype=torch.complex128, device=DEV)
        for stepno in range(2):
            ctx.pft_cl_step(a, b, B.pft_step(0.01, 1.0, 1.0, 5, 300 + r, stepno, 1), None, None, Qt)
            assert abs(host(log)[stepno, r, 0] - host(Qt)[0]) <= 1e-12 * abs(host(Qt)[0])
        assert np.abs(host(wp[r]) - host(a)).max() <= 1e-12 * np.abs(host(a)).max()
        assert np.abs(host(wm[r]) - host(b)).max() <= 1e-12 * np.abs(host(b)).max()
        ctx.close()


@pytest.mark.parametrize("model", [B.PFT_DIBLOCK, B.PFT_EDWARDS])
@pytest.mark.parametrize("prec", [B.PFT_C128, B.PFT_C64])
def test_batch_semi_implicit_between_reflecting_walls(prec, model):
    """Batched semi-implicit steps with reflecting walls (the filter on each
    replica's even image, one launch per pass over a group) equal the
    single-context steps, periodic replicas of the same grid included; both
    precisions, diblock and Edwards replicas."""
    W = inputs.Workload
    reps = [W("a", (16, 24, 20), (2.0, 3.0, 2.5), 30, 0.4, 15.0, C=20.0, seed=21),
            W("b", (24, 24, 24), (3.0, 3.0, 3.0), 36, 0.45, 16.0, C=20.0, seed=22),
            W("c", (24, 24, 24), (3.0, 3.0, 3.0), 28, 0.35, 14.0, C=20.0, seed=23),
            W("d", (16, 24, 20), (2.5, 2.0, 3.0), 33, 0.5, 18.0, C=20.0, seed=24)]
    bcs = [(1, 0, 1), (0, 0, 1), (0, 0, 0), (1, 0, 1)]
    ed = model == B.PFT_EDWARDS
    params = [B.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, prec, B.PFT_RQM4, model, 1.3 if ed else 0.0,
                       B.PFT_STORE_BOTH, bc) for w, bc in zip(reps, bcs)]
    fields = [inputs.fields(w) for w in reps]
    bat = B.Batch(params)
    wp = [dev(f[0]) for f in fields]
    wm = None if ed else [dev(f[1]) for f in fields]
    bat.pft_batch_cl_steps(wp, wm, B.pft_step(0.2, 1.0, 0.5, 17, 60, 0, 1, 1), 2, None)
    bat.pft_batch_sync()
    for r, w in enumerate(reps):
        print("replica", r, w.n, bcs[r], flush=True)
        ctx = single_like_batch(params[r], bcs[r])
        a = dev(fields[r][0])
        b = None if ed else dev(fields[r][1])
        for stepno in range(2):
            ctx.pft_cl_step(a, b, B.pft_step(0.2, 1.0, 0.5, 17, 60 + r, stepno, 1, 1))
        assert np.abs(host(wp[r]) - host(a)).max() <= 1e-12 * np.abs(host(a)).max()
        if not ed:
            assert np.abs(host(wm[r]) - host(b)).max() <= 1e-12 * np.abs(host(b)).max()
        ctx.close()


@pytest.mark.parametrize("model", [B.PFT_DIBLOCK, B.PFT_EDWARDS])
@pytest.mark.parametrize("prec", [B.PFT_C128, B.PFT_C64])
def test_batch_plain_split_matches_single(model, prec):
    """The plain split step (two strided passes per step) in batches, periodic
    and walled groups, diblock and Edwards: evaluations and graph-replayed
    explicit steps equal single contexts."""
    specs = [((24, 24, 24), (3.0, 3.0, 3.0), 30, (0, 0, 0)),
             ((16, 24, 20), (2.0, 3.0, 2.5), 21, (1, 0, 2)),
             ((24, 24, 24), (2.5, 3.5, 3.0), 37, (0, 0, 0))]
    params = [B.Params(*n, *L, ns, 0.4, 15.0, 10.0, prec, B.PFT_SPLIT2, model,
                       1.2 if model == B.PFT_EDWARDS else 0.0, B.PFT_STORE_BOTH, bc) for n, L, ns, bc in specs]
    rng = np.random.default_rng(31)
    fl = [(0.3 * rng.standard_normal(s[0]) + 0.05j * rng.standard_normal(s[0]),
           0.4 * rng.standard_normal(s[0]) + 0.05j * rng.standard_normal(s[0])) for s in specs]
    ed = model == B.PFT_EDWARDS
    k = len(specs)
    bat = B.Batch(params)
    wp = [dev(f[0]) for f in fl]
    wm = None if ed else [dev(f[1]) for f in fl]
    pa = [torch.empty(s[0], dtype=torch.complex128, device=DEV) for s in specs]
    pb = [torch.empty_like(t) for t in pa]
    Q = torch.empty(k, dtype=torch.complex128, device=DEV)
    H = torch.empty_like(Q)
    bat.pft_batch_evaluate(wp, wm, pa, pb, Q, H)
    bat.pft_batch_sync()
    for r in range(k):
        ctx = B.Context(params[r])
        out = ctx.evaluate(dev(fl[r][0]), None if ed else dev(fl[r][1]))
        assert np.abs(host(pa[r]) - host(out["phiA"])).max() <= 1e-13
        assert abs(host(Q)[r] - host(out["Q"])[0]) <= 1e-13 * abs(host(out["Q"])[0])
        assert abs(host(H)[r] - host(out["H"])[0]) <= 1e-12 * (abs(host(out["H"])[0]) + 10.0 * np.prod(specs[r][1]))
        ctx.close()
    bat.pft_batch_cl_steps(wp, wm, B.pft_step(0.01, 1.0, 1.0, 3, 80, 0, 1), 2, None)
    bat.pft_batch_sync()
    for r in range(k):
        print("replica", r, specs[r][0], specs[r][3], flush=True)
        ctx = B.Context(params[r])
        a = dev(fl[r][0])
        b = None if ed else dev(fl[r][1])
        for stepno in range(2):
            ctx.pft_cl_step(a, b, B.pft_step(0.01, 1.0, 1.0, 3, 80 + r, stepno, 1))
        assert np.abs(host(wp[r]) - host(a)).max() <= 1e-12 * np.abs(host(a)).max()
        if not ed:
            assert np.abs(host(wm[r]) - host(b)).max() <= 1e-12 * np.abs(host(b)).max()
        ctx.close()


def test_batch_unsynced_calls_with_changing_pointers():
    """Evaluations into new output buffers and re-captured field steps issued
    back to back without a sync: each call's job tables are rewritten only
    after the batch's queued work has drained, so every call lands in its own
    buffers with the values of single contexts."""
    reps, params, fields = replica_set(6, 81, B.PFT_C64)
    n = len(reps)
    bat = B.Batch(params)
    wp = [dev(f[0]) for f in fields]
    wm = [dev(f[1]) for f in fields]

    def outputs():
        pa = [torch.full(w.n, np.nan, dtype=torch.complex128, device=DEV) for w in reps]
        pb = [torch.full(w.n, np.nan, dtype=torch.complex128, device=DEV) for w in reps]
        return pa, pb, torch.zeros(n, dtype=torch.complex128, device=DEV), torch.zeros(n, dtype=torch.complex128, device=DEV)

    o1, o2, o3 = outputs(), outputs(), outputs()
    bat.pft_batch_evaluate(wp, wm, *o1)
    bat.pft_batch_evaluate(wp, wm, *o2)              # new pointers, no sync
    wp2 = [t.clone() for t in wp]
    wm2 = [t.clone() for t in wm]
    log = torch.zeros((2, n, 2), dtype=torch.complex128, device=DEV)
    bat.pft_batch_cl_steps(wp2, wm2, B.pft_step(0.01, 1.0, 1.0, 9, 0, 0, 1), 2, log)   # capture
    bat.pft_batch_evaluate(wp2, wm2, *o3)            # the stepped fields, new pointers
    wp3 = [t.clone() for t in wp]
    wm3 = [t.clone() for t in wm]
    bat.pft_batch_cl_steps(wp3, wm3, B.pft_step(0.01, 1.0, 1.0, 9, 0, 0, 1), 1, None)  # re-capture
    bat.pft_batch_sync()
    for r, w in enumerate(reps):
        ctx = B.Context(params[r])
        ref = ctx.evaluate(wp[r], wm[r])
        for o in (o1, o2):
            assert np.abs(host(o[0][r]) - host(ref["phiA"])).max() <= 1e-13
            assert np.abs(host(o[1][r]) - host(ref["phiB"])).max() <= 1e-13
            assert abs(host(o[2])[r] - host(ref["Q"])[0]) <= 1e-13 * abs(host(ref["Q"])[0])
        a, b = wp[r].clone(), wm[r].clone()
        Qt = torch.empty(1, dtype=torch.complex128, device=DEV)
        for stepno in range(2):
            ctx.pft_cl_step(a, b, B.pft_step(0.01, 1.0, 1.0, 9, r, stepno, 1), None, None, Qt)
            assert abs(host(log)[stepno, r, 0] - host(Qt)[0]) <= 1e-12 * abs(host(Qt)[0])
            if stepno == 0:
                assert np.abs(host(wp3[r]) - host(a)).max() <= 1e-12 * np.abs(host(a)).max()
        assert np.abs(host(wp2[r]) - host(a)).max() <= 1e-12 * np.abs(host(a)).max()
        ref2 = ctx.evaluate(a, b)
        assert np.abs(host(o3[0][r]) - host(ref2["phiA"])).max() <= 1e-13
        assert abs(host(o3[2])[r] - host(ref2["Q"])[0]) <= 1e-13 * abs(host(ref2["Q"])[0])
        ctx.close()
