"""The benchmark's other 128^3 workloads at full size in its launch
configuration: the Edwards homopolymer evaluation (edw128) and the lamellar
workload between walls (reflecting walls normal to z; absorbing walls on every
axis).  Checked by one-step parity of the GPU's own stored slices against the
oracle's step and by the exact invariants at full size: every node pair gives
Q, and the densities sum to the number of sites.  (The oracle's walled
transforms follow their O(N^2) definitions, too slow for whole walled 128^3
sweeps; the full Edwards evaluation is compared with the oracle's in
test_gpu_fullsize_oracle.py.)"""
import numpy as np
import pytest
import torch

from paper_1204_5434_amd import binding as B
from paper_1204_5434_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def say(*a):
    print(*a, flush=True)


def host(t):
    return t.detach().cpu().numpy()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def one_step_checks(orc, ctx, p_or, steps, fields_of_step, h, tol):
    n = (p_or.nx, p_or.ny, p_or.nz)
    qj = torch.empty(n, dtype=torch.complex128, device=DEV)
    qj1 = torch.empty_like(qj)
    K = ctx.K
    for which, j in steps:
        si = j if which == 0 else K - 1 - j
        say("  one-step check", which, j)
        ctx.pft_get_slice(which, j, qj)
        ctx.pft_get_slice(which, j + 1, qj1)
        ref = orc.step(p_or, h[si], fields_of_step(si), host(qj))
        assert np.abs(host(qj1) - ref).max() <= tol * np.abs(ref).max(), (which, j)


def invariants(ctx, out, M, prec):
    K = ctx.K
    qn = torch.empty(K + 1, dtype=torch.complex128, device=DEV)
    ctx.pft_node_q(qn)
    Q = host(out["Q"])[0]
    tol = 1e-11 if prec == B.PFT_C128 else 1e-5
    assert np.abs(host(qn) - Q).max() <= tol * abs(Q)
    assert abs(host(out["phiA"] + out["phiB"]).sum() - M) <= tol * M
    assert ctx.pft_status_flags() == 0


@pytest.mark.parametrize("prec", [B.PFT_C128, B.PFT_C64])
def test_full_size_edw128_sampled(orc, prec):
    w = inputs.EDW128
    say("full size", w.name, "precision", prec)
    om = inputs.fields(w)[0]
    Bv = w.extra["B"]
    ctx = B.Context(B.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, prec, B.PFT_RQM4, B.PFT_EDWARDS, Bv))
    out = ctx.evaluate(dev(om))
    p_or = orc.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, 0, False)
    h = np.full(w.ns, 1.0 / w.ns)
    field = 1j * om  # the propagator sees w = i omega
    tol = 1e-12 if prec == B.PFT_C128 else 2e-5
    one_step_checks(orc, ctx, p_or, ((0, 0), (0, ctx.K // 2), (0, ctx.K - 1)), lambda si: field, h, tol)
    invariants(ctx, out, w.M, prec)
    ctx.close()


@pytest.mark.parametrize("bc", [(0, 0, 1), (2, 2, 2)], ids=["film_z_reflecting", "box_absorbing"])
@pytest.mark.parametrize("prec", [B.PFT_C128, B.PFT_C64])
def test_full_size_walls_sampled(orc, prec, bc):
    w = inputs.LAM128
    say("full size", w.name, "walls", bc, "precision", prec)
    wp, wm = inputs.fields(w)
    ctx = B.Context(B.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, prec, B.PFT_RQM4, B.PFT_DIBLOCK, 0.0,
                             B.PFT_STORE_BOTH, bc))
    out = ctx.evaluate(dev(wp), dev(wm))
    p_or = orc.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, 0, False, bc)
    wA, wB = orc.block_fields(p_or, wp, wm)
    h, blk, _ = orc.contour(w.ns, w.f)
    tol = 1e-12 if prec == B.PFT_C128 else 2e-5
    one_step_checks(orc, ctx, p_or, ((0, 0), (1, ctx.K - 1)), lambda si: wA if blk[si] == 0 else wB, h, tol)
    invariants(ctx, out, w.M, prec)
    ctx.close()
