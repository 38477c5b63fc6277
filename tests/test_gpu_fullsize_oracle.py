"""End-to-end parity at full size against one full oracle run.

- The benchmark workload (lamellar cell, 128^3, Ns = 100, Richardson step of
  Eq. (12)), in the launch configuration the benchmark times: every phi_A,
  phi_B, the per-node Q and H against the oracle's complete evaluation (both
  sweeps over all 101 nodes, FP64).
- The Edwards homopolymer workload (128^3, Ns = 100, one sweep with
  q-dagger = q): phi, Q and H against the oracle's complete evaluation.
- The gradient workload (96^3, Ns = 128, f = 0.3 so that the A/B junction
  falls inside a step, lamellar-plus-noise w-): dH/dw+, dH/dw- and dH/dL of the
  checkpointed reverse mode (every 11 nodes) against the oracle's reverse mode
  over the same split steps.

Each result's error is printed for both propagator precisions (FP32 error
against the FP64 oracle, per result).  Scales: phi relative to max|phi|; Q
relative; H on |H| + C V (Q's relative error reaches H as C V times it);
dH/dw relative to max|dH/dw|; dH/dL_a on |dH/dL_a| + C V / L_a (the same
log Q term, differentiated)."""
import os

import numpy as np
import pytest
import torch

from paper_1204_5434_amd import binding as B
from paper_1204_5434_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL = {B.PFT_C128: 1e-10, B.PFT_C64: 2e-5}
TOL_Q = {B.PFT_C128: 1e-11, B.PFT_C64: 2e-5}
NAME = {B.PFT_C128: "f64", B.PFT_C64: "f32"}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def report(what, prec, err, bar):
    print(f"ERROR {what} {NAME[prec]} {err:.3e} (bar {bar:.0e})", flush=True)


@pytest.fixture(scope="module")
def threads(orc):
    orc.set_threads(max(1, min(16, len(os.sched_getaffinity(0)))))


@pytest.fixture(scope="module")
def lam128(orc, threads):
    w = inputs.LAM128
    wp, wm = inputs.fields(w)
    print("oracle: full lam128 evaluation", flush=True)
    ref = orc.evaluate(orc.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, 0, False), wp, wm)
    return w, wp, wm, ref


@pytest.mark.parametrize("prec", [B.PFT_C128, B.PFT_C64])
def test_lam128_full_evaluation(lam128, prec):
    w, wp, wm, ref = lam128
    ctx = B.Context(B.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, prec, B.PFT_RQM4))
    out = ctx.evaluate(dev(wp), dev(wm))
    qn = torch.empty(ctx.K + 1, dtype=torch.complex128, device=DEV)
    ctx.pft_node_q(qn)
    tol, tq = TOL[prec], TOL_Q[prec]
    scale = max(np.abs(ref["phiA"]).max(), np.abs(ref["phiB"]).max())
    ea = np.abs(host(out["phiA"]) - ref["phiA"]).max() / scale
    eb = np.abs(host(out["phiB"]) - ref["phiB"]).max() / scale
    Q = host(out["Q"])[0]
    eq = abs(Q - ref["Q"]) / abs(ref["Q"])
    en = np.abs(host(qn) - ref["Qnode"]).max() / abs(ref["Q"])
    eh = abs(host(out["H"])[0] - ref["H"]) / (abs(ref["H"]) + w.C * np.prod(w.L))
    ehr = abs(host(out["H"])[0] - ref["H"]) / abs(ref["H"])
    for name, e, bar in (("phiA", ea, tol), ("phiB", eb, tol), ("Q", eq, tq), ("Qnode", en, tq),
                         ("H", eh, tq), ("H_relative_to_H", ehr, tq)):
        report("lam128 " + name, prec, e, bar)
    assert ea <= tol and eb <= tol
    assert eq <= tq and en <= tq and eh <= tq
    assert ctx.pft_status_flags() == 0
    ctx.close()


@pytest.fixture(scope="module")
def edw128(orc, threads):
    w = inputs.EDW128
    om = inputs.fields(w)[0]
    print("oracle: full edw128 evaluation", flush=True)
    ref = orc.edwards_evaluate(orc.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, 0, False), w.extra["B"], om)
    return w, om, ref


@pytest.mark.parametrize("prec", [B.PFT_C128, B.PFT_C64])
def test_edw128_full_evaluation(edw128, prec):
    w, om, ref = edw128
    ctx = B.Context(B.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, prec, B.PFT_RQM4, B.PFT_EDWARDS,
                             w.extra["B"]))
    out = ctx.evaluate(dev(om))
    tol, tq = TOL[prec], TOL_Q[prec]
    ep = np.abs(host(out["phiA"]) - ref["phi"]).max() / np.abs(ref["phi"]).max()
    Q = host(out["Q"])[0]
    eq = abs(Q - ref["Q"]) / abs(ref["Q"])
    eh = abs(host(out["H"])[0] - ref["H"]) / (abs(ref["H"]) + w.C * np.prod(w.L))
    for name, e, bar in (("phi", ep, tol), ("Q", eq, tq), ("H", eh, tq)):
        report("edw128 " + name, prec, e, bar)
    assert ep <= tol and eq <= tq and eh <= tq
    assert np.abs(host(out["phiB"])).max() == 0.0
    assert ctx.pft_status_flags() == 0
    ctx.close()


@pytest.fixture(scope="module")
def grad96(orc, threads):
    w = inputs.GRAD96
    wp, wm = inputs.fields(w)
    print("oracle: full grad96 reverse mode", flush=True)
    p = orc.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, 0, False)
    gp, gm, dL = orc.adjoint(p, wp, wm)
    H = orc.evaluate(p, wp, wm)["H"]
    return w, wp, wm, gp, gm, dL, H


@pytest.mark.parametrize("prec", [B.PFT_C128, B.PFT_C64])
def test_grad96_full_adjoint(grad96, prec):
    w, wp, wm, rp, rm, rL, rH = grad96
    ctx = B.Context(B.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, prec, B.PFT_RQM4))
    gp = torch.empty(w.n, dtype=torch.complex128, device=DEV)
    gm = torch.empty_like(gp)
    dL = torch.empty(3, dtype=torch.complex128, device=DEV)
    H = torch.empty(1, dtype=torch.complex128, device=DEV)
    ctx.pft_adjoint(dev(wp), dev(wm), gp, gm, dL, H, 11)
    tol = TOL[prec]
    V = np.prod(w.L)
    ep = np.abs(host(gp) - rp).max() / np.abs(rp).max()
    em = np.abs(host(gm) - rm).max() / np.abs(rm).max()
    eL = max(abs(host(dL)[a] - rL[a]) / (abs(rL[a]) + w.C * V / w.L[a]) for a in range(3))
    eLr = max(abs(host(dL)[a] - rL[a]) / abs(rL[a]) for a in range(3))
    eh = abs(host(H)[0] - rH) / (abs(rH) + w.C * V)
    for name, e in (("dH_dwplus", ep), ("dH_dwminus", em), ("dH_dL", eL), ("dH_dL_relative_to_dL", eLr),
                    ("H", eh)):
        report("grad96 " + name, prec, e, tol)
    assert ep <= tol and em <= tol and eL <= tol and eh <= TOL_Q[prec]
    ctx.close()
