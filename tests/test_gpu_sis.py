"""GPU parity of the semi-implicit field step (Eqs. (10)-(11), pft_step.update
= 1) against the oracle.

The step runs in FP64 on the fields whatever the propagator precision, so it is
checked twice: against the oracle's step applied to the densities the GPU
itself produced (isolates the reciprocal-space filter: 1e-12), and end to end
against the oracle's evaluation + step (the evaluation's own bars).  Shapes
cover one-lane (8..20) and multi-lane (24..256) line transforms on every axis.
"""
import numpy as np
import pytest
import torch

from paper_1204_5434_amd import binding as B
from paper_1204_5434_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def fields(shape, seed):
    r = np.random.default_rng(seed)
    wp = 0.3 * r.standard_normal(shape) + 0.05j * r.standard_normal(shape)
    wm = 0.4 * r.standard_normal(shape) + 0.05j * r.standard_normal(shape)
    return wp, wm


SHAPES = [
    ((8, 12, 20), (2.0, 3.0, 5.0)),
    ((24, 32, 40), (3.0, 4.0, 5.0)),
    ((48, 16, 96), (6.0, 2.0, 12.0)),
    ((128, 8, 16), (16.0, 1.0, 2.0)),
    ((16, 256, 12), (2.0, 32.0, 1.5)),
    ((20, 64, 192), (2.5, 8.0, 24.0)),
]


@pytest.mark.parametrize("shape,L", SHAPES, ids=[str(s[0]) for s in SHAPES])
@pytest.mark.parametrize("noise", [0, 1])
def test_sis_step_matches_oracle(orc, shape, L, noise):
    say("sis", shape, noise)
    ns, f, chiN, C = 12, 0.4, 16.0, 3.0
    wp, wm = fields(shape, 60 + sum(shape))
    p_or = orc.Params(*shape, *L, ns, f, chiN, C, 0, False)
    ctx = B.Context(B.Params(*shape, *L, ns, f, chiN, C, B.PFT_C128, B.PFT_RQM4))
    gwp, gwm = dev(wp), dev(wm)
    pa = torch.empty(shape, dtype=torch.complex128, device=DEV)
    pb = torch.empty_like(pa)
    st = B.pft_step(0.8, 1.0, 0.7, 11, 2, 3, noise, 1)
    ctx.pft_cl_step(gwp, gwm, st, pa, pb)
    # the filter alone: the oracle's step on the GPU's densities
    np_, nm_ = orc.sis_update(p_or, wp, wm, host(pa), host(pb), 0.8, 1.0, 0.7, noise=bool(noise),
                              seed=11, replica=2, step_=3)
    scale = max(np.abs(np_).max(), np.abs(nm_).max())
    assert np.abs(host(gwp) - np_).max() <= 1e-12 * scale
    assert np.abs(host(gwm) - nm_).max() <= 1e-12 * scale
    # end to end
    ref = orc.evaluate(p_or, wp, wm)
    ep, em = orc.sis_update(p_or, wp, wm, ref["phiA"], ref["phiB"], 0.8, 1.0, 0.7, noise=bool(noise),
                            seed=11, replica=2, step_=3)
    assert np.abs(host(gwp) - ep).max() <= 1e-10 * scale
    assert np.abs(host(gwm) - em).max() <= 1e-10 * scale
    ctx.close()


@pytest.mark.parametrize("prec,tol", [(B.PFT_C128, 1e-10), (B.PFT_C64, 2e-5)])
def test_sis_edwards_step(orc, prec, tol):
    shape, L, ns, C, Bv = (24, 20, 32), (3.0, 2.5, 4.0), 16, 4.0, 1.5
    r = np.random.default_rng(61)
    om = 0.3 * r.standard_normal(shape) + 0.05j * r.standard_normal(shape)
    p_or = orc.Params(*shape, *L, ns, 0.5, 1.0, C, 0, False)
    ctx = B.Context(B.Params(*shape, *L, ns, 0.5, 1.0, C, prec, B.PFT_RQM4, B.PFT_EDWARDS, Bv))
    g = dev(om)
    phi = torch.empty(shape, dtype=torch.complex128, device=DEV)
    ctx.pft_cl_step(g, None, B.pft_step(0.5, 1.2, 1.0, 4, 0, 1, 1, 1), phi)
    filt = orc.edwards_sis_update(p_or, Bv, om, host(phi), 0.5, 1.2, noise=True, seed=4, replica=0, step_=1)
    scale = np.abs(filt).max()
    assert np.abs(host(g) - filt).max() <= 1e-12 * scale
    ref = orc.edwards_evaluate(p_or, Bv, om)
    e2e = orc.edwards_sis_update(p_or, Bv, om, ref["phi"], 0.5, 1.2, noise=True, seed=4, replica=0, step_=1)
    assert np.abs(host(g) - e2e).max() <= tol * scale


def test_sis_scft_relaxation_large_steps(orc):
    """SCFT relaxation at a step 20x the explicit one: the semi-implicit
    trajectory tracks the oracle's and the force decays."""
    w = inputs.SCFT16
    wp, wm = inputs.fields(w)
    dt = 20 * w.dt
    p_or = orc.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, 0, False)
    ctx = B.Context(B.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, B.PFT_C128, B.PFT_RQM4))
    gwp, gwm = dev(wp), dev(wm)
    pa = torch.empty(w.n, dtype=torch.complex128, device=DEV)
    pb = torch.empty_like(pa)
    st = B.pft_step(dt, 1.0, 1.0, 0, 0, 0, 0, 1)
    norms = []
    for it in range(12):
        ref = orc.evaluate(p_or, wp, wm)
        ctx.pft_cl_step(gwp, gwm, st, pa, pb)
        assert np.abs(host(pa) - ref["phiA"]).max() <= 1e-10, it
        Fp, Fm = orc.forces(p_or, wm, ref["phiA"], ref["phiB"])
        norms.append(np.sqrt(np.mean(np.abs(Fp) ** 2 + np.abs(Fm) ** 2)))
        wp, wm = orc.sis_update(p_or, wp, wm, ref["phiA"], ref["phiB"], dt)
        assert np.abs(host(gwp) - wp).max() <= 1e-10 and np.abs(host(gwm) - wm).max() <= 1e-10, it
    assert norms[-1] < 0.5 * norms[0]
