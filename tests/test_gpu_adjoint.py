"""GPU reverse mode (pft_adjoint) against the oracle's reverse mode, finite
differences of the GPU's own H, the plain-split force identity, and PyTorch's
gradcheck through the autograd Function."""
import numpy as np
import pytest
import torch

from paper_1204_5434_amd import binding as B
from paper_1204_5434_amd import inputs
from paper_1204_5434_amd.autograd import hamiltonian

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
    wp = 0.3 * r.standard_normal(shape) + 0.1j * r.standard_normal(shape)
    wm = 0.5 * r.standard_normal(shape) + 0.1j * r.standard_normal(shape)
    return wp, wm


def gpu_adjoint(ctx, wp, wm, kc=0):
    gp = torch.empty(ctx.shape, dtype=torch.complex128, device=DEV)
    gm = torch.empty_like(gp)
    dL = torch.empty(3, dtype=torch.complex128, device=DEV)
    H = torch.empty(1, dtype=torch.complex128, device=DEV)
    ctx.pft_adjoint(wp, wm, gp, gm, dL, H, kc)
    return host(gp), host(gm), host(dL), complex(host(H)[0])


CASES = [
    # n, L, ns, f, chiN, C, scheme
    ((16, 12, 20), (4.0, 3.0, 5.0), 20, 0.5, 15.0, 2.0, 0),
    ((12, 16, 8), (3.0, 4.0, 2.0), 25, 0.3, 18.0, 1.0, 0),   # junction inside a step
    ((8, 12, 16), (2.0, 3.0, 4.0), 13, 0.62, 12.0, 1.0, 1),  # plain split + junction
    ((24, 8, 12), (6.0, 2.0, 3.0), 10, 0.4, 14.4, 3.0, 1),
    ((8, 8, 8), (2.0, 2.0, 2.0), 2, 0.5, 15.0, 1.0, 0),       # shortest contour
    ((12, 8, 16), (3.0, 2.0, 4.0), 10, 0.03, 15.0, 1.0, 0),   # junction inside the first step
    ((8, 12, 12), (2.0, 3.0, 3.0), 10, 0.97, 15.0, 2.0, 1),   # junction inside the last step
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-ns{c[2]}-f{c[3]}-s{c[6]}" for c in CASES])
@pytest.mark.parametrize("prec", [B.PFT_C128, B.PFT_C64])
def test_adjoint_matches_oracle(orc, case, prec):
    n, L, ns, f, chiN, C, scheme = case
    say("adjoint parity", case, prec)
    wp, wm = fields(n, 21)
    rp, rm, rL = orc.adjoint(orc.Params(*n, *L, ns, f, chiN, C, scheme, False), wp, wm)
    ctx = B.Context(B.Params(*n, *L, ns, f, chiN, C, prec, scheme))
    gp, gm, dL, _ = gpu_adjoint(ctx, dev(wp), dev(wm))
    tol = 1e-10 if prec == B.PFT_C128 else 2e-5
    assert np.abs(gp - rp).max() <= tol * np.abs(rp).max()
    assert np.abs(gm - rm).max() <= tol * np.abs(rm).max()
    # dH/dL_a = C dV S / L_a - C (V / L_a) log Q - ...: like H it is a difference
    # of extensive terms, so Q's relative error reaches it as C V / L_a times it.
    V = np.prod(L)
    for a in range(3):
        assert abs(dL[a] - rL[a]) <= tol * (abs(rL[a]) + C * V / L[a]), a
    assert ctx.pft_status_flags() == 0


@pytest.mark.parametrize("scheme", [0, 1])
def test_checkpoint_interval_is_exact(scheme):
    n, L = (16, 16, 12), (4.0, 4.0, 3.0)
    wp, wm = fields(n, 22)
    ctx = B.Context(B.Params(*n, *L, 23, 0.41, 15.0, 1.0, B.PFT_C128, scheme))
    ref = gpu_adjoint(ctx, dev(wp), dev(wm), kc=1)
    for kc in (0, 2, 7, 24):
        got = gpu_adjoint(ctx, dev(wp), dev(wm), kc=kc)
        for a, b in zip(got[:3], ref[:3]):
            assert np.array_equal(a, b), kc
    # segments recomputed in place on one stream instead of beside the
    # adjoint steps on a second one: the same numbers
    ctx.pft_set_concurrent_sweeps(False)
    for kc in (2, 7):
        got = gpu_adjoint(ctx, dev(wp), dev(wm), kc=kc)
        for a, b in zip(got[:3], ref[:3]):
            assert np.array_equal(a, b), ("one stream", kc)


def test_split2_gradient_is_the_force():
    n, L, C = (16, 12, 16), (4.0, 3.0, 4.0), 2.5
    wp, wm = fields(n, 23)
    ctx = B.Context(B.Params(*n, *L, 16, 0.37, 15.0, C, B.PFT_C128, B.PFT_SPLIT2))
    gp, gm, _, _ = gpu_adjoint(ctx, dev(wp), dev(wm))
    out = ctx.evaluate(dev(wp), dev(wm))
    pa, pb = host(out["phiA"]), host(out["phiB"])
    dV = np.prod(L) / np.prod(n)
    Fp = 1j * (pa + pb - 1)
    Fm = 2 * wm / 15.0 + pb - pa
    assert np.abs(gp - C * dV * Fp).max() <= 1e-12 * np.abs(gp).max()
    assert np.abs(gm - C * dV * Fm).max() <= 1e-12 * np.abs(gm).max()


def test_gradient_state_fd_and_force():
    """96^3, Ns = 128, f = 0.3 (junction), checkpoints every 11 steps: per-site
    4th-order differences of the GPU's own H at 64 sites, a directional
    difference along the lamellar mode, and the analytic density force.

    The reverse mode runs the axis schedule; the differences of H are taken on
    that schedule too (the fused schedule's H agrees to rounding, checked
    first), so that only one rounding pattern enters the per-site noise floor."""
    w = inputs.GRAD96
    wp, wm = inputs.fields(w)
    ctx = B.Context(B.Params(*w.n, *w.L, w.ns, w.f, w.chiN, w.C, B.PFT_C128, B.PFT_RQM4))
    gwp, gwm = dev(wp), dev(wm)
    gp, gm, dL, H0 = gpu_adjoint(ctx, gwp, gwm, kc=11)
    Hbuf = torch.empty(1, dtype=torch.complex128, device=DEV)
    ctx.pft_set_fused_planes(1)
    ctx.pft_propagate(gwp, gwm)
    ctx.pft_hamiltonian(gwp, gwm, Hbuf)
    assert abs(complex(host(Hbuf)[0]) - H0) <= 1e-12 * abs(H0)
    ctx.pft_set_fused_planes(False)

    def H(ap, am):
        ctx.pft_propagate(ap, am)
        ctx.pft_hamiltonian(ap, am, Hbuf)
        return complex(host(Hbuf)[0])

    assert abs(H(gwp, gwm) - H0) <= 1e-12 * abs(H0)
    rng = np.random.default_rng(7)
    sites = [tuple(s) for s in rng.integers(0, 96, size=(64, 3))]
    # the step balances H's rounding noise (~1e-14 |H|, falling as 1/eps in the
    # difference) against the O(eps^4) truncation error (< 1e-7 up to eps = 6e-3)
    eps = 1e-3
    worst = 0.0
    for k, site in enumerate(sites):
        which = k % 2
        g = (gp if which == 0 else gm)[site]

        def Hs(e):
            d = torch.zeros(w.n, dtype=torch.complex128, device=DEV)
            d[site] = e
            return H(gwp + d, gwm) if which == 0 else H(gwp, gwm + d)
        fd = (-Hs(2 * eps) + 8 * Hs(eps) - 8 * Hs(-eps) + Hs(-2 * eps)) / (12 * eps)
        worst = max(worst, abs(fd - g) / abs(g))
    say("worst per-site relative FD difference", worst)
    assert worst <= 1e-4
    # directional derivative along the lamellar mode: an O(V) signal
    x = np.arange(96).reshape(-1, 1, 1) / 96
    d = dev(np.cos(2 * np.pi * x) * np.ones(w.n) + 0.3j)
    fd = (-H(gwp, gwm + 2e-4 * d) + 8 * H(gwp, gwm + 1e-4 * d) - 8 * H(gwp, gwm - 1e-4 * d)
          + H(gwp, gwm - 2e-4 * d)) / (12e-4)
    an = (gm * host(d)).sum()
    assert abs(fd - an) <= 1e-8 * abs(an)
    # analytic density force: equal to the gradient up to O(ds^2)
    out = ctx.evaluate(gwp, gwm)
    dV = np.prod(w.L) / w.M
    Fm = 2 * wm / w.chiN + host(out["phiB"]) - host(out["phiA"])
    assert np.abs(gm - w.C * dV * Fm).max() <= 2e-3 * np.abs(gm).max()
    # box stress by differences in each edge length (fresh contexts)
    for a in range(3):
        def HL(e):
            Ls = list(w.L)
            Ls[a] += e
            c2 = B.Context(B.Params(*w.n, *Ls, w.ns, w.f, w.chiN, w.C, B.PFT_C128, B.PFT_RQM4))
            c2.pft_set_fused_planes(False)
            c2.pft_propagate(gwp, gwm)
            c2.pft_hamiltonian(gwp, gwm, Hbuf)
            v = complex(host(Hbuf)[0])
            c2.close()
            return v
        fdL = (-HL(2e-3) + 8 * HL(1e-3) - 8 * HL(-1e-3) + HL(-2e-3)) / 12e-3
        say("dH/dL", a, dL[a], fdL)
        assert abs(fdL - dL[a]) <= 1e-7 * abs(dL[a])


def test_autograd_function_gradcheck():
    n, L = (8, 8, 12), (2.0, 2.0, 3.0)
    wp, wm = fields(n, 24)
    ctx = B.Context(B.Params(*n, *L, 12, 0.45, 15.0, 1.0, B.PFT_C128, B.PFT_RQM4))
    a = dev(wp).requires_grad_(True)
    b = dev(wm).requires_grad_(True)
    H = hamiltonian(ctx, a, b)
    H.real.backward()
    gp, gm, _, _ = gpu_adjoint(ctx, dev(wp), dev(wm))
    # d Re H / d w as PyTorch reports it: conj of the holomorphic derivative
    assert np.allclose(host(a.grad), np.conj(gp), rtol=0, atol=1e-14)
    assert torch.autograd.gradcheck(lambda x, y: hamiltonian(ctx, x, y), (a.detach().requires_grad_(True),
                                    b.detach().requires_grad_(True)), eps=1e-6, atol=1e-7, rtol=1e-5,
                                    fast_mode=True)


def test_set_box_equals_new_context(orc):
    """pft_set_box moves a context to new edges: the evaluation and the
    adjoint equal those of a context created with those edges, and the oracle."""
    n, ns = (12, 8, 16), 14
    wp, wm = fields(n, 26)
    p0 = B.Params(*n, 3.0, 2.0, 4.0, ns, 0.45, 15.0, 2.0, B.PFT_C128, B.PFT_RQM4)
    L1 = (3.3, 1.9, 4.4)
    ctx = B.Context(p0)
    ctx.evaluate(dev(wp), dev(wm))
    ctx.pft_set_box(*L1)
    out = ctx.evaluate(dev(wp), dev(wm))
    ref_ctx = B.Context(B.Params(*n, *L1, ns, 0.45, 15.0, 2.0, B.PFT_C128, B.PFT_RQM4))
    ref = ref_ctx.evaluate(dev(wp), dev(wm))
    assert np.abs(host(out["phiA"]) - host(ref["phiA"])).max() == 0
    assert host(out["H"])[0] == host(ref["H"])[0]
    a1 = gpu_adjoint(ctx, dev(wp), dev(wm))
    a2 = gpu_adjoint(ref_ctx, dev(wp), dev(wm))
    assert np.array_equal(a1[2], a2[2]) and np.array_equal(a1[0], a2[0])
    o = orc.evaluate(orc.Params(*n, *L1, ns, 0.45, 15.0, 2.0, 0, False), wp, wm)
    assert abs(host(out["H"])[0] - o["H"]) <= 1e-11 * (abs(o["H"]) + 2.0 * np.prod(L1))
    with pytest.raises(B.PftError):
        ctx.pft_set_box(0.0, 1.0, 1.0)
    ctx.close()
    ref_ctx.close()


def test_autograd_box_edges_gradcheck():
    """The box edges as a differentiable input: dRe H/dL from backward equals
    the real part of the box derivative, and gradcheck passes on L alone and
    on (w+, w-, L) together."""
    n = (8, 12, 8)
    wp, wm = fields(n, 27)
    ctx = B.Context(B.Params(*n, 2.0, 3.0, 2.0, 12, 0.4, 15.0, 1.5, B.PFT_C128, B.PFT_RQM4))
    L = torch.tensor([2.1, 2.9, 2.2], dtype=torch.float64, requires_grad=True)
    H = hamiltonian(ctx, dev(wp), dev(wm), L)
    H.real.backward()
    ref = gpu_adjoint(ctx, dev(wp), dev(wm))
    assert (ctx.params.lx, ctx.params.ly, ctx.params.lz) == (2.1, 2.9, 2.2)
    assert np.allclose(L.grad.numpy(), ref[2].real, rtol=1e-14, atol=0)
    a, b = dev(wp), dev(wm)
    assert torch.autograd.gradcheck(lambda x: hamiltonian(ctx, a, b, x), (L.detach().requires_grad_(True),),
                                    eps=1e-6, atol=1e-7, rtol=1e-5)
    assert torch.autograd.gradcheck(lambda x, y, z: hamiltonian(ctx, x, y, z),
                                    (a.clone().requires_grad_(True), b.clone().requires_grad_(True),
                                     L.detach().requires_grad_(True)),
                                    eps=1e-6, atol=1e-7, rtol=1e-5, fast_mode=True)
    ctx.close()


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 0, 0)])
def test_set_box_then_semi_implicit_step(bc):
    """After pft_set_box the semi-implicit step filters with the new box's
    |k|^2 (its tables, built on the first step, are rebuilt): the step equals
    that of a context created with the new edges, periodic and between
    reflecting walls."""
    n, ns = (16, 12, 20), 12
    wp, wm = fields(n, 28)
    L0, L1 = (3.0, 2.5, 4.0), (3.6, 2.2, 4.4)
    st = B.pft_step(0.3, 1.0, 0.7, 5, 0, 2, 1, 1)
    ctx = B.Context(B.Params(*n, *L0, ns, 0.45, 15.0, 20.0, B.PFT_C128, B.PFT_RQM4, B.PFT_DIBLOCK, 0.0,
                             B.PFT_STORE_BOTH, bc))
    a, b = dev(wp), dev(wm)
    ctx.pft_cl_step(a, b, st)          # builds the filter tables for L0
    ctx.pft_set_box(*L1)
    a, b = dev(wp), dev(wm)
    ctx.pft_cl_step(a, b, st)
    ref = B.Context(B.Params(*n, *L1, ns, 0.45, 15.0, 20.0, B.PFT_C128, B.PFT_RQM4, B.PFT_DIBLOCK, 0.0,
                             B.PFT_STORE_BOTH, bc))
    c, d = dev(wp), dev(wm)
    ref.pft_cl_step(c, d, st)
    assert torch.equal(a, c) and torch.equal(b, d)
    ctx.close()
    ref.close()
