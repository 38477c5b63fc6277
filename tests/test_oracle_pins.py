"""Pins of the oracle's propagator, densities, Q and H against results the
paper's equations fix independently of any implementation:

* constant fields solve the modified diffusion equation (Eq. (5)) in closed
  form under both split schemes;
* exact invariants of the discrete method (per-node Q, total density,
  chain reversal, grid symmetries, reality);
* the weak-field (Debye / random-phase) response of a Gaussian diblock;
* a single Fourier mode diffuses as exp(-|k|^2 s);
* self-convergence orders: 4 for the Richardson step (Eq. (12)), 2 for the
  plain split, 2 for the trapezoid contour sums;
* the homogeneous saddle point of Eq. (3) reproduces the textbook mean-field
  free energy chi N f (1 - f) of an incompressible AB melt.
"""
import numpy as np
import pytest


def P(orc, n=(6, 6, 6), L=(4.0, 4.0, 4.0), ns=20, f=0.5, chiN=15.0, C=1.0, scheme=0, naive=False):
    return orc.Params(n[0], n[1], n[2], L[0], L[1], L[2], ns, f, chiN, C, scheme, naive)


def smooth_fields(shape, seed, amp=0.4):
    r = np.random.default_rng(seed)
    x, y, z = np.meshgrid(*(np.arange(n) / n for n in shape), indexing="ij")
    wp = amp * (0.3 * np.cos(2 * np.pi * x) + 0.2j * np.sin(2 * np.pi * (y - z)))
    wm = amp * (np.cos(2 * np.pi * (x + y)) + 0.5 * np.sin(4 * np.pi * z) + 0.1j * np.cos(2 * np.pi * y))
    wp = wp + 0.05 * amp * (r.standard_normal(shape) + 1j * r.standard_normal(shape))
    wm = wm + 0.05 * amp * (r.standard_normal(shape) + 1j * r.standard_normal(shape))
    return wp, wm


# ---------------------------------------------------------------- contour ---

@pytest.mark.parametrize("ns,f", [(50, 0.5), (128, 0.3), (100, 0.4), (40, 0.33), (7, 0.05), (9, 0.95)])
def test_contour_plan(orc, ns, f):
    h, blk, J = orc.contour(ns, f)
    s = np.concatenate([[0.0], np.cumsum(h)])
    assert np.isclose(s[-1], 1.0, atol=1e-14)
    assert np.isclose(s[J], f, atol=1e-14)
    assert np.all(blk[:J] == 0) and np.all(blk[J:] == 1)
    assert np.all(h > 0)
    integer = abs(f * ns - round(f * ns)) <= 1e-9
    assert len(h) == (ns if integer else ns + 1)
    ta, tb = orc.trapezoid(h, blk)
    assert np.isclose(ta.sum(), f, atol=1e-14) and np.isclose(tb.sum(), 1 - f, atol=1e-14)


# --------------------------------------------------------- P1 constant fields

@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("ns,f", [(20, 0.5), (25, 0.3), (13, 0.62)])
def test_constant_fields_exact(orc, scheme, ns, f):
    p = P(orc, n=(4, 6, 5), ns=ns, f=f, scheme=scheme)
    a, b = 0.3 + 0.2j, -0.7 + 0.1j          # i w+ = a, w- = b
    wp = np.full(p.shape, -1j * a)
    wm = np.full(p.shape, b)
    wA, wB = a - b, a + b
    qs, qds = orc.propagate(p, wp, wm)
    h, blk, J = orc.contour(ns, f)
    s = np.concatenate([[0.0], np.cumsum(h)])
    for j, sj in enumerate(s):
        integral = wA * min(sj, f) + wB * max(sj - f, 0.0)
        assert np.allclose(qs[j], np.exp(-integral), rtol=1e-12, atol=0)
    phiA, phiB, Q, Qn = orc.densities(p, qs, qds)
    assert np.isclose(Q, np.exp(-(f * wA + (1 - f) * wB)), rtol=1e-12)
    assert np.allclose(phiA, f, atol=1e-12) and np.allclose(phiB, 1 - f, atol=1e-12)


def test_homopolymer_constant_field(orc):
    # w_A = w_B = w: q(s) = e^{-w s}, Q = e^{-w}
    p = P(orc, n=(4, 4, 4), ns=10, f=0.5)
    w = 0.45
    wp = np.full(p.shape, -1j * w)
    wm = np.zeros(p.shape, complex)
    qs, _ = orc.propagate(p, wp, wm, backward=False)
    for j in range(11):
        assert np.allclose(qs[j], np.exp(-w * j / 10), rtol=1e-13)
    assert np.isclose(qs[-1].mean(), np.exp(-w), rtol=1e-13)


# ------------------------------------------------------------ P2 invariants

@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("f,ns", [(0.5, 20), (0.3, 25)])
def test_invariants(orc, scheme, f, ns):
    p = P(orc, n=(6, 8, 4), L=(3.0, 4.0, 2.5), ns=ns, f=f, scheme=scheme)
    wp, wm = smooth_fields(p.shape, 3)
    r = orc.evaluate(p, wp, wm)
    assert np.allclose(r["Qnode"], r["Q"], rtol=1e-11, atol=0)
    assert np.isclose((r["phiA"] + r["phiB"]).sum(), p.M, rtol=1e-11)
    assert np.isclose(r["phiA"].sum(), f * p.M, rtol=1e-11)


@pytest.mark.parametrize("f,ns", [(0.5, 20), (0.3, 25), (0.41, 17)])
def test_chain_reversal(orc, f, ns):
    p1 = P(orc, n=(6, 4, 4), ns=ns, f=f)
    p2 = P(orc, n=(6, 4, 4), ns=ns, f=1 - f)
    wp, wm = smooth_fields(p1.shape, 4)
    r1 = orc.evaluate(p1, wp, wm)
    r2 = orc.evaluate(p2, wp, -wm)
    assert np.allclose(r1["phiA"], r2["phiB"], atol=1e-12)
    assert np.allclose(r1["phiB"], r2["phiA"], atol=1e-12)
    assert np.isclose(r1["Q"], r2["Q"], rtol=1e-12)


def test_grid_symmetries(orc):
    p = P(orc, n=(6, 6, 6), L=(4.0, 4.0, 4.0), ns=12, f=0.4)
    wp, wm = smooth_fields(p.shape, 5)
    r = orc.evaluate(p, wp, wm)
    sh = (1, -2, 3)
    rs = orc.evaluate(p, np.roll(wp, sh, (0, 1, 2)), np.roll(wm, sh, (0, 1, 2)))
    assert np.allclose(rs["phiA"], np.roll(r["phiA"], sh, (0, 1, 2)), atol=1e-12)
    perm = (2, 0, 1)
    rp = orc.evaluate(p, np.transpose(wp, perm), np.transpose(wm, perm))
    assert np.allclose(rp["phiB"], np.transpose(r["phiB"], perm), atol=1e-12)
    assert np.isclose(rp["Q"], r["Q"], rtol=1e-12)


def test_real_fields_give_real_densities(orc):
    p = P(orc, n=(6, 6, 4), ns=16, f=0.5)
    r = np.random.default_rng(6)
    wp = 1j * 0.3 * r.standard_normal(p.shape)   # i w+ real
    wm = 0.3 * r.standard_normal(p.shape)
    out = orc.evaluate(p, wp, wm)
    assert abs(out["Q"].imag) < 1e-15 and np.abs(out["phiA"].imag).max() < 1e-14


# -------------------------------------------------------- P3 Debye response

def g1(f, x):
    return 2.0 * (f * x + np.exp(-f * x) - 1.0) / x ** 2


def s_ab(f, x):
    return (1.0 - np.exp(-f * x)) * (1.0 - np.exp(-(1.0 - f) * x)) / x ** 2


@pytest.mark.parametrize("f", [0.5, 0.3])
@pytest.mark.parametrize("epsA,epsB", [(1.0, 0.0), (0.0, 1.0), (1.0, 1.0), (0.7, -0.4)])
def test_debye_response(orc, f, epsA, epsB):
    n, Lx, ns, eps = (8, 2, 2), 4.0, 200, 1e-3
    p = P(orc, n=n, L=(Lx, 1.0, 1.0), ns=ns, f=f)
    x = (2 * np.pi / Lx) ** 2                      # |k|^2 R_g^2 of the cosine mode
    cos = np.cos(2 * np.pi * np.arange(n[0]) / n[0]).reshape(-1, 1, 1) * np.ones(n)

    def run(e):
        wA, wB = e * epsA * cos, e * epsB * cos
        # w_A = i w+ - w-, w_B = i w+ + w-
        wp = -1j * (wA + wB) / 2
        wm = (wB - wA) / 2
        return orc.evaluate(p, wp, wm)

    rp, rm = run(eps), run(-eps)
    SAA, SBB, SAB = g1(f, x), g1(1 - f, x), s_ab(f, x)
    dphiA = (rp["phiA"] - rm["phiA"]) / (2 * eps)   # odd part: linear response
    dphiB = (rp["phiB"] - rm["phiB"]) / (2 * eps)
    assert np.allclose(dphiA.real, -(SAA * epsA + SAB * epsB) * cos, atol=2e-5)
    assert np.allclose(dphiB.real, -(SAB * epsA + SBB * epsB) * cos, atol=2e-5)
    lnQ = (np.log(rp["Q"]) + np.log(rm["Q"])).real / 2  # even part: quadratic response
    expect = 0.25 * (SAA * epsA ** 2 + 2 * SAB * epsA * epsB + SBB * epsB ** 2) * eps ** 2
    assert abs(lnQ - expect) <= 1e-4 * abs(expect) + 1e-14


def test_debye_homopolymer_limit(orc):
    # equal fields on both blocks: the Debye function g_D = 2 (e^-x + x - 1)/x^2
    n, Lx, eps = (10, 2, 2), 5.0, 1e-3
    p = P(orc, n=n, L=(Lx, 1.0, 1.0), ns=200, f=0.37)
    x = (2 * np.pi / Lx) ** 2
    cos = np.cos(2 * np.pi * np.arange(n[0]) / n[0]).reshape(-1, 1, 1) * np.ones(n)
    r1 = orc.evaluate(p, -1j * eps * cos, np.zeros(n))
    r2 = orc.evaluate(p, 1j * eps * cos, np.zeros(n))
    gD = 2 * (np.exp(-x) + x - 1) / x ** 2
    phi = (r1["phiA"] + r1["phiB"] - r2["phiA"] - r2["phiB"]) / (2 * eps)
    assert np.allclose(phi.real, -gD * cos, atol=2e-5)


# ----------------------------------------------------- P4 single free mode

@pytest.mark.parametrize("scheme", [0, 1])
def test_single_mode_diffusion(orc, scheme):
    n, L = (8, 6, 10), (3.0, 2.0, 5.0)
    p = P(orc, n=n, L=L, scheme=scheme)
    m = (1, 2, 3)
    x, y, z = np.meshgrid(*(np.arange(k) for k in n), indexing="ij")
    phase = 2 * np.pi * (m[0] * x / n[0] + m[1] * y / n[1] + m[2] * z / n[2])
    k2 = sum((2 * np.pi * m[a] / L[a]) ** 2 for a in range(3))
    u = np.cos(phase).astype(complex)
    h = 0.037
    assert np.allclose(orc.diffuse(p, h, u), np.exp(-k2 * h) * u, atol=1e-14)
    out = orc.step(p, h, np.zeros(n, complex), u, scheme=scheme)
    assert np.allclose(out, np.exp(-k2 * h) * u, atol=1e-14)


def test_diffusion_naive_equals_fft(orc):
    p1 = P(orc, n=(4, 6, 5), L=(2.0, 3.0, 2.5))
    p2 = P(orc, n=(4, 6, 5), L=(2.0, 3.0, 2.5), naive=True)
    u = np.random.default_rng(7).standard_normal(p1.shape) + 0j
    assert np.allclose(orc.diffuse(p1, 0.05, u), orc.diffuse(p2, 0.05, u), atol=1e-13)


def test_ksq_grid(orc):
    p = P(orc, n=(4, 6, 5), L=(2.0, 3.0, 2.5))
    k = [2 * np.pi * np.fft.fftfreq(p.shape[a], d=(p.lx, p.ly, p.lz)[a] / p.shape[a]) for a in range(3)]
    ref = k[0][:, None, None] ** 2 + k[1][None, :, None] ** 2 + k[2][None, None, :] ** 2
    assert np.allclose(orc.ksq_grid(p), ref, rtol=1e-14)


# ------------------------------------------------------ P6 convergence order

@pytest.mark.parametrize("scheme,pQ", [(0, 4), (1, 2)])
def test_convergence_orders(orc, scheme, pQ):
    wp, wm = smooth_fields((8, 8, 8), 8)
    Qs, phis = [], []
    for ns in (20, 40, 80, 160):
        r = orc.evaluate(P(orc, n=(8, 8, 8), ns=ns, f=0.5, scheme=scheme), wp, wm)
        Qs.append(r["Q"])
        phis.append(r["phiA"])
    eQ = [abs(Qs[i] - Qs[i + 1]) for i in range(3)]
    ratio = eQ[1] / eQ[2]
    assert abs(np.log2(ratio) - pQ) < 0.15
    ePhi = [np.abs(phis[i] - phis[i + 1]).max() for i in range(3)]
    assert abs(np.log2(ePhi[1] / ePhi[2]) - 2) < 0.1


# ------------------------------------------- homogeneous mean-field saddle

@pytest.mark.parametrize("f,chiN", [(0.5, 14.0), (0.4, 14.4), (0.3, 18.0)])
def test_homogeneous_saddle_free_energy(orc, f, chiN):
    # Stationary homogeneous fields: w- = chiN (2f - 1)/2, any constant i w+.
    # Textbook incompressible melt: F / (n k T) = chiN f (1 - f); the field
    # theory's H carries the extra constant -chiN/4 of the Gaussian transform.
    p = P(orc, n=(4, 4, 4), L=(2.0, 2.0, 2.0), ns=10, f=f, chiN=chiN, C=3.0)
    wm = np.full(p.shape, chiN * (2 * f - 1) / 2, complex)
    wp = np.full(p.shape, -1j * 0.37)
    r = orc.evaluate(p, wp, wm)
    V = 8.0
    assert np.isclose(r["H"] / (p.C * V) + chiN / 4, chiN * f * (1 - f), rtol=1e-12, atol=1e-12)
    Fp, Fm = orc.forces(p, wm, r["phiA"], r["phiB"])
    assert np.abs(Fp).max() < 1e-12 and np.abs(Fm).max() < 1e-12
    wp2, wm2 = orc.em_update(p, wp, wm, r["phiA"], r["phiB"], dt=0.1)
    assert np.allclose(wp2, wp, atol=1e-12) and np.allclose(wm2, wm, atol=1e-12)
