"""Pins of the oracle's Edwards-model functions (homopolymer in implicit
solvent, Eq. (2); the propagator feels w = i omega along the whole chain).

- uniform fields: q_j = exp(-i omega s_j), Q = exp(-i omega), phi = 1 exactly,
  H = (B/2) V omega^2 + i C V omega, F = (B/C) omega + i;
- the homogeneous saddle point omega* = -i C / B: F = 0 and H = C^2 V / (2 B)
  (the mean-field excluded-volume energy), the update leaves it fixed;
- weak-field response against the Debye function g_D(x) = 2 (e^-x + x - 1)/x^2;
- under the plain split, central differences of H equal C dV F site by site;
- symmetry: the single-sweep densities equal those of two independent sweeps
  (q-dagger computed, not assumed) with w_+ = omega, w_- = 0;
- the update's noise is the field-0 Gaussian stream with s^2 = 2 lam dt/(C dV).
"""
import numpy as np
import pytest


def P(orc, n=(6, 4, 8), L=(3.0, 2.0, 4.0), ns=20, C=2.0, scheme=0):
    return orc.Params(*n, *L, ns, 0.5, 10.0, C, scheme, False)


def rand_omega(shape, seed, s=0.3):
    r = np.random.default_rng(seed)
    return s * r.standard_normal(shape) + 0.1j * r.standard_normal(shape)


@pytest.mark.parametrize("scheme", [0, 1])
def test_uniform_field_closed_forms(orc, scheme):
    p = P(orc, scheme=scheme)
    B, om = 1.7, 0.35 - 0.2j
    omega = np.full(p.shape, om)
    qs = orc.edwards_propagate(p, omega)
    s = np.arange(p.ns + 1) / p.ns
    for j in (0, 7, p.ns):
        assert np.abs(qs[j] - np.exp(-1j * om * s[j])).max() < 1e-14
    out = orc.edwards_evaluate(p, B, omega)
    assert abs(out["Q"] - np.exp(-1j * om)) < 1e-14
    assert np.abs(out["phi"] - 1).max() < 1e-13
    V = p.volume
    assert abs(out["H"] - (0.5 * B * V * om ** 2 + 1j * p.C * V * om)) < 1e-12 * abs(out["H"])
    F = orc.edwards_force(p, B, omega, out["phi"])
    assert np.abs(F - ((B / p.C) * om + 1j)).max() < 1e-13


def test_homogeneous_saddle_point(orc):
    p = P(orc, C=3.0)
    B = 2.5
    omega = np.full(p.shape, -1j * p.C / B)
    out = orc.edwards_evaluate(p, B, omega)
    F = orc.edwards_force(p, B, omega, out["phi"])
    assert np.abs(F).max() < 1e-13
    assert abs(out["H"] - p.C ** 2 * p.volume / (2 * B)) < 1e-12 * p.C ** 2 * p.volume / B
    new = orc.edwards_em_update(p, B, omega, out["phi"], 0.1)
    assert np.abs(new - omega).max() < 1e-14


def test_debye_response(orc):
    # omega = eps cos(k.r): w = i eps cos, so delta phi = -i eps g_D cos and
    # ln Q = (i eps)^2 g_D / 4 to leading order
    n, Lx, eps = (10, 2, 2), 5.0, 1e-3
    p = P(orc, n=n, L=(Lx, 1.0, 1.0), ns=200)
    x = (2 * np.pi / Lx) ** 2
    cos = np.cos(2 * np.pi * np.arange(n[0]) / n[0]).reshape(-1, 1, 1) * np.ones(n)
    rp = orc.edwards_evaluate(p, 1.0, eps * cos)
    rm = orc.edwards_evaluate(p, 1.0, -eps * cos)
    gD = 2 * (np.exp(-x) + x - 1) / x ** 2
    dphi = (rp["phi"] - rm["phi"]) / (2 * eps)
    assert np.allclose(dphi, -1j * gD * cos, atol=2e-5)
    lnQ = (np.log(rp["Q"]) + np.log(rm["Q"])) / 2
    expect = -0.25 * gD * eps ** 2
    assert abs(lnQ - expect) <= 1e-4 * abs(expect)


@pytest.mark.parametrize("ns", [12, 9])
def test_split2_force_is_exact_gradient(orc, ns):
    p = P(orc, n=(4, 4, 6), L=(2.0, 2.0, 3.0), ns=ns, scheme=1)
    B = 1.3
    omega = rand_omega(p.shape, 30)
    out = orc.edwards_evaluate(p, B, omega)
    F = orc.edwards_force(p, B, omega, out["phi"])
    dV = p.volume / p.M
    eps = 1e-5
    for site in [(0, 0, 0), (1, 2, 3), (3, 3, 5)]:
        for direction in (1.0, 1j):
            e = np.zeros(p.shape, complex)
            e[site] = eps * direction
            fd = (orc.edwards_evaluate(p, B, omega + e)["H"] - orc.edwards_evaluate(p, B, omega - e)["H"]) / (2 * eps)
            expect = p.C * dV * F[site] * direction
            assert abs(fd - expect) < 1e-8 * (1 + abs(expect)), (site, direction)


def test_rqm4_force_is_gradient_to_second_order(orc):
    # the Richardson step's derivative differs from the trapezoid force by a
    # term that vanishes at least as fast as ds^2
    B = 0.8
    errs = []
    for ns in (10, 20, 40):
        p = P(orc, n=(4, 4, 4), L=(2.0, 2.0, 2.0), ns=ns, scheme=0)
        omega = rand_omega(p.shape, 31)
        out = orc.edwards_evaluate(p, B, omega)
        F = orc.edwards_force(p, B, omega, out["phi"])
        dV = p.volume / p.M
        eps = 1e-5
        site = (1, 2, 3)
        e = np.zeros(p.shape, complex)
        e[site] = eps
        fd = (orc.edwards_evaluate(p, B, omega + e)["H"] - orc.edwards_evaluate(p, B, omega - e)["H"]) / (2 * eps)
        errs.append(abs(fd - p.C * dV * F[site]))
    assert errs[0] / errs[1] > 2.5 and errs[1] / errs[2] > 2.5 and errs[2] < errs[0] / 10


@pytest.mark.parametrize("scheme", [0, 1])
def test_single_sweep_equals_two_sweeps(orc, scheme):
    # f * ns an integer, so the diblock contour has no junction; with w_- = 0
    # both blocks see i omega and the computed q-dagger must equal q
    p2 = orc.Params(6, 4, 8, 3.0, 2.0, 4.0, 20, 0.45, 10.0, 2.0, scheme, False)
    p1 = P(orc, ns=20, scheme=scheme)
    omega = rand_omega(p1.shape, 32)
    e = orc.edwards_evaluate(p1, 1.0, omega)
    d = orc.evaluate(p2, omega, np.zeros(p1.shape))
    assert abs(e["Q"] - d["Q"]) < 1e-14 * abs(d["Q"])
    assert np.abs(e["phi"] - (d["phiA"] + d["phiB"])).max() < 1e-13


def test_update_noise_stream_and_scale(orc):
    p = P(orc, n=(8, 8, 8), L=(4.0, 4.0, 4.0), C=5.0)
    B, dt, lam = 1.2, 0.02, 0.7
    omega = rand_omega(p.shape, 33)
    phi = orc.edwards_evaluate(p, B, omega)["phi"]
    det = orc.edwards_em_update(p, B, omega, phi, dt, lam)
    noisy = orc.edwards_em_update(p, B, omega, phi, dt, lam, noise=True, seed=9, replica=2, step_=5)
    dV = p.volume / p.M
    s = np.sqrt(2 * lam * dt / (p.C * dV))
    xi = orc.gaussian(9, 2, 5, 0, p.M).reshape(p.shape)
    assert np.abs((noisy - det) - s * xi).max() < 1e-14
    F = orc.edwards_force(p, B, omega, phi)
    assert np.abs(det - (omega - lam * dt * F)).max() < 1e-15


def test_em_drift_is_first_order_descent_of_H(orc):
    """One noise-free step of Eq. (9) on the Edwards field changes H by
    -lam dt C dV sum F^2 to first order (dH/domega = C dV F under the plain
    split, pinned above by central differences); the relative residual halves
    with dt.  A flipped drift or dt in place of lam dt fails."""
    p = P(orc, n=(6, 4, 8), L=(3.0, 2.0, 4.0), ns=16, C=2.0, scheme=1)
    B, lam = 1.3, 0.6
    omega = rand_omega(p.shape, 51)
    base = orc.edwards_evaluate(p, B, omega)
    F = orc.edwards_force(p, B, omega, base["phi"])
    dV = p.volume / p.M
    rel = []
    for dt in (4e-3, 2e-3, 1e-3):
        new = orc.edwards_em_update(p, B, omega, base["phi"], dt, lam)
        dH = orc.edwards_evaluate(p, B, new)["H"] - base["H"]
        pred = -lam * dt * p.C * dV * np.sum(F * F)
        rel.append((dH - pred) / pred)
    assert abs(rel[-1]) < 2e-2, rel
    for a, b in zip(rel, rel[1:]):
        assert 1.8 < abs(a / b) < 2.2, rel
