"""Pins of H's field derivative against the mean-field forces.

With the plain split step and trapezoid contour sums the derivative of the
discrete Hamiltonian is exactly C dV F (each step's derivative contributes
the trapezoid weight of its two end nodes), so central finite differences of
the oracle's H must reproduce the oracle's forces; and H is holomorphic, so
the derivative along i w equals i times the derivative along w.  Under the
Richardson step the agreement is O(ds^2) only.
"""
import numpy as np
import pytest


def fields(shape, seed):
    r = np.random.default_rng(seed)
    wp = 0.3 * r.standard_normal(shape) + 0.1j * r.standard_normal(shape)
    wm = 0.5 * r.standard_normal(shape) + 0.1j * r.standard_normal(shape)
    return wp, wm


def H(orc, p, wp, wm):
    return orc.evaluate(p, wp, wm)["H"]


@pytest.mark.parametrize("f,ns", [(0.5, 12), (0.3, 11)])
def test_split2_force_is_exact_gradient(orc, f, ns):
    p = orc.Params(4, 4, 6, 2.0, 2.0, 3.0, ns, f, 15.0, 2.0, 1, False)
    wp, wm = fields(p.shape, 10)
    r = orc.evaluate(p, wp, wm)
    Fp, Fm = orc.forces(p, wm, r["phiA"], r["phiB"])
    dV = p.volume / p.M
    eps = 1e-5
    for site in [(0, 0, 0), (1, 2, 3), (3, 3, 5)]:
        for which, F in ((0, Fp), (1, Fm)):
            for direction in (1.0, 1j):
                e = np.zeros(p.shape, complex)
                e[site] = eps * direction
                args_p = (wp + e, wm) if which == 0 else (wp, wm + e)
                args_m = (wp - e, wm) if which == 0 else (wp, wm - e)
                fd = (H(orc, p, *args_p) - H(orc, p, *args_m)) / (2 * eps)
                expect = p.C * dV * F[site] * direction
                assert abs(fd - expect) < 1e-8 * (1 + abs(expect)), (site, which, direction)


def test_split2_directional_derivative(orc):
    # a smooth direction gives an O(1) signal, so the check is tight
    p = orc.Params(6, 4, 4, 3.0, 2.0, 2.0, 10, 0.4, 12.0, 1.0, 1, False)
    wp, wm = fields(p.shape, 11)
    x = np.arange(6).reshape(-1, 1, 1) / 6
    d = np.cos(2 * np.pi * x) * np.ones(p.shape) + 0.3j
    r = orc.evaluate(p, wp, wm)
    Fp, Fm = orc.forces(p, wm, r["phiA"], r["phiB"])
    dV = p.volume / p.M
    eps = 1e-5
    fd = (H(orc, p, wp, wm + eps * d) - H(orc, p, wp, wm - eps * d)) / (2 * eps)
    assert abs(fd - p.C * dV * (Fm * d).sum()) < 1e-8 * abs(fd)


def test_rqm4_force_is_gradient_to_second_order(orc):
    wp, wm = fields((4, 4, 4), 12)
    errs = []
    for ns in (10, 20, 40):
        p = orc.Params(4, 4, 4, 2.0, 2.0, 2.0, ns, 0.5, 15.0, 1.0, 0, False)
        r = orc.evaluate(p, wp, wm)
        _, Fm = orc.forces(p, wm, r["phiA"], r["phiB"])
        dV = p.volume / p.M
        eps = 1e-5
        e = np.zeros(p.shape, complex)
        e[1, 2, 3] = eps
        fd = (H(orc, p, wp, wm + e) - H(orc, p, wp, wm - e)) / (2 * eps)
        errs.append(abs(fd - p.C * dV * Fm[1, 2, 3]))
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0
