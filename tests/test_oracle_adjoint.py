"""Pins of the oracle's reverse-mode derivatives of H (field gradient and box
stress) against finite differences of the oracle's own H, the exact plain-split
force identity, and holomorphy.  Fourth-order central differences with steps
where round-off and truncation balance (~3e-4) resolve the derivatives to
~1e-9 relative."""
import numpy as np
import pytest


def fields(shape, seed):
    r = np.random.default_rng(seed)
    wp = 0.3 * r.standard_normal(shape) + 0.1j * r.standard_normal(shape)
    wm = 0.5 * r.standard_normal(shape) + 0.1j * r.standard_normal(shape)
    return wp, wm


def fd4(f, eps):
    return (-f(2 * eps) + 8 * f(eps) - 8 * f(-eps) + f(-2 * eps)) / (12 * eps)


CASES = [(0, 0.5, 10), (0, 0.3, 11), (1, 0.5, 10), (1, 0.37, 9)]


@pytest.mark.parametrize("scheme,f,ns", CASES)
def test_field_gradient_fd(orc, scheme, f, ns):
    sh, L = (4, 6, 4), (2.0, 3.0, 2.5)
    p = orc.Params(*sh, *L, ns, f, 15.0, 2.0, scheme, False)
    wp, wm = fields(sh, 3)
    gp, gm, _ = orc.adjoint(p, wp, wm)
    for site in [(0, 0, 0), (1, 2, 3), (3, 5, 1)]:
        for which, g in ((0, gp), (1, gm)):
            for direction in (1.0, 1j):   # holomorphic: derivative along i w is i dH/dw
                def H(e):
                    d = np.zeros(sh, complex)
                    d[site] = e * direction
                    return orc.evaluate(p, wp + d, wm)["H"] if which == 0 else orc.evaluate(p, wp, wm + d)["H"]
                fd = fd4(H, 3e-4)
                # H carries ~1e-13 of FFT round-off, i.e. ~5e-10 after differencing
                assert abs(fd - g[site] * direction) <= 1e-7 * abs(g[site]) + 5e-10, (site, which, direction)


@pytest.mark.parametrize("bc,scheme", [((1, 0, 2), 0), ((2, 1, 0), 1), ((1, 1, 1), 0)])
def test_field_gradient_fd_with_walls(orc, bc, scheme):
    """Between walls the steps diffuse through the walled operator (cosine /
    sine modes), which is symmetric too: the same reverse mode, checked by
    finite differences of the oracle's walled H."""
    sh, L = (4, 6, 4), (2.0, 3.0, 2.5)
    p = orc.Params(*sh, *L, 9, 0.41, 15.0, 2.0, scheme, False, bc)
    wp, wm = fields(sh, 5)
    gp, gm, _ = orc.adjoint(p, wp, wm)
    for site in [(0, 0, 0), (3, 5, 3), (2, 1, 2)]:
        for which, g in ((0, gp), (1, gm)):
            def H(e):
                d = np.zeros(sh, complex)
                d[site] = e
                return orc.evaluate(p, wp + d, wm)["H"] if which == 0 else orc.evaluate(p, wp, wm + d)["H"]
            fd = fd4(H, 3e-4)
            assert abs(fd - g[site]) <= 1e-7 * abs(g[site]) + 5e-10, (site, which)


@pytest.mark.parametrize("scheme,f,ns", CASES)
def test_box_stress_fd(orc, scheme, f, ns):
    sh, L = (4, 6, 4), [2.0, 3.0, 2.5]
    wp, wm = fields(sh, 4)
    p = orc.Params(*sh, *L, ns, f, 15.0, 2.0, scheme, False)
    _, _, dL = orc.adjoint(p, wp, wm)
    for a in range(3):
        def H(e):
            La = list(L)
            La[a] += e
            return orc.evaluate(orc.Params(*sh, *La, ns, f, 15.0, 2.0, scheme, False), wp, wm)["H"]
        fd = fd4(H, 1e-3)
        assert abs(fd - dL[a]) <= 1e-8 * abs(dL[a]) + 1e-12, a


@pytest.mark.parametrize("bc,scheme", [((1, 0, 2), 0), ((2, 1, 0), 1), ((1, 1, 1), 0), ((2, 2, 2), 0)])
def test_box_stress_fd_with_walls(orc, bc, scheme):
    """Between walls each edge varied alone (the cell-centred grid scales with
    it; walled modes k = pi m / L): the reverse-mode dH/dL against finite
    differences of the oracle's walled H, periodic axes of the same box
    included."""
    sh, L = (4, 6, 4), [2.0, 3.0, 2.5]
    wp, wm = fields(sh, 8)
    p = orc.Params(*sh, *L, 9, 0.41, 15.0, 2.0, scheme, False, bc)
    _, _, dL = orc.adjoint(p, wp, wm)
    for a in range(3):
        def H(e):
            La = list(L)
            La[a] += e
            return orc.evaluate(orc.Params(*sh, *La, 9, 0.41, 15.0, 2.0, scheme, False, bc), wp, wm)["H"]
        fd = fd4(H, 1e-3)
        assert abs(fd - dL[a]) <= 1e-8 * abs(dL[a]) + 1e-12, (a, fd, dL[a])


@pytest.mark.parametrize("f,ns", [(0.5, 12), (0.3, 11)])
def test_split2_gradient_equals_force(orc, f, ns):
    sh, L = (6, 4, 4), (3.0, 2.0, 2.0)
    p = orc.Params(*sh, *L, ns, f, 12.0, 3.0, 1, False)
    wp, wm = fields(sh, 5)
    gp, gm, _ = orc.adjoint(p, wp, wm)
    r = orc.evaluate(p, wp, wm)
    Fp, Fm = orc.forces(p, wm, r["phiA"], r["phiB"])
    dV = p.volume / p.M
    assert np.abs(gp - p.C * dV * Fp).max() <= 1e-12 * np.abs(gp).max()
    assert np.abs(gm - p.C * dV * Fm).max() <= 1e-12 * np.abs(gm).max()


def test_rqm4_gradient_approaches_force(orc):
    # the analytic density force is the gradient only up to O(ds^2) under Eq. (12)
    sh, L = (4, 4, 4), (2.0, 2.0, 2.0)
    wp, wm = fields(sh, 6)
    errs = []
    for ns in (10, 20, 40):
        p = orc.Params(*sh, *L, ns, 0.5, 15.0, 1.0, 0, False)
        _, gm, _ = orc.adjoint(p, wp, wm)
        r = orc.evaluate(p, wp, wm)
        _, Fm = orc.forces(p, wm, r["phiA"], r["phiB"])
        errs.append(np.abs(gm - p.volume / p.M * Fm).max())
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5
