"""Pins of the oracle's semi-implicit step between reflecting walls (Eqs.
(10)-(11) with the linear response taken in the cosine basis of the walled
axes, k = pi m / L there):

- one cosine mode of the force moves w_+ by exactly -lam dt A / (1 + lam dt g_D(k^2));
- any fields: equal to the periodic step (Fourier basis, already pinned) on the
  even mirror image of period 2L along each walled axis, restricted to the
  physical half -- an independent route through the periodic code;
- the Edwards step likewise;
- absorbing walls are refused (their linear response is not diagonal in any
  mode basis).
"""
import numpy as np
import pytest


def P(orc, n, L, bc, ns=8, f=0.4, chiN=15.0, C=2.0):
    return orc.Params(*n, *L, ns, f, chiN, C, 0, False, tuple(bc))


def mirror(a, bc):
    for axis in range(3):
        if bc[axis]:
            a = np.concatenate([a, np.flip(a, axis=axis)], axis=axis)
    return a


def fields(shape, seed):
    r = np.random.default_rng(seed)
    z = lambda s: s * r.standard_normal(shape) + 0.05j * r.standard_normal(shape)
    return z(0.3), z(0.4), 0.5 + z(0.1), 0.5 + z(0.1)


@pytest.mark.parametrize("axis,m", [(0, 0), (0, 1), (1, 3), (2, 5)])
def test_single_cosine_mode(orc, axis, m):
    n, L = (8, 10, 12), (2.0, 2.5, 3.0)
    bc = [0, 0, 0]
    bc[axis] = 1
    p = P(orc, n, L, bc)
    idx = np.arange(n[axis]).reshape([-1 if a == axis else 1 for a in range(3)])
    s = np.broadcast_to(np.cos(np.pi * m * (idx + 0.5) / n[axis]), n).astype(complex)
    # phi_A = 1 - i s, phi_B = 0 gives F_+ = i (phi_A + phi_B - 1) = s
    phiA, phiB = 1.0 - 1j * s, np.zeros(n, complex)
    wp0 = np.zeros(n, complex)
    wm0 = np.zeros(n, complex)
    dt, lam = 0.3, 1.7
    wp, _ = orc.sis_update(p, wp0, wm0, phiA, phiB, dt, lam, 1.0)
    k = np.pi * m / L[axis]
    expect = -lam * dt * s / (1.0 + lam * dt * orc.debye(k * k))
    assert np.abs(wp - expect).max() < 1e-13


@pytest.mark.parametrize("bc", [(1, 0, 0), (0, 1, 1), (1, 1, 1)])
def test_reflecting_step_equals_periodic_mirror(orc, bc):
    # without noise: the draws are per site of each grid, so the image would not
    # carry the same numbers
    n, L = (6, 8, 10), (1.5, 2.0, 2.5)
    p = P(orc, n, L, bc)
    wp, wm, pa, pb = fields(n, 3)
    got_p, got_m = orc.sis_update(p, wp, wm, pa, pb, 0.4, 1.3, 0.8)
    ne = tuple(2 * n[a] if bc[a] else n[a] for a in range(3))
    Le = tuple(2 * L[a] if bc[a] else L[a] for a in range(3))
    pe = P(orc, ne, Le, (0, 0, 0))
    ref_p, ref_m = orc.sis_update(pe, mirror(wp, bc), mirror(wm, bc), mirror(pa, bc), mirror(pb, bc), 0.4, 1.3, 0.8)
    sl = tuple(slice(0, n[a]) for a in range(3))
    assert np.abs(got_p - ref_p[sl]).max() < 1e-13
    assert np.abs(got_m - ref_m[sl]).max() < 1e-13


def test_reflecting_edwards_step_equals_periodic_mirror(orc):
    n, L, bc = (8, 6, 10), (2.0, 1.5, 2.5), (0, 1, 1)
    p = P(orc, n, L, bc)
    om, _, phi, _ = fields(n, 4)
    got = orc.edwards_sis_update(p, 1.5, om, phi, 0.3, 1.1)
    ne = tuple(2 * n[a] if bc[a] else n[a] for a in range(3))
    Le = tuple(2 * L[a] if bc[a] else L[a] for a in range(3))
    ref = orc.edwards_sis_update(P(orc, ne, Le, (0, 0, 0)), 1.5, mirror(om, bc), mirror(phi, bc), 0.3, 1.1)
    assert np.abs(got - ref[tuple(slice(0, k) for k in n)]).max() < 1e-13


def test_absorbing_walls_refused(orc):
    p = P(orc, (8, 8, 8), (2.0,) * 3, (0, 2, 0))
    z = np.zeros((8, 8, 8), complex)
    with pytest.raises(ValueError):
        orc.sis_update(p, z, z, z, z, 0.1)
