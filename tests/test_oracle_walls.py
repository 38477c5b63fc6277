"""Pins of the oracle's walled diffusion (reflecting = Neumann through the cosine
transform, absorbing = Dirichlet through the sine transform, on the cell-centred
grid x_n = (n + 1/2) L / N; Sec. III on boundary conditions).

- single eigenmodes cos / sin(pi m (n+1/2)/N) decay by exactly exp(-(pi m/L)^2 h);
- any field: equal to the periodic diffusion of its even / odd mirror image on
  [0, 2L) (numpy's FFT), restricted to the physical half -- the classical
  construction of the DCT-II / DST-II, independent of the oracle's sums;
- reflecting walls conserve the integral; with constant fields phi_A = f and
  Q = exp(-(f w_A + (1-f) w_B)) exactly, as with periodic boundaries;
- the walled operator is symmetric, so the per-node Q_j = Q and sum(phi) = M hold;
- with zero field and absorbing walls, Q is the survival fraction of the 1-D
  heat kernel.
"""
import numpy as np
import pytest


def P(orc, n=(8, 6, 10), L=(3.0, 2.5, 4.0), bc=(0, 0, 0), ns=10, f=0.4, scheme=0):
    return orc.Params(*n, *L, ns, f, 14.0, 1.0, scheme, False, tuple(bc))


def grid_axis(shape, axis):
    idx = np.arange(shape[axis]).reshape([-1 if a == axis else 1 for a in range(3)])
    return np.broadcast_to(idx, shape).astype(float)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("kind,m", [(1, 0), (1, 1), (1, 3), (2, 1), (2, 2), (2, 5)])
def test_single_wall_mode(orc, axis, kind, m):
    bc = [0, 0, 0]
    bc[axis] = kind
    p = P(orc, bc=bc)
    N, L = p.shape[axis], (p.lx, p.ly, p.lz)[axis]
    n = grid_axis(p.shape, axis)
    arg = np.pi * m * (n + 0.5) / N
    u = (np.cos(arg) if kind == 1 else np.sin(arg)) + 0j
    h = 0.07
    out = orc.diffuse(p, h, u)
    assert np.abs(out - np.exp(-(np.pi * m / L) ** 2 * h) * u).max() < 1e-13


def mirror_diffuse(u, L, bc, h):
    """Periodic diffusion of the mirror image (even for reflecting, odd for
    absorbing walls) on [0, 2L), axis by axis, with numpy's FFT."""
    u = u.copy()
    for axis in range(3):
        N = u.shape[axis]
        if bc[axis] == 0:
            k = 2 * np.pi * np.fft.fftfreq(N, d=L[axis] / N)
            shape = [-1 if a == axis else 1 for a in range(3)]
            u = np.fft.ifft(np.fft.fft(u, axis=axis) * np.exp(-k ** 2 * h).reshape(shape), axis=axis)
            continue
        sign = 1.0 if bc[axis] == 1 else -1.0
        ext = np.concatenate([u, sign * np.flip(u, axis=axis)], axis=axis)
        k = 2 * np.pi * np.fft.fftfreq(2 * N, d=L[axis] / N)
        shape = [-1 if a == axis else 1 for a in range(3)]
        ext = np.fft.ifft(np.fft.fft(ext, axis=axis) * np.exp(-k ** 2 * h).reshape(shape), axis=axis)
        u = np.take(ext, np.arange(N), axis=axis)
    return u


@pytest.mark.parametrize("bc", [(1, 0, 0), (0, 2, 0), (1, 2, 1), (2, 2, 2), (1, 1, 1)])
def test_walls_equal_mirror_image(orc, bc):
    p = P(orc, bc=bc)
    r = np.random.default_rng(7)
    u = r.standard_normal(p.shape) + 1j * r.standard_normal(p.shape)
    h = 0.05
    out = orc.diffuse(p, h, u)
    ref = mirror_diffuse(u, (p.lx, p.ly, p.lz), bc, h)
    assert np.abs(out - ref).max() < 1e-12


def test_reflecting_walls_conserve_mass(orc):
    p = P(orc, bc=(1, 1, 0))
    u = np.random.default_rng(8).standard_normal(p.shape) + 0j
    assert abs(orc.diffuse(p, 0.3, u).sum() - u.sum()) < 1e-12 * np.abs(u).sum()


@pytest.mark.parametrize("scheme", [0, 1])
def test_constant_fields_with_reflecting_walls(orc, scheme):
    p = P(orc, bc=(1, 1, 1), ns=13, f=0.37, scheme=scheme)
    a, b = 0.3 + 0.2j, -0.7 + 0.1j
    out = orc.evaluate(p, np.full(p.shape, -1j * a), np.full(p.shape, b))
    Q = np.exp(-(p.f * (a - b) + (1 - p.f) * (a + b)))
    assert abs(out["Q"] - Q) < 1e-13 * abs(Q)
    assert np.abs(out["phiA"] - p.f).max() < 1e-13


@pytest.mark.parametrize("bc", [(2, 0, 1), (1, 2, 2)])
def test_walled_invariants(orc, bc):
    p = P(orc, bc=bc, ns=12, f=0.45)
    r = np.random.default_rng(9)
    wp = 0.3 * r.standard_normal(p.shape) + 0.1j * r.standard_normal(p.shape)
    wm = 0.3 * r.standard_normal(p.shape) + 0.1j * r.standard_normal(p.shape)
    out = orc.evaluate(p, wp, wm)
    assert np.abs(out["Qnode"] - out["Q"]).max() < 1e-12 * abs(out["Q"])
    assert abs((out["phiA"] + out["phiB"]).sum() - p.M) < 1e-10 * p.M


def test_zero_field_absorbing_survival(orc):
    p = P(orc, n=(12, 4, 4), L=(3.0, 1.0, 1.0), bc=(2, 0, 0), ns=20, f=0.5, scheme=0)
    out = orc.evaluate(p, np.zeros(p.shape, complex), np.zeros(p.shape, complex))
    survival = mirror_diffuse(np.ones(p.shape, complex), (p.lx, p.ly, p.lz), p.bc, 1.0).mean()
    # Richardson steps of the exact diffusion with no field: the sweep is exact
    assert abs(out["Q"] - survival) < 1e-13
    assert abs(out["Q"]) < 1.0
