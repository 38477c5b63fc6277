"""Pins of the oracle's semi-implicit field step (Eq. (10), effective step
Eq. (11)): every Fourier mode of the explicit increment is divided by
1 + lam dt g(k), with g = g_D(|k|^2) for w_+, 2/chiN for w_-, B/C + g_D for the
Edwards field.

- g_D against its series summed in exact rational arithmetic (x < 1) and the
  direct form (x >= 1);
- a force made of one cosine mode (any axis mix, distinct box edges) moves the
  field by exactly -lam dt A cos / (1 + lam dt g(|k|^2)), and a uniform force
  by -lam dt A / (1 + lam dt g(0)), g_D(0) = 1;
- the noise goes through the same filter: checked against numpy's FFT;
- the w_- update is local: -(lam dt F_- - s xi) / (1 + 2 lam dt / chiN).
"""
import math
from fractions import Fraction

import numpy as np
import pytest


def P(orc, n=(8, 6, 10), L=(3.0, 2.5, 4.0), ns=10, chiN=14.0, C=2.0):
    return orc.Params(*n, *L, ns, 0.5, chiN, C, 0, False)


def gd_ref(x):
    """g_D(x) = 2 (e^-x + x - 1)/x^2: for x < 1 its series summed in exact
    rational arithmetic, above that the direct form (no cancellation there)."""
    if x >= 1.0:
        return 2.0 * (math.exp(-x) + x - 1.0) / x ** 2
    X = Fraction(x)
    return float(sum(2 * (-X) ** m / math.factorial(m + 2) for m in range(40)))


@pytest.mark.parametrize("x", [0.0, 1e-8, 1e-4, 0.03, 0.0999, 0.1, 0.35, 0.4999, 0.5, 0.9, 2.0, 40.0])
def test_debye_function(orc, x):
    assert abs(orc.debye(x) - gd_ref(x)) <= 4e-16


def mode(p, m):
    """cos(k.r) on the grid for integer mode m, and |k|^2."""
    idx = np.meshgrid(*(np.arange(k) for k in p.shape), indexing="ij")
    ph = sum(2 * np.pi * m[a] * idx[a] / p.shape[a] for a in range(3))
    k2 = sum((2 * np.pi * m[a] / (p.lx, p.ly, p.lz)[a]) ** 2 for a in range(3))
    return np.cos(ph), k2


@pytest.mark.parametrize("m", [(1, 0, 0), (0, 2, -1), (3, -1, 4), (4, 3, 5)])
def test_single_mode_pressure_force(orc, m):
    p = P(orc)
    cos, k2 = mode(p, m)
    A, dt, lam = 0.7, 0.3, 1.3
    # phi_A + phi_B = 1 - i A cos gives F_+ = A cos; phi_A = phi_B, w_- = 0 gives F_- = 0
    phi = 0.5 * (1 - 1j * A * cos)
    wp = np.zeros(p.shape, complex)
    wm = np.zeros(p.shape, complex)
    nwp, nwm = orc.sis_update(p, wp, wm, phi, phi, dt, lam, lam)
    expect = -lam * dt * A * cos / (1 + lam * dt * gd_ref(k2))
    assert np.abs(nwp - expect).max() < 1e-14
    assert np.abs(nwm).max() == 0.0


def test_uniform_pressure_force(orc):
    p = P(orc)
    A, dt = 0.4, 0.2
    phi = np.full(p.shape, 0.5 * (1 - 1j * A))
    nwp, _ = orc.sis_update(p, np.zeros(p.shape), np.zeros(p.shape), phi, phi, dt)
    assert np.abs(nwp - (-dt * A / (1 + dt))).max() < 1e-15


def test_exchange_field_is_local(orc):
    p = P(orc)
    r = np.random.default_rng(3)
    wm = 0.3 * r.standard_normal(p.shape) + 0.1j * r.standard_normal(p.shape)
    phiA = 0.5 + 0.1 * r.standard_normal(p.shape)
    phiB = 1 - phiA
    dt, lam = 0.5, 0.8
    _, nwm = orc.sis_update(p, np.zeros(p.shape), wm, phiA, phiB, dt, 1.0, lam)
    Fm = 2 * wm / p.chiN + phiB - phiA
    assert np.abs(nwm - (wm - lam * dt * Fm / (1 + 2 * lam * dt / p.chiN))).max() < 1e-15


def test_noise_filtered_like_the_force(orc):
    p = P(orc, n=(8, 8, 12), L=(4.0, 3.0, 5.0), C=3.0)
    dt, lam = 0.25, 1.1
    phi = np.full(p.shape, 0.5 + 0j)    # zero forces
    wp0 = np.zeros(p.shape, complex)
    nwp, nwm = orc.sis_update(p, wp0, wp0, phi, phi, dt, lam, lam, noise=True, seed=5, replica=1, step_=9)
    dV = np.prod((p.lx, p.ly, p.lz)) / p.M
    s = math.sqrt(2 * lam * dt / (p.C * dV))
    xp = orc.gaussian(5, 1, 9, 0, p.M).reshape(p.shape)
    xm = orc.gaussian(5, 1, 9, 1, p.M).reshape(p.shape)
    k = [2 * np.pi * np.fft.fftfreq(n, d=L / n) for n, L in zip(p.shape, (p.lx, p.ly, p.lz))]
    K2 = k[0][:, None, None] ** 2 + k[1][None, :, None] ** 2 + k[2][None, None, :] ** 2
    g = np.vectorize(gd_ref)(K2)
    expect = np.fft.ifftn(np.fft.fftn(s * xp) / (1 + lam * dt * g))
    assert np.abs(nwp - expect).max() < 1e-13
    assert np.abs(nwm - s * xm / (1 + 2 * lam * dt / p.chiN)).max() < 1e-14


@pytest.mark.parametrize("m", [(0, 0, 0), (2, -1, 3)])
def test_edwards_single_mode(orc, m):
    p = P(orc, C=4.0)
    Bv, A, dt, lam = 2.0, 0.3, 0.4, 0.9
    cos, k2 = mode(p, m)
    phi = 1 - 1j * A * cos                # F = (B/C) 0 + i phi = i + A cos
    om = orc.edwards_sis_update(p, Bv, np.zeros(p.shape), phi, dt, lam)
    g0 = Bv / p.C + 1.0
    gk = Bv / p.C + gd_ref(k2)
    if m == (0, 0, 0):
        expect = -lam * dt * (1j + A) / (1 + lam * dt * g0) * np.ones(p.shape)
    else:
        expect = -lam * dt * 1j / (1 + lam * dt * g0) - lam * dt * A * cos / (1 + lam * dt * gk)
    assert np.abs(om - expect).max() < 1e-14
