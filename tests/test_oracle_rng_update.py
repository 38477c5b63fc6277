"""Pins of the oracle's noise stream and field update.

* Philox4x64-10 words equal numpy's independent implementation of the same
  published generator (numpy increments the counter before encrypting, so
  its state is set one below the counter the oracle encrypts).
* The Box-Muller normals have the moments of N(0, 1) and no lag correlation,
  and the update's noise has the discrete variance 2 lam dt / (C dV) stated
  after Eq. (10).
* The deterministic update is the drift -lam dt F, and F_+ has no k = 0 mode
  because the total density sums to M.
* Independently of the update's own formula: under the plain split step
  dH/dw = C dV F exactly, so one noise-free step must lower H by
  lam dt C dV sum F^2 to first order, with a residual that halves with dt
  (this fixes the drift's sign, its lam dt scale and which force drives
  which field).
"""
import numpy as np
import pytest


@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (0, 0, 0, 0)),
    ((1206, 3), (17, 1, 999, 0)),
    ((2 ** 64 - 1, 12345), (2 ** 63 + 5, 2 ** 40, 7, 2 ** 64 - 2)),
])
def test_philox_matches_numpy(orc, key, ctr):
    got = orc.philox4x64_10(np.array(ctr, np.uint64), np.array(key, np.uint64))
    # numpy's Philox adds one to the 256-bit counter (word 0 least significant)
    # before each block, so start it one below.
    value = sum(int(w) << (64 * i) for i, w in enumerate(ctr))
    value = (value - 1) % 2 ** 256
    c = [(value >> (64 * i)) & (2 ** 64 - 1) for i in range(4)]
    bg = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(c, np.uint64))
    ref = bg.random_raw(4)
    assert np.array_equal(got, ref)


def test_gaussian_moments_and_independence(orc):
    M = 1 << 18
    xi = orc.gaussian(1206, 0, 5, 0, M)
    assert abs(xi.mean()) < 5 / np.sqrt(M)
    assert abs(xi.var() - 1) < 5 * np.sqrt(2 / M)
    assert abs(np.mean(xi[1:] * xi[:-1])) < 5 / np.sqrt(M)
    assert abs(np.mean(xi ** 4) - 3) < 0.05
    # distinct field / step / replica give uncorrelated streams
    for other in (orc.gaussian(1206, 0, 5, 1, M), orc.gaussian(1206, 0, 6, 0, M),
                  orc.gaussian(1206, 1, 5, 0, M)):
        assert abs(np.mean(xi * other)) < 5 / np.sqrt(M)
    # counter-based: a prefix of the stream does not depend on the length asked for
    assert np.array_equal(orc.gaussian(1206, 0, 5, 0, 10), xi[:10])


def test_em_update_drift_and_noise(orc):
    p = orc.Params(8, 8, 8, 3.0, 3.0, 3.0, 10, 0.4, 20.0, 50.0, 0, False)
    r = np.random.default_rng(9)
    wp = 0.2 * r.standard_normal(p.shape) + 0.05j * r.standard_normal(p.shape)
    wm = 0.2 * r.standard_normal(p.shape) + 0.05j * r.standard_normal(p.shape)
    out = orc.evaluate(p, wp, wm)
    Fp, Fm = orc.forces(p, wm, out["phiA"], out["phiB"])
    assert abs(Fp.sum()) < 1e-10 * p.M          # no k = 0 mode in F_+
    dt, lp, lm = 0.01, 1.0, 0.5
    wp1, wm1 = orc.em_update(p, wp, wm, out["phiA"], out["phiB"], dt, lp, lm)
    assert np.allclose(wp1, wp - lp * dt * Fp, atol=1e-15)
    assert np.allclose(wm1, wm - lm * dt * Fm, atol=1e-15)
    wp2, wm2 = orc.em_update(p, wp, wm, out["phiA"], out["phiB"], dt, lp, lm, noise=True,
                             seed=1206, replica=0, step_=3)
    dV = 27.0 / p.M
    np_ = (wp2 - wp1) / np.sqrt(2 * lp * dt / (p.C * dV))
    nm = (wm2 - wm1) / np.sqrt(2 * lm * dt / (p.C * dV))
    assert np.abs(np_.imag).max() < 1e-12 and np.abs(nm.imag).max() < 1e-12   # real noise
    assert np.allclose(np_.real.ravel(), orc.gaussian(1206, 0, 3, 0, p.M), atol=1e-9)
    assert np.allclose(nm.real.ravel(), orc.gaussian(1206, 0, 3, 1, p.M), atol=1e-9)


def _descent_ratios(dH_of_dt, predicted_of_dt, dts):
    """(dH - predicted) / predicted for each dt; the drift is right in sign and
    scale when this tends to 0 and halves with dt (a first-order residual)."""
    return [(dH_of_dt(dt) - predicted_of_dt(dt)) / predicted_of_dt(dt) for dt in dts]


def _check_first_order(rel):
    assert abs(rel[-1]) < 2e-2, rel
    for a, b in zip(rel, rel[1:]):
        assert 1.8 < abs(a / b) < 2.2, rel


@pytest.mark.parametrize("moving", ["plus", "minus"])
def test_em_drift_is_first_order_descent_of_H(orc, moving):
    """Eq. (9) without noise moves a field against its force.  Under the plain
    split step with trapezoid contour sums dH/dw = C dV F exactly (pinned by
    central differences of H elsewhere), so one step changes H by
    -lam dt C dV sum_x F^2 (complex square: H is holomorphic) to first order in
    dt.  The update is taken from em_update and H from evaluate, so a sign flip
    of the drift, dt in place of lam dt, or the wrong force on a field fails."""
    p = orc.Params(6, 8, 4, 3.0, 3.5, 2.5, 16, 0.4, 15.0, 7.0, orc.SPLIT2, False)
    r = np.random.default_rng(41)
    wp = 0.3 * r.standard_normal(p.shape) + 0.08j * r.standard_normal(p.shape)
    wm = 0.4 * r.standard_normal(p.shape) + 0.08j * r.standard_normal(p.shape)
    base = orc.evaluate(p, wp, wm)
    Fp, Fm = orc.forces(p, wm, base["phiA"], base["phiB"])
    dV = p.volume / p.M
    lam_p, lam_m = (0.7, 0.0) if moving == "plus" else (0.0, 1.3)
    F, lam = (Fp, lam_p) if moving == "plus" else (Fm, lam_m)

    def dH(dt):
        wp1, wm1 = orc.em_update(p, wp, wm, base["phiA"], base["phiB"], dt, lam_p, lam_m)
        # the field that is not driven stays put
        assert np.array_equal(wm1 if moving == "plus" else wp1, wm if moving == "plus" else wp)
        return orc.evaluate(p, wp1, wm1)["H"] - base["H"]

    def predicted(dt):
        return -lam * dt * p.C * dV * np.sum(F * F)

    _check_first_order(_descent_ratios(dH, predicted, [4e-3, 2e-3, 1e-3]))


def test_em_drift_both_fields_adds_the_two_descents(orc):
    """Both fields moving at once: the first-order change of H is the sum of
    the two fields' -lam dt C dV sum F^2 terms, each with its own mobility."""
    p = orc.Params(4, 6, 6, 2.5, 3.0, 3.0, 12, 0.5, 12.0, 3.0, orc.SPLIT2, False)
    r = np.random.default_rng(42)
    wp = 0.2 * r.standard_normal(p.shape) + 0.05j * r.standard_normal(p.shape)
    wm = 0.5 * r.standard_normal(p.shape) + 0.05j * r.standard_normal(p.shape)
    base = orc.evaluate(p, wp, wm)
    Fp, Fm = orc.forces(p, wm, base["phiA"], base["phiB"])
    dV = p.volume / p.M
    lam_p, lam_m = 1.6, 0.45

    def dH(dt):
        wp1, wm1 = orc.em_update(p, wp, wm, base["phiA"], base["phiB"], dt, lam_p, lam_m)
        return orc.evaluate(p, wp1, wm1)["H"] - base["H"]

    def predicted(dt):
        return -dt * p.C * dV * (lam_p * np.sum(Fp * Fp) + lam_m * np.sum(Fm * Fm))

    _check_first_order(_descent_ratios(dH, predicted, [4e-3, 2e-3, 1e-3]))
