"""Pins of the oracle's discrete Fourier transforms.

The oracle's recursive FFT is checked against the O(M^2) definition, both
against numpy's FFT (an independent library routine), and against the
transform's own identities (impulse <-> constant, Parseval, inversion)."""
import numpy as np
import pytest

SHAPES = [(4, 4, 4), (6, 8, 10), (3, 5, 2), (12, 12, 12), (8, 9, 5), (7, 4, 11)]


def rand(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft_matches_definition(orc, shape, sign):
    a = rand(shape, 1)
    ref = orc.dft3_naive(a, sign)
    got = orc.fft3(a, sign)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("shape", SHAPES)
def test_definition_matches_numpy(orc, shape):
    a = rand(shape, 2)
    assert np.allclose(orc.dft3_naive(a, -1), np.fft.fftn(a), rtol=0, atol=1e-11)
    assert np.allclose(orc.dft3_naive(a, +1), np.fft.ifftn(a) * a.size, rtol=0, atol=1e-11)


@pytest.mark.parametrize("n", [16, 24, 32, 40, 48, 64, 96, 128, 256])
def test_fft_numpy_every_axis_length(orc, n):
    a = rand((n, 4, 3), 3)
    assert np.abs(orc.fft3(a, -1) - np.fft.fftn(a)).max() <= 1e-12 * np.abs(a).sum() ** 0.5 * n
    b = rand((2, 3, n), 4)
    assert np.abs(orc.fft3(b, -1) - np.fft.fftn(b)).max() <= 1e-12 * np.abs(b).sum() ** 0.5 * n


def test_impulse_and_constant(orc):
    shape = (6, 10, 8)
    imp = np.zeros(shape, complex)
    imp[0, 0, 0] = 1.0
    assert np.allclose(orc.fft3(imp), 1.0, atol=1e-15)
    const = np.ones(shape, complex)
    out = orc.fft3(const)
    expect = np.zeros(shape, complex)
    expect[0, 0, 0] = const.size
    assert np.allclose(out, expect, atol=1e-12)


def test_parseval_and_inversion(orc):
    a = rand((10, 12, 6), 5)
    A = orc.fft3(a, -1)
    assert np.isclose((np.abs(A) ** 2).sum(), a.size * (np.abs(a) ** 2).sum(), rtol=1e-13)
    back = orc.fft3(A, +1) / a.size
    assert np.abs(back - a).max() < 1e-13


def test_linearity(orc):
    a, b = rand((6, 6, 6), 6), rand((6, 6, 6), 7)
    lhs = orc.fft3(2.5 * a - 1j * b)
    rhs = 2.5 * orc.fft3(a) - 1j * orc.fft3(b)
    assert np.abs(lhs - rhs).max() < 1e-12


def test_integer_modes(orc):
    # m(j) = j for j <= n/2, j - n above: numpy's fftfreq * n, except the
    # Nyquist sign, which never matters because only m^2 enters.
    for n in (4, 5, 16, 24, 25, 128):
        m = np.array([orc.mode(j, n) for j in range(n)])
        ref = np.rint(np.fft.fftfreq(n) * n).astype(int)
        assert np.array_equal(m ** 2, ref ** 2)
        assert np.array_equal(np.abs(m), np.abs(ref))
