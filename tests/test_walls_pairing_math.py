"""The construction the walled kernels implement, checked on the CPU in numpy:
a line of N points between walls, reordered as (x0, x2, ..., x_{N-2}, x_{N-1},
..., x3, x1) (odd points sign-flipped between absorbing walls), transformed by
one N-point DFT in the four-step split the kernels use (N1 points per lane,
N2 lanes, spectrum element (k1, k2) = frequency k1 + N1 k2), with each
frequency m mixed with its partner N - m through
alpha_m = (g_m + g_{N-m}) / 2, beta_m = (g_m - g_{N-m}) exp(i pi m / N) / 2,
and transformed back, equals the periodic diffusion of the even / odd mirror
image on [0, 2L) (numpy's FFT), i.e. the cosine / sine mode diffusion.  The
partner of row k1 is row (N1 - k1) mod N1, column N2 - 1 - k2 (k1 > 0) or
(N2 - k2) mod N2 (k1 = 0)."""
import numpy as np
import pytest


def mirror_diffuse(x, L, h, bc):
    N = len(x)
    sign = 1.0 if bc == 1 else -1.0
    ext = np.concatenate([x, sign * x[::-1]])
    k = 2 * np.pi * np.fft.fftfreq(2 * N, d=L / N)
    return np.fft.ifft(np.fft.fft(ext) * np.exp(-k ** 2 * h))[:N]


def pair_factors(N, L, h, bc):
    def g(m):
        mode = (N - m) if bc == 2 else m
        return np.exp(-(np.pi * mode / L) ** 2 * h) / N
    al = np.zeros(N)
    be = np.zeros(N, complex)
    al[0] = g(0)
    for m in range(1, N):
        al[m] = 0.5 * (g(m) + g(N - m))
        be[m] = 0.5 * (g(m) - g(N - m)) * np.exp(1j * np.pi * m / N)
    return al, be


def four_step_pair_diffuse(v, N1, N2, al, be):
    N = N1 * N2
    S = np.empty((N1, N2), complex)  # S[k1, t]: lane t after its N1-point DFT and twiddle
    for t in range(N2):
        S[:, t] = np.fft.fft(v[t::N2]) * np.exp(-2j * np.pi * t * np.arange(N1) / N)
    X = np.fft.fft(S, axis=1)  # X[k1, k2] = V[k1 + N1 k2]
    Z = np.empty_like(X)
    for k1 in range(N1):
        k1p = (N1 - k1) % N1
        for k2 in range(N2):
            k2p = (N2 - k2) % N2 if k1 == 0 else N2 - 1 - k2
            m = k1 + N1 * k2
            assert k1p + N1 * k2p == (N - m) % N
            Z[k1, k2] = al[m] * X[k1, k2] + be[m] * X[k1p, k2p]
    S2 = np.fft.ifft(Z, axis=1) * N2
    out = np.empty(N, complex)
    for t in range(N2):
        out[t::N2] = np.fft.ifft(S2[:, t] * np.exp(2j * np.pi * t * np.arange(N1) / N)) * N1
    return out


SPLITS = [(8, 1), (12, 1), (20, 1), (12, 2), (16, 2), (20, 2), (12, 4), (16, 4), (20, 4), (24, 4), (16, 8), (24, 8),
          (16, 16)]


@pytest.mark.parametrize("N1,N2", SPLITS)
@pytest.mark.parametrize("bc", [1, 2])
def test_pairing_equals_mirror_image(N1, N2, bc):
    N = N1 * N2
    rng = np.random.default_rng(N + bc)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    L, h = 0.2 * N, 0.05
    idx = np.array([2 * n if n < N // 2 else 2 * (N - 1 - n) + 1 for n in range(N)])
    sgn = np.array([-1.0 if (bc == 2 and n >= N // 2) else 1.0 for n in range(N)])
    al, be = pair_factors(N, L, h, bc)
    v = four_step_pair_diffuse(sgn * x[idx], N1, N2, al, be)
    out = np.empty(N, complex)
    out[idx] = sgn * v
    ref = mirror_diffuse(x, L, h, bc)
    assert np.abs(out - ref).max() < 1e-13 * np.abs(ref).max()
