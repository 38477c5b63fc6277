// Device building blocks of the pseudo-spectral diffusion operator: complex
// arithmetic, compile-time unit roots, in-register DFTs, and the two-stage
// (four-step) line transform spread over a few lanes with one LDS exchange
// per direction.
//
// The diffusion factor exp(-k^2 h) of the modified diffusion equation
// (Eq. (5)) is separable over the axes, so a three-dimensional diffusion is
// three commuting one-dimensional ones (Sec. III, the pseudo-spectral split
// step).  Each one-dimensional diffusion here runs forward DFT -> multiply by
// the axis factor g(k) = exp(-(2 pi m / L)^2 h) / N -> inverse DFT entirely on
// chip; the spectrum is never written to memory and never reordered.
//
// Twiddles are evaluated in double precision at compile time (Taylor series on
// an exact integer reduction of the angle) and rounded once to the working
// precision; a twiddle that depends on the lane is the product of at most two
// such table entries, and nothing comes from a recurrence.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace pft {

// ---------------------------------------------------------------- complex --
template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
// multiply by -i (forward) or +i (inverse) quarter turns
template <typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return {a.im, -a.re}; }
template <typename T>
__device__ __forceinline__ cx<T> mul_pi(cx<T> a) { return {-a.im, a.re}; }

// Streaming access to data that is written once and read back only much later
// (the stored propagator slices): nontemporal, so that it does not displace the
// arrays every pass re-reads from the caches.
template <typename T>
__device__ __forceinline__ void store_stream(cx<T>* p, cx<T> v)
{
    using V2 = T __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(V2{v.re, v.im}, reinterpret_cast<V2*>(p));
}
template <typename T>
__device__ __forceinline__ cx<T> load_stream(const cx<T>* p)
{
    using V2 = T __attribute__((ext_vector_type(2)));
    const V2 v = __builtin_nontemporal_load(reinterpret_cast<const V2*>(p));
    return {v.x, v.y};
}

// ------------------------------------------------------ compile-time loops --
template <int B, int E, class F>
__device__ __forceinline__ void sfor(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

// ------------------------------------------------- compile-time unit roots --
namespace detail {
constexpr double kHalfPi = 1.57079632679489661923132169163975144;

constexpr double sin_series(double x)
{
    // |x| <= pi/4; terms summed smallest first
    double terms[14] = {};
    double t = x;
    terms[0] = x;
    for (int k = 1; k < 14; ++k) {
        t *= -x * x / double((2 * k) * (2 * k + 1));
        terms[k] = t;
    }
    double s = 0.0;
    for (int k = 13; k >= 0; --k) s += terms[k];
    return s;
}

constexpr double cos_series(double x)
{
    double terms[14] = {};
    double t = 1.0;
    terms[0] = 1.0;
    for (int k = 1; k < 14; ++k) {
        t *= -x * x / double((2 * k - 1) * (2 * k));
        terms[k] = t;
    }
    double s = 0.0;
    for (int k = 13; k >= 0; --k) s += terms[k];
    return s;
}

// cos and sin of 2 pi a / n: exact quadrant reduction in integers, then a
// series on an angle of at most pi/4.
constexpr double root_cs(long a, long n, bool want_sin)
{
    const long r = ((a % n) + n) % n;
    const long q = (4 * r) / n;
    const long rem = 4 * r - q * n;  // angle within the quadrant = (pi/2) rem / n
    double c0 = 0.0, s0 = 0.0;
    if (2 * rem <= n) {
        const double p = kHalfPi * double(rem) / double(n);
        c0 = cos_series(p);
        s0 = sin_series(p);
    } else {
        const double p = kHalfPi * double(n - rem) / double(n);
        c0 = sin_series(p);
        s0 = cos_series(p);
    }
    double c = 0.0, s = 0.0;
    switch (q) {
    case 0: c = c0; s = s0; break;
    case 1: c = -s0; s = c0; break;
    case 2: c = -c0; s = -s0; break;
    default: c = s0; s = -c0; break;
    }
    return want_sin ? s : c;
}
}  // namespace detail

// Table of e^{-2 pi i j / N}, j < N, in working precision T.
template <typename T, int N>
struct RootTable {
    cx<T> w[N];
    constexpr RootTable() : w()
    {
        for (int j = 0; j < N; ++j) {
            w[j].re = T(detail::root_cs(j, N, false));
            w[j].im = T(-detail::root_cs(j, N, true));
        }
    }
};

template <typename T, int N>
__constant__ constexpr RootTable<T, N> kRoots = RootTable<T, N>();

// x * e^{-+2 pi i A / N} with A, N known at compile time (forward: minus).
template <int A, int N, bool INV, typename T>
__device__ __forceinline__ cx<T> rot(cx<T> x)
{
    constexpr int a = ((A % N) + N) % N;
    if constexpr (a == 0) {
        return x;
    } else if constexpr (2 * a == N) {
        return {-x.re, -x.im};
    } else if constexpr (4 * a == N) {
        return INV ? mul_pi(x) : mul_mi(x);
    } else if constexpr (4 * a == 3 * N) {
        return INV ? mul_mi(x) : mul_pi(x);
    } else {
        constexpr T c = T(detail::root_cs(a, N, false));
        constexpr T s = T(detail::root_cs(a, N, true));
        // forward factor c - i s, inverse c + i s
        if constexpr (INV)
            return {c * x.re - s * x.im, c * x.im + s * x.re};
        else
            return {c * x.re + s * x.im, c * x.im - s * x.re};
    }
}

// a[k1] *= W_N^{-+ t k1} for k1 = 1 .. N1-1 (forward: minus).  With k1 = 4 m + l
// the factor is the product of the table entries W^{t l} and W^{4 t m}, so a
// lane reads 3 + (N1 - 1) / 4 roots instead of N1 - 1.
template <int N1, int N, bool INV, typename T>
__device__ __forceinline__ void twiddle(cx<T> (&a)[N1], int t)
{
    constexpr int ML = (N1 - 1) / 4;
    cx<T> lo[4], hi[ML + 1];
    sfor<1, (N1 < 4 ? N1 : 4)>([&](auto L) {
        constexpr int l = decltype(L)::value;
        lo[l] = kRoots<T, N>.w[(t * l) % N];
    });
    sfor<1, ML + 1>([&](auto Mi) {
        constexpr int m = decltype(Mi)::value;
        hi[m] = kRoots<T, N>.w[(t * 4 * m) % N];
    });
    sfor<1, N1>([&](auto K1) {
        constexpr int k1 = decltype(K1)::value;
        constexpr int l = k1 % 4, m = k1 / 4;
        cx<T> w;
        if constexpr (m == 0) {
            w = lo[l];
        } else if constexpr (l == 0) {
            w = hi[m];
        } else {
            w = lo[l] * hi[m];
        }
        const cx<T> x = a[k1];
        if constexpr (INV)
            a[k1] = {w.re * x.re + w.im * x.im, w.re * x.im - w.im * x.re};
        else
            a[k1] = {w.re * x.re - w.im * x.im, w.re * x.im + w.im * x.re};
    });
}

// ------------------------------------------------------ in-register DFTs --
// dft<R, INV>(v): v[k] <- sum_n v[n] e^{-+2 pi i n k / R}, unnormalised.
template <int R, bool INV, typename T>
__device__ __forceinline__ void dft(cx<T>* v);

template <bool INV, typename T>
__device__ __forceinline__ void dft2(cx<T>* v)
{
    const cx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
}

template <bool INV, typename T>
__device__ __forceinline__ void dft3(cx<T>* v)
{
    constexpr T h = T(0.5);
    constexpr T s = T(0.86602540378443864676372317075293618);  // sin(2 pi / 3)
    const cx<T> a0 = v[0], t = v[1] + v[2], d = v[1] - v[2];
    const cx<T> m = {a0.re - h * t.re, a0.im - h * t.im};
    const cx<T> sd = s * d;
    v[0] = a0 + t;
    if constexpr (INV) {
        v[1] = m + mul_pi(sd);
        v[2] = m + mul_mi(sd);
    } else {
        v[1] = m + mul_mi(sd);
        v[2] = m + mul_pi(sd);
    }
}

template <bool INV, typename T>
__device__ __forceinline__ void dft4(cx<T>* v)
{
    const cx<T> s02 = v[0] + v[2], d02 = v[0] - v[2];
    const cx<T> s13 = v[1] + v[3], d13 = v[1] - v[3];
    v[0] = s02 + s13;
    v[2] = s02 - s13;
    if constexpr (INV) {
        v[1] = d02 + mul_pi(d13);
        v[3] = d02 + mul_mi(d13);
    } else {
        v[1] = d02 + mul_mi(d13);
        v[3] = d02 + mul_pi(d13);
    }
}

template <bool INV, typename T>
__device__ __forceinline__ void dft5(cx<T>* v)
{
    constexpr T c1 = T(0.30901699437494742410229341718281906);   // cos(2 pi / 5)
    constexpr T c2 = T(-0.80901699437494742410229341718281906);  // cos(4 pi / 5)
    constexpr T s1 = T(0.95105651629515357211643933337938214);   // sin(2 pi / 5)
    constexpr T s2 = T(0.58778525229247312916870595463907277);   // sin(4 pi / 5)
    const cx<T> a0 = v[0];
    const cx<T> b1 = v[1] + v[4], d1 = v[1] - v[4];
    const cx<T> b2 = v[2] + v[3], d2 = v[2] - v[3];
    const cx<T> r1 = a0 + c1 * b1 + c2 * b2;
    const cx<T> r2 = a0 + c2 * b1 + c1 * b2;
    const cx<T> i1 = s1 * d1 + s2 * d2;
    const cx<T> i2 = s2 * d1 - s1 * d2;
    v[0] = a0 + b1 + b2;
    if constexpr (INV) {
        v[1] = r1 + mul_pi(i1);
        v[4] = r1 + mul_mi(i1);
        v[2] = r2 + mul_pi(i2);
        v[3] = r2 + mul_mi(i2);
    } else {
        v[1] = r1 + mul_mi(i1);
        v[4] = r1 + mul_pi(i1);
        v[2] = r2 + mul_mi(i2);
        v[3] = r2 + mul_pi(i2);
    }
}

template <int R>
constexpr int first_factor()
{
    return (R % 4 == 0 && R > 4) ? 4 : (R % 2 == 0) ? 2 : (R % 3 == 0) ? 3 : 5;
}

// Composite R = A * B by the four-step split, all indices compile-time so the
// whole transform lives in registers:
//   X[k1 + A k2] = sum_n2 W_B^{n2 k2} W_R^{n2 k1} sum_n1 v[B n1 + n2] W_A^{n1 k1}.
template <int R, bool INV, typename T>
__device__ __forceinline__ void dft(cx<T>* v)
{
    if constexpr (R == 1) {
    } else if constexpr (R == 2) {
        dft2<INV>(v);
    } else if constexpr (R == 3) {
        dft3<INV>(v);
    } else if constexpr (R == 4) {
        dft4<INV>(v);
    } else if constexpr (R == 5) {
        dft5<INV>(v);
    } else {
        constexpr int A = first_factor<R>();
        constexpr int B = R / A;
        static_assert(A * B == R, "unsupported radix");
        cx<T> u[B][A];
        sfor<0, B>([&](auto N2) {
            constexpr int n2 = decltype(N2)::value;
            sfor<0, A>([&](auto N1) { u[n2][decltype(N1)::value] = v[B * decltype(N1)::value + n2]; });
            dft<A, INV>(u[n2]);
            sfor<1, A>([&](auto K1) {
                constexpr int k1 = decltype(K1)::value;
                u[n2][k1] = rot<n2 * k1, R, INV>(u[n2][k1]);
            });
        });
        sfor<0, A>([&](auto K1) {
            constexpr int k1 = decltype(K1)::value;
            cx<T> s[B];
            sfor<0, B>([&](auto N2) { s[decltype(N2)::value] = u[decltype(N2)::value][k1]; });
            dft<B, INV>(s);
            sfor<0, B>([&](auto K2) { v[k1 + A * decltype(K2)::value] = s[decltype(K2)::value]; });
        });
    }
}

// ---------------------------------------------------- line diffusion -------
// One line of N = N1 * N2 points is held by N2 lanes; lane t owns the points
// n = n1 * N2 + t (n1 < N1) in a[n1].  diffuse() replaces the line by
// IDFT( g(k) DFT(line) ), with g in natural frequency order (1/N folded in).
//
// Forward: an N1-point DFT in registers over n1, the twiddle W_N^{t k1}, an
// LDS transpose, then N1/N2 DFTs of N2 points per lane give X[k1 + N1 k2] for
// the lane's k1 = t + N2 i.  The factor g is applied there, and the inverse
// retraces the same steps, so the spectrum never needs natural order.  Two
// barriers per direction change suffice: the rows k1 of the stage-two matrix
// belong to one lane each.
//
// lay(k1, n2) maps an element of the exchanged N1 x N2 matrix of this lane's
// line to its LDS slot.  Every lane of the workgroup must call diffuse()
// (it contains barriers); lanes without a line pass zeros.
//
// MEAN (diffusion factors, whose k = 0 entry is 1/N): in complex float the
// k = 0 mode is divided by N in double and rounded once, instead of being
// multiplied by 1/N rounded to float.  1/N is not a float for N with a factor
// 3 or 5, and its rounding error would scale the mean of q by the same factor
// in every pass of every contour step, an error that grows linearly with the
// number of steps in Q.
template <int N, typename T>
__device__ __forceinline__ cx<T> mean_over_n(cx<T> x)
{
    constexpr double inv = 1.0 / N;
    return {T(double(x.re) * inv), T(double(x.im) * inv)};
}

template <int N1, int N2, bool MEAN = false, typename T, class Lay, class G>
__device__ __forceinline__ void diffuse(cx<T> (&a)[N1], int t, cx<T>* __restrict__ sh, const Lay& lay, const G& g)
{
    constexpr int N = N1 * N2;
    constexpr bool kMean = MEAN && std::is_same<T, float>::value;
    if constexpr (N2 == 1) {
        dft<N1, false>(a);
        sfor<0, N1>([&](auto K) {
            constexpr int k = decltype(K)::value;
            if constexpr (kMean && k == 0) {
                a[0] = mean_over_n<N>(a[0]);
            } else {
                const T gk = g[k];
                a[k] = gk * a[k];
            }
        });
        dft<N1, true>(a);
    } else {
        static_assert(N1 % N2 == 0, "each lane must own whole stage-two transforms");
        constexpr int NB = N1 / N2;
        dft<N1, false>(a);
        twiddle<N1, N, false>(a, t);
        __syncthreads();
        sfor<0, N1>([&](auto K1) { sh[lay(decltype(K1)::value, t)] = a[decltype(K1)::value]; });
        __syncthreads();
        // stage two: row k1 of the exchanged matrix is read and written back by
        // its owning lane only, so each row goes back as soon as it is done
        sfor<0, NB>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const int k1 = t + N2 * i;
            cx<T> b[N2];
            sfor<0, N2>([&](auto M2) { b[decltype(M2)::value] = sh[lay(k1, decltype(M2)::value)]; });
            dft<N2, false>(b);
            sfor<0, N2>([&](auto K2) {
                constexpr int k2 = decltype(K2)::value;
                const T gk = g[k1 + N1 * k2];
                if constexpr (kMean && i == 0 && k2 == 0)
                    b[0] = (t == 0) ? mean_over_n<N>(b[0]) : gk * b[0];  // k1 = t: lane 0 holds k = 0
                else
                    b[k2] = gk * b[k2];
            });
            dft<N2, true>(b);
            sfor<0, N2>([&](auto M2) { sh[lay(k1, decltype(M2)::value)] = b[decltype(M2)::value]; });
        });
        __syncthreads();
        sfor<0, N1>([&](auto K1) { a[decltype(K1)::value] = sh[lay(decltype(K1)::value, t)]; });
        twiddle<N1, N, true>(a, t);
        dft<N1, true>(a);
    }
}

// ------------------------------------------------- diffusion between walls --
// A line of N points between walls (Sec. III: cosine modes for reflecting,
// sine modes for absorbing walls) is held in the order v[n] = x[2n] for
// n < N/2 and v[n] = x[2(N-1-n)+1] for n >= N/2, absorbing walls with the
// sign of the odd points x flipped.  One N-point DFT V of v then carries the
// cosine coefficients of x as C[m] = (w_m V[m] + conj(w_m) V[N-m]) / 2,
// w_m = exp(-i pi m / 2N), so multiplying each mode by g_m and transforming
// back is, per frequency,
//   V'[m] = alpha_m V[m] + beta_m V[(N-m) mod N],
//   alpha_m = (g_m + g_{N-m}) / 2,  beta_m = (g_m - g_{N-m}) exp(i pi m / N) / 2
// (alpha_0 = g_0, beta_0 = 0; absorbing walls use g_m of sine mode N - m).
// ab holds (alpha_m, Re beta_m, Im beta_m) for m = 0..N-1 with 1/N folded in.
// The pairing of m with N - m crosses lanes, so the stage-two spectrum goes
// through LDS once more than in diffuse(); same calling rules as diffuse().
template <int N1, int N2, typename T, class Lay>
__device__ __forceinline__ void pair_diffuse(cx<T> (&a)[N1], int t, cx<T>* __restrict__ sh, const Lay& lay,
                                             const T* __restrict__ ab)
{
    constexpr int N = N1 * N2;
    auto mix = [&](int m, cx<T> z, cx<T> zp) -> cx<T> {
        const T al = ab[3 * m];
        const cx<T> be{ab[3 * m + 1], ab[3 * m + 2]};
        return al * z + be * zp;
    };
    if constexpr (N2 == 1) {
        dft<N1, false>(a);
        cx<T> b[N1];
        sfor<0, N1>([&](auto K) {
            constexpr int m = decltype(K)::value;
            b[m] = mix(m, a[m], a[(N - m) % N]);
        });
        sfor<0, N1>([&](auto K) { a[decltype(K)::value] = b[decltype(K)::value]; });
        dft<N1, true>(a);
    } else {
        static_assert(N1 % N2 == 0, "each lane must own whole stage-two transforms");
        constexpr int NB = N1 / N2;
        dft<N1, false>(a);
        twiddle<N1, N, false>(a, t);
        __syncthreads();
        sfor<0, N1>([&](auto K1) { sh[lay(decltype(K1)::value, t)] = a[decltype(K1)::value]; });
        __syncthreads();
        // stage two forward: row k1 becomes V[k1 + N1 k2], k2 = 0..N2-1, in place
        sfor<0, NB>([&](auto I) {
            const int k1 = t + N2 * decltype(I)::value;
            cx<T> b[N2];
            sfor<0, N2>([&](auto M2) { b[decltype(M2)::value] = sh[lay(k1, decltype(M2)::value)]; });
            dft<N2, false>(b);
            sfor<0, N2>([&](auto K2) { sh[lay(k1, decltype(K2)::value)] = b[decltype(K2)::value]; });
        });
        __syncthreads();
        // pair each frequency with N - m (row (N1 - k1) mod N1, held by another lane)
        cx<T> z[NB][N2];
        sfor<0, NB>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const int k1 = t + N2 * i;
            const int k1p = (N1 - k1) % N1;
            sfor<0, N2>([&](auto K2) {
                constexpr int k2 = decltype(K2)::value;
                const int k2p = (k1 == 0) ? (N2 - k2) % N2 : N2 - 1 - k2;
                z[i][k2] = mix(k1 + N1 * k2, sh[lay(k1, k2)], sh[lay(k1p, k2p)]);
            });
        });
        __syncthreads();
        sfor<0, NB>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const int k1 = t + N2 * i;
            dft<N2, true>(z[i]);
            sfor<0, N2>([&](auto M2) { sh[lay(k1, decltype(M2)::value)] = z[i][decltype(M2)::value]; });
        });
        __syncthreads();
        sfor<0, N1>([&](auto K1) { a[decltype(K1)::value] = sh[lay(decltype(K1)::value, t)]; });
        twiddle<N1, N, true>(a, t);
        dft<N1, true>(a);
    }
}

// ------------------------------------------- one-way line transforms ------
// line_forward: the line held as in diffuse() (lane t owns n = n1 N2 + t) is
// replaced by its unnormalised DFT, handed out in natural order: store(k, X[k])
// is called once for every k the lane ends up owning.  line_inverse is the
// reverse: load(k) supplies X[k] in natural order and the lane receives its
// points of the unnormalised inverse DFT in a[].  Both contain barriers.
template <int N1, int N2, typename T, class Lay, class Store>
__device__ __forceinline__ void line_forward(cx<T> (&a)[N1], int t, cx<T>* __restrict__ sh, const Lay& lay,
                                             const Store& store)
{
    constexpr int N = N1 * N2;
    if constexpr (N2 == 1) {
        dft<N1, false>(a);
        sfor<0, N1>([&](auto K) { store(decltype(K)::value, a[decltype(K)::value]); });
    } else {
        constexpr int NB = N1 / N2;
        dft<N1, false>(a);
        twiddle<N1, N, false>(a, t);
        __syncthreads();
        sfor<0, N1>([&](auto K1) { sh[lay(decltype(K1)::value, t)] = a[decltype(K1)::value]; });
        __syncthreads();
        sfor<0, NB>([&](auto I) {
            const int k1 = t + N2 * decltype(I)::value;
            cx<T> b[N2];
            sfor<0, N2>([&](auto M2) { b[decltype(M2)::value] = sh[lay(k1, decltype(M2)::value)]; });
            dft<N2, false>(b);
            sfor<0, N2>([&](auto K2) { store(k1 + N1 * decltype(K2)::value, b[decltype(K2)::value]); });
        });
    }
}

template <int N1, int N2, typename T, class Lay, class Load>
__device__ __forceinline__ void line_inverse(cx<T> (&a)[N1], int t, cx<T>* __restrict__ sh, const Lay& lay,
                                             const Load& load)
{
    constexpr int N = N1 * N2;
    if constexpr (N2 == 1) {
        sfor<0, N1>([&](auto K) { a[decltype(K)::value] = load(decltype(K)::value); });
        dft<N1, true>(a);
    } else {
        constexpr int NB = N1 / N2;
        __syncthreads();
        sfor<0, NB>([&](auto I) {
            const int k1 = t + N2 * decltype(I)::value;
            cx<T> b[N2];
            sfor<0, N2>([&](auto K2) { b[decltype(K2)::value] = load(k1 + N1 * decltype(K2)::value); });
            dft<N2, true>(b);
            sfor<0, N2>([&](auto M2) { sh[lay(k1, decltype(M2)::value)] = b[decltype(M2)::value]; });
        });
        __syncthreads();
        sfor<0, N1>([&](auto K1) { a[decltype(K1)::value] = sh[lay(decltype(K1)::value, t)]; });
        twiddle<N1, N, true>(a, t);
        dft<N1, true>(a);
    }
}

}  // namespace pft
