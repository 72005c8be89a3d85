// fft_reg.hpp - register-resident mixed-radix DFTs for one pencil per thread.
//
// The lifted grids of the method (Sec. 3.2, K*_{K,L} of extent 2K x 2L) have
// short axes (typically 10..64 points), so every 1-D transform along an axis
// is done by one thread holding the whole pencil in registers.  The size is a
// template parameter: the Cooley-Tukey recursion below is fully unrolled at
// compile time, every array index is a constant, and every twiddle factor is
// a compile-time constant computed by our own constexpr sine/cosine (Taylor
// series after reduction to [-pi/4, pi/4]).  Trivial twiddles (1, -1, +-i)
// cost no multiplies.
//
// Sign convention: SIGN = +1 computes X[k] = sum_n x[n] e^{+2 pi i n k / S}
// (the unnormalised inverse transform, coefficients -> grid values);
// SIGN = -1 the forward transform without the 1/S factor.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>

namespace iwfpm {

template <typename R>
struct cplx {
    R x, y;
};

template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> cscale(cplx<R> a, R s) { return {a.x * s, a.y * s}; }
// multiply by SIGN * i
template <int SIGN, typename R>
__device__ __forceinline__ cplx<R> cmul_si(cplx<R> a) {
    if constexpr (SIGN > 0) return {-a.y, a.x};
    else return {a.y, -a.x};
}

// ---------------------------------------------------------------------------
// compile-time trigonometry: e^{2 pi i a / b}
// ---------------------------------------------------------------------------
namespace ct {
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double sin_series(double x) {  // |x| <= pi/4
    double x2 = x * x, term = x, sum = x;
    for (int i = 1; i < 16; ++i) {
        term *= -x2 / double((2 * i) * (2 * i + 1));
        sum += term;
    }
    return sum;
}
constexpr double cos_series(double x) {  // |x| <= pi/4
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int i = 1; i < 16; ++i) {
        term *= -x2 / double((2 * i - 1) * (2 * i));
        sum += term;
    }
    return sum;
}
constexpr long mod_pos(long a, long b) { return ((a % b) + b) % b; }
// nearest quadrant q with 2 pi a / b = q pi/2 + phi, |phi| <= pi/4
constexpr long quadrant(long a, long b) {
    // round(4a/b) with a in [0, b)
    return (8 * a + b) / (2 * b);
}
constexpr double cos2pi(long a, long b) {
    a = mod_pos(a, b);
    long q = quadrant(a, b);
    double phi = (kPi / 2.0) * double(4 * a - q * b) / double(b);
    switch (q & 3) {
        case 0: return cos_series(phi);
        case 1: return -sin_series(phi);
        case 2: return -cos_series(phi);
        default: return sin_series(phi);
    }
}
constexpr double sin2pi(long a, long b) {
    a = mod_pos(a, b);
    long q = quadrant(a, b);
    double phi = (kPi / 2.0) * double(4 * a - q * b) / double(b);
    switch (q & 3) {
        case 0: return sin_series(phi);
        case 1: return cos_series(phi);
        case 2: return -sin_series(phi);
        default: return -cos_series(phi);
    }
}
constexpr int smallest_factor(int s) {
    for (int p = 2; p * p <= s; ++p)
        if (s % p == 0) return p;
    return s;
}
// leaf radix used by the recursion: 4 when possible, else the smallest prime
constexpr int radix_of(int s) { return (s % 4 == 0 && s > 4) ? 4 : smallest_factor(s); }
}  // namespace ct

template <int I>
using ic = std::integral_constant<int, I>;

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(ic<B>{});
        static_for<B + 1, E>(f);
    }
}

// x * e^{SIGN 2 pi i A / B}, specialised for the trivial angles
template <int A, int B, int SIGN, typename R>
__device__ __forceinline__ cplx<R> twiddle(cplx<R> v) {
    constexpr long a = ct::mod_pos(A, B);
    if constexpr (a == 0) {
        return v;
    } else if constexpr (2 * a == B) {
        return {-v.x, -v.y};
    } else if constexpr (4 * a == B) {
        return cmul_si<SIGN>(v);
    } else if constexpr (4 * a == 3 * B) {
        return cmul_si<-SIGN>(v);
    } else {
        constexpr R c = R(ct::cos2pi(a, B));
        constexpr R s = R(SIGN * ct::sin2pi(a, B));
        return {v.x * c - v.y * s, v.x * s + v.y * c};
    }
}

// Direct DFT of a prime (or otherwise leaf) size P.  For odd P the inputs
// are paired, x[n] +- x[P-n], so that cosines and sines are applied once.
template <int P, int SIGN, typename R>
__device__ __forceinline__ void dft_leaf(cplx<R> (&x)[P]) {
    if constexpr (P == 1) {
        return;
    } else if constexpr (P == 2) {
        cplx<R> a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    } else if constexpr (P == 4) {
        cplx<R> s02 = cadd(x[0], x[2]), d02 = csub(x[0], x[2]);
        cplx<R> s13 = cadd(x[1], x[3]), d13 = cmul_si<SIGN>(csub(x[1], x[3]));
        x[0] = cadd(s02, s13);
        x[2] = csub(s02, s13);
        x[1] = cadd(d02, d13);
        x[3] = csub(d02, d13);
    } else if constexpr (P % 2 == 1) {
        constexpr int H = (P - 1) / 2;
        cplx<R> a[H], b[H];
        cplx<R> x0 = x[0];
        cplx<R> sum = x[0];
        static_for<1, H + 1>([&](auto n_) {
            constexpr int n = decltype(n_)::value;
            a[n - 1] = cadd(x[n], x[P - n]);
            b[n - 1] = csub(x[n], x[P - n]);
            sum = cadd(sum, a[n - 1]);
        });
        x[0] = sum;
        static_for<1, H + 1>([&](auto k_) {
            constexpr int k = decltype(k_)::value;
            cplx<R> A = x0, Bv = {R(0), R(0)};
            static_for<1, H + 1>([&](auto n_) {
                constexpr int n = decltype(n_)::value;
                constexpr R c = R(ct::cos2pi(long(n) * k, P));
                constexpr R s = R(ct::sin2pi(long(n) * k, P));
                A.x += a[n - 1].x * c;
                A.y += a[n - 1].y * c;
                Bv.x += b[n - 1].x * s;
                Bv.y += b[n - 1].y * s;
            });
            cplx<R> iB = cmul_si<SIGN>(Bv);
            x[k] = cadd(A, iB);
            x[P - k] = csub(A, iB);
        });
    } else {
        static_assert(P % 2 == 1 || P <= 4, "leaf sizes are 1, 2, 4 or odd");
    }
}

// In-place DFT of size S in registers (decimation in time over the leading
// radix p = radix_of(S), S = p m; output in natural order).
template <int S, int SIGN, typename R>
__device__ __forceinline__ void fft_inplace(cplx<R> (&x)[S]) {
    constexpr int p = ct::radix_of(S);
    constexpr int m = S / p;
    if constexpr (m == 1) {
        dft_leaf<S, SIGN>(x);
    } else {
        cplx<R> z[p][m];
        static_for<0, m>([&](auto n2_) {
            constexpr int n2 = decltype(n2_)::value;
            cplx<R> t[p];
            static_for<0, p>([&](auto n1_) {
                constexpr int n1 = decltype(n1_)::value;
                t[n1] = x[m * n1 + n2];
            });
            dft_leaf<p, SIGN>(t);
            static_for<0, p>([&](auto k1_) {
                constexpr int k1 = decltype(k1_)::value;
                z[k1][n2] = twiddle<(n2 * k1) % S, S, SIGN>(t[k1]);
            });
        });
        static_for<0, p>([&](auto k1_) {
            constexpr int k1 = decltype(k1_)::value;
            fft_inplace<m, SIGN>(z[k1]);
            static_for<0, m>([&](auto k2_) {
                constexpr int k2 = decltype(k2_)::value;
                x[k1 + p * k2] = z[k1][k2];
            });
        });
    }
}

}  // namespace iwfpm
