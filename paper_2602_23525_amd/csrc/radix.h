// Butterflies of the generic tile kernel: the radices of butterfly.h, the
// composites 6, 9, 10, 12, 14 and 15 (fewer LDS exchanges for sizes with
// factors 3, 5 and 7: 9 as one step of eq. ct with constant twiddles, the
// others of coprime factors by the prime-factor map, without twiddles), and the
// primes 11, 13, 17, 19 and 23 by the definition with paired terms (17 to 23
// only in the kernel variant that holds 24 elements per thread).
#pragma once
#include <utility>

#include "butterfly.h"

namespace mfft {

// ------------------------------------------------------------ composite radices
// cos and sin of 2 pi m / R at compile time: the angle is split as
// q pi/2 + pi j/(2R) with q = round(4m/R) (exact integers, |j| <= R/2), the
// remainder evaluated by its Taylor series (|x| <= pi/4, 12 terms: below one
// FP64 ulp) and rotated back by the quadrant exactly.
struct CPair {
    double c, s;
};

constexpr CPair cx_cis_small(int j, int R)
{
    const double x = 3.14159265358979323846 * j / (2.0 * R);
    double s = 0, c = 0, ts = x, tc = 1;
    for (int k = 0; k < 12; ++k) {
        s += ts;
        c += tc;
        ts *= -x * x / ((2.0 * k + 2) * (2.0 * k + 3));
        tc *= -x * x / ((2.0 * k + 1) * (2.0 * k + 2));
    }
    return {c, s};
}

constexpr CPair cx_root(int m, int R)
{
    m %= R;
    const int q = (8 * m + R) / (2 * R);   // round(4m / R)
    const CPair r = cx_cis_small(4 * m - q * R, R);
    switch (q & 3) {
    case 0: return {r.c, r.s};
    case 1: return {-r.s, r.c};
    case 2: return {-r.c, -r.s};
    default: return {r.s, -r.c};
    }
}

// z * w_R^M (forward sign), quarter turns exact
template <typename T, int R, int M>
__device__ __forceinline__ cpx<T> twiddle_const(cpx<T> z)
{
    constexpr int m = M % R;
    if constexpr (m == 0) return z;
    else if constexpr (4 * m == R) return mul_mi(z);
    else if constexpr (2 * m == R) return cpx<T>{-z.re, -z.im};
    else if constexpr (4 * m == 3 * R) return cpx<T>{-z.im, z.re};
    else {
        constexpr CPair p = cx_root(m, R);
        return cmul(z, cpx<T>{T(p.c), T(-p.s)});
    }
}

template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}

template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <typename T, int R>
__device__ __forceinline__ void dftx(cpx<T> *v);

// R = A * B by eq. ct with constant twiddles: DFT-A over l1 of x[B l1 + l2]
// for each l2, twiddle w_R^(l2 k1), DFT-B over l2, output y[k1 + A k2].
template <typename T, int A, int B>
__device__ __forceinline__ void dft_ab(cpx<T> *v)
{
    cpx<T> z[B][A];
#pragma unroll
    for (int l2 = 0; l2 < B; ++l2) {
#pragma unroll
        for (int l1 = 0; l1 < A; ++l1) z[l2][l1] = v[B * l1 + l2];
        dftx<T, A>(z[l2]);
    }
    static_for<B>([&](auto l2c) {
        constexpr int l2 = decltype(l2c)::value;
        static_for<A>([&](auto k1c) {
            constexpr int k1 = decltype(k1c)::value;
            z[l2][k1] = twiddle_const<T, A * B, l2 * k1>(z[l2][k1]);
        });
    });
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
        cpx<T> w[B];
#pragma unroll
        for (int l2 = 0; l2 < B; ++l2) w[l2] = z[l2][k1];
        dftx<T, B>(w);
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = w[k2];
    }
}

// Inverse of b modulo m (gcd(b, m) = 1), at compile time.
constexpr int inv_mod(int b, int m)
{
    for (int x = 1; x < m; ++x)
        if ((b * x) % m == 1) return x;
    return 1;   // m = 1
}

// R = A * B with gcd(A, B) = 1 by the prime-factor (Good-Thomas) algorithm,
// which Section 2 names beside Cooley-Tukey and Section 5 uses for hard-coded
// codelets: input x[(B n1 + A n2) mod R] as a B x A array, DFT-A over n1,
// DFT-B over n2, output index k with k = k1 (mod A) and k = k2 (mod B), i.e.
// (B bA k1 + A aB k2) mod R with bA = B^-1 mod A, aB = A^-1 mod B.  The
// exponent of w_R splits into w_A^(n1 k1) w_B^(n2 k2) exactly, so no twiddle
// factors sit between the two sets of DFTs (a plain register permutation).
template <typename T, int A, int B>
__device__ __forceinline__ void dft_pfa(cpx<T> *v)
{
    constexpr int R = A * B;
    constexpr int bA = inv_mod(B % A, A), aB = inv_mod(A % B, B);
    cpx<T> z[B][A];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) z[n2][n1] = v[(B * n1 + A * n2) % R];
        dftx<T, A>(z[n2]);
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
        cpx<T> w[B];
#pragma unroll
        for (int n2 = 0; n2 < B; ++n2) w[n2] = z[n2][k1];
        dftx<T, B>(w);
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) v[(B * bA * k1 + A * aB * k2) % R] = w[k2];
    }
}

// Odd prime R by the definition with paired terms: for k = 1 .. (R-1)/2,
//   a_k = v0 + sum_j cos(2 pi jk/R) (v_j + v_(R-j)),
//   b_k = sum_j sin(2 pi jk/R) (v_j - v_(R-j)),
//   y_k = a_k - i b_k,  y_(R-k) = a_k + i b_k  (forward sign), y_0 = sum v.
template <typename T, int R>
__device__ __forceinline__ void dft_odd_prime(cpx<T> *v)
{
    constexpr int H = (R - 1) / 2;
    cpx<T> s[H], d[H];
    cpx<T> y0 = v[0];
#pragma unroll
    for (int j = 1; j <= H; ++j) {
        s[j - 1] = cadd(v[j], v[R - j]);
        d[j - 1] = csub(v[j], v[R - j]);
        y0 = cadd(y0, s[j - 1]);
    }
    cpx<T> out[R];
    out[0] = y0;
    static_for<H>([&](auto kc) {
        constexpr int k = decltype(kc)::value + 1;
        cpx<T> a = v[0], b = {T(0), T(0)};
        static_for<H>([&](auto jc) {
            constexpr int j = decltype(jc)::value + 1;
            constexpr CPair w = cx_root((j * k) % R, R);
            a = {a.re + T(w.c) * s[j - 1].re, a.im + T(w.c) * s[j - 1].im};
            b = {b.re + T(w.s) * d[j - 1].re, b.im + T(w.s) * d[j - 1].im};
        });
        out[k] = {a.re + b.im, a.im - b.re};       // a - i b
        out[R - k] = {a.re - b.im, a.im + b.re};   // a + i b
    });
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = out[k];
}

template <typename T, int R>
__device__ __forceinline__ void dftx(cpx<T> *v)
{
    if constexpr (R == 6) dft_pfa<T, 3, 2>(v);
    else if constexpr (R == 9) dft_ab<T, 3, 3>(v);
    else if constexpr (R == 10) dft_pfa<T, 5, 2>(v);
    else if constexpr (R == 12) dft_pfa<T, 4, 3>(v);
    else if constexpr (R == 14) dft_pfa<T, 7, 2>(v);
    else if constexpr (R == 15) dft_pfa<T, 5, 3>(v);
    else if constexpr (R == 11 || R == 13 || R == 17 || R == 19 || R == 23) dft_odd_prime<T, R>(v);
    else dft<T, R>(v);
}

}  // namespace mfft
