// Complex arithmetic and the register-resident butterflies shared by the
// tile kernel and the specialized leaf kernel: forward (sign -1) DFTs of
// length R in 2, 3, 4, 5, 7, 8, 16 on values held in VGPRs, natural order in
// and out (the codelets of Section 5, written by hand).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mfft {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// multiply by -i
template <typename T>
__device__ __forceinline__ cpx<T> mul_mi(cpx<T> a) { return {a.im, -a.re}; }
template <typename T>
__device__ __forceinline__ cpx<T> conj(cpx<T> a) { return {a.re, -a.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> scale(cpx<T> a, T s) { return {a.re * s, a.im * s}; }

// ------------------------------------------------------------ butterflies
// Forward (sign -1) DFTs of length R, natural order in and out, in place.

template <typename T>
__device__ __forceinline__ void dft2(cpx<T> *v)
{
    cpx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename T>
__device__ __forceinline__ void dft3(cpx<T> *v)
{
    const T s3 = T(0.86602540378443864676);  // sin(2 pi / 3)
    cpx<T> t = cadd(v[1], v[2]);
    cpx<T> u = scale(mul_mi(csub(v[1], v[2])), s3);
    cpx<T> a = csub(v[0], scale(t, T(0.5)));
    v[0] = cadd(v[0], t);
    v[1] = cadd(a, u);
    v[2] = csub(a, u);
}

template <typename T>
__device__ __forceinline__ void dft4(cpx<T> *v)
{
    cpx<T> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    cpx<T> s13 = cadd(v[1], v[3]), d13 = mul_mi(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
}

template <typename T>
__device__ __forceinline__ void dft5(cpx<T> *v)
{
    const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
    const T s1 = T(0.95105651629515357212), s2 = T(0.58778525229247312917);
    cpx<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    cpx<T> u1 = csub(v[1], v[4]), u2 = csub(v[2], v[3]);
    cpx<T> x0 = v[0];
    cpx<T> a1 = {x0.re + c1 * t1.re + c2 * t2.re, x0.im + c1 * t1.im + c2 * t2.im};
    cpx<T> a2 = {x0.re + c2 * t1.re + c1 * t2.re, x0.im + c2 * t1.im + c1 * t2.im};
    cpx<T> b1 = {s1 * u1.re + s2 * u2.re, s1 * u1.im + s2 * u2.im};
    cpx<T> b2 = {s2 * u1.re - s1 * u2.re, s2 * u1.im - s1 * u2.im};
    v[0] = cadd(x0, cadd(t1, t2));
    v[1] = cadd(a1, mul_mi(b1));
    v[4] = csub(a1, mul_mi(b1));
    v[2] = cadd(a2, mul_mi(b2));
    v[3] = csub(a2, mul_mi(b2));
}

template <typename T>
__device__ __forceinline__ void dft7(cpx<T> *v)
{
    const T c1 = T(0.62348980185873353053), c2 = T(-0.22252093395631440429),
            c3 = T(-0.90096886790241912624);
    const T s1 = T(0.78183148246802980871), s2 = T(0.97492791218182360702),
            s3 = T(0.43388373911755812048);
    cpx<T> x0 = v[0];
    cpx<T> t1 = cadd(v[1], v[6]), t2 = cadd(v[2], v[5]), t3 = cadd(v[3], v[4]);
    cpx<T> u1 = csub(v[1], v[6]), u2 = csub(v[2], v[5]), u3 = csub(v[3], v[4]);
    cpx<T> a1 = {x0.re + c1 * t1.re + c2 * t2.re + c3 * t3.re,
                 x0.im + c1 * t1.im + c2 * t2.im + c3 * t3.im};
    cpx<T> a2 = {x0.re + c2 * t1.re + c3 * t2.re + c1 * t3.re,
                 x0.im + c2 * t1.im + c3 * t2.im + c1 * t3.im};
    cpx<T> a3 = {x0.re + c3 * t1.re + c1 * t2.re + c2 * t3.re,
                 x0.im + c3 * t1.im + c1 * t2.im + c2 * t3.im};
    cpx<T> b1 = {s1 * u1.re + s2 * u2.re + s3 * u3.re, s1 * u1.im + s2 * u2.im + s3 * u3.im};
    cpx<T> b2 = {s2 * u1.re - s3 * u2.re - s1 * u3.re, s2 * u1.im - s3 * u2.im - s1 * u3.im};
    cpx<T> b3 = {s3 * u1.re - s1 * u2.re + s2 * u3.re, s3 * u1.im - s1 * u2.im + s2 * u3.im};
    v[0] = cadd(x0, cadd(t1, cadd(t2, t3)));
    v[1] = cadd(a1, mul_mi(b1));
    v[6] = csub(a1, mul_mi(b1));
    v[2] = cadd(a2, mul_mi(b2));
    v[5] = csub(a2, mul_mi(b2));
    v[3] = cadd(a3, mul_mi(b3));
    v[4] = csub(a3, mul_mi(b3));
}

template <typename T>
__device__ __forceinline__ void dft8(cpx<T> *v)
{
    const T h = T(0.70710678118654752440);
    cpx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cpx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft4(e);
    dft4(o);
    // o_k *= w_8^k
    o[1] = {h * (o[1].re + o[1].im), h * (o[1].im - o[1].re)};
    o[2] = mul_mi(o[2]);
    o[3] = {h * (o[3].im - o[3].re), -h * (o[3].re + o[3].im)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = cadd(e[k], o[k]);
        v[k + 4] = csub(e[k], o[k]);
    }
}

template <typename T>
__device__ __forceinline__ void dft16(cpx<T> *v)
{
    // 16 = 4 x 4: inner DFT-4 over l1 of x[4 l1 + l2], twiddle w_16^(l2 k1),
    // outer DFT-4 over l2, output y[k1 + 4 k2]  (eq. ct with n1 = n2 = 4).
    const T h = T(0.70710678118654752440);
    const T c = T(0.92387953251128675613), s = T(0.38268343236508977173);
    cpx<T> z[4][4];
#pragma unroll
    for (int l2 = 0; l2 < 4; ++l2) {
#pragma unroll
        for (int l1 = 0; l1 < 4; ++l1) z[l2][l1] = v[4 * l1 + l2];
        dft4(z[l2]);
    }
    // twiddles w_16^(l2 k1), l2, k1 in 1..3
    z[1][1] = cmul(z[1][1], cpx<T>{c, -s});
    z[1][2] = cmul(z[1][2], cpx<T>{h, -h});
    z[1][3] = cmul(z[1][3], cpx<T>{s, -c});
    z[2][1] = cmul(z[2][1], cpx<T>{h, -h});
    z[2][2] = mul_mi(z[2][2]);
    z[2][3] = cmul(z[2][3], cpx<T>{-h, -h});
    z[3][1] = cmul(z[3][1], cpx<T>{s, -c});
    z[3][2] = cmul(z[3][2], cpx<T>{-h, -h});
    z[3][3] = cmul(z[3][3], cpx<T>{-c, s});
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cpx<T> w[4] = {z[0][k1], z[1][k1], z[2][k1], z[3][k1]};
        dft4(w);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = w[k2];
    }
}

template <typename T, int R>
__device__ __forceinline__ void dft(cpx<T> *v)
{
    if constexpr (R == 2) dft2(v);
    else if constexpr (R == 3) dft3(v);
    else if constexpr (R == 4) dft4(v);
    else if constexpr (R == 5) dft5(v);
    else if constexpr (R == 7) dft7(v);
    else if constexpr (R == 8) dft8(v);
    else if constexpr (R == 16) dft16(v);
}

}  // namespace mfft
