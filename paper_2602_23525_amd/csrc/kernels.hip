// HIP kernels for gfx950 besides the tile kernel: the rank-0 copy kernel, the
// FP64 table generators (Section 6: twiddles computed accurately, here in FP64
// on the GPU and rounded once), and the launch dispatch over the tile-kernel
// variants.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>

#include "butterfly.h"
#include "internal.h"
#include "kernels.h"

namespace mfft {

// ------------------------------------------------------------ rank-0 copy

__global__ void copy_kernel(CopyArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.total) return;
    int64_t rem = i, oi = 0, oo = 0;
    for (int d = a.rank - 1; d >= 0; --d) {
        const int64_t q = rem / a.n[d];
        const int64_t idx = rem - q * a.n[d];
        rem = q;
        oi += idx * a.is[d];
        oo += idx * a.os[d];
    }
    if (a.elem_bytes == 8) {
        ((uint2 *)a.out)[oo] = ((const uint2 *)a.in)[oi];
    } else {
        ((uint4 *)a.out)[oo] = ((const uint4 *)a.in)[oi];
    }
}

// ------------------------------------------------------------ FP64 tables

// exp(-2 pi i e / N) in FP64.  The angle is reduced with exact integer
// arithmetic to at most an eighth of a turn before sincospi, so the
// eighth roots of unity come out exact and the table is conjugate-symmetric.
__device__ double2 root_fp64(int64_t e, int64_t N)
{
    e %= N;
    if (e < 0) e += N;
    // angle = num / den turns
    int64_t num = e, den = N;
    double ssign = 1.0, csign = 1.0;
    bool swap = false;
    if (2 * num > den) {          // a -> 1 - a : sin flips
        num = den - num;
        ssign = -1.0;
    }
    if (4 * num > den) {          // a -> 1/2 - a : cos flips
        num = den - 2 * num;
        den *= 2;
        csign = -1.0;
    }
    if (8 * num > den) {          // a -> 1/4 - a : cos <-> sin
        num = den - 4 * num;
        den *= 4;
        swap = true;
    }
    double s, c;
    sincospi(2.0 * (double)num / (double)den, &s, &c);
    if (swap) {
        const double t = s;
        s = c;
        c = t;
    }
    return make_double2(csign * c, -(ssign * s));
}

// Entry e of a stage table: (j, k) with the twiddle w_(Ns*R)^(j*k).
// k-major (the specialized leaf kernel): e = k*Ns + j, k < R.
// j-major (the generic tile kernel): e = j*(R-1) + k - 1, 1 <= k < R, so that
// a butterfly's R-1 twiddles are consecutive.
__device__ __forceinline__ void stage_entry(int64_t e, int32_t Ns, int32_t R, bool jmajor,
                                            int64_t *j, int64_t *k)
{
    if (jmajor) {
        *j = e / (R - 1);
        *k = e % (R - 1) + 1;
    } else {
        *k = e / Ns;
        *j = e % Ns;
    }
}

template <typename T>
__global__ void gen_stage_twiddles(cpx<T> *out, int32_t Ns, int32_t R, bool jmajor)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)Ns * (jmajor ? R - 1 : R)) return;
    int64_t j, k;
    stage_entry(e, Ns, R, jmajor, &j, &k);
    const double2 w = root_fp64(j * k, (int64_t)Ns * R);
    out[e] = {T(w.x), T(w.y)};
}

// Accuracy ablation: the same FP32 table with the angle 2 pi m / N and its
// sine and cosine evaluated in FP32 (m = j*k reduced exactly in integer).
__global__ void gen_stage_twiddles_f32(cpx<float> *out, int32_t Ns, int32_t R, bool jmajor)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = (int64_t)Ns * R;
    if (e >= (int64_t)Ns * (jmajor ? R - 1 : R)) return;
    int64_t j, k;
    stage_entry(e, Ns, R, jmajor, &j, &k);
    const int64_t m = (j * k) % N;
    const float ang = -2.0f * 3.14159265358979f * (float)m / (float)N;
    float s, c;
    sincosf(ang, &s, &c);
    out[e] = {c, s};
}

__global__ void gen_tw4(double2 *hi, int64_t nhi, double2 *lo, int64_t nlo, int32_t shift, int64_t N)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nhi) hi[e] = root_fp64(e << shift, N);
    if (e < nlo) lo[e] = root_fp64(e, N);
}

// Bluestein chirp c_k = exp(-pi i (k^2 mod 2n) / n), k < n, FP64.
__global__ void gen_chirp(double2 *c, int64_t n)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t km = k % (2 * n);
    const int64_t q = (int64_t)(((uint64_t)km * (uint64_t)km) % (uint64_t)(2 * n));   // n < 2^31
    c[k] = root_fp64(q, 2 * n);
}

template <typename T>
__global__ void gen_roots(cpx<T> *out, int64_t count, int64_t N)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const double2 w = root_fp64(k, N);
    out[k] = {T(w.x), T(w.y)};
}

// ------------------------------------------------------------ real-data steps
// A real sequence of even length n = 2h packed as z[j] = x[2j] + i x[2j+1]
// has Z = DFT_h(z) = E + iO with E, O the transforms of the even and odd
// samples, both conjugate-symmetric; X[k] = E[k] + w_n^k O[k] (the DIT step of
// eq. ct with radix 2).  With A = Z[k], B = Z[h-k]:
//   E = (A + conj B)/2,  O = -i (A - conj B)/2,
//   X[k] = E + w O,  X[h-k] = conj(E - w O),  w = w_n^k.
// The inverse builds Z'[k] = E'[k] + i O'[k] with E' = X[k] + conj X[h-k] and
// O' = w_n^-k (X[k] - conj X[h-k]); an unnormalized inverse DFT of length h
// then yields x[2j] + i x[2j+1].
template <typename T>
__global__ void real_kernel(RealArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.total) return;
    int64_t line = i / a.cnt;
    const int64_t k = i - line * a.cnt;
    int64_t bi = 0, bo = 0;
    for (int d = a.vrank - 1; d >= 0; --d) {
        const int64_t q = line / a.vn[d];
        const int64_t idx = line - q * a.vn[d];
        line = q;
        bi += idx * a.vis[d];
        bo += idx * a.vos[d];
    }
    const T half = T(0.5);
    if (a.mode == RK_UNTANGLE) {
        const cpx<T> *Z = (const cpx<T> *)a.in + bi;
        cpx<T> *X = (cpx<T> *)a.out + bo;
        const int64_t h = a.n / 2;
        const cpx<T> A = Z[(k % h) * a.is];
        if (k == 0) {
            X[0] = {A.re + A.im, T(0)};
            X[h * a.os] = {A.re - A.im, T(0)};
            return;
        }
        const cpx<T> B = Z[(h - k) * a.is];
        const cpx<T> E = {half * (A.re + B.re), half * (A.im - B.im)};
        const cpx<T> O = {half * (A.im + B.im), half * (B.re - A.re)};   // -i (A - conj B) / 2
        const cpx<T> w = ((const cpx<T> *)a.tw)[k];
        const cpx<T> wO = cmul(w, O);
        X[k * a.os] = cadd(E, wO);
        if (2 * k != h) X[(h - k) * a.os] = conj(csub(E, wO));
    } else if (a.mode == RK_TANGLE) {
        const cpx<T> *X = (const cpx<T> *)a.in + bi;
        cpx<T> *Z = (cpx<T> *)a.out + bo;
        const int64_t h = a.n / 2;
        cpx<T> A = X[k * a.is], B = X[(h - k) * a.is];
        if (k == 0) {
            // bins 0 and n/2 of a conjugate-symmetric spectrum are real
            Z[0] = {A.re + B.re, A.re - B.re};
            return;
        }
        const cpx<T> P = {A.re + B.re, A.im - B.im};    // A + conj B
        const cpx<T> M = {A.re - B.re, A.im + B.im};    // A - conj B
        const cpx<T> w = ((const cpx<T> *)a.tw)[k];
        const cpx<T> wM = cmul(conj(w), M);
        const cpx<T> iwM = {-wM.im, wM.re};
        Z[k * a.os] = cadd(P, iwM);
        if (2 * k != h) Z[(h - k) * a.os] = conj(csub(P, iwM));
    } else if (a.mode == RK_WIDEN) {
        const T x = ((const T *)a.in)[bi + k * a.is];
        ((cpx<T> *)a.out)[bo + k * a.os] = {x, T(0)};
    } else if (a.mode == RK_HERM) {
        const cpx<T> *X = (const cpx<T> *)a.in + bi;
        cpx<T> y = k <= a.n / 2 ? X[k * a.is] : conj(X[(a.n - k) * a.is]);
        if (k == 0 || 2 * k == a.n) y.im = T(0);
        ((cpx<T> *)a.out)[bo + k * a.os] = y;
    } else {
        ((T *)a.out)[bo + k * a.os] = ((const cpx<T> *)a.in)[bi + k * a.is].re;
    }
}

// Wrapped conj(chirp) sequence of length M for the convolution kernel.
__global__ void gen_bluestein_v(double2 *v, const double2 *c, int64_t n, int64_t M)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    double2 r = make_double2(0.0, 0.0);
    if (m < n) r = make_double2(c[m].x, -c[m].y);
    else if (M - m < n) r = make_double2(c[M - m].x, -c[M - m].y);
    v[m] = r;
}

__device__ int64_t modpow(int64_t b, int64_t e, int64_t p)
{
    int64_t r = 1 % p;
    b %= p;
    while (e > 0) {
        if (e & 1) r = (r * b) % p;
        b = (b * b) % p;
        e >>= 1;
    }
    return r;
}

// Rader tables for prime p with generator g: gather[j] = g^j, scatter[q] =
// g^-q (mod p), and the sequence b_m = w_p^(g^-m) in FP64.
__global__ void gen_rader(int32_t *gather, int32_t *scatter, double2 *b, int64_t p, int64_t g)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p - 1) return;
    gather[j] = (int32_t)modpow(g, j, p);
    const int64_t inv = modpow(g, (p - 1 - j) % (p - 1), p);
    scatter[j] = (int32_t)inv;
    b[j] = root_fp64(inv, p);
}

// out[k] = T(in[k] * s) (FP64 product, one rounding)
template <typename T>
__global__ void convert_scale(cpx<T> *out, const double2 *in, int64_t count, double s)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    out[k] = {T(in[k].x * s), T(in[k].y * s)};
}

// ------------------------------------------------------------ launchers

static inline unsigned blocks_for(int64_t count, int threads)
{
    return (unsigned)((count + threads - 1) / threads);
}

// per-variant launchers (k_c32_k0.hip, ...)
#define MFFT_VARIANT(P, K)                                                                   \
    hipError_t launch_pass_##P##_k##K(const PassArgs &a, size_t lds, hipStream_t s);          \
    hipError_t launch_batch_##P##_k##K(const PassArgs *items, const int64_t *prefix,         \
                                       const int32_t *owner, int64_t total, int block,        \
                                       size_t lds, hipStream_t s);                            \
    int pass_blocks_per_cu_##P##_k##K(int block, size_t lds);
MFFT_VARIANT(c32, 0)
MFFT_VARIANT(c32, 1)
MFFT_VARIANT(c32, 5)
MFFT_VARIANT(c32, 7)
MFFT_VARIANT(c64, 0)
MFFT_VARIANT(c64, 1)
MFFT_VARIANT(c64, 5)
MFFT_VARIANT(c64, 7)
MFFT_VARIANT(c32, 0_e24)
MFFT_VARIANT(c32, 1_e24)
MFFT_VARIANT(c64, 0_e24)
MFFT_VARIANT(c64, 1_e24)
#undef MFFT_VARIANT

// Kernel kind needed by a pass (bits of tile.h's K_*): 0 plain, 1 Cooley-Tukey
// twiddles, 5 in-kernel convolution (with twiddles), 7 all features.
int pass_kind(uint32_t flags)
{
    const uint32_t ext = PF_PRE_MUL | PF_GATHER | PF_CONJ_A | PF_POST_MUL | PF_SCATTER |
                         PF_RADER | PF_AUX_X0 | PF_AUX_ADD;
    // PF_XCD only changes the tile order and is handled by every kind
    if (flags & ext) return 7;
    if (flags & (PF_CONV | PF_AUX_A0)) return 5;
    if (flags & PF_TW4) return 1;
    return 0;
}

hipError_t launch_pass(const PassArgs &a, int prec, int emax, size_t lds_bytes, hipStream_t s)
{
    if (a.ntiles <= 0) return hipSuccess;
    if (a.ntiles > 0x7fffffffLL - kXcds) return hipErrorInvalidValue;
    const int k = pass_kind(a.flags);
    if (emax > 16) {
        // radices 17, 19, 23: plain and twiddled lines only
        if (emax > 24 || k > 1) return hipErrorInvalidValue;
        if (prec == 0) return k ? launch_pass_c32_k1_e24(a, lds_bytes, s) : launch_pass_c32_k0_e24(a, lds_bytes, s);
        return k ? launch_pass_c64_k1_e24(a, lds_bytes, s) : launch_pass_c64_k0_e24(a, lds_bytes, s);
    }
    if (prec == 0) {
        if (k == 0) return launch_pass_c32_k0(a, lds_bytes, s);
        if (k == 1) return launch_pass_c32_k1(a, lds_bytes, s);
        if (k == 5) return launch_pass_c32_k5(a, lds_bytes, s);
        return launch_pass_c32_k7(a, lds_bytes, s);
    }
    if (k == 0) return launch_pass_c64_k0(a, lds_bytes, s);
    if (k == 1) return launch_pass_c64_k1(a, lds_bytes, s);
    if (k == 5) return launch_pass_c64_k5(a, lds_bytes, s);
    return launch_pass_c64_k7(a, lds_bytes, s);
}

static int query_blocks_per_cu(int prec, int kind, int emax, int block, size_t lds)
{
    if (emax > 16) {
        if (kind > 1) return 1;
        if (prec == 0) return kind ? pass_blocks_per_cu_c32_k1_e24(block, lds) : pass_blocks_per_cu_c32_k0_e24(block, lds);
        return kind ? pass_blocks_per_cu_c64_k1_e24(block, lds) : pass_blocks_per_cu_c64_k0_e24(block, lds);
    }
    if (prec == 0) {
        if (kind == 0) return pass_blocks_per_cu_c32_k0(block, lds);
        if (kind == 1) return pass_blocks_per_cu_c32_k1(block, lds);
        if (kind == 5) return pass_blocks_per_cu_c32_k5(block, lds);
        return pass_blocks_per_cu_c32_k7(block, lds);
    }
    if (kind == 0) return pass_blocks_per_cu_c64_k0(block, lds);
    if (kind == 1) return pass_blocks_per_cu_c64_k1(block, lds);
    if (kind == 5) return pass_blocks_per_cu_c64_k5(block, lds);
    return pass_blocks_per_cu_c64_k7(block, lds);
}

// The occupancy answers, kept per device and question: the planner asks for
// every size class of every line length it plans (10,000 plans of a batch
// repeat a few hundred questions).
int pass_blocks_per_cu(int prec, int kind, int emax, int block, size_t lds)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, int, size_t>, int> seen;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return query_blocks_per_cu(prec, kind, emax, block, lds);
    }
    const auto key = std::make_tuple(dev, prec, kind, emax, block, lds);
    {
        std::lock_guard<std::mutex> g(mu);
        const auto it = seen.find(key);
        if (it != seen.end()) return it->second;
    }
    const int b = query_blocks_per_cu(prec, kind, emax, block, lds);
    std::lock_guard<std::mutex> g(mu);
    seen[key] = b;
    return b;
}

hipError_t launch_batch(const PassArgs *items_dev, const int64_t *prefix_dev,
                        const int32_t *owner_dev, int64_t total, int prec, int kind, int block,
                        size_t lds_bytes, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    if (total > 0x7fffffffLL) return hipErrorInvalidValue;
#define MFFT_BATCH_ARGS items_dev, prefix_dev, owner_dev, total, block, lds_bytes, s
    if (kind == kWideKind || kind == kWideKind + 1) {
        if (prec == 0)
            return kind == kWideKind ? launch_batch_c32_k0_e24(MFFT_BATCH_ARGS)
                                     : launch_batch_c32_k1_e24(MFFT_BATCH_ARGS);
        return kind == kWideKind ? launch_batch_c64_k0_e24(MFFT_BATCH_ARGS)
                                 : launch_batch_c64_k1_e24(MFFT_BATCH_ARGS);
    }
    if (prec == 0) {
        if (kind == 0) return launch_batch_c32_k0(MFFT_BATCH_ARGS);
        if (kind == 1) return launch_batch_c32_k1(MFFT_BATCH_ARGS);
        if (kind == 5) return launch_batch_c32_k5(MFFT_BATCH_ARGS);
        return launch_batch_c32_k7(MFFT_BATCH_ARGS);
    }
    if (kind == 0) return launch_batch_c64_k0(MFFT_BATCH_ARGS);
    if (kind == 1) return launch_batch_c64_k1(MFFT_BATCH_ARGS);
    if (kind == 5) return launch_batch_c64_k5(MFFT_BATCH_ARGS);
    return launch_batch_c64_k7(MFFT_BATCH_ARGS);
#undef MFFT_BATCH_ARGS
}

// Contiguous copy, 16-byte vectors, four per thread: the rank-0 plan of a
// unit-stride loop (and the reference copy for bandwidth calibration).
__global__ __launch_bounds__(256) void copy_contig_kernel(const uint4 *__restrict__ in,
                                                          uint4 *__restrict__ out, int64_t n16)
{
    const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    uint4 v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (base + j * 256 < n16) v[j] = in[base + j * 256];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (base + j * 256 < n16) out[base + j * 256] = v[j];
}

// ------------------------------------------------------------ in-place square transpose
// One workgroup per pair of 32 x 32 tiles (ti <= tj) of one block: both tiles
// are read into LDS (rows of 32 elements, coalesced), then each is written to
// the other's place transposed; a diagonal tile is transposed onto itself.
// Every element of the pair is read before the barrier and written after it,
// and the pairs partition the block, so the transpose is race-free in place.
constexpr int kTrTile = 32;

template <typename E>
__global__ __launch_bounds__(256) void transpose_sq_kernel(TransposeArgs a, int64_t pairs,
                                                           int nt)
{
    __shared__ E ta[kTrTile][kTrTile + 1], tb[kTrTile][kTrTile + 1];
    const int64_t g = blockIdx.x;
    const int64_t blk = g / pairs;
    int rem = (int)(g - blk * pairs);
    // pair index -> (ti, tj), ti <= tj, row by row of the upper triangle
    int ti = 0;
    while (rem >= nt - ti) {
        rem -= nt - ti;
        ++ti;
    }
    const int tj = ti + rem;
    int64_t base = 0, r = blk;
    for (int d = a.rank - 1; d >= 0; --d) {
        const int64_t qd = r / a.n[d];
        base += (r - qd * a.n[d]) * a.s[d];
        r = qd;
    }
    E *data = (E *)a.data + base;
    const int x = threadIdx.x & (kTrTile - 1), y0 = threadIdx.x / kTrTile;
    const int64_t q = a.q;
    // tile A = rows ti*32.., columns tj*32..; tile B = rows tj*32.., columns ti*32..
#pragma unroll
    for (int y = y0; y < kTrTile; y += 256 / kTrTile) {
        const int64_t ra = (int64_t)ti * kTrTile + y, ca = (int64_t)tj * kTrTile + x;
        if (ra < q && ca < q) ta[y][x] = data[ra * a.rs + ca * a.cs];
        const int64_t rb = (int64_t)tj * kTrTile + y, cb = (int64_t)ti * kTrTile + x;
        if (ti != tj && rb < q && cb < q) tb[y][x] = data[rb * a.rs + cb * a.cs];
    }
    __syncthreads();
#pragma unroll
    for (int y = y0; y < kTrTile; y += 256 / kTrTile) {
        // B's place (rows tj.., columns ti..) gets A transposed
        const int64_t rb = (int64_t)tj * kTrTile + y, cb = (int64_t)ti * kTrTile + x;
        if (rb < q && cb < q) data[rb * a.rs + cb * a.cs] = ta[x][y];
        if (ti != tj) {
            const int64_t ra = (int64_t)ti * kTrTile + y, ca = (int64_t)tj * kTrTile + x;
            if (ra < q && ca < q) data[ra * a.rs + ca * a.cs] = tb[x][y];
        }
    }
}

hipError_t launch_transpose_sq(const TransposeArgs &a, hipStream_t s)
{
    if (a.total <= 0 || a.q <= 1) return hipSuccess;
    const int nt = (int)((a.q + kTrTile - 1) / kTrTile);
    const int64_t pairs = (int64_t)nt * (nt + 1) / 2;
    const int64_t grid = pairs * a.total;
    if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
    if (a.elem_bytes == 8)
        hipLaunchKernelGGL(transpose_sq_kernel<uint2>, dim3((unsigned)grid), dim3(256), 0, s, a,
                           pairs, nt);
    else
        hipLaunchKernelGGL(transpose_sq_kernel<uint4>, dim3((unsigned)grid), dim3(256), 0, s, a,
                           pairs, nt);
    return hipGetLastError();
}

// ------------------------------------------------------------ in-place item permutation
// One workgroup per (cycle, block): the item at the cycle's start is read,
// then along the cycle each item is read before the previous one is written
// into its place.  A lane always handles the same elements of every item
// (element t + 256*j), so lanes need no synchronization.  Elements move as W
// 8-byte words (W = 1 FP32 complex, 2 FP64 complex); local arrays of 64-bit
// words stay in registers.
constexpr int kPermMax = 8;   // elements per lane: items up to 2048 elements

template <int W>
__global__ __launch_bounds__(256) void permute_items_kernel(PermuteArgs a)
{
    using U = unsigned long long;
    const int64_t g = blockIdx.x;
    const int64_t blk = g / a.ncycles;
    const int c = (int)(g - blk * a.ncycles);
    int64_t base = 0, r = blk;
    for (int d = a.rank - 1; d >= 0; --d) {
        const int64_t qd = r / a.n[d];
        base += (r - qd * a.n[d]) * a.s[d];
        r = qd;
    }
    U *data = (U *)a.data + base * W;
    const int t = threadIdx.x;
    const int x0 = a.starts[c];
    U cur[kPermMax * W], nxt[kPermMax * W];
#pragma unroll
    for (int j = 0; j < kPermMax; ++j) {
        const int64_t e = t + 256 * j;
        if (e < a.len) {
            const U *src = data + (x0 * a.xs + e * a.es) * W;
#pragma unroll
            for (int w = 0; w < W; ++w) cur[j * W + w] = src[w];
        }
    }
    int x = x0;
    for (int step = 0; step < a.nitems; ++step) {   // a cycle has at most nitems steps
        const int y = a.next[x];
        U *item = data + (int64_t)y * a.xs * W;
        if (y != x0) {
#pragma unroll
            for (int j = 0; j < kPermMax; ++j) {
                const int64_t e = t + 256 * j;
                if (e < a.len) {
#pragma unroll
                    for (int w = 0; w < W; ++w) nxt[j * W + w] = item[e * a.es * W + w];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kPermMax; ++j) {
            const int64_t e = t + 256 * j;
            if (e < a.len) {
#pragma unroll
                for (int w = 0; w < W; ++w) item[e * a.es * W + w] = cur[j * W + w];
            }
        }
        if (y == x0) break;
#pragma unroll
        for (int k = 0; k < kPermMax * W; ++k) cur[k] = nxt[k];
        x = y;
    }
}

hipError_t launch_permute_items(const PermuteArgs &a, hipStream_t s)
{
    if (a.total <= 0 || a.ncycles <= 0) return hipSuccess;
    if (a.len > 256 * kPermMax) return hipErrorInvalidValue;
    const int64_t grid = (int64_t)a.ncycles * a.total;
    if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
    if (a.elem_bytes == 8)
        hipLaunchKernelGGL(permute_items_kernel<1>, dim3((unsigned)grid), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(permute_items_kernel<2>, dim3((unsigned)grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_copy(const CopyArgs &a, hipStream_t s)
{
    if (a.total <= 0) return hipSuccess;
    const int64_t bytes = a.total * a.elem_bytes;
    if (a.rank == 1 && a.is[0] == 1 && a.os[0] == 1 && bytes % 16 == 0 &&
        ((uintptr_t)a.in % 16) == 0 && ((uintptr_t)a.out % 16) == 0) {
        const int64_t n16 = bytes / 16;
        hipLaunchKernelGGL(copy_contig_kernel, dim3((unsigned)((n16 + 1023) / 1024)), dim3(256), 0,
                           s, (const uint4 *)a.in, (uint4 *)a.out, n16);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(copy_kernel, dim3(blocks_for(a.total, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gen_stage_twiddles(void *out, int prec, int Ns, int R, hipStream_t s,
                                     bool fp32_math, bool jmajor)
{
    const int64_t cnt = (int64_t)Ns * (jmajor ? R - 1 : R);
    if (cnt <= 0) return hipSuccess;
    if (prec == 0 && fp32_math)
        hipLaunchKernelGGL(gen_stage_twiddles_f32, dim3(blocks_for(cnt, 256)), dim3(256), 0, s,
                           (cpx<float> *)out, Ns, R, jmajor);
    else if (prec == 0)
        hipLaunchKernelGGL(gen_stage_twiddles<float>, dim3(blocks_for(cnt, 256)), dim3(256), 0, s,
                           (cpx<float> *)out, Ns, R, jmajor);
    else
        hipLaunchKernelGGL(gen_stage_twiddles<double>, dim3(blocks_for(cnt, 256)), dim3(256), 0,
                           s, (cpx<double> *)out, Ns, R, jmajor);
    return hipGetLastError();
}

hipError_t launch_gen_tw4(void *hi, int64_t nhi, void *lo, int64_t nlo, int shift, int64_t N,
                          hipStream_t s)
{
    const int64_t cnt = nhi > nlo ? nhi : nlo;
    hipLaunchKernelGGL(gen_tw4, dim3(blocks_for(cnt, 256)), dim3(256), 0, s, (double2 *)hi, nhi,
                       (double2 *)lo, nlo, shift, N);
    return hipGetLastError();
}

hipError_t launch_real(const RealArgs &a, int prec, hipStream_t s)
{
    if (a.total <= 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL(real_kernel<float>, dim3(blocks_for(a.total, 256)), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(real_kernel<double>, dim3(blocks_for(a.total, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gen_roots(void *out, int prec, int64_t count, int64_t N, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL(gen_roots<float>, dim3(blocks_for(count, 256)), dim3(256), 0, s,
                           (cpx<float> *)out, count, N);
    else
        hipLaunchKernelGGL(gen_roots<double>, dim3(blocks_for(count, 256)), dim3(256), 0, s,
                           (cpx<double> *)out, count, N);
    return hipGetLastError();
}

hipError_t launch_gen_chirp(void *c, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(gen_chirp, dim3(blocks_for(n, 256)), dim3(256), 0, s, (double2 *)c, n);
    return hipGetLastError();
}

hipError_t launch_gen_bluestein_v(void *v, const void *c, int64_t n, int64_t M, hipStream_t s)
{
    hipLaunchKernelGGL(gen_bluestein_v, dim3(blocks_for(M, 256)), dim3(256), 0, s, (double2 *)v,
                       (const double2 *)c, n, M);
    return hipGetLastError();
}

hipError_t launch_gen_rader(int32_t *gather, int32_t *scatter, void *b, int64_t p, int64_t g,
                            hipStream_t s)
{
    hipLaunchKernelGGL(gen_rader, dim3(blocks_for(p - 1, 256)), dim3(256), 0, s, gather, scatter,
                       (double2 *)b, p, g);
    return hipGetLastError();
}

hipError_t launch_convert_scale(void *out, int prec, const void *in, int64_t count, double scale,
                                hipStream_t s)
{
    if (prec == 0)
        hipLaunchKernelGGL(convert_scale<float>, dim3(blocks_for(count, 256)), dim3(256), 0, s,
                           (cpx<float> *)out, (const double2 *)in, count, scale);
    else
        hipLaunchKernelGGL(convert_scale<double>, dim3(blocks_for(count, 256)), dim3(256), 0, s,
                           (cpx<double> *)out, (const double2 *)in, count, scale);
    return hipGetLastError();
}

}  // namespace mfft
