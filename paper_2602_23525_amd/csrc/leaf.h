// Specialized leaf kernel: unit-stride lines of a compile-time power-of-two
// length N, 16 elements per thread, all index arithmetic folded at compile
// time.  This is the direct plan of Section 4.2 ("Direct plans") for the sizes
// that dominate batched workloads; the generic tile kernel covers the rest.
//
// Data flow per line (Stockham autosort, Section 2):
//   thread t loads x[t + e*TPT], e < 16  (coalesced: consecutive lanes read
//   consecutive elements), which are exactly the inputs of its stage-1
//   butterflies; each stage twiddles, runs radix-R butterflies in VGPRs and
//   exchanges through LDS; the last stage's outputs are y[t + e*TPT], stored
//   coalesced.
//
// Workgroups are persistent over tiles (BT lines each).  With PF, the loads of
// the next tile are issued before the current tile's butterflies so that each
// workgroup keeps two tiles of HBM traffic in flight; the stage twiddles of a
// thread do not depend on the tile and are loaded into registers once.
#pragma once
#include "butterfly.h"
#include "gmem.h"
#include "internal.h"
#include "leaf_shape.h"
#include "twiddle4.h"

namespace mfft {

template <int... Rs>
struct Radices {};

template <int R, int... Rest>
constexpr int first_radix(Radices<R, Rest...>) { return R; }

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }

// Twiddles of one stage held in registers: for butterfly i the powers
// w^(2^m), m < log2 R, of its base twiddle w = w_(NS*R)^j, read from the FP64-
// generated table; the other powers are products of at most four of them
// (Section 6: a small table plus a bounded number of complex multiplications).
template <typename T, int R>
struct StageTw {
    cpx<T> w[16 / R][ilog2c(R)];
};

template <typename T, int N, int TPT, int NS, int R>
__device__ __forceinline__ void load_stage_tw(StageTw<T, R> &tw, gptr<const cpx<T>> table, int t)
{
    constexpr int NB = 16 / R;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int b = t + i * TPT;
        const int j = b & (NS - 1);
#pragma unroll
        for (int m = 0; m < ilog2c(R); ++m) tw.w[i][m] = table[(1 << m) * NS + j];
    }
}

// Opaque copy: keeps the compiler from hoisting the twiddle expansion out of
// the tile loop (which would pin all R powers in registers for the kernel's
// lifetime).
template <typename T>
__device__ __forceinline__ cpx<T> opaque(cpx<T> z)
{
    __asm__ volatile("" : "+v"(z.re), "+v"(z.im));
    return z;
}

// All R twiddle powers of butterfly i from its power-of-two powers.
template <typename T, int R>
__device__ __forceinline__ void expand_tw(const cpx<T> *pin, cpx<T> (&w)[R])
{
    cpx<T> p[ilog2c(R)];
#pragma unroll
    for (int m = 0; m < ilog2c(R); ++m) p[m] = opaque(pin[m]);
    w[0] = {T(1), T(0)};
#pragma unroll
    for (int k = 1; k < R; ++k) {
        const int low = k & -k;                  // lowest set bit
        if (k == low) w[k] = p[ilog2c(low)];
        else w[k] = cmul(w[k - low], p[ilog2c(low)]);
    }
}

// Padded LDS slot of element b + k*STEP, k < 16, as one address plus a
// compile-time offset: for STEP a multiple of 16 the padded index grows by
// STEP + STEP/16 per step, and for STEP 1 with b % 16 + 15 inside one block of
// 16 (b a multiple of a radix dividing 16 and k below that radix) by 1, so the
// compiler keeps one address register instead of one per element.
template <int STEP, typename T>
__device__ __forceinline__ cpx<T> *lds_slot(cpx<T> *line, int b, int k)
{
    if constexpr (STEP % 16 == 0) return line + lds_pad(b) + k * (STEP + STEP / 16);
    else if constexpr (STEP == 1) return line + lds_pad(b) + k;
    else return line + lds_pad(b + k * STEP);
}

// One stage on registers: x[i + k*NB] is element k of butterfly i.
template <typename T, int N, int TPT, int NS, int R, bool LAST>
__device__ __forceinline__ void fast_stage(cpx<T> (&x)[16], const StageTw<T, R> &tw, cpx<T> *line,
                                           int t)
{
    constexpr int NB = 16 / R;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        cpx<T> v[R];
#pragma unroll
        for (int k = 0; k < R; ++k) v[k] = x[i + k * NB];
        if constexpr (NS > 1) {
            cpx<T> w[R];
            expand_tw<T, R>(tw.w[i], w);
#pragma unroll
            for (int k = 1; k < R; ++k) v[k] = cmul(v[k], w[k]);
        }
        dft<T, R>(v);
        if constexpr (LAST) {
#pragma unroll
            for (int k = 0; k < R; ++k) x[i + k * NB] = v[k];
        } else {
            const int b = t + i * TPT;
            const int j = b & (NS - 1);
            const int q = b >> ilog2c(NS);
            const int base = q * NS * R + j;
#pragma unroll
            for (int k = 0; k < R; ++k) *lds_slot<NS>(line, base, k) = v[k];
        }
    }
}

template <typename T, int N, int TPT, int NS, int R, int... Rest>
struct StageChain {
    StageTw<T, R> tw;
    StageChain<T, N, TPT, NS * R, Rest...> next;
    __device__ __forceinline__ void load(gptr<const cpx<T>> table, int off, int t)
    {
        if constexpr (NS > 1) load_stage_tw<T, N, TPT, NS, R>(tw, table + off, t);
        next.load(table, off + NS * R, t);
    }
    __device__ __forceinline__ void run(cpx<T> (&x)[16], cpx<T> *line, int t)
    {
        fast_stage<T, N, TPT, NS, R, false>(x, tw, line, t);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 16; ++e) x[e] = *lds_slot<TPT>(line, t, e);
        __syncthreads();
        next.run(x, line, t);
    }
};

template <typename T, int N, int TPT, int NS, int R>
struct StageChain<T, N, TPT, NS, R> {
    StageTw<T, R> tw;
    __device__ __forceinline__ void load(gptr<const cpx<T>> table, int off, int t)
    {
        if constexpr (NS > 1) load_stage_tw<T, N, TPT, NS, R>(tw, table + off, t);
    }
    __device__ __forceinline__ void run(cpx<T> (&x)[16], cpx<T> *line, int t)
    {
        fast_stage<T, N, TPT, NS, R, true>(x, tw, line, t);
    }
};

// Global loads and stores of one element, non-temporal when the pass does
// not reuse what it reads (NT bit 1) or writes (NT bit 0).
template <int NT, typename T>
__device__ __forceinline__ cpx<T> ld_elem(gptr<const cpx<T>> p)
{
    if constexpr (NT & 2) {
        return {__builtin_nontemporal_load(&p->re), __builtin_nontemporal_load(&p->im)};
    } else {
        return *p;
    }
}

template <int NT, typename T>
__device__ __forceinline__ void st_elem(gptr<cpx<T>> p, cpx<T> v)
{
    if constexpr (NT & 1) {
        __builtin_nontemporal_store(v.re, &p->re);
        __builtin_nontemporal_store(v.im, &p->im);
    } else {
        *p = v;
    }
}

// RD: 0 plain; 1 the line is the transform of a packed real sequence, split
// into the n+1 outputs of the real transform on store (PF_R2C); 2 the line is
// combined from n+1 values of a half spectrum on load (PF_C2R); 3 columns
// (PF_LEAF_COL): the BT lines of a tile are adjacent in memory (unit vector
// stride) and their elements strided, so consecutive lanes take consecutive
// lines (runs of BT elements per load and store) and each line's thread index
// t is the lane's rank among the lanes of its line; 4 columns in, rows out and
// 5 rows in, columns out (PF_LEAF_CR, PF_LEAF_RC): the loads use one
// lane mapping, the stores the other, the results passing through LDS once
// more.  Column tiles (3-5) may multiply element k of inner line c by the
// Cooley-Tukey twiddle w_N^(c*k) on store (PF_TW4).  The outer passes of a
// three-pass Bluestein convolution, compiled apart so that the plain column
// tiles keep their registers: RD 6 is RD 4 loading element l of line c as
// x[j] * pre[j], j = c*li_c + l*li_l, zero for j >= li_lim (the chirp product
// and the zero padding); RD 7 is RD 5 storing element k of line c only for
// g = c*lo_c + k*lo_k < lo_lim, as conj(y) * post[g] (PF_CONJ_A) or
// y * post[g]; RD 8 is RD 3 running the convolution of Bluestein's middle
// pass: transform, product with conj, conj(y * conv[c*conv_c + k*conv_k]),
// transform again (the inverse by conjugation); RD 9 is RD 0 running a whole
// Bluestein convolution of length N in one tile: the chirp product and zero
// padding of RD 6 on load, the convolution of RD 8, the chirp product and
// truncation of RD 7 on store.
// WPE: occupancy floor in waves per SIMD (caps VGPRs at 512 / WPE).
// NT: bit 0 streams the output with non-temporal stores, bit 1 the input with
// non-temporal loads (neither is reused by this pass).
template <int N>
constexpr int leaf_lds_stride() { return (lds_pad(N - 1) + 1) | 1; }

// The leaf pass from tile `tile` on, every G-th tile, with the tile's LDS at
// lds (BT lines of leaf_lds_stride<N>() elements).
// The compile-time radix list Rs... is the one the planner lays the stage
// twiddle table out for (leaf_radix_at).
template <int N, int... Rs>
constexpr bool leaf_radices_match()
{
    constexpr int r[] = {Rs...};
    if ((int)sizeof...(Rs) != leaf_radix_count(N)) return false;
    for (int i = 0; i < (int)sizeof...(Rs); ++i)
        if (r[i] != leaf_radix_at(N, i)) return false;
    return true;
}

template <typename T, int N, int BT, bool PF, int NT, int RD, int... Rs>
__device__ __forceinline__ void leaf_body(const PassArgs &a, cpx<T> *lds, int64_t tile,
                                          const int64_t G)
{
    static_assert(leaf_radices_match<N, Rs...>(), "radix list differs from the planner's table layout");
    constexpr int TPT = N / 16;
    constexpr int STRIDE = leaf_lds_stride<N>();
    constexpr bool cols_in = RD == 3 || RD == 4 || RD == 6 || RD == 8;
    constexpr bool cols_out = RD == 3 || RD == 5 || RD == 7 || RD == 8;
    constexpr bool xpose = cols_in != cols_out;
    static_assert(!(xpose && PF), "transposing tiles are one tile per workgroup");
    const int tid = threadIdx.x;
    // lane -> (line, thread of the line) for the loads and the stages, and for
    // the stores of a transposing tile
    const int tr = cols_in ? (tid & (BT - 1)) : tid / TPT;
    const int t = cols_in ? tid / BT : tid - tr * TPT;
    const int trs = cols_out ? (tid & (BT - 1)) : tid / TPT;
    const int ts = cols_out ? tid / BT : tid - trs * TPT;
    // element strides of the line (compile-time 1 for row lines)
    const int64_t eis = cols_in ? a.is : 1, eos = cols_out ? a.os : 1;
    cpx<T> *line = lds + tr * STRIDE;
    const bool cin = (a.flags & PF_CONJ_IN) != 0, cout = (a.flags & PF_CONJ_OUT) != 0;

    StageChain<T, N, TPT, 1, Rs...> chain;
    chain.load(glob((const cpx<T> *)a.tw_leaf), 0, t);

    // column tiles: inner index of the lane's store line (for the twiddle);
    // Bluestein modes: index of the lane's load line clamped to the vector
    // loop (for the chirp, spectrum and, in row tiles, the store tables)
    int64_t cst = 0, lc = 0;
    constexpr bool pre = RD == 6 || RD == 9, conv = RD == 8 || RD == 9;
    constexpr bool post = RD == 7 || RD == 9;
    static_assert(!(PF && (pre || conv)), "lc belongs to the tile being computed");
    auto line_base = [&](int64_t tile, int64_t *ib, int64_t *obs, bool *ok) {
        const int64_t o = tile / a.ntiles_inner;
        const int64_t c0 = (tile - o * a.ntiles_inner) * BT;
        const int64_t c = c0 + tr;
        if constexpr (cols_in || cols_out) cst = c0 + (xpose ? trs : tr);
        if constexpr (pre || conv) lc = c < a.vn ? c : a.vn - 1;
        int64_t rem = o, bi = 0, bo = 0;
        for (int d = a.nouter - 1; d >= 0; --d) {
            const int64_t qd = rem / a.on[d];
            const int64_t idx = rem - qd * a.on[d];
            rem = qd;
            bi += idx * a.ois[d];
            bo += idx * a.oos[d];
        }
        // a padding line of a partial last tile reads the last line (its
        // results are never stored), so that every load is unconditional
        *ib = bi + (c < a.vn ? c : a.vn - 1) * a.vis;
        const int64_t cs = xpose ? cst : c;
        *ok = cs < a.vn;
        *obs = bo + cs * a.vos;
    };
    auto load_line = [&](cpx<T>(&x)[16], int64_t ib) {
        const gptr<const cpx<T>> src = glob((const cpx<T> *)a.in) + ib + t * eis;
        if constexpr (pre) {
            // elements past li_lim read element 0 of the line (in range) and
            // become zero
            const gptr<const cpx<T>> pm = glob((const cpx<T> *)a.pre);
            const int64_t j0 = lc * a.li_c + (int64_t)t * a.li_l, js = (int64_t)TPT * a.li_l;
#pragma unroll
            for (int e = 0; e < 16; ++e)
                x[e] = ld_elem<NT>(j0 + e * js < a.li_lim ? &src[e * TPT * eis]
                                                          : glob((const cpx<T> *)a.in) + ib);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t j = j0 + e * js;
                const bool v = j < a.li_lim;
                const cpx<T> w = pm[v ? j : 0];
                const cpx<T> y = cin ? conj(x[e]) : x[e];
                x[e] = v ? cmul(y, w) : cpx<T>{T(0), T(0)};
            }
            return;
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) x[e] = ld_elem<NT>(&src[e * TPT * eis]);
    };

    // Real-data fusions (one line = the n-point complex transform of a packed
    // real sequence of length 2n): PF_C2R combines the n+1 values of a half
    // spectrum into the packed input on load, PF_R2C splits the result into the
    // n+1 outputs on store (both as the elementwise real-data steps, through
    // LDS since the partners k and n-k sit in different lanes).
    constexpr bool r2c = RD == 1, c2r = RD == 2;
    const gptr<const cpx<T>> rtw = glob((const cpx<T> *)a.post);   // w_2n^k, k <= n/2
    // half spectrum X (n+1 values from ib) -> packed Z' in LDS, lane t taking
    // the pairs (k, n-k), k = t + j*TPT <= n/2 (j <= 8); the loads of a group
    // of JC pairs (all nine in FP32, two groups in FP64 to bound registers)
    // are issued before their first use; ends with a barrier
    constexpr int J = N / 2 / TPT + 1;
    constexpr int JC = sizeof(T) == 4 ? J : (J + 1) / 2;
    auto combine_half_spectrum = [&](int64_t ib) {
        const gptr<const cpx<T>> X = glob((const cpx<T> *)a.in) + ib;
        // an opaque copy of the lane index keeps the compiler from hoisting
        // the J table and line addresses out of the tile loop
        int tq = t;
        __asm__ volatile("" : "+v"(tq));
#pragma unroll
        for (int j0 = 0; j0 < J; j0 += JC) {
            cpx<T> A[JC], B[JC], W[JC];
#pragma unroll
            for (int q = 0; q < JC; ++q) {
                const int k = min(tq + (j0 + q) * TPT, N / 2);
                A[q] = ld_elem<NT>(&X[k]);
                B[q] = ld_elem<NT>(&X[N - k]);
                W[q] = rtw[k];
            }
#pragma unroll
            for (int q = 0; q < JC; ++q) {
                const int k = t + (j0 + q) * TPT;
                if (j0 + q >= J || k > N / 2) break;
                if (k == 0) {   // bins 0 and n of the real transform are real
                    line[0] = {A[q].re + B[q].re, A[q].re - B[q].re};
                    continue;
                }
                const cpx<T> P = {A[q].re + B[q].re, A[q].im - B[q].im};
                const cpx<T> M = {A[q].re - B[q].re, A[q].im + B[q].im};
                const cpx<T> wM = cmul(conj(W[q]), M);
                const cpx<T> iwM = {-wM.im, wM.re};
                line[lds_pad(k)] = {P.re + iwM.re, P.im + iwM.im};
                if (2 * k != N) line[lds_pad(N - k)] = {P.re - iwM.re, iwM.im - P.im};
            }
        }
        __syncthreads();
    };
    // packed transform Z (in x, element t + e*TPT) -> the n+1 outputs of the
    // real transform at ob; ends with a barrier so the next tile may reuse LDS
    auto split_to_half_spectrum = [&](const cpx<T>(&z)[16], int64_t ob, bool ok) {
#pragma unroll
        for (int e = 0; e < 16; ++e) *lds_slot<TPT>(line, t, e) = z[e];
        __syncthreads();
        if (ok) {
            const gptr<cpx<T>> X = glob((cpx<T> *)a.out) + ob;
            const T half = T(0.5);
            int tq = t;   // opaque, as in the combine
            __asm__ volatile("" : "+v"(tq));
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int k = tq + j * TPT;
                if (k > N / 2) break;
                const cpx<T> A = line[lds_pad(k)];
                if (k == 0) {
                    st_elem<NT>(&X[0], {A.re + A.im, T(0)});
                    st_elem<NT>(&X[N], {A.re - A.im, T(0)});
                    continue;
                }
                const cpx<T> B = line[lds_pad(N - k)];
                const cpx<T> E = {half * (A.re + B.re), half * (A.im - B.im)};
                const cpx<T> O = {half * (A.im + B.im), half * (B.re - A.re)};
                const cpx<T> wO = cmul(rtw[k], O);
                st_elem<NT>(&X[k], {E.re + wO.re, E.im + wO.im});
                if (2 * k != N) st_elem<NT>(&X[N - k], {E.re - wO.re, wO.im - E.im});
            }
        }
        __syncthreads();
    };

    if (tile >= a.ntiles) return;
    int64_t ib, ob;
    bool ok;
    line_base(tile, &ib, &ob, &ok);
    cpx<T> x[16];
    if constexpr (!c2r) load_line(x, ib);
    for (;;) {
        const int64_t next = tile + G;
        int64_t ib2 = 0, ob2 = 0;
        bool ok2 = false;
        cpx<T> xn[16];
        if constexpr (PF) {
            if (next < a.ntiles && !c2r) {
                line_base(next, &ib2, &ob2, &ok2);
                load_line(xn, ib2);
            }
        }
        if constexpr (c2r) {
            combine_half_spectrum(ib);
#pragma unroll
            for (int e = 0; e < 16; ++e) x[e] = *lds_slot<TPT>(line, t, e);
            __syncthreads();   // the first stage overwrites the line
        }
        if (cin && !pre) {
#pragma unroll
            for (int e = 0; e < 16; ++e) x[e] = conj(x[e]);
        }
        chain.run(x, line, t);
        if constexpr (conv) {
            // every LDS read of the first transform came before its last
            // barrier, so the second may start at once
            const gptr<const cpx<T>> cv = glob((const cpx<T> *)a.conv) + lc * a.conv_c + (int64_t)t * a.conv_k;
            const int64_t cks = (int64_t)TPT * a.conv_k;
#pragma unroll
            for (int e = 0; e < 16; ++e) x[e] = conj(cmul(x[e], cv[e * cks]));
            chain.run(x, line, t);
        }
        if constexpr (xpose) {
            // results to LDS in the stage mapping, back in the store mapping
#pragma unroll
            for (int e = 0; e < 16; ++e) *lds_slot<TPT>(line, t, e) = x[e];
            __syncthreads();
            cpx<T> *sl = lds + trs * STRIDE;
#pragma unroll
            for (int e = 0; e < 16; ++e) x[e] = *lds_slot<TPT>(sl, ts, e);
        }
        if constexpr (cols_in || cols_out) {
            if (a.flags & PF_TW4) {
                // element k = k0 + e*TPT of inner line c (k0 the lane's store
                // rank): w_N^(c*k).  FP32 data: the powers of w_N^(c*TPT) by an
                // FP64 recurrence from w_N^(c*k0) (16 steps, far below FP32
                // rounding); FP64 data: each twiddle from the two tables
                // (Section 6: no recurrence where it would reach the data's
                // precision)
                const int64_t cw = ok ? cst : 0;
                const int64_t k0 = xpose ? ts : t;
                if constexpr (sizeof(T) == 8) {
#pragma unroll
                    for (int e = 0; e < 16; ++e)
                        x[e] = mul_d(x[e], tw4_root(a, cw * (k0 + e * TPT)));
                } else {
                    double2 w = tw4_root(a, cw * k0);
                    const double2 ws = tw4_root(a, cw * TPT);
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        x[e] = mul_d(x[e], w);
                        w = zmul(w, ws);
                    }
                }
            }
        }
        if constexpr (post) {
            if (ok) {
                // the store line and the lane's rank in it (row tiles: the
                // load line, in range when ok)
                const int64_t sc = xpose ? cst : lc;
                const int sr = xpose ? ts : t;
                const gptr<cpx<T>> dst = glob((cpx<T> *)a.out) + ob + sr * eos;
                const gptr<const cpx<T>> pm = glob((const cpx<T> *)a.post);
                const bool ca = (a.flags & PF_CONJ_A) != 0;
                const int64_t g0 = sc * a.lo_c + (int64_t)sr * a.lo_k, gs = (int64_t)TPT * a.lo_k;
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int64_t g = g0 + e * gs;
                    if (g < a.lo_lim) {
                        const cpx<T> y = cmul(ca ? conj(x[e]) : x[e], pm[g]);
                        st_elem<NT>(&dst[e * TPT * eos], cout ? conj(y) : y);
                    }
                }
            }
        } else if constexpr (r2c) {
            split_to_half_spectrum(x, ob, ok);
        } else if (ok) {
            const gptr<cpx<T>> dst = glob((cpx<T> *)a.out) + ob + (xpose ? ts : t) * eos;
#pragma unroll
            for (int e = 0; e < 16; ++e)
                st_elem<NT>(&dst[e * TPT * eos], cout ? conj(x[e]) : x[e]);
        }
        if (next >= a.ntiles) break;
        // no barrier needed here (except after a transposing store): every
        // LDS read of this tile came before the barrier that ends the last
        // exchange
        if constexpr (xpose) __syncthreads();
        tile = next;
        bool prefetched = false;
        if constexpr (PF) {
            if (!c2r) {
                ib = ib2;
                ob = ob2;
                ok = ok2;
#pragma unroll
                for (int e = 0; e < 16; ++e) x[e] = xn[e];
                prefetched = true;
            }
        }
        if (!prefetched) {
            line_base(tile, &ib, &ob, &ok);
            if constexpr (!c2r) load_line(x, ib);
        }
    }
}

template <typename T, int N, int BT, bool PF, int WPE, int NT, int RD, int... Rs>
__global__ __launch_bounds__(BT *N / 16) __attribute__((amdgpu_waves_per_eu(WPE))) void leaf_kernel(PassArgs)
{
    __shared__ cpx<T> lds[BT * leaf_lds_stride<N>()];
    const PassArgs &a = *(const PassArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    leaf_body<T, N, BT, PF, NT, RD, Rs...>(a, lds, blockIdx.x, gridDim.x);
}

// Leaf passes of one length and tile kind from many plans in one launch (a
// batch across plans): one tile per workgroup, tiles numbered pass by pass
// (prefix[i] = tiles of passes before i, owner[t] = the pass of tile t, so a
// workgroup finds its pass with one load instead of a search); the workgroup
// runs that pass's tile with the pass's own arguments.  Non-temporal loads and
// stores, as the one-pass default.
template <typename T, int N, int BT, int RD, int... Rs>
__global__ __launch_bounds__(BT *N / 16) __attribute__((amdgpu_waves_per_eu(2))) void leaf_batch_kernel(
    const PassArgs *__restrict__ items, const int64_t *__restrict__ prefix,
    const int32_t *__restrict__ owner)
{
    __shared__ cpx<T> lds[BT * leaf_lds_stride<N>()];
    const int64_t tile = blockIdx.x;
    const int i = owner[tile];
    leaf_body<T, N, BT, false, 3, RD, Rs...>(items[i], lds, tile - prefix[i], int64_t(1) << 62);
}

}  // namespace mfft
