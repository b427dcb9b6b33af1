// Device code of the FFT tile kernel, included by one translation unit per
// (precision, registers-per-thread) variant.
//
// Tile kernel (one workgroup = one tile of `bt` lines of length n):
//   load   -> LDS (lanes along the lines' vector loop, for strided lines) or
//             straight into registers for the first stage (unit-stride lines);
//   stages -> Stockham autosort (Section 2: transforms back and forth between
//             two arrays, one digit per stage, in-order output, no bit
//             reversal).  Each stage loads R elements per butterfly into VGPRs,
//             multiplies by the stage twiddles, runs a register-resident radix-R
//             butterfly (R in 2,3,4,5,7,8,16) and writes back to LDS;
//   store  -> from registers (unit-stride lines) or through LDS (strided).
// The leaf is the "large base case" of Section 3.3: one workgroup completes a
// whole sub-transform held in LDS, so every pass costs one HBM round trip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gmem.h"
#include "internal.h"
#include "radix.h"
#include "twiddle4.h"

namespace mfft {

// ------------------------------------------------------------ kernel kinds
// Feature sets compiled into separate kernels so that plain leaf passes carry
// no code (or registers) for the fused plan steps they do not use.
enum : int {
    K_TW4 = 1,    // Cooley-Tukey twiddles on store
    K_EXT = 2,    // table-driven loads and stores: pre/post multiplies, gather/scatter,
                  // Rader's per-transform terms
    K_CONV = 4,   // in-kernel convolution between two transforms of the line
};

// ------------------------------------------------------------ tile context

template <typename T>
struct Tile {
    int tid, tr, t;
    bool act;           // thread belongs to the tile's bt * tpt lanes
    int64_t o;          // flattened outer index of the tile
    int64_t c0;         // first line of the tile along the inner vector loop
    int64_t ob_in, ob_out;
    cpx<T> *lds;        // tile base
    cpx<T> *my;         // this thread's line
    cpx<T> x0, a0;      // Rader: x[0] and the zero-frequency sum of the permuted input
};

// Element load that marks the data as not reused (PF_NT_IN).
template <typename T>
__device__ __forceinline__ cpx<T> ld_nt(gptr<const cpx<T>> p)
{
    return {__builtin_nontemporal_load(&p->re), __builtin_nontemporal_load(&p->im)};
}

// Elements per chunk of the table-driven (K_EXT) stores.
template <typename T>
constexpr int ext_chunk() { return sizeof(T) == 4 ? 3 : 4; }

// Plain tile load: all loads of the lane issued, then the LDS writes.  Element
// idx0 + k*step of the lane's line sits at p0 + k*pst; past the line's end (or
// past the vector loop, where the lane reads line c0) the lane re-reads an
// in-range element.
template <typename T, int EMAX>
__device__ __forceinline__ void issue_plain(const PassArgs &a, const Tile<T> &tl, int line,
                                            int idx0, cpx<T> (&r)[EMAX + 2])
{
    constexpr int KMAX = EMAX + 2;
    const int n = a.n, step = a.tpt;
    const int64_t c = tl.c0 + line;
    const gptr<const cpx<T>> p0 = glob((const cpx<T> *)a.in) + tl.ob_in +
                                  (c < a.vn ? c : tl.c0) * a.vis + (int64_t)idx0 * a.is;
    const int64_t pst = (int64_t)step * a.is;
    // slots past ceil(n / step) hold no element of any lane: skipped by a
    // uniform branch rather than loaded from p0
    const int kn = (n + step - 1) / step;
    gptr<const cpx<T>> p = p0;
    if (a.flags & PF_NT_IN) {
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            if (k < kn) r[k] = ld_nt(idx0 + k * step < n ? p : p0);
            p += pst;
        }
    } else {
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            if (k < kn) r[k] = *(idx0 + k * step < n ? p : p0);
            p += pst;
        }
    }
}

template <typename T, int EMAX>
__device__ __forceinline__ void commit_plain(const PassArgs &a, cpx<T> *lds, int line, int idx0,
                                             const cpx<T> (&r)[EMAX + 2])
{
    constexpr int KMAX = EMAX + 2;
    const int n = a.n, step = a.tpt;
    // the tile load's layout is unpadded: element idx at idx
    cpx<T> *d0 = lds + line * a.lds_stride + idx0;
    const bool cj = (a.flags & PF_CONJ_IN) != 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
        if (idx0 + k * step < n) d0[k * step] = cj ? conj(r[k]) : r[k];
}

// Tile load of one lane: elements idx0 + k*tpt (k < EMAX + 2, below n) of
// tile line `line` go to LDS.  Every global load of the lane is issued before
// the first LDS write, so a tile costs one memory round trip (two with a
// gather table).  Lanes past the vector loop or past the logical range read an
// in-range address and drop the value (zero padding beyond li_lim).
template <typename T, int EMAX, int KIND>
__device__ __forceinline__ void load_line(const PassArgs &a, const Tile<T> &tl, cpx<T> *lds,
                                          int line, int idx0)
{
    constexpr int KMAX = EMAX + 2;
    const int n = a.n, step = a.tpt;
    const int64_t c = tl.c0 + line;
    const bool okc = c < a.vn;
    const gptr<const cpx<T>> in = glob((const cpx<T> *)a.in) + tl.ob_in + (okc ? c : tl.c0) * a.vis;
    cpx<T> *dst = lds + line * a.lds_stride;
    const bool cj = (a.flags & PF_CONJ_IN) != 0;
    cpx<T> r[KMAX];
    if constexpr (KIND & K_EXT) {
        // one chunk: every index load of the lane, then every element and
        // table load, so that a gathered tile costs two memory round trips
        // (the load phase has registers to spare; the store side, which runs
        // inside the stages, keeps small chunks)
        constexpr int CH = KMAX;
        const uint32_t f = a.flags;
        const int64_t cl = c * a.li_c;
#pragma unroll
        for (int k0 = 0; k0 < KMAX; k0 += CH) {
            int li[CH], e[CH];
            bool val[CH];
            cpx<T> pm[CH];
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                const int idx = idx0 + (k0 + q) * step;
                const int64_t l = cl + (int64_t)idx * a.li_l;
                val[q] = k0 + q < KMAX && okc && idx < n && l < a.li_lim;
                li[q] = val[q] ? (int)l : 0;
                e[q] = val[q] ? idx : 0;
            }
            if (f & PF_GATHER) {
#pragma unroll
                for (int q = 0; q < CH; ++q) e[q] = glob(a.gather)[li[q]];
            }
            if (f & PF_NT_IN) {
#pragma unroll
                for (int q = 0; q < CH; ++q) r[q] = ld_nt(&in[(int64_t)e[q] * a.is]);
            } else {
#pragma unroll
                for (int q = 0; q < CH; ++q) r[q] = in[(int64_t)e[q] * a.is];
            }
            if (f & PF_PRE_MUL) {
#pragma unroll
                for (int q = 0; q < CH; ++q) pm[q] = glob((const cpx<T> *)a.pre)[li[q]];
            }
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                const int idx = idx0 + (k0 + q) * step;
                if (k0 + q < KMAX && idx < n) {
                    cpx<T> x = val[q] ? r[q] : cpx<T>{T(0), T(0)};
                    if (cj) x = conj(x);
                    if (f & PF_PRE_MUL) x = cmul(x, pm[q]);
                    dst[idx] = x;
                }
            }
        }
    } else {
        issue_plain<T, EMAX>(a, tl, line, idx0, r);
        commit_plain<T, EMAX>(a, lds, line, idx0, r);
    }
}

// Store M elements k0 + m*ks (m < M) of line c, values y[m]; with CHECK,
// only those below n.  With K_EXT, the table reads of a chunk (post multiply,
// scatter index) are issued before its first store.
template <typename T, int M, int KIND, bool CHECK>
__device__ __forceinline__ void store_run(const PassArgs &a, const Tile<T> &tl, int64_t c, bool okc,
                                          int64_t base, int k0, int ks, const cpx<T> (&y)[M])
{
    const gptr<cpx<T>> out = glob((cpx<T> *)a.out) + base;
    const uint32_t f = a.flags;
    const int n = a.n;
    if constexpr (KIND & K_EXT) {
        constexpr int CH = ext_chunk<T>();
        const int64_t l0 = c * a.lo_c + (int64_t)k0 * a.lo_k, lst = (int64_t)ks * a.lo_k;
#pragma unroll
        for (int m0 = 0; m0 < M; m0 += CH) {
            int lo[CH], e[CH];
            bool val[CH];
            cpx<T> pm[CH];
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                const int m = m0 + q;
                const int64_t l = l0 + m * lst;
                val[q] = m < M && okc && (!CHECK || k0 + m * ks < n) && l < a.lo_lim;
                lo[q] = val[q] ? (int)l : 0;
                e[q] = k0 + m * ks;
            }
            if (f & PF_SCATTER) {
#pragma unroll
                for (int q = 0; q < CH; ++q) e[q] = glob(a.scatter)[lo[q]];
            }
            if (f & PF_POST_MUL) {
#pragma unroll
                for (int q = 0; q < CH; ++q) pm[q] = glob((const cpx<T> *)a.post)[lo[q]];
            }
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                if (!val[q]) continue;
                cpx<T> v = y[m0 + q < M ? m0 + q : M - 1];
                if (f & PF_CONJ_A) v = conj(v);
                if ((f & PF_AUX_A0) && !(f & PF_CONV) && lo[q] == 0)
                    glob((cpx<T> *)a.aux)[2 * tl.o + 1] = v;
                if (f & PF_POST_MUL) v = cmul(v, pm[q]);
                if (f & (PF_RADER | PF_AUX_ADD)) v = cadd(v, tl.x0);
                if (f & PF_CONJ_OUT) v = conj(v);
                out[(int64_t)e[q] * a.os] = v;
                if ((f & (PF_RADER | PF_AUX_ADD)) && lo[q] == 0) {
                    cpx<T> y0 = cadd(tl.x0, tl.a0);
                    if (f & PF_CONJ_OUT) y0 = conj(y0);
                    out[0] = y0;
                }
            }
        }
    } else {
        if (okc) {
            const bool cj = (f & PF_CONJ_OUT) != 0;
            const int64_t pst = (int64_t)ks * a.os;
            gptr<cpx<T>> p = out + (int64_t)k0 * a.os;
            if (f & PF_NT_OUT) {
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    if (!CHECK || k0 + m * ks < n) {
                        const cpx<T> v = cj ? conj(y[m]) : y[m];
                        __builtin_nontemporal_store(v.re, &p->re);
                        __builtin_nontemporal_store(v.im, &p->im);
                    }
                    p += pst;
                }
            } else {
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    if (!CHECK || k0 + m * ks < n) *p = cj ? conj(y[m]) : y[m];
                    p += pst;
                }
            }
        }
    }
}

__device__ __forceinline__ int fast_div(int b, uint32_t magic, int shift)
{
    return (int)((__umulhi((uint32_t)b, magic) + (uint32_t)b) >> shift);
}

// Where a stage's inputs come from: LDS; LDS times the convolution spectrum;
// the pass's input in global memory (the first stage of a row tile: element
// b + k*nb of the line, so the lanes of a wave read consecutive elements)
enum { F_LDS = 0, F_GLOBAL = 1, F_LDS_CONV = 2 };
enum { E_LDS = 0, E_GLOBAL = 1 };

template <typename T, int R, int EMAX, int KIND>
__device__ __forceinline__ void stage(const PassArgs &a, const StageDesc &sd, Tile<T> &tl,
                                      int fetch, int emit)
{
    constexpr int NB = EMAX / R;
    // nb comes from the stage descriptor (not n / R) so that LDS addresses are
    // computed inside the stage rather than hoisted for every radix up front
    const int nb = sd.nb, tpt = a.tpt, Ns = sd.Ns;
    // opaque copies of the lane's thread and line indices: keep the compiler
    // from hoisting each radix's address arithmetic out of the stage loop
    // (registers held for the whole kernel; FP32 plain kind 102 -> 79 VGPRs)
    int t = tl.t, tr = tl.tr;
    __asm__ volatile("" : "+v"(t), "+v"(tr));
    cpx<T> *const my = tl.lds + tr * a.lds_stride;
    const int64_t c = tl.c0 + tr;
    const bool ok = c < a.vn;
    // lines past the vector loop (the last tile's padding) compute on an
    // in-range line's tables and store nothing: table reads stay in bounds
    const int64_t cs = ok ? c : tl.c0;
    const int64_t out_base = tl.ob_out + c * a.vos;
    // lanes past the tile's bt*tpt threads (batched launches with a larger
    // block) only take part in the barriers
    const int nbl = tl.act ? nb : 0;
    cpx<T> v[NB][R];
    int qv[NB];

#pragma unroll
    for (int i = 0; i < NB; ++i) qv[i] = fast_div(t + i * tpt, sd.magic, sd.shift);
    if (fetch == F_GLOBAL) {
        // straight from the input: line c (padding lines read line c0),
        // element b + k*nb, every load of the lane issued before the first use
        const gptr<const cpx<T>> src =
            glob((const cpx<T> *)a.in) + tl.ob_in + (ok ? c : tl.c0) * a.vis;
        const bool nt = (a.flags & PF_NT_IN) != 0, cj = (a.flags & PF_CONJ_IN) != 0;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int b = t + i * tpt;
            if (b < nbl) {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const gptr<const cpx<T>> e = src + (int64_t)(b + k * nb) * a.is;
                    if (nt) v[i][k] = ld_nt(e);
                    else v[i][k] = *e;
                }
            }
        }
        if (cj) {
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int k = 0; k < R; ++k) v[i][k] = conj(v[i][k]);
        }
    } else {
        // butterfly b = q*Ns + j reads element b + k*nb of the previous layout
        // (one address per butterfly, the k-th element rd_stride further)
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int b = t + i * tpt;
            if (b < nbl) {
                const cpx<T> *src = my + b + (qv[i] >> sd.rd_shift);
#pragma unroll
                for (int k = 0; k < R; ++k) v[i][k] = src[k * sd.rd_stride];
            }
        }
    }
    if constexpr (KIND & K_CONV) {
        if (fetch == F_LDS_CONV) {
            // in-kernel convolution: element idx of line c times the spectrum
            // entry conv[c*conv_c + idx*conv_k], conjugated (inverse by conjugation)
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int b = t + i * tpt;
                if (b < nbl) {
                    const gptr<const cpx<T>> cv =
                        glob((const cpx<T> *)a.conv) + cs * a.conv_c + (int64_t)b * a.conv_k;
                    const int64_t cst = (int64_t)nb * a.conv_k;
#pragma unroll
                    for (int k = 0; k < R; ++k) v[i][k] = conj(cmul(v[i][k], cv[k * cst]));
                }
            }
        }
    }
    // every read of the previous layout done before it is overwritten (a
    // stage that read the input has nothing to wait for: the tile's LDS was
    // released by the barrier that ended the previous tile)
    if (fetch != F_GLOBAL) __syncthreads();

    const gptr<const cpx<T>> tw = glob((const cpx<T> *)a.tw) + sd.tw_off;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int b = t + i * tpt;
        if (b < nbl) {
            const int q = qv[i];
            const int j = b - q * Ns;
            if (Ns > 1) {
                if constexpr (sizeof(T) == 4) {
                    // FP32: j-major table, the butterfly's R-1 twiddles are
                    // consecutive (one address, immediate offsets, 16-byte loads)
                    const gptr<const cpx<T>> w = tw + (uint32_t)j * (uint32_t)(R - 1);
                    cpx<T> wk[R - 1];
#pragma unroll
                    for (int k = 1; k < R; ++k) wk[k - 1] = w[k - 1];
#pragma unroll
                    for (int k = 1; k < R; ++k) v[i][k] = cmul(v[i][k], wk[k - 1]);
                } else {
                    // FP64: k-major table, lanes with consecutive j read
                    // consecutive entries (16-byte elements: wide rows of the
                    // j-major form spread a wave's load over too many lines)
                    const gptr<const cpx<T>> w = tw + j;
#pragma unroll
                    for (int k = 1; k < R; ++k) v[i][k] = cmul(v[i][k], w[k * Ns]);
                }
            }
            dftx<T, R>(v[i]);
            const int base = q * Ns * R + j;
            if (emit == E_GLOBAL) {
                if constexpr (KIND & K_TW4) {
                    if (a.flags & PF_TW4) {
                        // element base + k*Ns of line c takes w_N^(c*(j + k*Ns)):
                        // FP32 data: start w_N^(c*j), step w_N^(c*Ns), products
                        // in FP64; FP64 data: every twiddle from the tables
                        if constexpr (sizeof(T) == 8) {
#pragma unroll
                            for (int k = 0; k < R; ++k)
                                v[i][k] = mul_d(v[i][k], tw4_root(a, cs * (j + k * Ns)));
                        } else {
                            double2 w = tw4_root(a, cs * j);
                            const double2 ws = tw4_root(a, cs * Ns);
#pragma unroll
                            for (int k = 0; k < R; ++k) {
                                v[i][k] = mul_d(v[i][k], w);
                                w = zmul(w, ws);
                            }
                        }
                    }
                }
                store_run<T, R, KIND, false>(a, tl, c, ok, out_base, base, Ns, v[i]);
            } else {
                cpx<T> *dst = my + base + (q >> sd.wr_shift);
#pragma unroll
                for (int k = 0; k < R; ++k) dst[k * Ns] = v[i][k];
            }
        }
    }
    if (emit != E_GLOBAL) __syncthreads();
}

template <typename T, int EMAX, int KIND>
__device__ __forceinline__ void run_fft(const PassArgs &a, Tile<T> &tl, int first_fetch,
                                        int last_emit)
{
    for (int s = 0; s < a.nst; ++s) {
        const StageDesc &sd = a.st[s];
        const int fetch = s == 0 ? first_fetch : F_LDS;
        const int emit = s == a.nst - 1 ? last_emit : E_LDS;
        switch (sd.R) {
        case 2: stage<T, 2, EMAX, KIND>(a, sd, tl, fetch, emit); break;
        case 3: stage<T, 3, EMAX, KIND>(a, sd, tl, fetch, emit); break;
        case 4: stage<T, 4, EMAX, KIND>(a, sd, tl, fetch, emit); break;
        case 5: stage<T, 5, EMAX, KIND>(a, sd, tl, fetch, emit); break;
        case 7: stage<T, 7, EMAX, KIND>(a, sd, tl, fetch, emit); break;
        case 8: stage<T, 8, EMAX, KIND>(a, sd, tl, fetch, emit); break;
        case 6: stage<T, 6, EMAX, KIND>(a, sd, tl, fetch, emit); break;
        case 9: stage<T, 9, EMAX, KIND>(a, sd, tl, fetch, emit); break;
        case 10: stage<T, 10, EMAX, KIND>(a, sd, tl, fetch, emit); break;
        case 12: stage<T, 12, EMAX, KIND>(a, sd, tl, fetch, emit); break;
        case 14: stage<T, 14, EMAX, KIND>(a, sd, tl, fetch, emit); break;
        case 15: stage<T, 15, EMAX, KIND>(a, sd, tl, fetch, emit); break;
        case 11: stage<T, 11, EMAX, KIND>(a, sd, tl, fetch, emit); break;
        case 13: stage<T, 13, EMAX, KIND>(a, sd, tl, fetch, emit); break;
        // primes above 16: only the variant with 24 elements per thread
        case 17:
            if constexpr (EMAX >= 17) stage<T, 17, EMAX, KIND>(a, sd, tl, fetch, emit);
            break;
        case 19:
            if constexpr (EMAX >= 19) stage<T, 19, EMAX, KIND>(a, sd, tl, fetch, emit);
            break;
        case 23:
            if constexpr (EMAX >= 23) stage<T, 23, EMAX, KIND>(a, sd, tl, fetch, emit);
            break;
        default: stage<T, 16, EMAX, KIND>(a, sd, tl, fetch, emit); break;
        }
    }
}

// Tile context: lines c0 .. c0+bt-1 of the inner vector loop at outer index o.
template <typename T>
__device__ __forceinline__ Tile<T> tile_setup(const PassArgs &a, int64_t tile, cpx<T> *lds)
{
    Tile<T> tl;
    tl.tid = threadIdx.x;
    tl.tr = tl.tid / a.tpt;
    tl.t = tl.tid - tl.tr * a.tpt;
    tl.act = tl.tr < a.bt;
    if (!tl.act) tl.tr = 0;
    tl.o = tile / a.ntiles_inner;
    tl.c0 = (tile - tl.o * a.ntiles_inner) * a.bt;
    int64_t rem = tl.o, bi = 0, bo = 0;
    for (int d = a.nouter - 1; d >= 0; --d) {
        const int64_t q = rem / a.on[d];
        const int64_t idx = rem - q * a.on[d];
        rem = q;
        bi += idx * a.ois[d];
        bo += idx * a.oos[d];
    }
    tl.ob_in = bi;
    tl.ob_out = bo;
    tl.lds = lds;
    tl.my = lds + tl.tr * a.lds_stride;
    tl.x0 = {T(0), T(0)};
    tl.a0 = {T(0), T(0)};

    return tl;
}

// Lane's line and first element in the tile load.  Row mode: consecutive
// lanes walk one line's elements (unit line stride).  Column mode: nthr is a
// multiple of bt and consecutive lanes take consecutive lines (unit vector
// stride), each lane walking its line in steps of tpt.
template <typename T>
__device__ __forceinline__ void load_lane(const PassArgs &a, const Tile<T> &tl, int *line, int *idx0)
{
    if (a.load_mode == kModeCol) {
        *line = tl.tid & (a.bt - 1);
        *idx0 = tl.tid >> a.bt_log2;
    } else {
        *line = tl.tr;
        *idx0 = tl.t;
    }
}

// Everything after the tile load: the stages (two transforms around the
// spectrum product for an in-kernel convolution) and the store.  Ends with a
// barrier, so the workgroup may load its next tile into LDS.
template <typename T, int EMAX, int KIND>
__device__ __forceinline__ void tile_body(const PassArgs &a, Tile<T> &tl, cpx<T> *lds,
                                          int first_fetch)
{
    const int n = a.n, bt = a.bt;
    const uint32_t f = a.flags;
    cpx<T> *slots = lds + a.bt * a.lds_stride;   // 2 per line: x0, a0
    const int last_emit = a.store_mode == kModeCol ? E_LDS : E_GLOBAL;

    bool conv = false;
    if constexpr (KIND & K_CONV) conv = (f & PF_CONV) != 0;
    if (conv) {
        run_fft<T, EMAX, KIND>(a, tl, first_fetch, E_LDS);   // ends with a barrier
        if constexpr (KIND & K_EXT) {
            if (f & PF_RADER) {
                // x0 and the zero-frequency term of the permuted sequence, read
                // before the second transform overwrites the line
                tl.x0 = slots[2 * tl.tr];
                tl.a0 = tl.my[0];
                if (tl.act && tl.t == 0) slots[2 * tl.tr + 1] = tl.a0;
            }
        }
        if ((f & PF_AUX_A0) && tl.act && tl.t == 0 && tl.c0 + tl.tr == 0)
            glob((cpx<T> *)a.aux)[2 * tl.o + 1] = tl.my[0];   // zero frequency of line 0
        run_fft<T, EMAX, KIND>(a, tl, F_LDS_CONV, last_emit);
    } else {
        run_fft<T, EMAX, KIND>(a, tl, first_fetch, last_emit);
    }

    if (a.store_mode == kModeCol) {
        if (tl.act) {
            constexpr int KMAX = EMAX + 2;
            const int trq = tl.tid & (bt - 1);
            const int64_t c = tl.c0 + trq;
            const bool okc = c < a.vn;
            const int64_t base = tl.ob_out + c * a.vos;
            const cpx<T> *src = lds + trq * a.lds_stride;
            const int step = a.tpt;
            const int idx = tl.tid >> a.bt_log2;
            Tile<T> tq = tl;
            if constexpr (KIND & K_EXT) {
                if (f & PF_RADER) {
                    tq.x0 = slots[2 * trq];
                    tq.a0 = slots[2 * trq + 1];
                }
            }
            // this lane's elements idx + k*step of line c take the Cooley-Tukey
            // twiddle w_N^(c*idx) times powers of w_N^(c*step): two table
            // lookups per lane, FP64 products
            // (FP64 data: every twiddle from the tables instead)
            double2 w = make_double2(1.0, 0.0), ws = w;
            bool tw = false;
            int64_t cs = 0;
            if constexpr (KIND & K_TW4) {
                tw = (f & PF_TW4) != 0;
                if (tw) {
                    cs = okc ? c : tl.c0;   // padding lines: in-range tables
                    if constexpr (sizeof(T) != 8) {
                        w = tw4_root(a, (int64_t)idx * cs);
                        ws = tw4_root(a, (int64_t)step * cs);
                    }
                }
            }
            constexpr int CH = (KIND & K_EXT) ? ext_chunk<T>() : KMAX;
            // the last stage's layout is unpadded
#pragma unroll
            for (int k0 = 0; k0 < KMAX; k0 += CH) {
                // the last chunk may run past KMAX: those elements lie past
                // the line's end (n <= KMAX * step) and are not stored
                cpx<T> y[CH];
#pragma unroll
                for (int q = 0; q < CH; ++q) {
                    const int kk = idx + (k0 + q) * step;
                    y[q] = kk < n ? src[kk] : cpx<T>{T(0), T(0)};
                    if (tw) {
                        if constexpr (sizeof(T) == 8) {
                            if (kk < n) y[q] = mul_d(y[q], tw4_root(a, (int64_t)kk * cs));
                        } else {
                            y[q] = mul_d(y[q], w);
                            w = zmul(w, ws);
                        }
                    }
                }
                store_run<T, CH, KIND, true>(a, tq, c, okc, base, idx + k0 * step, step, y);
            }
        }
    }
    __syncthreads();  // the next tile of a persistent workgroup reuses LDS
}


// DIRECT: the single-pass kernel lets wide row tiles read the input in their
// first stage; the batched kernel keeps the LDS load (the direct path costs
// it 7 VGPRs, one wave per SIMD: the uneven batch's 7-smooth class ran 4.70
// -> 4.90 ms with it).
template <typename T, int EMAX, int KIND, bool DIRECT>
__device__ __forceinline__ void run_tile(const PassArgs &a, int64_t tile, cpx<T> *lds)
{
    Tile<T> tl = tile_setup<T>(a, tile, lds);
    const uint32_t f = a.flags;
    cpx<T> *slots = lds + a.bt * a.lds_stride;   // 2 per line: x0, a0
    if constexpr (KIND & K_EXT) {
        // per-transform scalars for Rader
        if (f & (PF_RADER | PF_AUX_X0)) {
            if (tl.act && tl.t == 0) {
                const int64_t c = tl.c0 + tl.tr;
                cpx<T> x0 = {T(0), T(0)};
                if (c < a.vn) {
                    x0 = glob((const cpx<T> *)a.in)[tl.ob_in + c * a.vis];
                    if (f & PF_CONJ_IN) x0 = conj(x0);
                }
                slots[2 * tl.tr] = x0;
                if ((f & PF_AUX_X0) && c == 0) glob((cpx<T> *)a.aux)[2 * tl.o] = x0;
            }
        }
        if (f & PF_AUX_ADD) {
            const gptr<const cpx<T>> aux = glob((const cpx<T> *)a.aux);
            tl.x0 = aux[2 * tl.o];
            tl.a0 = aux[2 * tl.o + 1];
        }
    }

    // plain and twiddled row tiles of lines at least a wave wide: the first
    // stage reads the input itself (no LDS round trip and barrier for the
    // load).  Measured on MI355X against the LDS load: 1000 x 16384 FP32
    // 66.5 -> 64.7 us, 3000 x 8192 110 -> 105, 6561 x 4096 142 -> 136, 6561 x
    // 2048 FP64 161 -> 153; lines of fewer lanes lost (60 x 131072 42 -> 47,
    // 200 x 32768 34.8 -> 36.7 us) and keep the LDS load.
    if constexpr (DIRECT && !(KIND & (K_EXT | K_CONV))) {
        if (a.load_mode == kModeRow && a.tpt >= 64) {
            tile_body<T, EMAX, KIND>(a, tl, lds, F_GLOBAL);
            return;
        }
    }
    if (tl.act) {
        int line, idx0;
        load_lane(a, tl, &line, &idx0);
        load_line<T, EMAX, KIND>(a, tl, lds, line, idx0);
    }
    __syncthreads();
    tile_body<T, EMAX, KIND>(a, tl, lds, F_LDS);
}

// Largest workgroup of the generic kernels: FP64 lines, and FP32 lines with 24
// elements per thread, keep 512 threads so the compiler may use up to 256
// VGPRs without spilling.
template <typename T>
constexpr int max_block(int emax) { return sizeof(T) == 8 || emax > 16 ? 512 : 1024; }

template <typename T, int EMAX, int KIND>
__global__ __launch_bounds__(max_block<T>(EMAX)) void pass_kernel(PassArgs a)
{
    extern __shared__ unsigned char smem[];
    cpx<T> *lds = (cpx<T> *)smem;
    // Read the argument block through the kernarg segment pointer so that the
    // per-stage descriptors indexed at run time are scalar loads rather than a
    // private copy of the whole block.
    const PassArgs *ap = (const PassArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    // one tile per workgroup; with PF_XCD consecutive tiles go to one XCD
    int64_t tile = blockIdx.x;
    if (ap->flags & PF_XCD) {
        const int64_t per = gridDim.x / kXcds;
        tile = (int64_t)(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
        if (tile >= ap->ntiles) return;   // whole workgroup leaves together
    }
    run_tile<T, EMAX, KIND, true>(*ap, tile, lds);
}

// Batched kernel over the passes of many plans, one tile per workgroup:
// workgroup g runs tile g of the concatenated tile list (items[i] covers tiles
// [prefix[i], prefix[i+1]), owner[g] is the item of tile g).  The hardware
// dispatcher starts each next workgroup where one finishes, as in a
// single-pass launch (measured on MI355X against a persistent grid popping
// tiles from a counter: the 7-smooth class of the uneven batch 5.10 -> 4.70 ms).
template <typename T, int EMAX, int KIND>
__global__ __launch_bounds__(max_block<T>(EMAX)) void batch_kernel(const PassArgs *__restrict__ items,
                                                     const int64_t *__restrict__ prefix,
                                                     const int32_t *__restrict__ owner)
{
    extern __shared__ unsigned char smem[];
    cpx<T> *lds = (cpx<T> *)smem;
    const int64_t g = blockIdx.x;
    const int i = owner[g];
    run_tile<T, EMAX, KIND, false>(items[i], g - prefix[i], lds);
}

}  // namespace mfft
