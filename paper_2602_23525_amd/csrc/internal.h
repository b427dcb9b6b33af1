// Internal types shared by the planner (host) and the pass kernels (device).
//
// A plan is a list of passes (Section 4.2: a plan is a composition of
// algorithmic steps).  Every pass is one launch of the tile kernel: it runs a
// loop of 1-D transforms ("lines") of one leaf length n over one or more vector
// loops, reading one buffer and writing another, with the plan steps that the
// paper treats separately fused into its loads and stores:
//   - the decimation-in-time twiddle multiply of the Cooley-Tukey step
//     (Section 4.2, "Cooley-Tukey plans"; the paper fuses it into the
//     "twiddle codelet", here it is fused into the store of the first pass);
//   - strided and transposed access, i.e. the indirect plan's rank-0 shuffle
//     (Section 4.2, "Indirect plans"), done through LDS tiles;
//   - the chirp and spectrum multiplies of Bluestein's algorithm and the
//     index permutations of Rader's algorithm (Section 4.2, "Plans for prime
//     sizes").
#pragma once
#include <cstdint>

namespace mfft {

constexpr int kMaxStages = 16;
constexpr int kMaxOuter = 6;

// How lanes map to memory in the load / store phase of a pass.
enum : int32_t {
    kModeRow = 0,  // consecutive lanes walk one line's elements (unit line stride)
    kModeCol = 1,  // consecutive lanes walk the tile's lines (unit vector stride)
};

enum : uint32_t {
    PF_CONJ_IN = 1u << 0,    // conjugate each loaded element
    PF_PRE_MUL = 1u << 1,    // multiply loaded element li by pre[li]
    PF_GATHER = 1u << 2,     // element address from gather[li] instead of the line index
    PF_CONV = 1u << 3,       // in-kernel cyclic convolution: y *= conv[k]; inverse DFT
    PF_TW4 = 1u << 4,        // Cooley-Tukey twiddle w_N^(k*c) on store
    PF_CONJ_A = 1u << 5,     // conjugate before the post multiply (inverse via conj)
    PF_POST_MUL = 1u << 6,   // multiply stored element lo by post[lo]
    PF_CONJ_OUT = 1u << 7,   // conjugate each stored element last
    PF_SCATTER = 1u << 8,    // element address from scatter[lo]
    PF_RADER = 1u << 9,      // single-kernel Rader: add x0, write Y[0] = x0 + sum
    PF_AUX_X0 = 1u << 10,    // save x0 of each transform to aux (multi-pass Rader)
    PF_AUX_A0 = 1u << 11,    // save the k=0 output (before post multiply) to aux
    PF_AUX_ADD = 1u << 12,   // add aux x0 on store, write Y[0] = x0 + A0 (multi-pass Rader)
    PF_XCD = 1u << 13,       // map consecutive tiles to one XCD (L2 locality of gathers)
    PF_R2C = 1u << 14,       // leaf kernel: split the packed real transform on store (n+1 out)
    PF_C2R = 1u << 15,       // leaf kernel: combine a half spectrum on load (n+1 in)
    PF_NT_IN = 1u << 16,     // generic kernel: non-temporal element loads
    PF_NT_OUT = 1u << 17,    // generic kernel: non-temporal element stores (plain stores)
    PF_LEAF_COL = 1u << 18,  // leaf kernel: tile of adjacent lines with strided elements
    PF_LEAF_CR = 1u << 19,   // leaf kernel: adjacent lines in, unit-stride lines out
    PF_LEAF_RC = 1u << 20,   // leaf kernel: unit-stride lines in, adjacent lines out
};

// Workgroups are dispatched round-robin over the chip's 8 XCDs, each with its
// own L2.  With PF_XCD the launch has a multiple of 8 workgroups and workgroup
// b runs tile (b % 8) * (grid / 8) + b / 8, so each XCD walks a contiguous
// range of tiles (all tiles of one transform share an L2).
constexpr int kXcds = 8;

// One Stockham stage of radix R after sub-transforms of size Ns are complete.
struct StageDesc {
    int32_t R;       // radix
    int32_t Ns;      // product of the radices of the earlier stages
    uint32_t magic;  // b / Ns == (umulhi(b, magic) + b) >> shift  for b < 2^24
    int32_t shift;
    int32_t tw_off;  // offset of this stage's twiddles in the stage table
    int32_t nb;      // butterflies of the stage, n / R
    // LDS layouts (generic tile kernel).  The layout a stage writes puts one
    // spare slot after every 2^wr_shift groups of Ns*R elements (none:
    // wr_shift 31), so element q*Ns*R + j + k*Ns sits at
    // q*Ns*R + j + (q >> wr_shift) + k*Ns.  The next stage reads element
    // b + k*nb at b + (q >> rd_shift) + k*rd_stride (q = b / Ns), the period
    // of the layout dividing nb.  Tile loads and the last stage's layout are
    // unpadded.
    int32_t rd_stride;
    int16_t rd_shift;
    int16_t wr_shift;
};

// Kernel argument block of one pass (also the descriptor of a batched item).
struct PassArgs {
    const void *in;
    void *out;
    const void *tw;       // stage twiddles, element type of the pass (generic
                          // kernel layout, offsets in st[].tw_off)
    const void *tw_leaf;  // the same twiddles in the specialized leaf kernel's
                          // layout (passes planned for that kernel)
    const void *tw4_hi;   // two-level Cooley-Tukey twiddle tables (FP64 pairs)
    const void *tw4_lo;
    const void *pre;      // pre-multiply table (element type)
    const void *post;     // post-multiply table
    const void *conv;     // in-kernel convolution spectrum
    const int32_t *gather;
    const int32_t *scatter;
    void *aux;            // per-transform (x0, A0) pairs for multi-pass Rader

    int32_t n;            // line length (leaf transform size)
    int32_t nst;          // number of stages
    int32_t tpt;          // threads per line
    int32_t bt;           // lines per tile (power of two)
    int32_t bt_log2;
    int32_t lds_stride;   // LDS complex elements per line (odd)
    int32_t load_mode;
    int32_t store_mode;
    uint32_t flags;
    int32_t nouter;
    StageDesc st[kMaxStages];

    int64_t is, os;             // element strides of the line
    int64_t vn, vis, vos;       // the tiled (inner) vector loop
    int64_t on[kMaxOuter], ois[kMaxOuter], oos[kMaxOuter];  // outer loops, on[0] slowest
    int64_t ntiles_inner;       // ceil(vn / bt)
    int64_t ntiles;             // ntiles_inner * prod(on)

    // logical element indices: li = c*li_c + l*li_l (load), lo = c*lo_c + k*lo_k (store)
    int64_t li_c, li_l, li_lim;
    int64_t lo_c, lo_k, lo_lim;

    int64_t tw4_N;
    int32_t tw4_shift;
    int32_t tw4_mask;

    // in-kernel convolution: element idx of line c is multiplied by
    // conv[c * conv_c + idx * conv_k]
    int64_t conv_c, conv_k;
};

// LDS index padding of the specialized leaf kernel: one spare slot every 16
// elements keeps radix-16 stride writes free of bank conflicts.  Lines of the
// generic tile kernel hold up to lds_pad(n - 1) + 1 elements in every layout.
__host__ __device__ constexpr int lds_pad(int i) { return i + (i >> 4); }

}  // namespace mfft
