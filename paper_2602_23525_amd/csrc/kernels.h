// Host-side launchers of the HIP kernels (definitions in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "leaf_shape.h"

namespace mfft {

// Rank-0 plan (Section 4.2, "Rank-0 plans"): strided element copy over up to
// 8 loops.  elem_bytes is 8 (FP32 complex) or 16 (FP64 complex).
struct CopyArgs {
    const void *in;
    void *out;
    int32_t rank;
    int32_t elem_bytes;
    int64_t total;
    int64_t n[8], is[8], os[8];
};

// Elementwise steps of the real-data plans (one line = one transform, the
// vector loops as for copies).  n is the real length, h = n/2.
enum : int {
    RK_UNTANGLE = 0,  // Z (h complex) -> X (h+1 complex): split the transform of the
                      // packed sequence x[2j] + i x[2j+1] into the real transform
    RK_TANGLE = 1,    // X (h+1 complex) -> Z' (h complex): the reverse, for the inverse
    RK_WIDEN = 2,     // real -> complex with zero imaginary part (n elements)
    RK_HERM = 3,      // X (n/2+1 complex) -> conjugate-symmetric extension (n complex)
    RK_REAL = 4,      // complex -> its real part (n elements)
};

struct RealArgs {
    const void *in;
    void *out;
    const void *tw;      // RK_UNTANGLE / RK_TANGLE: w_n^k, k <= h/2 (element type)
    int32_t mode;
    int32_t vrank;
    int64_t n;           // real length of the transform
    int64_t cnt;         // work items per line
    int64_t total;       // lines * cnt
    int64_t is, os;      // line strides, in elements of the input / output type
    int64_t vn[8], vis[8], vos[8];
};

hipError_t launch_real(const RealArgs &a, int prec, hipStream_t s);
// w_N^k (sign -1), k < count, FP64-evaluated and rounded to the precision
hipError_t launch_gen_roots(void *out, int prec, int64_t count, int64_t N, hipStream_t s);

hipError_t launch_pass(const PassArgs &a, int prec, int emax, size_t lds_bytes, hipStream_t s);
// Batched generic-kernel launch: one workgroup of `block` threads per tile of
// the concatenated tile list (items, prefix sums and tile owners in device
// memory).
hipError_t launch_batch(const PassArgs *items_dev, const int64_t *prefix_dev,
                        const int32_t *owner_dev, int64_t total, int prec, int kind, int block,
                        size_t lds_bytes, hipStream_t s);
int pass_kind(uint32_t flags);
// Resident workgroups per CU of the single-pass generic kernel for a pass of
// kind `kind` (pass_kind) with `emax` elements per thread.
int pass_blocks_per_cu(int prec, int kind, int emax, int block, size_t lds);
// Batched-launch family of the variants with 24 elements per thread (lines
// with radices 17, 19, 23): kWideKind + pass_kind, for kinds 0 and 1.
constexpr int kWideKind = 16;
hipError_t launch_copy(const CopyArgs &a, hipStream_t s);

// In-place transpose of q x q blocks (the last step of an in-place two-pass
// Cooley-Tukey plan without scratch): in every block, element (i, j) at
// base + i*rs + j*cs trades places with (j, i); blocks at the offsets of up to
// 8 outer loops (n[d], s[d]).  elem_bytes 8 or 16.
struct TransposeArgs {
    void *data;
    int32_t elem_bytes;
    int32_t rank;
    int64_t q, rs, cs;
    int64_t total;            // number of blocks (product of n[d])
    int64_t n[8], s[8];
};
hipError_t launch_transpose_sq(const TransposeArgs &a, hipStream_t s);

// In-place permutation of equal runs (items) of a block: item x (len elements
// at base + x*xs, element stride es) moves to item next[x].  The permutation's
// cycles of length >= 2 start at starts[0 .. ncycles); blocks at the offsets of
// up to 8 outer loops (n[d], s[d]).  len <= 2048, elem_bytes 8 or 16.
struct PermuteArgs {
    void *data;
    int32_t elem_bytes;
    int32_t rank;
    int64_t len, es, xs;
    const int32_t *next, *starts;
    int32_t ncycles;
    int32_t nitems;           // items per block (bounds every cycle's length)
    int64_t total;            // number of blocks (product of n[d])
    int64_t n[8], s[8];
};
hipError_t launch_permute_items(const PermuteArgs &a, hipStream_t s);
// Stage table of Ns*R (k-major, leaf kernel) or Ns*(R-1) (j-major, generic
// kernel) twiddles w_(Ns*R)^(j*k).
hipError_t launch_gen_stage_twiddles(void *out, int prec, int Ns, int R, hipStream_t s,
                                     bool fp32_math, bool jmajor);
hipError_t launch_gen_tw4(void *hi, int64_t nhi, void *lo, int64_t nlo, int shift, int64_t N,
                          hipStream_t s);
hipError_t launch_gen_chirp(void *c, int64_t n, hipStream_t s);
hipError_t launch_gen_bluestein_v(void *v, const void *c, int64_t n, int64_t M, hipStream_t s);
hipError_t launch_gen_rader(int32_t *gather, int32_t *scatter, void *b, int64_t p, int64_t g,
                            hipStream_t s);
hipError_t launch_convert_scale(void *out, int prec, const void *in, int64_t count, double scale,
                                hipStream_t s);

}  // namespace mfft

namespace mfft {
// Specialized power-of-two leaf kernel (leaf.h): unit-stride lines, or tiles of
// adjacent lines with strided elements (shapes in leaf_shape.h).
// variant bit 0: prefetch next tile; bit 1: lower occupancy floor (more VGPRs)
int leaf_blocks_per_cu(int prec, int n, int variant);
hipError_t launch_leaf(const PassArgs &a, int prec, int n, int variant, int grid, hipStream_t s);
// Leaf passes of one length and tile kind (mode: 0 rows, 3 columns, 4 columns
// in / rows out, 5 rows in / columns out; leaf_batch_mode of the pass flags)
// from many plans in one launch: items[i] with prefix[i] = tiles before item
// i, owner[t] = the item of tile t.
int leaf_batch_mode(uint32_t flags);
hipError_t launch_leaf_batch(const PassArgs *items, const int64_t *prefix, const int32_t *owner,
                             int64_t tiles, int prec, int n, int mode, hipStream_t s);
}  // namespace mfft
