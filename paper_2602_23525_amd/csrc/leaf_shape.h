// Shapes of the specialized power-of-two leaf kernel (leaf.h) that the
// planner needs on the host: which lengths it takes and how many lines one
// tile holds.  Plain constexpr arithmetic, shared by the kernel instantiations
// and the planner.
#pragma once
#include <cstdint>

namespace mfft {

// Lines per tile.  Row tiles: 256 threads (FP32) or 128 (FP64) of 16 elements,
// at least one line (n = 4096 FP64: one line of 256 threads).  Column tiles:
// 64 lines of 64 points up to 16 of 256 (FP32; half as many in FP64, same
// bytes), then 16 / 8 (FP32) and 8 / 4 (FP64) lines as the LDS allows.
constexpr int leaf_row_lines(int prec, int n)
{
    return (prec == 0 ? 4096 : 2048) / n > 0 ? (prec == 0 ? 4096 : 2048) / n : 1;
}
constexpr int leaf_col_lines(int prec, int n)
{
    if (prec == 0) return n <= 256 ? 4096 / n : (n <= 512 ? 16 : 8);
    return n <= 256 ? 2048 / n : (n <= 512 ? 8 : 4);
}

// 16384 points (FP32) and 8192 (FP64) fill the LDS of one CU with one line
constexpr int leaf_max_n(int prec) { return prec == 0 ? 16384 : 8192; }

// Row tiles: powers of two from 64 to leaf_max_n
constexpr bool leaf_supported(int prec, int64_t n)
{
    return n >= 64 && n <= leaf_max_n(prec) && (n & (n - 1)) == 0;
}
inline int leaf_lines_per_tile(int prec, int n) { return leaf_row_lines(prec, n); }

// Radix sequence of the leaf kernel for a supported length n = 2^e, in
// execution order: e/4 stages of radix 16, then one of radix 2^(e mod 4)
// when that is above 1.  The kernel's stage twiddle table is laid out for
// this sequence, whatever sequence a generic-kernel plan of n would use.
constexpr int leaf_log2(int64_t n) { return n > 1 ? 1 + leaf_log2(n / 2) : 0; }
constexpr int leaf_radix_count(int64_t n) { return leaf_log2(n) / 4 + (leaf_log2(n) % 4 ? 1 : 0); }
constexpr int leaf_radix_at(int64_t n, int i) { return i < leaf_log2(n) / 4 ? 16 : 1 << (leaf_log2(n) % 4); }

// Column tiles: 64-2048 points; transposing ones (columns in, rows out or the
// reverse) from 256, so that a row run is at least 16 lanes
constexpr bool leaf_col_supported(int prec, int64_t n, bool transposing)
{
    return (void)prec, n >= (transposing ? 256 : 64) && n <= 2048 && (n & (n - 1)) == 0;
}
inline int leaf_col_lines_per_tile(int prec, int n) { return leaf_col_lines(prec, n); }

}  // namespace mfft
