// Instantiations of the specialized power-of-two leaf kernel (leaf.h) and
// their launcher.  256 threads per workgroup for FP32, 128 for FP64, so that
// one tile's LDS stays near 35 KB (n = 4096: one line of 256 threads in both
// precisions, 35 KB FP32, 70 KB FP64).
#include "kernels.h"
#include "leaf.h"

namespace mfft {

template <typename T, int N, int BT, bool PF, int WPE, int NT, int RD, int... Rs>
static hipError_t go(const PassArgs &a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((leaf_kernel<T, N, BT, PF, WPE, NT, RD, Rs...>), dim3(grid), dim3(BT * N / 16), 0, s, a);
    return hipGetLastError();
}

template <typename T, int N, int BT, bool PF, int WPE, int NT, int RD, int... Rs>
static int occ()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, leaf_kernel<T, N, BT, PF, WPE, NT, RD, Rs...>,
                                                     BT * N / 16, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return blocks > 0 ? blocks : 1;
}

// kind: 0 = launch, 1 = occupancy query
template <typename T, int THREADS, bool PF, int WPE, int NT, int RD = 0>
static int dispatch(int kind, const PassArgs &a, int n, int grid, hipStream_t s, hipError_t *err)
{
#define LEAF_CASE(N, ...)                                                                  \
    case N:                                                                                \
        if (kind == 1) return occ<T, N, THREADS * 16 / N, PF, WPE, NT, RD, __VA_ARGS__>(); \
        *err = go<T, N, THREADS * 16 / N, PF, WPE, NT, RD, __VA_ARGS__>(a, grid, s);       \
        return 0;
    switch (n) {
        LEAF_CASE(64, 16, 4)
        LEAF_CASE(128, 16, 8)
        LEAF_CASE(256, 16, 16)
        LEAF_CASE(512, 16, 16, 2)
        LEAF_CASE(1024, 16, 16, 4)
        LEAF_CASE(2048, 16, 16, 8)
    default:
        break;
    }
    if (n == 4096) {
        // one line of 256 threads per workgroup in both precisions
        if (kind == 1) return occ<T, 4096, 1, PF, WPE, NT, RD, 16, 16, 16>();
        *err = go<T, 4096, 1, PF, WPE, NT, RD, 16, 16, 16>(a, grid, s);
        return 0;
    }
    if constexpr (!PF && (RD == 0 || RD == 9)) {
        // one line of 512 (8192 points) or 1024 threads (16384, FP32 only)
        if (n == 8192) {
            if (kind == 1) return occ<T, 8192, 1, PF, WPE, NT, RD, 16, 16, 16, 2>();
            *err = go<T, 8192, 1, PF, WPE, NT, RD, 16, 16, 16, 2>(a, grid, s);
            return 0;
        }
        if constexpr (sizeof(T) == 4) {
            if (n == 16384) {
                if (kind == 1) return occ<T, 16384, 1, PF, WPE, NT, RD, 16, 16, 16, 4>();
                *err = go<T, 16384, 1, PF, WPE, NT, RD, 16, 16, 16, 4>(a, grid, s);
                return 0;
            }
        }
    }
#undef LEAF_CASE
    *err = hipErrorInvalidValue;
    return 0;
}

// Column tiles (PF_LEAF_COL, ...): leaf_col_lines adjacent lines, so that each
// load and store instruction of a wave moves runs of that many elements.  One
// tile per workgroup, non-temporal loads and stores, as the row default.
constexpr int col_lines(int prec, int n) { return leaf_col_lines(prec, n); }

// RD 3: columns in and out (64-2048 points); 4 / 5: columns in, rows out and
// the reverse (256-2048 points, so that a row run is at least 16 lanes); 6 / 7:
// 4 / 5 with Bluestein's chirp products; 8: 3 with Bluestein's convolution
template <typename T, int RD>
static int dispatch_cols(int kind, const PassArgs &a, int n, int grid, hipStream_t s,
                         hipError_t *err)
{
    constexpr int P = sizeof(T) == 4 ? 0 : 1;
#define COL_CASE(N, ...)                                                                   \
    case N:                                                                                \
        if (kind == 1) return occ<T, N, col_lines(P, N), false, 2, 3, RD, __VA_ARGS__>();  \
        *err = go<T, N, col_lines(P, N), false, 2, 3, RD, __VA_ARGS__>(a, grid, s);        \
        return 0;
    if constexpr (RD == 3 || RD == 8) {
        switch (n) {
            COL_CASE(64, 16, 4)
            COL_CASE(128, 16, 8)
        default:
            break;
        }
    }
    switch (n) {
        COL_CASE(256, 16, 16)
        COL_CASE(512, 16, 16, 2)
        COL_CASE(1024, 16, 16, 4)
        COL_CASE(2048, 16, 16, 8)
    default:
        break;
    }
#undef COL_CASE
    *err = hipErrorInvalidValue;
    return 0;
}

// variant bits: 0 prefetch; 1-2 occupancy floor (1: 3 waves per SIMD, 2: 4,
// else 2; FP32 only); 3 non-temporal stores; 4 non-temporal loads (only
// together with stores).
template <typename T, int THREADS, bool PF, int WPE>
static int run_nt(int kind, const PassArgs &a, int n, int nt, int grid, hipStream_t s,
                  hipError_t *e)
{
    if (nt == 3) return dispatch<T, THREADS, PF, WPE, 3>(kind, a, n, grid, s, e);
    if (nt == 1) return dispatch<T, THREADS, PF, WPE, 1>(kind, a, n, grid, s, e);
    return dispatch<T, THREADS, PF, WPE, 0>(kind, a, n, grid, s, e);
}

template <typename T, int THREADS, bool PF>
static int run_wpe(int kind, const PassArgs &a, int n, int w, int nt, int grid, hipStream_t s,
                   hipError_t *e)
{
    if (w == 2) return run_nt<T, THREADS, PF, 4>(kind, a, n, nt, grid, s, e);
    if (w & 1) return run_nt<T, THREADS, PF, 3>(kind, a, n, nt, grid, s, e);
    return run_nt<T, THREADS, PF, 2>(kind, a, n, nt, grid, s, e);
}

static int run(int kind, const PassArgs &a, int prec, int n, int variant, int grid,
               hipStream_t s, hipError_t *e)
{
    if (a.flags & PF_LEAF_COL) {
        if (a.flags & PF_CONV)   // Bluestein's middle pass
            return prec == 0 ? dispatch_cols<float, 8>(kind, a, n, grid, s, e)
                             : dispatch_cols<double, 8>(kind, a, n, grid, s, e);
        return prec == 0 ? dispatch_cols<float, 3>(kind, a, n, grid, s, e)
                         : dispatch_cols<double, 3>(kind, a, n, grid, s, e);
    }
    if (a.flags & PF_LEAF_CR) {
        if (a.flags & PF_PRE_MUL)   // Bluestein's first pass
            return prec == 0 ? dispatch_cols<float, 6>(kind, a, n, grid, s, e)
                             : dispatch_cols<double, 6>(kind, a, n, grid, s, e);
        return prec == 0 ? dispatch_cols<float, 4>(kind, a, n, grid, s, e)
                         : dispatch_cols<double, 4>(kind, a, n, grid, s, e);
    }
    if (a.flags & PF_LEAF_RC) {
        if (a.flags & PF_POST_MUL)   // Bluestein's last pass
            return prec == 0 ? dispatch_cols<float, 7>(kind, a, n, grid, s, e)
                             : dispatch_cols<double, 7>(kind, a, n, grid, s, e);
        return prec == 0 ? dispatch_cols<float, 5>(kind, a, n, grid, s, e)
                         : dispatch_cols<double, 5>(kind, a, n, grid, s, e);
    }
    // real-data fusions: one configuration each, non-temporal loads and
    // stores as the plain default (prefetch only for FP32 r2c, where it pays
    // with a persistent grid)
    if (a.flags & (PF_R2C | PF_C2R)) {
        const bool pf = variant & 1;
        if (a.flags & PF_R2C) {
            if (prec == 0)
                return pf ? dispatch<float, 256, true, 2, 3, 1>(kind, a, n, grid, s, e)
                          : dispatch<float, 256, false, 2, 3, 1>(kind, a, n, grid, s, e);
            return dispatch<double, 128, false, 2, 3, 1>(kind, a, n, grid, s, e);
        }
        if (prec == 0) return dispatch<float, 256, false, 2, 3, 2>(kind, a, n, grid, s, e);
        return dispatch<double, 128, false, 2, 3, 2>(kind, a, n, grid, s, e);
    }
    // Bluestein in one tile: one configuration, as the column tiles
    if (a.flags & PF_CONV)
        return prec == 0 ? dispatch<float, 256, false, 2, 3, 9>(kind, a, n, grid, s, e)
                         : dispatch<double, 128, false, 2, 3, 9>(kind, a, n, grid, s, e);
    // lines above 4096 points are one tile per workgroup (no prefetch variant)
    const bool pf = (variant & 1) && n <= 4096;
    const int w = (variant >> 1) & 3, nt = (variant >> 3) & 3;
    if (prec == 0) {
        if (pf) return run_wpe<float, 256, true>(kind, a, n, w, nt, grid, s, e);
        return run_wpe<float, 256, false>(kind, a, n, w, nt, grid, s, e);
    }
    if (pf) return run_wpe<double, 128, true>(kind, a, n, 0, nt, grid, s, e);
    return run_wpe<double, 128, false>(kind, a, n, 0, nt, grid, s, e);
}

int leaf_blocks_per_cu(int prec, int n, int variant)
{
    hipError_t e = hipSuccess;
    return run(1, PassArgs{}, prec, n, variant, 0, 0, &e);
}

hipError_t launch_leaf(const PassArgs &a, int prec, int n, int variant, int grid, hipStream_t s)
{
    hipError_t e = hipSuccess;
    if (grid <= 0) return hipSuccess;
    run(0, a, prec, n, variant, grid, s, &e);
    return e;
}

}  // namespace mfft
