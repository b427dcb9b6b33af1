// Instantiations of the batched leaf kernel (leaf.h, leaf_batch_kernel): leaf
// passes of one length and tile kind from many plans in one launch, with the
// lines per tile of the one-pass kernel (the passes' tile counts assume them).
#include "kernels.h"
#include "leaf.h"

namespace mfft {

template <typename T, int N, int RD, int... Rs>
static hipError_t gob(const PassArgs *items, const int64_t *prefix, const int32_t *owner,
                      int64_t tiles, hipStream_t s)
{
    constexpr int P = sizeof(T) == 4 ? 0 : 1;
    constexpr int BT = (RD == 0 || RD == 9) ? leaf_row_lines(P, N) : leaf_col_lines(P, N);
    constexpr int THREADS = BT * N / 16;
    hipLaunchKernelGGL((leaf_batch_kernel<T, N, BT, RD, Rs...>), dim3((unsigned)tiles),
                       dim3(THREADS), 0, s, items, prefix, owner);
    return hipGetLastError();
}

// RD 0 rows (64-16384 points FP32, 64-8192 FP64), 3 columns (64-2048), 4 / 5
// transposing column tiles (256-2048), 6 / 7 the same with Bluestein's chirp
// products, 8 columns with Bluestein's convolution, 9 rows with a whole
// Bluestein convolution
template <typename T, int RD>
static hipError_t dispatch_b(const PassArgs *items, const int64_t *prefix, const int32_t *owner,
                             int64_t tiles, int n, hipStream_t s)
{
    if constexpr (RD == 0 || RD == 3 || RD == 8 || RD == 9) {
        if (n == 64) return gob<T, 64, RD, 16, 4>(items, prefix, owner, tiles, s);
        if (n == 128) return gob<T, 128, RD, 16, 8>(items, prefix, owner, tiles, s);
    }
    if constexpr (RD == 0 || RD == 9) {
        if (n == 4096) return gob<T, 4096, RD, 16, 16, 16>(items, prefix, owner, tiles, s);
        if (n == 8192) return gob<T, 8192, RD, 16, 16, 16, 2>(items, prefix, owner, tiles, s);
        if constexpr (sizeof(T) == 4) {
            if (n == 16384) return gob<T, 16384, RD, 16, 16, 16, 4>(items, prefix, owner, tiles, s);
        }
    }
    switch (n) {
    case 256: return gob<T, 256, RD, 16, 16>(items, prefix, owner, tiles, s);
    case 512: return gob<T, 512, RD, 16, 16, 2>(items, prefix, owner, tiles, s);
    case 1024: return gob<T, 1024, RD, 16, 16, 4>(items, prefix, owner, tiles, s);
    case 2048: return gob<T, 2048, RD, 16, 16, 8>(items, prefix, owner, tiles, s);
    default: break;
    }
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t dispatch_mode(const PassArgs *items, const int64_t *prefix,
                                const int32_t *owner, int64_t tiles, int n, int mode,
                                hipStream_t s)
{
    switch (mode) {
    case 0: return dispatch_b<T, 0>(items, prefix, owner, tiles, n, s);
    case 3: return dispatch_b<T, 3>(items, prefix, owner, tiles, n, s);
    case 4: return dispatch_b<T, 4>(items, prefix, owner, tiles, n, s);
    case 5: return dispatch_b<T, 5>(items, prefix, owner, tiles, n, s);
    case 6: return dispatch_b<T, 6>(items, prefix, owner, tiles, n, s);
    case 7: return dispatch_b<T, 7>(items, prefix, owner, tiles, n, s);
    case 8: return dispatch_b<T, 8>(items, prefix, owner, tiles, n, s);
    case 9: return dispatch_b<T, 9>(items, prefix, owner, tiles, n, s);
    default: return hipErrorInvalidValue;
    }
}

int leaf_batch_mode(uint32_t flags)
{
    if (flags & PF_LEAF_COL) return (flags & PF_CONV) ? 8 : 3;
    if (flags & PF_LEAF_CR) return (flags & PF_PRE_MUL) ? 6 : 4;
    if (flags & PF_LEAF_RC) return (flags & PF_POST_MUL) ? 7 : 5;
    if (flags & PF_CONV) return 9;
    return 0;
}

hipError_t launch_leaf_batch(const PassArgs *items, const int64_t *prefix, const int32_t *owner,
                             int64_t tiles, int prec, int n, int mode, hipStream_t s)
{
    if (tiles <= 0) return hipSuccess;
    if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
    return prec == 0 ? dispatch_mode<float>(items, prefix, owner, tiles, n, mode, s)
                     : dispatch_mode<double>(items, prefix, owner, tiles, n, mode, s);
}

}  // namespace mfft
