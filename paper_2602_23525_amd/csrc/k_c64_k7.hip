// Tile-kernel variant: double complex, kernel kind 7 (see tile.h), up to 16
// elements per thread.
#include "tile.h"

namespace mfft {

hipError_t launch_pass_c64_k7(const PassArgs &a, size_t lds, hipStream_t s)
{
    static size_t big = 65536;   // dynamic LDS allowed so far (gfx950: up to 160 KB)
    if (lds > big) {
        (void)hipFuncSetAttribute((const void *)pass_kernel<double, 16, 7>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        big = lds;
    }
    const int64_t grid = (a.flags & PF_XCD) ? (a.ntiles + kXcds - 1) / kXcds * kXcds : a.ntiles;
    hipLaunchKernelGGL((pass_kernel<double, 16, 7>), dim3((unsigned)grid),
                       dim3(a.bt * a.tpt), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_batch_c64_k7(const PassArgs *items, const int64_t *prefix, const int32_t *owner,
                                int64_t total, unsigned long long *counter, int block, int grid,
                                size_t lds, hipStream_t s)
{
    static size_t big = 65536;
    if (lds > big) {
        (void)hipFuncSetAttribute((const void *)batch_kernel<double, 16, 7>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        big = lds;
    }
    hipLaunchKernelGGL((batch_kernel<double, 16, 7>), dim3(grid), dim3(block), lds, s, items,
                       prefix, owner, total, counter);
    return hipGetLastError();
}

int batch_blocks_per_cu_c64_k7(int block, size_t lds)
{
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, batch_kernel<double, 16, 7>, block, lds) !=
        hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return b > 0 ? b : 1;
}

}  // namespace mfft
