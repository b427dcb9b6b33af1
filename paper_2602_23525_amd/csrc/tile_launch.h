// Launchers of one variant (element type, kernel kind, elements per thread)
// of the generic tile kernel: the single-pass launch and the batched launch.  Each variant is instantiated by a
// translation unit of its own (k_c{32,64}_k{0,1,5,7}.hip, and
// k_c{32,64}_k{0,1}_e24.hip for lines with radices 17, 19, 23) so that the
// variants compile in parallel.
#pragma once
#include <mutex>

#include "tile.h"

namespace mfft {

// Raise a kernel's dynamic-LDS limit to at least `lds` bytes (gfx950: up to
// 160 KB per workgroup).  The limit only grows; calls from several host
// threads are serialized so that a smaller request never lowers it.
inline hipError_t allow_dynamic_lds(const void *fn, size_t lds, size_t *granted, std::mutex *m)
{
    std::lock_guard<std::mutex> lk(*m);
    if (lds <= *granted) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) *granted = lds;
    return e;
}

template <typename T, int KIND, int EMAX = 16>
struct TileLaunch {
    static std::mutex &mu()
    {
        static std::mutex m;
        return m;
    }

    static hipError_t pass(const PassArgs &a, size_t lds, hipStream_t s)
    {
        static size_t granted = 65536;
        hipError_t e = allow_dynamic_lds((const void *)pass_kernel<T, EMAX, KIND>, lds, &granted, &mu());
        if (e != hipSuccess) return e;
        const int64_t grid = (a.flags & PF_XCD) ? (a.ntiles + kXcds - 1) / kXcds * kXcds : a.ntiles;
        hipLaunchKernelGGL((pass_kernel<T, EMAX, KIND>), dim3((unsigned)grid), dim3(a.bt * a.tpt), lds,
                           s, a);
        return hipGetLastError();
    }

    // resident workgroups per CU of the single-pass kernel
    static int pass_blocks_per_cu(int block, size_t lds)
    {
        static size_t granted = 65536;
        if (allow_dynamic_lds((const void *)pass_kernel<T, EMAX, KIND>, lds, &granted, &mu()) != hipSuccess) {
            (void)hipGetLastError();
            return 1;
        }
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, pass_kernel<T, EMAX, KIND>, block, lds) !=
            hipSuccess) {
            (void)hipGetLastError();
            return 1;
        }
        return b > 0 ? b : 1;
    }

    // batched launch: one workgroup per tile of the concatenated list
    static hipError_t batch(const PassArgs *items, const int64_t *prefix, const int32_t *owner,
                            int64_t total, int block, size_t lds, hipStream_t s)
    {
        static size_t granted = 65536;
        hipError_t e = allow_dynamic_lds((const void *)batch_kernel<T, EMAX, KIND>, lds, &granted, &mu());
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((batch_kernel<T, EMAX, KIND>), dim3((unsigned)total), dim3(block), lds, s,
                           items, prefix, owner);
        return hipGetLastError();
    }
};

}  // namespace mfft

// The entry points of variant NAME (kernels.hip dispatches to them).
#define MFFT_TILE_LAUNCHERS(T, NAME, KIND) MFFT_TILE_LAUNCHERS_E(T, NAME, KIND, 16)
#define MFFT_TILE_LAUNCHERS_E(T, NAME, KIND, EMAX)                                                \
    namespace mfft {                                                                              \
    hipError_t launch_pass_##NAME(const PassArgs &a, size_t lds, hipStream_t s)                   \
    {                                                                                             \
        return TileLaunch<T, KIND, EMAX>::pass(a, lds, s);                                        \
    }                                                                                             \
    hipError_t launch_batch_##NAME(const PassArgs *items, const int64_t *prefix,                  \
                                   const int32_t *owner, int64_t total, int block, size_t lds,    \
                                   hipStream_t s)                                                 \
    {                                                                                             \
        return TileLaunch<T, KIND, EMAX>::batch(items, prefix, owner, total, block, lds, s);      \
    }                                                                                             \
    int pass_blocks_per_cu_##NAME(int block, size_t lds)                                          \
    {                                                                                             \
        return TileLaunch<T, KIND, EMAX>::pass_blocks_per_cu(block, lds);                         \
    }                                                                                             \
    }
