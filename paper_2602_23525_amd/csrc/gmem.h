// Global-memory pointers for data reached through pass descriptors.
//
// A pointer read from a descriptor in memory (a batch's item table) is a
// generic pointer, and the compiler would access it with flat instructions,
// which wait on both the LDS and the memory counters and take a 64-bit
// address per lane.  Converted once to the global address space, every
// access derived from it is a global load or store (scalar base plus 32-bit
// lane offset where the compiler can form one).  Only device memory is ever
// passed to the kernels, so the conversion is exact.
#pragma once
#include <hip/hip_runtime.h>

namespace mfft {

// (The host pass of the compiler, which parses but never emits device code,
// sees plain pointers: its targets have no global address space.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename P>
using gptr = __attribute__((address_space(1))) P *;
#else
template <typename P>
using gptr = P *;
#endif

template <typename P>
__device__ __forceinline__ gptr<P> glob(P *p)
{
    return (gptr<P>)p;
}

}  // namespace mfft
