// Host-only stand-in for the HIP runtime header, so that host code of the
// library compiles as ordinary C++ for CPU tests: the butterfly headers (plain
// arithmetic on register values) and the planner.  For the planner, "device"
// allocations are address ranges handed out by a counter (never dereferenced:
// every kernel launch is a stub of the test driver), and copies, waits and
// errors succeed.
#pragma once
#include <cstddef>
#include <cstdint>

#define __device__
#define __host__
#define __forceinline__ inline
#define __global__

typedef int hipError_t;
typedef struct ihipStream_t *hipStream_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2 };
enum hipMemcpyKind {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
};

struct HostStubHeap {
    static uintptr_t &top()
    {
        static uintptr_t t = (uintptr_t)1 << 44;
        return t;
    }
};

inline hipError_t hipMalloc(void **p, size_t bytes)
{
    uintptr_t &t = HostStubHeap::top();
    *p = (void *)t;
    t += (bytes + 4095) / 4096 * 4096 + 4096;
    return hipSuccess;
}
inline hipError_t hipFree(void *) { return hipSuccess; }
inline hipError_t hipMemcpy(void *, const void *, size_t, hipMemcpyKind) { return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipGetDevice(int *d)
{
    *d = 0;
    return hipSuccess;
}
inline const char *hipGetErrorString(hipError_t) { return "host stub"; }
