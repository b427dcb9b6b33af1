// Host-only stand-in for the HIP runtime header, so that the butterfly headers
// (plain arithmetic on register values) compile as ordinary C++ for CPU tests.
#pragma once
#define __device__
#define __host__
#define __forceinline__ inline
