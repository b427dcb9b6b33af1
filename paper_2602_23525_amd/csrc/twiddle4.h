// Cooley-Tukey twiddles w_N^e from the two-level FP64 tables of a pass
// (Section 6: a small table plus one complex multiplication per twiddle),
// shared by the generic tile kernel and the leaf kernel's transposing tiles.
#pragma once
#include "butterfly.h"
#include "gmem.h"
#include "internal.h"

namespace mfft {

__device__ __forceinline__ double2 tw4_root(const PassArgs &a, int64_t e)
{
    // w_N^e = hi[e >> s] * lo[e & mask], both factors and the product in FP64
    // (the two-table scheme of Section 6)
    const double2 h = glob((const double2 *)a.tw4_hi)[e >> a.tw4_shift];
    const double2 l = glob((const double2 *)a.tw4_lo)[e & a.tw4_mask];
    return make_double2(h.x * l.x - h.y * l.y, h.x * l.y + h.y * l.x);
}

__device__ __forceinline__ double2 zmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <typename T>
__device__ __forceinline__ cpx<T> mul_d(cpx<T> y, double2 w)
{
    // twiddle rounded once to T, product in T
    const cpx<T> wt = {T(w.x), T(w.y)};
    return cmul(y, wt);
}

}  // namespace mfft
