// Red-black SOR cell update shared by every relaxation kernel, so that the
// untiled and the streamed kernels produce identical bits.
#pragma once

#include <hip/hip_runtime.h>

namespace twg {

// FP32: d = avg4 (+ f) - old with the exact quarter folded into one fma,
// then old + w * d in a second fma.
template <bool RHS>
__device__ __forceinline__ float upd(float old, float ew, float sn, float w, float f)
{
    const float s = ew + sn;
    const float d = RHS ? __builtin_fmaf(0.25f, s, f) - old : __builtin_fmaf(0.25f, s, -old);
    return __builtin_fmaf(w, d, old);
}

// FP64: in the order of the definition (this file is compiled with
// contraction off), so one sweep reproduces a plain FP64 sweep bit for bit.
// Without a source the quarter is folded into the subtraction: the product
// (E + W + S + N) / 4 is exact (unless it is subnormal), so the fma rounds
// once where the plain form rounds once as well.
template <bool RHS>
__device__ __forceinline__ double upd(double old, double ew, double sn, double w, double f)
{
    double d;
    if (RHS) {
        const double g = (ew + sn) * 0.25 + f;
        d = g - old;
    } else {
        d = __builtin_fma(0.25, ew + sn, -old);
    }
    return old + w * d;
}


}  // namespace twg
