// Red-black SOR cell update shared by every relaxation kernel, so that the
// untiled and the streamed kernels produce identical bits.
#pragma once

#include <hip/hip_runtime.h>

namespace twg {

// The update of a FREE cell with neighbours E, W, N (the row above) and S
// (the row below):
//   d    = fma(1/4, ((E + W) + N) + S, f - old)     (f = 0 without a source)
//   new  = fma(w, d, old)
// in the element type, each operation rounded once (this file is compiled
// with contraction off).  S is added last because in the streamed kernels it
// is the neighbour the previous half-sweep of the same row step has just
// produced: the order keeps that dependency three operations deep.  The
// oracle's FP64 sweep evaluates the same expression, so FP64 sweeps match it
// bit for bit.
__device__ __forceinline__ float fused(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fused(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <bool RHS, typename T>
__device__ __forceinline__ T upd(T old, T ewn, T s, T w, T f)
{
    const T sum = ewn + s;
    const T d = fused(T(0.25), sum, RHS ? f - old : -old);
    return fused(w, d, old);
}

}  // namespace twg
