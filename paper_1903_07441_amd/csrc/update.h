// Red-black SOR cell update shared by every relaxation kernel, so that the
// untiled and the streamed kernels produce identical bits.
#pragma once

#include <hip/hip_runtime.h>

namespace twg {

// The update of a cell with neighbours E, W, N (the row above) and S (the
// row below) and factor w (omega on a FREE cell, 0 on a fixed one):
//   d    = fma(1/4, ((E + W) + N) + S, -old)
//   new  = fma(w, d, old)
// in the element type, each operation rounded once (this file is compiled
// with contraction off).  S is added last because in the streamed kernels it
// is the neighbour the previous half-sweep of the same row step has just
// produced: the order keeps that dependency three operations deep.  The
// oracle's FP64 sweep evaluates the same expression, so FP64 sweeps match it
// bit for bit.
__device__ __forceinline__ float fused(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fused(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ T upd(T old, T ewn, T s, T w)
{
    const T sum = ewn + s;
    const T d = fused(T(0.25), sum, -old);
    return fused(w, d, old);
}

// With a source term f (the correction solves of the defect correction) the
// same relaxation, old + w (avg4 + f - old), is evaluated from three
// per-cell constants formed once per row load,
//   a = w / 4,  b = 1 - w,  c = w f        (a fixed cell: a = 0, b = 1, c = 0)
//   new = fma(a, ((E + W) + N) + S, fma(b, old, c))
// which costs no more per update than the plain form.  1 - w is exact for w
// in [1, 2] (and for w = 0), and w / 4 is exact.
template <typename T> struct SrcConst { T a, b, c; };

template <typename T>
__device__ __forceinline__ SrcConst<T> src_const(T w, T f)
{
    return {w * T(0.25), T(1) - w, w * f};
}

template <typename T>
__device__ __forceinline__ T upd_src(T old, T ewn, T s, SrcConst<T> k)
{
    const T sum = ewn + s;
    return fused(k.a, sum, fused(k.b, old, k.c));
}

}  // namespace twg
