// Device helpers shared by the fused step (fused_step.hip) and the other
// kernels of liblbm.so (aux_kernels.hip): storage formats with their
// encode/decode rules, the wrap / mirror index maps of the boundaries, and
// the dispatch over the storage precisions.  Each translation unit gets its
// own copy (anonymous namespace).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "lbm_internal.h"

namespace lbm {
namespace {

// ---------------------------------------------------------------------------
// Storage formats
// ---------------------------------------------------------------------------
// bfloat16 storage: the upper 16 bits of an IEEE binary32
using bf16_t = uint16_t;

template <class T>
using gptr = __attribute__((address_space(1))) T*;

struct PF64 { using TM = double;   using TP = double; using R = double; };
struct PF32 { using TM = float;    using TP = float;  using R = float; };
struct PF16 { using TM = _Float16; using TP = float;  using R = float; };
struct PBF16 { using TM = bf16_t;  using TP = float;  using R = float; };

__device__ __forceinline__ float bf16_to_f32(bf16_t v) {
  return __uint_as_float(static_cast<uint32_t>(v) << 16);
}
// round to nearest even; NaN stays NaN (v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ bf16_t f32_to_bf16(float f) {
  return __builtin_bit_cast(bf16_t, static_cast<__bf16>(f));
}

template <class R> __device__ __forceinline__ R dec(double v, float, float) { return static_cast<R>(v); }
template <class R> __device__ __forceinline__ R dec(float v, float, float) { return static_cast<R>(v); }
template <class R> __device__ __forceinline__ R dec(_Float16 v, float off, float inv) {
  return static_cast<R>(static_cast<float>(v) * inv + off);
}
template <class R> __device__ __forceinline__ R dec(bf16_t v, float off, float inv) {
  return static_cast<R>(bf16_to_f32(v) * inv + off);
}

// Encoding of a stored value: identity for FP64 / FP32 storage; for the
// 16-bit formats (v - off) * scale in FP32, rounded to nearest even.
template <class T> struct Enc;
template <> struct Enc<double> {
  template <class R> __device__ static double go(R v, float, float) { return static_cast<double>(v); }
};
template <> struct Enc<float> {
  template <class R> __device__ static float go(R v, float, float) { return static_cast<float>(v); }
};
template <> struct Enc<_Float16> {
  template <class R> __device__ static _Float16 go(R v, float off, float scale) {
    return static_cast<_Float16>((static_cast<float>(v) - off) * scale);
  }
};
template <> struct Enc<bf16_t> {
  template <class R> __device__ static bf16_t go(R v, float off, float scale) {
    return f32_to_bf16((static_cast<float>(v) - off) * scale);
  }
};

// ---------------------------------------------------------------------------
// Index maps
// ---------------------------------------------------------------------------
// Coordinate i on an axis of length n: periodic wrap, or the half-way mirror
// of a wall (-1 -> 0, -2 -> 1, n -> n-1, n+1 -> n-2).  Columns far outside
// (never consumed) are clamped into range.
__device__ __forceinline__ int map_axis(int i, int n, int wall, int& crossed) {
  if (!wall) {
    int r = i % n;
    crossed = 0;
    return r < 0 ? r + n : r;
  }
  crossed = 0;
  if (i < 0) { i = -1 - i; crossed = 1; }
  else if (i >= n) { i = 2 * n - 1 - i; crossed = 1; }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

__device__ __forceinline__ int map_axis(int i, int n, int wall) {
  int c;
  return map_axis(i, n, wall, c);
}

// 1 / (sqrt(s) + 1e-12): IEEE sqrt and division in FP64; in FP32 the
// hardware square root and reciprocal (about 1 ulp), which the FP32 modes'
// error budget absorbs.
__device__ __forceinline__ double inv_norm_eps(double s) { return 1.0 / (sqrt(s) + 1e-12); }

// 1 / d for d > 0 (finite, normal): the hardware reciprocal estimate refined by
// two Newton steps r <- r + r (1 - d r), each squaring the relative error, so
// the result is within a rounding or two of the correctly rounded quotient --
// 5 instructions instead of the ~11 of the IEEE division sequence.
__device__ __forceinline__ double rcp_newton(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}
// FP32: the hardware reciprocal (1 ulp) and one Newton step
__device__ __forceinline__ float rcp_newton(float d) {
  const float r = __builtin_amdgcn_rcpf(d);
  return fmaf(r, fmaf(-d, r, 1.0f), r);
}
__device__ __forceinline__ float inv_norm_eps(float s) {
  return __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(s) + 1e-12f);
}

template <class F>
hipError_t dispatch(int precision, F&& f) {
  switch (precision) {
    case kF64: return f(PF64{});
    case kF32: return f(PF32{});
    case kF16: return f(PF16{});
    case kBF16: return f(PBF16{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace
}  // namespace lbm
