// Device-side phase arithmetic shared by the forward and adjoint kernels.
//
// Phases are kept in revolutions (1 revolution = 2 pi rad): the gfx950
// transcendental unit evaluates cos(2 pi t) and sin(2 pi t) directly
// (v_cos_f32 / v_sin_f32) with exact internal range reduction for
// |t| <= 256, so a phase reduced to a few revolutions needs no multiply by
// 2 pi and no further fract.
#pragma once

#include <hip/hip_runtime.h>

namespace cgh {

__device__ __forceinline__ float cos_rev(float t) { return __builtin_amdgcn_cosf(t); }
__device__ __forceinline__ float sin_rev(float t) { return __builtin_amdgcn_sinf(t); }
__device__ __forceinline__ float fract(float t) { return __builtin_amdgcn_fractf(t); }

// One axis of the compensated phase, Prev (h - v)^2 reduced mod 1 revolution
// up to an integer, for a pixel coordinate h (integer-valued float) and an
// axis record {c, Ph, Pl, b, d}:
//   m = h - c                      exact (integers below 2^24)
//   m^2                            exact for |m| < 4096
//   Ph m^2 = hi + e                exact two-product (fma)
//   fract(hi)                      exact
//   result = fract(hi) + ((b m + d + Pl m^2) + e)
// The result lies in about (-1.3, 2.3) revolutions; its absolute error is a
// few 1e-8 revolutions whatever the size of Prev (h - v)^2.
__device__ __forceinline__ float axis_phase(float h, float c, float ph, float pl, float b,
                                            float d) {
  const float m = h - c;
  const float mm = m * m;
  const float hi = ph * mm;
  const float e = __builtin_fmaf(ph, mm, -hi);
  const float r = fract(hi);
  float l = __builtin_fmaf(b, m, d);
  l = __builtin_fmaf(pl, mm, l);
  l = l + e;
  return r + l;
}

}  // namespace cgh
