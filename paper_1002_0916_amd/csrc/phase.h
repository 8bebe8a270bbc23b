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
// axis record {c, Ph, Pl, b, d} (c = rint(v), f = v - c, Prev = Ph + Pl,
// b ~ -2 Prev f, d ~ Prev f^2, so Prev (h - v)^2 = Prev m^2 + b m + d):
//   m = h - c                        exact for |m| < 2^24
//   m^2 = mm + mm_lo                 exact pair (two-product by fma)
//   Ph mm = hi + e                   exact two-product
//   fract(hi)                        exact
//   l = ((Pl mm + d) + Ph mm_lo + e) + b m     small terms first, the
//                                              largest one last in one fma
//   l - rint(l)                      exact, in [-0.5, 0.5]
//   result = fract(hi) + (l - rint(l))         in [-0.5, 1.5)
// Pl mm_lo (below Prev m^2 2^-48) is dropped.  The error is one rounding of
// the result (<= 2^-24 rev) plus the roundings of l (|b m| <= Prev |m|, and
// b, d are FP32 roundings of their FP64 values): at most about
// 2^-24 (1 + 1.5 Prev |m|) + 2^-46 Prev m^2.  With Prev <= 2.5e-4 rev/px^2
// (pitch 8 um, 633 nm, z >= 0.2 m) that is below 5e-7 rev for |m| <= 16384
// and a few 1e-5 rev at |m| = 2^20, where the phase itself is 3e8 rev.
// The result stays within [-0.5, 1.5) for every input, so the cosine's
// exact-reduction range is never left.
__device__ __forceinline__ float axis_phase(float h, float c, float ph, float pl, float b,
                                            float d) {
  const float m = h - c;
  const float mm = m * m;
  const float mm_lo = __builtin_fmaf(m, m, -mm);
  const float hi = ph * mm;
  const float e = __builtin_fmaf(ph, mm, -hi);
  const float r = fract(hi);
  float l = __builtin_fmaf(pl, mm, d);
  l = __builtin_fmaf(ph, mm_lo, l);
  l = l + e;
  l = __builtin_fmaf(b, m, l);
  l = l - __builtin_rintf(l);
  return r + l;
}

}  // namespace cgh
