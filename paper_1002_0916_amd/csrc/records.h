// Per-point records from the FP32 inputs, computed in FP64 (every source that
// includes this is compiled with contraction off, so the records are the same
// bits wherever they are formed).
//
// The phase coefficient of Eq. (1) (Section 1) is P_j = pi p^2 / (lambda z_j)
// in radians per pixel^2; the kernels work in revolutions, so the record holds
// Prev_j = P_j / (2 pi) = p^2 / (2 lambda z_j), as an FP32 hi/lo pair.  Per
// axis (v = x_j or y_j): c = rint(v), f = v - c (exact), b = fl32(-2 Prev f)
// and d = fl32(Prev f^2), so that Prev (h - v)^2 = Prev m^2 + b m + d with
// m = h - c an integer (the compensated axis phase).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cgh {

struct PointRecord {
  float x, y, a;        // the inputs (padding: 0, 0, 0)
  double prev;          // Prev in FP64
  float ph, pl;         // Prev = ph + pl (FP32 hi/lo)
  float xc, xb, xd;     // x axis {c, b, d}
  float yc, yb, yd;     // y axis {c, b, d}
};

// Point j of n; j >= n is padding: zero amplitude at a valid position (x = y =
// 0, z = 1), which adds exactly 0 to every sum.
__device__ __forceinline__ PointRecord point_record(const float* __restrict__ x,
                                                    const float* __restrict__ y,
                                                    const float* __restrict__ z,
                                                    const float* __restrict__ a, int64_t j,
                                                    int64_t n, double pitch, double wavelength) {
  float xs = 0.0f, ys = 0.0f, zs = 1.0f, as = 0.0f;
  if (j < n) {
    xs = x[j];
    ys = y[j];
    zs = z[j];
    as = a[j];
  }
  const double prev = (pitch * pitch) / (2.0 * wavelength * (double)zs);
  PointRecord r;
  r.x = xs;
  r.y = ys;
  r.a = as;
  r.prev = prev;
  r.ph = (float)prev;
  r.pl = (float)(prev - (double)r.ph);
  r.xc = rintf(xs);
  r.yc = rintf(ys);
  const double xf = (double)(xs - r.xc), yf = (double)(ys - r.yc);  // both exact
  r.xb = (float)(-2.0 * prev * xf);
  r.xd = (float)(prev * xf * xf);
  r.yb = (float)(-2.0 * prev * yf);
  r.yd = (float)(prev * yf * yf);
  return r;
}

}  // namespace cgh
