// Per-point precompute (FP64 arithmetic, O(N)) and the per-row phase table of
// the compensated forward, plus small fill kernels.
//
// The phase coefficient of Eq. (1) (Section 1) is P_j = pi p^2 / (lambda z_j)
// in radians per pixel^2; the kernels work in revolutions, so the record holds
// Prev_j = P_j / (2 pi) = p^2 / (2 lambda z_j).
#include "cgh_internal.h"
#include "phase.h"

namespace cgh {

namespace {

__global__ __launch_bounds__(256) void prep_kernel(const float* __restrict__ x,
                                                   const float* __restrict__ y,
                                                   const float* __restrict__ z,
                                                   const float* __restrict__ a, int64_t n,
                                                   int64_t npad, double pitch, double wavelength,
                                                   float4* __restrict__ plain,
                                                   float* __restrict__ amp,
                                                   float* __restrict__ xrec,
                                                   float* __restrict__ yrec,
                                                   double4* __restrict__ rec64,
                                                   unsigned* __restrict__ clear) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (clear && j == 0) *clear = 0u;
  if (j >= npad) return;
  // Padding points have zero amplitude at a valid position, so they add
  // exactly 0 to every sum.
  float xs = 0.0f, ys = 0.0f, zs = 1.0f, as = 0.0f;
  if (j < n) {
    xs = x[j];
    ys = y[j];
    zs = z[j];
    as = a[j];
  }
  const double prev = (pitch * pitch) / (2.0 * wavelength * (double)zs);
  const float ph = (float)prev;
  const float pl = (float)(prev - (double)ph);
  plain[j] = make_float4(xs, ys, ph, as);
  amp[j] = as;

  const float xc = rintf(xs), yc = rintf(ys);
  const double xf = (double)(xs - xc), yf = (double)(ys - yc);  // both exact
  float* rx = xrec + j * kAxisRec;
  float* ry = yrec + j * kAxisRec;
  rx[0] = xc;
  rx[1] = ph;
  rx[2] = pl;
  rx[3] = (float)(-2.0 * prev * xf);
  rx[4] = (float)(prev * xf * xf);
  rx[5] = as;
  rx[6] = xs;
  rx[7] = 0.0f;
  ry[0] = yc;
  ry[1] = ph;
  ry[2] = pl;
  ry[3] = (float)(-2.0 * prev * yf);
  ry[4] = (float)(prev * yf * yf);
  ry[5] = as;
  ry[6] = ys;
  ry[7] = 0.0f;
  if (rec64) rec64[j] = make_double4((double)xs, (double)ys, prev, (double)as);
}

// ytab[g][j][i] = y-axis phase of point j at row g * kCompRows + i.
__global__ __launch_bounds__(256) void ytab_kernel(const float* __restrict__ yrec, int64_t npad,
                                                   int64_t total, float* __restrict__ ytab) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int64_t i = t % kCompRows;
  const int64_t j = (t / kCompRows) % npad;
  const int64_t g = t / (kCompRows * npad);
  const float* r = yrec + j * kAxisRec;
  const float h = (float)(g * kCompRows + i);
  ytab[t] = axis_phase(h, r[0], r[1], r[2], r[3], r[4]);
}

__global__ __launch_bounds__(256) void zero_f32_kernel(float* __restrict__ p, int64_t count) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = 0.0f;
}

__global__ __launch_bounds__(256) void zero_f64_kernel(double* __restrict__ p, int64_t count) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = 0.0;
}

inline unsigned blocks_for(int64_t count, int threads) {
  return (unsigned)((count + threads - 1) / threads);
}

}  // namespace

hipError_t launch_prep(const float* x, const float* y, const float* z, const float* a, int64_t n,
                       int64_t npad, double pitch, double wavelength, const Workspace& w,
                       bool want64, hipStream_t s) {
  hipLaunchKernelGGL(prep_kernel, dim3(blocks_for(npad, 256)), dim3(256), 0, s, x, y, z, a, n,
                     npad, pitch, wavelength, w.plain, w.amp, w.xrec, w.yrec,
                     want64 ? w.rec64 : (double4*)nullptr, w.hmax);
  return hipGetLastError();
}

hipError_t launch_ytab(const Plan& p, const Workspace& w, hipStream_t s) {
  const int64_t total = (int64_t)p.groups * p.npad * kCompRows;
  hipLaunchKernelGGL(ytab_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, w.yrec, p.npad,
                     total, w.ytab);
  return hipGetLastError();
}

hipError_t launch_fill_zero_f32(float* p, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_f32_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

hipError_t launch_fill_zero_f64(double* p, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_f64_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

}  // namespace cgh
