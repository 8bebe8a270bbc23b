// Forward kernels: the direct point-source sum of Eq. (1) (Section 1).
//
// Work mapping (all three kernels): one hologram pixel per lane.  The FP32
// kernels give lane l of a wave column x0 + l and kRows consecutive rows, so a
// wave writes kRows fully coalesced 256-byte row segments, and every point
// record is read once per wave through scalar loads (the loop index is
// wave-uniform), i.e. broadcast to all 64 lanes from SGPRs.  Points are
// unrolled kUnroll at a time so the scalar loads of the next points are in
// flight while the current ones are used.
#include "cgh_internal.h"
#include "phase.h"

namespace cgh {

namespace {

// Plain FP32: per interaction the phase Prev ((x_h - x_j)^2 + (y_h - y_j)^2)
// in revolutions, fract range reduction, native cosine, accumulate.
__global__ __launch_bounds__(kFwdThreads) void fwd_plain_kernel(const float4* __restrict__ rec,
                                                                int npad, int nx, int ny,
                                                                float* __restrict__ out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int col = blockIdx.x * kWave + lane;
  const int y0 = (blockIdx.y * kFwdWaves + wave) * kRows;
  const float xh = (float)col;
  float yh[kRows];
  float acc[kRows];
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    yh[i] = (float)(y0 + i);
    acc[i] = 0.0f;
  }
  for (int j = 0; j < npad; j += kUnroll) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const float4 r = rec[j + u];
      const float dx = xh - r.x;
      const float dx2 = dx * dx;
#pragma unroll
      for (int i = 0; i < kRows; ++i) {
        const float dy = yh[i] - r.y;
        const float r2 = __builtin_fmaf(dy, dy, dx2);
        const float t = fract(r.z * r2);
        acc[i] = __builtin_fmaf(r.w, cos_rev(t), acc[i]);
      }
    }
  }
  if (col < nx) {
#pragma unroll
    for (int i = 0; i < kRows; ++i)
      if (y0 + i < ny) out[(int64_t)(y0 + i) * nx + col] = acc[i];
  }
}

// Compensated FP32: the phase separates exactly as X_j(x_h) + Y_j(y_h) with
// X_j(x_h) = Prev (x_h - x_j)^2 and Y_j(y_h) = Prev (y_h - y_j)^2.  Each part
// is formed on the integer pixel grid as a compensated split product reduced
// mod 1 (axis_phase).  Y comes from the per-row table (wave-uniform, scalar
// loads); X is computed once per point per lane and reused for the lane's
// kRows pixels.  Per interaction: one add, the native cosine (no fract: the
// sum stays within a few revolutions) and one fma.
__global__ __launch_bounds__(kFwdThreads) void fwd_comp_kernel(const float* __restrict__ xrec,
                                                               const float* __restrict__ ytab,
                                                               int npad, int nx, int ny,
                                                               float* __restrict__ out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int col = blockIdx.x * kWave + lane;
  const int grp = blockIdx.y * kFwdWaves + wave;
  const float xh = (float)col;
  const float* __restrict__ yt = ytab + (int64_t)grp * npad * kRows;
  float acc[kRows];
#pragma unroll
  for (int i = 0; i < kRows; ++i) acc[i] = 0.0f;
  for (int j = 0; j < npad; j += kUnroll) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const float* r = xrec + (int64_t)(j + u) * kAxisRec;
      const float X = axis_phase(xh, r[0], r[1], r[2], r[3], r[4]);
      const float A = r[5];
      const float* yv = yt + (int64_t)(j + u) * kRows;
#pragma unroll
      for (int i = 0; i < kRows; ++i) acc[i] = __builtin_fmaf(A, cos_rev(X + yv[i]), acc[i]);
    }
  }
  const int y0 = grp * kRows;
  if (col < nx) {
#pragma unroll
    for (int i = 0; i < kRows; ++i)
      if (y0 + i < ny) out[(int64_t)(y0 + i) * nx + col] = acc[i];
  }
}

// FP64 reference: rho = Prev ((x_h - x_j)^2 + (y_h - y_j)^2) in revolutions,
// reduced exactly by rint, cosine by the device cospi.  One pixel per lane.
__global__ __launch_bounds__(256) void fwd_f64_kernel(const double4* __restrict__ rec, int npad,
                                                      int nx, int64_t npix,
                                                      double* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const double xh = (double)(p % nx);
  const double yh = (double)(p / nx);
  double acc = 0.0;
  for (int j = 0; j < npad; ++j) {
    const double4 r = rec[j];
    const double dx = xh - r.x;
    const double dy = yh - r.y;
    const double rho = r.z * (dx * dx + dy * dy);
    const double f = rho - rint(rho);
    acc += r.w * cospi(2.0 * f);
  }
  out[p] = acc;
}

}  // namespace

hipError_t launch_fwd_plain(const Plan& p, const Workspace& w, float* out, hipStream_t s) {
  hipLaunchKernelGGL(fwd_plain_kernel, dim3(p.fwd_gx, p.fwd_gy), dim3(kFwdThreads), 0, s,
                     (const float4*)w.plain, (int)p.npad, p.nx, p.ny, out);
  return hipGetLastError();
}

hipError_t launch_fwd_comp(const Plan& p, const Workspace& w, float* out, hipStream_t s) {
  hipLaunchKernelGGL(fwd_comp_kernel, dim3(p.fwd_gx, p.fwd_gy), dim3(kFwdThreads), 0, s,
                     (const float*)w.xrec, (const float*)w.ytab, (int)p.npad, p.nx, p.ny, out);
  return hipGetLastError();
}

hipError_t launch_fwd_f64(const Plan& p, const Workspace& w, double* out, hipStream_t s) {
  const int64_t npix = (int64_t)p.nx * p.ny;
  hipLaunchKernelGGL(fwd_f64_kernel, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, s,
                     (const double4*)w.rec64, (int)p.npad, p.nx, npix, out);
  return hipGetLastError();
}

}  // namespace cgh
