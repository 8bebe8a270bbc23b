// Per-point precompute (FP64 arithmetic, O(N)), the per-row phase tables of
// the compensated forward (fused with the precompute) and of the compensated
// adjoint, and small fill kernels.  The records themselves are defined in
// records.h.
#include "cgh_internal.h"
#include "phase.h"
#include "records.h"

namespace cgh {

namespace {

// Writes point j's records (plain, amp, axis records, optional FP64 record).
__device__ __forceinline__ void store_records(const PointRecord& r, int64_t j,
                                              float4* __restrict__ plain,
                                              float* __restrict__ amp, float* __restrict__ xrec,
                                              float* __restrict__ yrec,
                                              double4* __restrict__ rec64) {
  plain[j] = make_float4(r.x, r.y, r.ph, r.a);
  amp[j] = r.a;
  float* rx = xrec + j * kAxisRec;
  float* ry = yrec + j * kAxisRec;
  rx[0] = r.xc;
  rx[1] = r.ph;
  rx[2] = r.pl;
  rx[3] = r.xb;
  rx[4] = r.xd;
  rx[5] = r.a;
  rx[6] = r.x;
  rx[7] = 0.0f;
  ry[0] = r.yc;
  ry[1] = r.ph;
  ry[2] = r.pl;
  ry[3] = r.yb;
  ry[4] = r.yd;
  ry[5] = r.a;
  ry[6] = r.y;
  ry[7] = 0.0f;
  if (rec64) rec64[j] = make_double4((double)r.x, (double)r.y, r.prev, (double)r.a);
}

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
  store_records(point_record(x, y, z, a, j, n, pitch, wavelength), j, plain, amp, xrec, yrec,
                rec64);
}

// The compensated forward's precompute in one launch.  Thread (g, j) with
// g < groups forms point j's records, writes them when g = 0, and writes the
// y-axis phases of point j at the kCompRows rows of row group g:
//   ytab[g][j][i] = axis_phase(g * kCompRows + i) of point j.
// The threads after those (when xtab is given) write the x-axis phases of
// point j at the kXtabCols columns of column group g - groups:
//   xtab[col][j] = axis_phase(col) of point j.
constexpr int kXtabCols = 8;
__global__ __launch_bounds__(256) void prep_ytab_kernel(
    const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ z,
    const float* __restrict__ a, int64_t n, int64_t npad, int64_t groups, int64_t xgroups,
    double pitch, double wavelength, float4* __restrict__ plain, float* __restrict__ amp,
    float* __restrict__ xrec, float* __restrict__ yrec, float* __restrict__ ytab,
    float* __restrict__ xtab) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (groups + xgroups) * npad) return;
  const int64_t g = t / npad, j = t - g * npad;
  const PointRecord r = point_record(x, y, z, a, j, n, pitch, wavelength);
  if (g < groups) {
    if (g == 0) store_records(r, j, plain, amp, xrec, yrec, nullptr);
    float* dst = ytab + t * kCompRows;
#pragma unroll
    for (int i = 0; i < kCompRows; ++i)
      dst[i] = axis_phase((float)(g * kCompRows + i), r.yc, r.ph, r.pl, r.yb, r.yd);
  } else {
    const int64_t c0 = (g - groups) * kXtabCols;
#pragma unroll
    for (int k = 0; k < kXtabCols; ++k)
      xtab[(c0 + k) * npad + j] = axis_phase((float)(c0 + k), r.xc, r.ph, r.pl, r.xb, r.xd);
  }
}

// The compensated adjoint's tables: thread (g, j) forms point j's records
// and, for g < groups, writes for the kRtabRows rows y_h of row group g
//   rtab[y_h][j] = {cos, sin of axis_phase(y_h) of point j};
// the threads after those write, for the kRtabRows columns x_h of column
// group g - groups (columns up to the last strip's end),
//   ctab[x_h][j] = axis_phase(x_h) of point j:
// the values the adjoint kernel would otherwise form per strip.
constexpr int kRtabRows = 8;
__global__ __launch_bounds__(256) void prep_rtab_kernel(
    const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ z,
    const float* __restrict__ a, int64_t n, int64_t npad, int ny, int64_t groups,
    int64_t cgroups, double pitch, double wavelength, float2* __restrict__ rtab,
    float* __restrict__ ctab) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (groups + cgroups) * npad) return;
  const int64_t g = t / npad, j = t - g * npad;
  const PointRecord r = point_record(x, y, z, a, j, n, pitch, wavelength);
  if (g < groups) {
    const int row0 = (int)(g * kRtabRows);
    const int rows = min(kRtabRows, ny - row0);
    for (int i = 0; i < rows; ++i) {
      const float yh = (float)(row0 + i);
      const float ry = axis_phase(yh, r.yc, r.ph, r.pl, r.yb, r.yd);
      rtab[(int64_t)(row0 + i) * npad + j] = make_float2(cos_rev(ry), sin_rev(ry));
    }
  } else {
    const int64_t c0 = (g - groups) * kRtabRows;
#pragma unroll
    for (int k = 0; k < kRtabRows; ++k)
      ctab[(c0 + k) * npad + j] = axis_phase((float)(c0 + k), r.xc, r.ph, r.pl, r.xb, r.xd);
  }
}

__global__ __launch_bounds__(256) void zero_f32_kernel(float* __restrict__ p, int64_t count) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = 0.0f;
}

__global__ __launch_bounds__(256) void zero_f64_kernel(double* __restrict__ p, int64_t count) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = 0.0;
}

}  // namespace

hipError_t launch_prep(const float* x, const float* y, const float* z, const float* a, int64_t n,
                       int64_t npad, double pitch, double wavelength, const Workspace& w,
                       bool want64, hipStream_t s) {
  hipLaunchKernelGGL(prep_kernel, dim3(grid_blocks(npad, 256)), dim3(256), 0, s, x, y, z, a, n,
                     npad, pitch, wavelength, w.plain, w.amp, w.xrec, w.yrec,
                     want64 ? w.rec64 : (double4*)nullptr, w.hmax);
  return hipGetLastError();
}

hipError_t launch_prep_ytab(const float* x, const float* y, const float* z, const float* a,
                            double pitch, double wavelength, const Plan& p, const Workspace& w,
                            hipStream_t s) {
  static_assert(kWave % kXtabCols == 0, "column groups tile the forward's 64-column blocks");
  const int64_t xgroups = w.xtab ? (int64_t)p.fwd_gx * kWave / kXtabCols : 0;
  const int64_t total = ((int64_t)p.groups + xgroups) * p.npad;
  const unsigned blocks = grid_blocks(total, 256);
  if (!blocks) return hipErrorInvalidValue;
  hipLaunchKernelGGL(prep_ytab_kernel, dim3(blocks), dim3(256), 0, s, x, y, z, a,
                     p.n, p.npad, (int64_t)p.groups, xgroups, pitch, wavelength, w.plain, w.amp,
                     w.xrec, w.yrec, w.ytab, w.xtab);
  return hipGetLastError();
}

hipError_t launch_prep_rtab(const float* x, const float* y, const float* z, const float* a,
                            double pitch, double wavelength, const Plan& p, const Workspace& w,
                            hipStream_t s) {
  static_assert(kAdjCols % kRtabRows == 0, "column groups tile the adjoint's strips");
  const int64_t groups = (p.ny + kRtabRows - 1) / kRtabRows;
  const int64_t cgroups = (int64_t)p.nsx * kAdjCols / kRtabRows;
  const unsigned blocks = grid_blocks((groups + cgroups) * p.npad, 256);
  if (!blocks || !w.rtab || !w.ctab) return hipErrorInvalidValue;
  hipLaunchKernelGGL(prep_rtab_kernel, dim3(blocks), dim3(256), 0, s, x, y, z, a, p.n, p.npad,
                     p.ny, groups, cgroups, pitch, wavelength, w.rtab, w.ctab);
  return hipGetLastError();
}

hipError_t launch_fill_zero_f32(float* p, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const unsigned blocks = grid_blocks(count, 256);
  if (!blocks) return hipErrorInvalidValue;
  hipLaunchKernelGGL(zero_f32_kernel, dim3(blocks), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

hipError_t launch_fill_zero_f64(double* p, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const unsigned blocks = grid_blocks(count, 256);
  if (!blocks) return hipErrorInvalidValue;
  hipLaunchKernelGGL(zero_f64_kernel, dim3(blocks), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

}  // namespace cgh
