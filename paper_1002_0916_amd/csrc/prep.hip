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

// The compensated forward's precompute in one launch.  A block is 256
// points (blockIdx.y selects them) and one slice of a table (blockIdx.x): for
// x < yslices, kYtabSlice row groups of the row table,
//   ytab[g][j][i] = axis_phase(g * kCompRows + i) of point j,
// and after those (when xtab is given) kXtabSlice columns of the column table,
//   xtab[col][j] = axis_phase(col) of point j.
// Each thread forms its point's records once for the slice (and writes them in
// slice 0).  Index arithmetic is uniform per block: a per-lane 64-bit division
// of a flat index took a fifth of the instructions when each thread wrote 4 to
// 8 values.
constexpr int kYtabSlice = 4;   // row groups (16 rows) per thread
constexpr int kXtabSlice = 16;  // columns per thread
constexpr int kPrepBlock = 256;
__global__ __launch_bounds__(kPrepBlock) void prep_ytab_kernel(
    const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ z,
    const float* __restrict__ a, int64_t n, int64_t npad, int64_t groups, int64_t yslices,
    double pitch, double wavelength, float4* __restrict__ plain, float* __restrict__ amp,
    float* __restrict__ xrec, float* __restrict__ yrec, float4* __restrict__ ytab,
    float* __restrict__ xtab) {
  const int64_t j = (int64_t)blockIdx.y * kPrepBlock + threadIdx.x;
  if (j >= npad) return;
  const int64_t slice = blockIdx.x;
  const PointRecord r = point_record(x, y, z, a, j, n, pitch, wavelength);
  if (slice < yslices) {
    if (slice == 0) store_records(r, j, plain, amp, xrec, yrec, nullptr);
    const int64_t g0 = slice * kYtabSlice;
#pragma unroll
    for (int q = 0; q < kYtabSlice; ++q) {
      const int64_t g = g0 + q;
      if (g >= groups) break;
      const float h = (float)(g * kCompRows);
      ytab[g * npad + j] =
          make_float4(axis_phase(h, r.yc, r.ph, r.pl, r.yb, r.yd),
                      axis_phase(h + 1.0f, r.yc, r.ph, r.pl, r.yb, r.yd),
                      axis_phase(h + 2.0f, r.yc, r.ph, r.pl, r.yb, r.yd),
                      axis_phase(h + 3.0f, r.yc, r.ph, r.pl, r.yb, r.yd));
    }
  } else {
    const int64_t c0 = (slice - yslices) * kXtabSlice;
    float* dst = xtab + c0 * npad + j;
#pragma unroll
    for (int k = 0; k < kXtabSlice; ++k)
      dst[k * npad] = axis_phase((float)(c0 + k), r.xc, r.ph, r.pl, r.xb, r.xd);
  }
}

// The compensated adjoint's tables, laid out like the forward's: a block is
// 256 points (blockIdx.y) and one slice (blockIdx.x).  Slices x < rslices
// write kRtabSlice rows y_h of
//   rtab[y_h][j] = {cos, sin of axis_phase(y_h) of point j},
// the slices after those kRtabSlice columns x_h (columns up to the last
// strip's end) of
//   ctab[x_h][j] = axis_phase(x_h) of point j:
// the values the adjoint kernel would otherwise form per strip.
constexpr int kRtabSlice = 16;
__global__ __launch_bounds__(kPrepBlock) void prep_rtab_kernel(
    const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ z,
    const float* __restrict__ a, int64_t n, int64_t npad, int ny, int64_t rslices,
    double pitch, double wavelength, float2* __restrict__ rtab, float* __restrict__ ctab) {
  const int64_t j = (int64_t)blockIdx.y * kPrepBlock + threadIdx.x;
  if (j >= npad) return;
  const int64_t slice = blockIdx.x;
  const PointRecord r = point_record(x, y, z, a, j, n, pitch, wavelength);
  if (slice < rslices) {
    const int row0 = (int)(slice * kRtabSlice);
    const int rows = min(kRtabSlice, ny - row0);
    float2* dst = rtab + (int64_t)row0 * npad + j;
    for (int i = 0; i < rows; ++i) {
      const float ry = axis_phase((float)(row0 + i), r.yc, r.ph, r.pl, r.yb, r.yd);
      dst[i * npad] = make_float2(cos_rev(ry), sin_rev(ry));
    }
  } else {
    const int64_t c0 = (slice - rslices) * kRtabSlice;
    float* dst = ctab + c0 * npad + j;
#pragma unroll
    for (int k = 0; k < kRtabSlice; ++k)
      dst[k * npad] = axis_phase((float)(c0 + k), r.xc, r.ph, r.pl, r.xb, r.xd);
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
  static_assert(kWave % kXtabSlice == 0, "column slices tile the forward's 64-column blocks");
  static_assert(kCompRows == 4, "a row group of one point is one float4");
  const int64_t yslices = ((int64_t)p.groups + kYtabSlice - 1) / kYtabSlice;
  const int64_t xslices = w.xtab ? (int64_t)p.fwd_gx * kWave / kXtabSlice : 0;
  const int64_t pblocks = (p.npad + kPrepBlock - 1) / kPrepBlock;
  // blockIdx.y: at most 4000000 / 256 blocks of points
  if (yslices + xslices > 0x7fffffff || pblocks > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(prep_ytab_kernel, dim3((unsigned)(yslices + xslices), (unsigned)pblocks),
                     dim3(kPrepBlock), 0, s, x, y, z, a, p.n, p.npad, (int64_t)p.groups,
                     yslices, pitch, wavelength, w.plain, w.amp, w.xrec, w.yrec,
                     (float4*)w.ytab, w.xtab);
  return hipGetLastError();
}

hipError_t launch_prep_rtab(const float* x, const float* y, const float* z, const float* a,
                            double pitch, double wavelength, const Plan& p, const Workspace& w,
                            hipStream_t s) {
  static_assert(kAdjCols % kRtabSlice == 0, "column slices tile the adjoint's strips");
  const int64_t rslices = (p.ny + kRtabSlice - 1) / kRtabSlice;
  const int64_t cslices = (int64_t)p.nsx * kAdjCols / kRtabSlice;
  const int64_t pblocks = (p.npad + kPrepBlock - 1) / kPrepBlock;
  if (!w.rtab || !w.ctab || rslices + cslices > 0x7fffffff || pblocks > 65535)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(prep_rtab_kernel, dim3((unsigned)(rslices + cslices), (unsigned)pblocks),
                     dim3(kPrepBlock), 0, s, x, y, z, a, p.n, p.npad, p.ny, rslices, pitch,
                     wavelength, w.rtab, w.ctab);
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
