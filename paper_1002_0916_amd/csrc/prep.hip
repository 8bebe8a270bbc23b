// Per-point precompute (FP64 arithmetic, O(N)) and, in the same launch, the
// axis-phase tables of the compensated kernels; plus small fill kernels.
//
// The phase coefficient of Eq. (1) (Section 1) is P_j = pi p^2 / (lambda z_j)
// in radians per pixel^2; the kernels work in revolutions, so the record holds
// Prev_j = P_j / (2 pi) = p^2 / (2 lambda z_j).
#include "../../include/cgh.h"
#include "cgh_internal.h"
#include "phase.h"

namespace cgh {

namespace {

// Lane -> point j = blockIdx.x * 256 + threadIdx.x.  The workgroups with
// blockIdx.y == 0 store the records; when tables are requested (rows > 0),
// every workgroup also forms the compensated axis phases of its point for
// the table rows r = blockIdx.y, blockIdx.y + gridDim.y, ... (the records are
// recomputed per workgroup row, identically, so no second launch waits for
// them):
//   r < groups                    ytab[r][j][i] = Y_j(r * kCompRows + i)
//   groups <= r < groups + xcols  xtab[x][j] = X_j(x), x = r - groups
//   then yrows more rows          rowtab[y][j] = Y_j(y)
// (X_j, Y_j the compensated axis phases, axis_phase).
__global__ __launch_bounds__(256) void prep_kernel(
    const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ z,
    const float* __restrict__ a, int64_t n, int64_t npad, double pitch, double wavelength,
    float4* __restrict__ plain, float* __restrict__ amp, float* __restrict__ xrec,
    float* __restrict__ yrec, double4* __restrict__ rec64, unsigned* __restrict__ clear,
    int groups, int xcols, int yrows, float* __restrict__ ytab, float* __restrict__ xtab,
    float* __restrict__ rowtab) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool store = blockIdx.y == 0;
  if (store && clear && j == 0) *clear = 0u;
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
  const float xc = rintf(xs), yc = rintf(ys);
  const double xf = (double)(xs - xc), yf = (double)(ys - yc);  // both exact
  const float xb = (float)(-2.0 * prev * xf), xd = (float)(prev * xf * xf);
  const float yb = (float)(-2.0 * prev * yf), yd = (float)(prev * yf * yf);
  if (store) {
    plain[j] = make_float4(xs, ys, ph, as);
    amp[j] = as;
    float* rx = xrec + j * kAxisRec;
    float* ry = yrec + j * kAxisRec;
    rx[0] = xc;
    rx[1] = ph;
    rx[2] = pl;
    rx[3] = xb;
    rx[4] = xd;
    rx[5] = as;
    rx[6] = xs;
    rx[7] = 0.0f;
    ry[0] = yc;
    ry[1] = ph;
    ry[2] = pl;
    ry[3] = yb;
    ry[4] = yd;
    ry[5] = as;
    ry[6] = ys;
    ry[7] = 0.0f;
    if (rec64) rec64[j] = make_double4((double)xs, (double)ys, prev, (double)as);
  }
  const int rows = groups + xcols + yrows;
  for (int r = blockIdx.y; r < rows; r += gridDim.y) {
    if (r < groups) {
      float* dst = ytab + ((int64_t)r * npad + j) * kCompRows;
#pragma unroll
      for (int i = 0; i < kCompRows; ++i)
        dst[i] = axis_phase((float)(r * kCompRows + i), yc, ph, pl, yb, yd);
    } else if (r < groups + xcols) {
      const int xx = r - groups;
      xtab[(int64_t)xx * npad + j] = axis_phase((float)xx, xc, ph, pl, xb, xd);
    } else {
      const int yy = r - groups - xcols;
      rowtab[(int64_t)yy * npad + j] = axis_phase((float)yy, yc, ph, pl, yb, yd);
    }
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

inline unsigned blocks_for(int64_t count, int threads) {
  return (unsigned)((count + threads - 1) / threads);
}

}  // namespace

hipError_t launch_prep(const Plan& p, const float* x, const float* y, const float* z,
                       const float* a, double pitch, double wavelength, const Workspace& w,
                       bool want64, hipStream_t s) {
  // Compensated forward: ytab and xtab; compensated adjoint: xtab and rowtab.
  const bool tables = p.variant == CGH_COMPENSATED && !want64 &&
                      (p.op == CGH_OP_FORWARD || p.op == CGH_OP_BACKWARD);
  const bool fwd = p.op == CGH_OP_FORWARD;
  const int groups = tables && fwd ? p.groups : 0;
  const int xcols = !tables ? 0 : fwd ? p.fwd_gx * kWave : p.nsx * kAdjCols;
  const int yrows = tables && !fwd ? p.ny : 0;
  const int rows = groups + xcols + yrows;
  const dim3 grid = rows > 0 ? table_grid(p.npad, rows) : dim3(blocks_for(p.npad, 256));
  hipLaunchKernelGGL(prep_kernel, grid, dim3(256), 0, s, x, y, z, a, p.n, p.npad, pitch,
                     wavelength, w.plain, w.amp, w.xrec, w.yrec,
                     want64 ? w.rec64 : (double4*)nullptr, w.hmax, groups, xcols, yrows, w.ytab,
                     w.xtab, w.rowtab);
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
