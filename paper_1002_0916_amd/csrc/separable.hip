// Separable form of the hologram sum, evaluated as dense contractions on the
// matrix cores.
//
// The phase of Eq. (1) (Section 1) separates exactly by axis,
// theta_j(x_h, y_h) = 2 pi (X_j(x_h) + Y_j(y_h)) with X_j = Prev (x_h - x_j)^2
// and Y_j = Prev (y_h - y_j)^2 (both formed by the compensated axis_phase), so
// cos(theta) = cX cY - sX sY and
//
//   I[y][x] = sum_j A_j (cY_j(y) cX_j(x) - sY_j(y) sX_j(x)) = sum_k P[y][k] Q[x][k]
//
// with P[y][2j] = A_j cY_j(y), P[y][2j+1] = -A_j sY_j(y), Q[x][2j] = cX_j(x),
// Q[x][2j+1] = sX_j(x): one real GEMM of size ny x nx x 2N.  The adjoint sums
// (see adjoint.hip) factor the same way:
//
//   U_j(x) = sum_y G cY,  V_j(x) = sum_y G sY            (GEMM 2N x nx x ny)
//   Pc_j(y) = sum_x G cX, Ps_j(y) = sum_x G sX           (GEMM 2N x ny x nx)
//   Sc = sum_x (cX U - sX V);  column sums of G sin = sX U + cX V
//   row sums of G sin = cY Ps + sY Pc
//
// and Sx, Sr (x part) and Sy, Sr (y part) fold those with dx, dx^2, dy, dy^2.
// The adjoint GEMMs apply these folds to their own output tiles (fold.h), so
// U and Pm are never stored; a last pass adds the per-tile sums per point.
// This changes the algorithm (no per-interaction cosine): the per-point
// tables cost O(N (nx + ny)) transcendentals and the bulk is matrix-core
// work.
#include "cgh_internal.h"
#include "phase.h"

namespace cgh {

namespace {

// Both axis tables in one launch: tab[h][2j], tab[h][2j+1] = (s0 cos 2 pi
// phi, s1 sin 2 pi phi), phi the axis phase of point j at coordinate h;
// (s0, s1) = (1, 1), or (A_j, -A_j) for the y table when amp is given.
// Table rows r in [0, nxp) are the x table [nxp][npad] (float2 entries),
// rows [nxp, nxp + nyp) the y table [nyp][npad]; rows h >= nx (resp. ny) are
// zero.  Lane -> point j = blockIdx.x * 256 + threadIdx.x; the workgroups of
// one x index stride over the rows.
__global__ __launch_bounds__(256) void sep_table_kernel(
    const float* __restrict__ xrec, const float* __restrict__ yrec,
    const float* __restrict__ amp, int64_t npad, int nx, int nxp, int ny, int nyp,
    float2* __restrict__ tab_x, float2* __restrict__ tab_y) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= npad) return;
  float xr[5], yr[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    xr[i] = xrec[j * kAxisRec + i];
    yr[i] = yrec[j * kAxisRec + i];
  }
  const float A = amp ? amp[j] : 1.0f;
  for (int r = blockIdx.y; r < nxp + nyp; r += gridDim.y) {
    const bool is_x = r < nxp;
    const int h = is_x ? r : r - nxp;
    float2 v = make_float2(0.0f, 0.0f);
    if (h < (is_x ? nx : ny)) {
      const float* q = is_x ? xr : yr;
      const float phi = axis_phase((float)h, q[0], q[1], q[2], q[3], q[4]);
      const float c = cos_rev(phi), s = sin_rev(phi);
      v = (!is_x && amp) ? make_float2(A * c, -(A * s)) : make_float2(c, s);
    }
    (is_x ? tab_x : tab_y)[(int64_t)h * npad + j] = v;
  }
}

// I[y][x] = sum over split slices of C[s][y][x] (fixed order).
__global__ __launch_bounds__(256) void sep_sum_slices_kernel(const float* __restrict__ C,
                                                             int splits, int64_t slice_stride,
                                                             int64_t ldc, int nx, int ny,
                                                             float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nx * ny) return;
  const int64_t y = t / nx;
  const int x = (int)(t - y * nx);
  const float* p = C + y * ldc + x;
  float s = p[0];
  for (int z = 1; z < splits; ++z) s += p[(int64_t)z * slice_stride];
  out[t] = s;
}

// G copied into a zero-padded [rows_pad][cols_pad] grid.
__global__ __launch_bounds__(256) void sep_pad_kernel(const float* __restrict__ g, int nx, int ny,
                                                      int cols_pad, int64_t total,
                                                      float* __restrict__ gp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int64_t y = t / cols_pad;
  const int x = (int)(t - y * cols_pad);
  gp[t] = (x < nx && y < ny) ? g[y * nx + x] : 0.0f;
}

// Per point j: sums its fold planes (x part: s0 -> Sc, s1 -> Sx, s2 -> Sr;
// y part: s1 -> Sy, s2 -> Sr) in FP64 and scales them into the gradients.
// kFinSlices threads per point (threadIdx.y) each add the planes slice,
// slice + kFinSlices, ... in increasing order; the slice sums are then added
// in slice order (a fixed tree: bitwise reproducible).
__global__ __launch_bounds__(kWave* kFinSlices) void sep_finalize_kernel(
    const float4* __restrict__ fold_x, int planes_x, const float4* __restrict__ fold_y,
    int planes_y, int64_t npad, int64_t n, const float* __restrict__ z,
    const float* __restrict__ a, double pitch, double wavelength, float* __restrict__ gx,
    float* __restrict__ gy, float* __restrict__ gz, float* __restrict__ ga) {
  __shared__ double part[kFinSlices][5][kWave];
  const int lane = threadIdx.x, slice = threadIdx.y;
  const int64_t j = (int64_t)blockIdx.x * kWave + lane;
  double Sc = 0.0, Sx = 0.0, Srx = 0.0, Sy = 0.0, Sry = 0.0;
  if (j < npad) {
    // Planes slice, slice + kFinSlices, ... in increasing order; the loads of
    // kFinBatch planes are issued together, then added in order.
    constexpr int kFinBatch = 4;
    int k = slice;
    for (; k + (kFinBatch - 1) * kFinSlices < planes_x; k += kFinBatch * kFinSlices) {
      float4 v[kFinBatch];
#pragma unroll
      for (int q = 0; q < kFinBatch; ++q) v[q] = fold_x[(int64_t)(k + q * kFinSlices) * npad + j];
#pragma unroll
      for (int q = 0; q < kFinBatch; ++q) {
        Sc += (double)v[q].x;
        Sx += (double)v[q].y;
        Srx += (double)v[q].z;
      }
    }
    for (; k < planes_x; k += kFinSlices) {
      const float4 v = fold_x[(int64_t)k * npad + j];
      Sc += (double)v.x;
      Sx += (double)v.y;
      Srx += (double)v.z;
    }
    k = slice;
    for (; k + (kFinBatch - 1) * kFinSlices < planes_y; k += kFinBatch * kFinSlices) {
      float4 v[kFinBatch];
#pragma unroll
      for (int q = 0; q < kFinBatch; ++q) v[q] = fold_y[(int64_t)(k + q * kFinSlices) * npad + j];
#pragma unroll
      for (int q = 0; q < kFinBatch; ++q) {
        Sy += (double)v[q].y;
        Sry += (double)v[q].z;
      }
    }
    for (; k < planes_y; k += kFinSlices) {
      const float4 v = fold_y[(int64_t)k * npad + j];
      Sy += (double)v.y;
      Sry += (double)v.z;
    }
  }
  part[slice][0][lane] = Sc;
  part[slice][1][lane] = Sx;
  part[slice][2][lane] = Srx;
  part[slice][3][lane] = Sy;
  part[slice][4][lane] = Sry;
  __syncthreads();
  if (slice != 0 || j >= n) return;
  Sc = Sx = Srx = Sy = Sry = 0.0;
  for (int k = 0; k < kFinSlices; ++k) {
    Sc += part[k][0][lane];
    Sx += part[k][1][lane];
    Srx += part[k][2][lane];
    Sy += part[k][3][lane];
    Sry += part[k][4][lane];
  }
  const double Sr = Srx + Sry;
  const double zj = (double)z[j], aj = (double)a[j];
  // P_j = pi p^2 / (lambda z_j), Section 1.
  const double P = M_PI * pitch * pitch / (wavelength * zj);
  ga[j] = (float)Sc;
  gx[j] = (float)(2.0 * aj * P * Sx);
  gy[j] = (float)(2.0 * aj * P * Sy);
  gz[j] = (float)(aj * P / zj * Sr);
}

}  // namespace

dim3 table_grid(int64_t npad, int rows) {
  // About 1024 workgroups: enough to fill the chip, few enough that each
  // thread reuses its point's records over many rows.
  const unsigned bx = grid_blocks(npad, 256);
  unsigned gy = bx >= 1024 ? 1 : 1024 / bx;
  if (gy > (unsigned)rows) gy = (unsigned)rows;
  return dim3(bx, gy);
}

hipError_t launch_sep_tables(const float* xrec, const float* yrec, const float* amp, int64_t npad,
                             int nx, int nxp, int ny, int nyp, float* tab_x, float* tab_y,
                             hipStream_t s) {
  const dim3 grid = table_grid(npad, nxp + nyp);
  hipLaunchKernelGGL(sep_table_kernel, grid, dim3(256), 0, s, xrec, yrec, amp, npad, nx, nxp, ny,
                     nyp, (float2*)tab_x, (float2*)tab_y);
  return hipGetLastError();
}

hipError_t launch_sep_sum_slices(const float* C, int splits, int64_t slice_stride, int64_t ldc,
                                 int nx, int ny, float* out, hipStream_t s) {
  const unsigned blocks = grid_blocks((int64_t)nx * ny, 256);
  if (!blocks) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sep_sum_slices_kernel, dim3(blocks), dim3(256), 0, s, C, splits, slice_stride,
                     ldc, nx, ny, out);
  return hipGetLastError();
}

hipError_t launch_sep_pad(const float* g, int nx, int ny, int rows_pad, int cols_pad, float* gp,
                          hipStream_t s) {
  const int64_t total = (int64_t)rows_pad * cols_pad;
  const unsigned blocks = grid_blocks(total, 256);
  if (!blocks) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sep_pad_kernel, dim3(blocks), dim3(256), 0, s, g, nx, ny,
                     cols_pad, total, gp);
  return hipGetLastError();
}

hipError_t launch_sep_finalize(const Plan& p, const Workspace& w, const float* z, const float* a,
                               double pitch, double wavelength, float* gx, float* gy, float* gz,
                               float* ga, hipStream_t s) {
  const int planes_x = p.sep_splits_u * (p.nxp / 128);
  const int planes_y = p.sep_splits_p * (p.nyp / 128);
  hipLaunchKernelGGL(sep_finalize_kernel, dim3(grid_blocks(p.n, kWave)), dim3(kWave, kFinSlices),
                     0, s,
                     (const float4*)w.fold_x, planes_x, (const float4*)w.fold_y, planes_y, p.npad,
                     p.n, z, a, pitch, wavelength, gx, gy, gz, ga);
  return hipGetLastError();
}

}  // namespace cgh
