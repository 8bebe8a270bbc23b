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
// This changes the algorithm (no per-interaction cosine): the per-point
// tables cost O(N (nx + ny)) transcendentals and the bulk is FP32 MFMA work.
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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One workgroup (4 waves) per point: waves 0-1 fold the x part (columns
// h = 64 k + lane, k even / odd), waves 2-3 the y part (rows, likewise).  Each
// wave adds its terms in FP64 in a fixed lane-strided order and reduces them
// with a butterfly; the workgroup then combines the four wave sums in a fixed
// order and scales them into the gradients.
__global__ __launch_bounds__(256) void sep_fold_kernel(
    const float* __restrict__ xrec, const float* __restrict__ yrec, const float* __restrict__ Uc,
    int su, int64_t u_stride, int64_t ldu, const float* __restrict__ Pc, int sp,
    int64_t p_stride, int64_t ldp, int64_t n, int nx, int ny, const float* __restrict__ x,
    const float* __restrict__ y, const float* __restrict__ z, const float* __restrict__ a,
    double pitch, double wavelength, float* __restrict__ gx, float* __restrict__ gy,
    float* __restrict__ gz, float* __restrict__ ga) {
  __shared__ double part[4][3];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t j = blockIdx.x;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (wave < 2) {
    // x part: Sc, Sx, Sr_x
    const float* rx = xrec + j * kAxisRec;
    const double xj = (double)x[j];
    const float* urow = Uc + (2 * j) * ldu;
    for (int h = lane + 64 * wave; h < nx; h += 128) {
      float U = 0.0f, V = 0.0f;
      for (int s = 0; s < su; ++s) {
        U += urow[s * u_stride + h];
        V += urow[s * u_stride + ldu + h];
      }
      const float phi = axis_phase((float)h, rx[0], rx[1], rx[2], rx[3], rx[4]);
      const double c = cos_rev(phi), sn = sin_rev(phi);
      s0 += c * U - sn * V;
      const double sg = sn * U + c * V;
      const double dx = (double)h - xj;
      s1 += dx * sg;
      s2 += dx * dx * sg;
    }
  } else {
    // y part: Sy, Sr_y
    const float* ry = yrec + j * kAxisRec;
    const double yj = (double)y[j];
    const float* prow = Pc + (2 * j) * ldp;
    for (int h = lane + 64 * (wave - 2); h < ny; h += 128) {
      float Pcos = 0.0f, Psin = 0.0f;
      for (int s = 0; s < sp; ++s) {
        Pcos += prow[s * p_stride + h];
        Psin += prow[s * p_stride + ldp + h];
      }
      const float phi = axis_phase((float)h, ry[0], ry[1], ry[2], ry[3], ry[4]);
      const double c = cos_rev(phi), sn = sin_rev(phi);
      const double sr = c * Psin + sn * Pcos;
      const double dy = (double)h - yj;
      s1 += dy * sr;
      s2 += dy * dy * sr;
    }
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (lane == 0) {
    part[wave][0] = s0;
    part[wave][1] = s1;
    part[wave][2] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double Sc = part[0][0] + part[1][0];
    const double Sx = part[0][1] + part[1][1];
    const double Sy = part[2][1] + part[3][1];
    const double Sr = (part[0][2] + part[1][2]) + (part[2][2] + part[3][2]);
    const double zj = (double)z[j], aj = (double)a[j];
    // P_j = pi p^2 / (lambda z_j), Section 1.
    const double P = M_PI * pitch * pitch / (wavelength * zj);
    ga[j] = (float)Sc;
    gx[j] = (float)(2.0 * aj * P * Sx);
    gy[j] = (float)(2.0 * aj * P * Sy);
    gz[j] = (float)(aj * P / zj * Sr);
  }
}

inline unsigned blocks_for(int64_t count, int threads) {
  return (unsigned)((count + threads - 1) / threads);
}

}  // namespace

dim3 table_grid(int64_t npad, int rows) {
  // About 1024 workgroups: enough to fill the chip, few enough that each
  // thread reuses its point's records over many rows.
  const unsigned bx = blocks_for(npad, 256);
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
  hipLaunchKernelGGL(sep_sum_slices_kernel, dim3(blocks_for((int64_t)nx * ny, 256)), dim3(256), 0,
                     s, C, splits, slice_stride, ldc, nx, ny, out);
  return hipGetLastError();
}

hipError_t launch_sep_pad(const float* g, int nx, int ny, int rows_pad, int cols_pad, float* gp,
                          hipStream_t s) {
  const int64_t total = (int64_t)rows_pad * cols_pad;
  hipLaunchKernelGGL(sep_pad_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, g, nx, ny,
                     cols_pad, total, gp);
  return hipGetLastError();
}

hipError_t launch_sep_fold(const Plan& p, const Workspace& w, const float* U, int su,
                           int64_t u_stride, int64_t ldu, const float* Pm, int sp, int64_t p_stride,
                           int64_t ldp, const float* x, const float* y, const float* z,
                           const float* a, double pitch, double wavelength, float* gx, float* gy,
                           float* gz, float* ga, hipStream_t s) {
  hipLaunchKernelGGL(sep_fold_kernel, dim3((unsigned)p.n), dim3(256), 0, s,
                     (const float*)w.xrec, (const float*)w.yrec, U, su, u_stride, ldu, Pm, sp,
                     p_stride, ldp, p.n, p.nx, p.ny, x, y, z, a, pitch, wavelength, gx, gy, gz,
                     ga);
  return hipGetLastError();
}

}  // namespace cgh
