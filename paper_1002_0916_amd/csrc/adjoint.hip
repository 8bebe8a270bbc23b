// Adjoint kernels: gradients of a loss through Eq. (1) (Section 1).
//
// For theta = P_j r^2 (the chain rule on Eq. (1)) every point j needs four
// sums over all pixels h of the upstream gradient G = dL/dI:
//   Sc = sum G cos(theta)        Sx = sum G sin(theta) (x_h - x_j)
//   Sr = sum G sin(theta) r^2    Sy = sum G sin(theta) (y_h - y_j)
//
// Work mapping: the transpose of the forward.  Lane = point, so each of the
// four per-point reductions over pixels runs inside one lane and no
// cross-lane reduction is needed at all.  A wave takes 64 points and a region
// of 16 x 16 pixel blocks; G is wave-uniform and reaches the lanes through
// scalar loads (one s_load_dwordx16 per block row).  Within a block the
// pixel-dependent factors separate by axis: r^2 = dx^2 + dy^2, so the lane
// accumulates the column sums and row sums of g_s = G sin(theta) and folds
// them with dx_c, dx_c^2, dy_r, dy_r^2 once per block, leaving per
// interaction: the phase, sin and cos, and four accumulations.
//
// Second pass: one thread per point adds the region partials in region
// order (fixed, so the result is bitwise reproducible) in FP64 and applies
// the per-point factors 2 A_j P_j and A_j P_j / z_j.
#include "cgh_internal.h"
#include "phase.h"

namespace cgh {

namespace {

template <int VARIANT>
__global__ __launch_bounds__(kAdjThreads) void adj_partial_kernel(
    const float4* __restrict__ plain, const float* __restrict__ xrec,
    const float* __restrict__ yrec, const float* __restrict__ g, int64_t ldg, int nbx,
    int nblocks, int bpr, int npad, float4* __restrict__ partial) {
  const int region = blockIdx.x;
  const int j = blockIdx.y * kWave + threadIdx.x;

  // Per-lane point data.
  float px, py, prev;
  float xc = 0.f, xph = 0.f, xpl = 0.f, xb = 0.f, xd = 0.f;
  float yc = 0.f, yph = 0.f, ypl = 0.f, yb = 0.f, yd = 0.f;
  {
    const float4 r = plain[j];
    px = r.x;
    py = r.y;
    prev = r.z;
    if (VARIANT == 1) {
      const float* rx = xrec + (int64_t)j * kAxisRec;
      const float* ry = yrec + (int64_t)j * kAxisRec;
      xc = rx[0]; xph = rx[1]; xpl = rx[2]; xb = rx[3]; xd = rx[4];
      yc = ry[0]; yph = ry[1]; ypl = ry[2]; yb = ry[3]; yd = ry[4];
    }
  }

  float Sc = 0.f, Sx = 0.f, Sy = 0.f, Sr = 0.f;
  const int b0 = region * bpr;
  const int b1 = min(b0 + bpr, nblocks);
  for (int b = b0; b < b1; ++b) {
    const int by = b / nbx;
    const int bx = b - by * nbx;
    const float x0 = (float)(bx * kBlk);
    const float y0 = (float)(by * kBlk);
    // Column terms (per lane): compensated x-phase, or dx for the plain form.
    float CX[kBlk], RY[kBlk];
#pragma unroll
    for (int c = 0; c < kBlk; ++c) {
      const float h = x0 + (float)c;
      CX[c] = VARIANT == 1 ? axis_phase(h, xc, xph, xpl, xb, xd) : h - px;
    }
#pragma unroll
    for (int r = 0; r < kBlk; ++r) {
      const float h = y0 + (float)r;
      if (VARIANT == 1) {
        RY[r] = axis_phase(h, yc, yph, ypl, yb, yd);
      } else {
        const float dy = h - py;
        RY[r] = dy * dy;
      }
    }
    float SgC[kBlk], SgR[kBlk];
#pragma unroll
    for (int c = 0; c < kBlk; ++c) SgC[c] = 0.f;
    const float* __restrict__ gb = g + (int64_t)(by * kBlk) * ldg + bx * kBlk;
#pragma unroll
    for (int r = 0; r < kBlk; ++r) {
      const float* __restrict__ gr = gb + (int64_t)r * ldg;
      float sr = 0.f;
#pragma unroll
      for (int c = 0; c < kBlk; ++c) {
        const float G = gr[c];
        float t;
        if (VARIANT == 1) {
          t = CX[c] + RY[r];
        } else {
          t = fract(prev * __builtin_fmaf(CX[c], CX[c], RY[r]));
        }
        const float s = sin_rev(t);
        const float co = cos_rev(t);
        Sc = __builtin_fmaf(G, co, Sc);
        const float gs = G * s;
        SgC[c] += gs;
        sr += gs;
      }
      SgR[r] = sr;
    }
#pragma unroll
    for (int c = 0; c < kBlk; ++c) {
      const float dx = (x0 + (float)c) - px;
      Sx = __builtin_fmaf(dx, SgC[c], Sx);
      Sr = __builtin_fmaf(dx * dx, SgC[c], Sr);
    }
#pragma unroll
    for (int r = 0; r < kBlk; ++r) {
      const float dy = (y0 + (float)r) - py;
      Sy = __builtin_fmaf(dy, SgR[r], Sy);
      Sr = __builtin_fmaf(dy * dy, SgR[r], Sr);
    }
  }
  partial[(int64_t)region * npad + j] = make_float4(Sc, Sx, Sy, Sr);
}

__global__ __launch_bounds__(256) void adj_finalize_kernel(
    const float4* __restrict__ partial, int regions, int64_t npad, int64_t n,
    const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ z,
    const float* __restrict__ a, double pitch, double wavelength, float* __restrict__ gx,
    float* __restrict__ gy, float* __restrict__ gz, float* __restrict__ ga) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double Sc = 0.0, Sx = 0.0, Sy = 0.0, Sr = 0.0;
  for (int r = 0; r < regions; ++r) {
    const float4 v = partial[(int64_t)r * npad + j];
    Sc += (double)v.x;
    Sx += (double)v.y;
    Sy += (double)v.z;
    Sr += (double)v.w;
  }
  const double zj = (double)z[j];
  const double aj = (double)a[j];
  // P_j = pi p^2 / (lambda z_j), Section 1.
  const double P = M_PI * pitch * pitch / (wavelength * zj);
  ga[j] = (float)Sc;
  gx[j] = (float)(2.0 * aj * P * Sx);
  gy[j] = (float)(2.0 * aj * P * Sy);
  gz[j] = (float)(aj * P / zj * Sr);
}

__global__ __launch_bounds__(256) void pad_g_kernel(const float* __restrict__ g, int nx, int ny,
                                                    int ldp, int64_t total,
                                                    float* __restrict__ gpad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int64_t yy = t / ldp;
  const int xx = (int)(t - yy * ldp);
  gpad[t] = (xx < nx && yy < ny) ? g[yy * nx + xx] : 0.0f;
}

}  // namespace

hipError_t launch_pad_g(const Plan& p, const float* g, float* gpad, hipStream_t s) {
  const int ldp = p.nbx * kBlk;
  const int64_t total = (int64_t)ldp * p.nby * kBlk;
  hipLaunchKernelGGL(pad_g_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, g,
                     p.nx, p.ny, ldp, total, gpad);
  return hipGetLastError();
}

hipError_t launch_adj_partial(const Plan& p, const Workspace& w, const float* g, int64_t ldg,
                              hipStream_t s) {
  const dim3 grid(p.regions, p.ngroups);
  const int nblocks = p.nbx * p.nby;
  if (p.variant == 1) {
    hipLaunchKernelGGL(adj_partial_kernel<1>, grid, dim3(kAdjThreads), 0, s,
                       (const float4*)w.plain, (const float*)w.xrec, (const float*)w.yrec, g, ldg,
                       p.nbx, nblocks, p.blocks_per_region, (int)p.npad, (float4*)w.partial);
  } else {
    hipLaunchKernelGGL(adj_partial_kernel<0>, grid, dim3(kAdjThreads), 0, s,
                       (const float4*)w.plain, (const float*)w.xrec, (const float*)w.yrec, g, ldg,
                       p.nbx, nblocks, p.blocks_per_region, (int)p.npad, (float4*)w.partial);
  }
  return hipGetLastError();
}

hipError_t launch_adj_finalize(const Plan& p, const Workspace& w, const float* x, const float* y,
                               const float* z, const float* a, double pitch, double wavelength,
                               float* gx, float* gy, float* gz, float* ga, hipStream_t s) {
  hipLaunchKernelGGL(adj_finalize_kernel, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, s,
                     (const float4*)w.partial, p.regions, p.npad, p.n, x, y, z, a, pitch,
                     wavelength, gx, gy, gz, ga);
  return hipGetLastError();
}

}  // namespace cgh
