// Forward kernels: the direct point-source sum of Eq. (1) (Section 1).
//
// Work mapping: one hologram column per lane.  The plain and compensated FP32
// kernels give lane l of a wave column x0 + l and a few consecutive rows, so a
// wave writes fully coalesced 256-byte row segments, and every point record
// is read once per wave through scalar loads (the loop index is
// wave-uniform), i.e. broadcast to all 64 lanes from SGPRs.  Points are
// unrolled a group at a time so the scalar loads of the next points are in
// flight while the current ones are used.  The recurrence kernel gives a lane
// K consecutive columns of R rows instead (Eq. (2) steps along x), and the
// FP64 reference one pixel per lane.
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
  const unsigned tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int bx = (int)(tile % gridDim.x), by = (int)(tile / gridDim.x);
  const int col = bx * kWave + lane;
  const int y0 = (by * kFwdWaves + wave) * kRows;
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

// Recurrence FP32, Eq. (2) (Section 2.1): along a row the phase of pixel
// x_h + n follows from two additions, Gamma_n = Gamma_{n-1} + delta_{n-1} and
// delta_n = delta_{n-1} + Delta, from Gamma_0 = P r^2 at x_h,
// delta_0 = P (2 (x_h - x_j) + 1) and Delta = 2 P (here in revolutions, P ->
// Prev).  Lane l covers the K consecutive pixels x0 + K l ... x0 + K l + K - 1
// of R rows (the paper's work-item covers eight consecutive pixels of one
// row).  delta and Delta depend on the column only, so the lane's R rows
// share them: per point the lane forms dx, delta_0 and Delta once and
// Gamma_0 = fract(Prev r^2) (the plain phase) once per row, and per
// interaction the recurrence costs one add for Gamma (plus 1/R of an add for
// delta) before the native cosine and the accumulate.  Gamma_0 is in [0, 1)
// and delta_0, Delta are reduced mod 1 (exactly; cos is 1-periodic in
// revolutions), so |Gamma_n| < 1 + n (1 + n) stays well inside the cosine's
// exact-reduction range without a fract per step.  Points are read four at a
// time through scalar loads (the paper unrolls four points per iteration),
// one group ahead of their use.
//
// S > 1 splits the points of a workgroup's pixels over S groups of kRecWaves
// waves (point subset s = [s npad / S, (s + 1) npad / S)): more waves per SIMD
// for the same pixels, when the hologram is too small to give every SIMD
// several.  Groups 1 .. S-1 leave their sums in LDS and group 0 adds them in
// group order and stores (deterministic).
template <int K, int R, int S>
__global__ __launch_bounds__(kRecThreads * S) void fwd_rec_kernel(const float4* __restrict__ rec,
                                                                  int npad, int nx, int ny,
                                                                  float* __restrict__ out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave_all = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int wave = wave_all % kRecWaves;  // rows
  const int part = wave_all / kRecWaves;  // point subset
  // Row blocks run along the grid's x dimension (up to 2^20 / 4 of them),
  // column blocks along y.
  const unsigned tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int by = (int)(tile % gridDim.x), bx = (int)(tile / gridDim.x);
  const int x0 = (bx * kWave + lane) * K;
  const int y0 = (by * kRecWaves + wave) * R;
  const float xh = (float)x0;
  float acc[R][K];
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int n = 0; n < K; ++n) acc[i][n] = 0.0f;

  auto point = [&](const float4& r) {
    const float dx = xh - r.x;
    const float dx2 = dx * dx;
    float d = fract(r.z * __builtin_fmaf(2.0f, dx, 1.0f));
    const float D = fract(r.z + r.z);
    float g[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const float dy = (float)(y0 + i) - r.y;
      g[i] = fract(r.z * __builtin_fmaf(dy, dy, dx2));
    }
#pragma unroll
    for (int n = 0; n < K; ++n) {
#pragma unroll
      for (int i = 0; i < R; ++i) acc[i][n] = __builtin_fmaf(r.w, cos_rev(g[i]), acc[i][n]);
      if (n + 1 < K) {
#pragma unroll
        for (int i = 0; i < R; ++i) g[i] += d;
        d += D;
      }
    }
  };
  // Two ping-pong groups of records in SGPRs; the next group's loads are
  // issued after the first point of the current one (whose use waits for
  // every outstanding scalar load), so the other points cover their latency.
  // The last group of the subset re-reads itself (in bounds).
  auto load = [&](int j, float4* dst) {
#pragma unroll
    for (int u = 0; u < kRecUnroll; ++u) dst[u] = rec[j + u];
  };
  auto group = [&](int j, const float4* cur, float4* nxt, int jend) {
    point(cur[0]);
    __builtin_amdgcn_sched_barrier(0);
    load(min(j + kRecUnroll, jend - kRecUnroll), nxt);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 1; u < kRecUnroll; ++u) point(cur[u]);
  };
  const int jbeg = part * (npad / S), jend = jbeg + npad / S;
  float4 A[kRecUnroll], B[kRecUnroll];
  load(jbeg, A);
  for (int j = jbeg; j < jend; j += 2 * kRecUnroll) {
    group(j, A, B, jend);
    group(j + kRecUnroll, B, A, jend);
  }
  if constexpr (S > 1) {
    // [subset - 1][element][thread of the group]: consecutive lanes hit
    // consecutive words.
    constexpr int kGroupThreads = kRecThreads;
    __shared__ float part_sums[(S - 1) * R * K * kGroupThreads];
    const int t = wave * kWave + lane;
    if (part > 0) {
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int n = 0; n < K; ++n)
          part_sums[((part - 1) * R * K + i * K + n) * kGroupThreads + t] = acc[i][n];
    }
    __syncthreads();
    if (part > 0) return;
#pragma unroll
    for (int q = 1; q < S; ++q)
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int n = 0; n < K; ++n)
          acc[i][n] += part_sums[((q - 1) * R * K + i * K + n) * kGroupThreads + t];
  }
#pragma unroll
  for (int i = 0; i < R; ++i) {
    if (y0 + i >= ny) continue;
    float* row = out + (int64_t)(y0 + i) * nx;
#pragma unroll
    for (int n = 0; n < K; ++n)
      if (x0 + n < nx) row[x0 + n] = acc[i][n];
  }
}

// Compensated FP32: the phase separates exactly as X_j(x_h) + Y_j(y_h) with
// X_j(x_h) = Prev (x_h - x_j)^2 and Y_j(y_h) = Prev (y_h - y_j)^2.  Each part
// is formed on the integer pixel grid as a compensated split product reduced
// mod 1 (axis_phase).  Lane l of a wave owns column col0 + l and the wave
// kCompRows rows; the kCompWaves waves of a workgroup share their 64
// columns.  Per tile of kTile points the workgroup stages in LDS the x-phases
// [point][column] (from the column table xtab[col][npad] with TAB, else
// formed from each point's record: the same bits), each wave's row phases
// [point] (one float4 of the row table: its kCompRows rows) and the
// amplitudes.  The inner loop reads X per lane and Y and A as broadcast LDS
// reads (every lane the same address), so every operand of the per-
// interaction add, cosine and fma is a VGPR: on gfx950 such FP32 instructions
// issue about 1.7 times as fast as ones reading an SGPR, and without SGPR
// buffers the kernel fits eight waves per SIMD.  The tile is single-buffered
// (25 KB of LDS): the next tile's values are loaded into registers while the
// current one is consumed and stored between two barriers.  Per interaction:
// one add, the native cosine (no fract: the sum stays within a few
// revolutions) and one fma.
template <bool TAB, bool RES>
__device__ __forceinline__ void fwd_comp_body(const float* __restrict__ xrec,
                                                  const float* __restrict__ xtab,
                                                  const float* __restrict__ amp,
                                                  const float* __restrict__ ytab, int npad,
                                                  int nx, int ny, float* __restrict__ out,
                                                  const float* __restrict__ tgt,
                                                  float* __restrict__ res) {
  static_assert(kCompRows == 4, "a wave's row phases of one point are one float4");
  __shared__ float xs[kTile * kTilePitch];
  __shared__ float4 ys[kCompWaves][kTile];
  __shared__ float4 as4[kTile / 4];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  // Tiles in column-major order, so each XCD takes a band of columns: it
  // reads only its columns' share of the column table (the larger table),
  // and all of the row table.
  const unsigned tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int by = (int)(tile % gridDim.y), bx = (int)(tile / gridDim.y);
  const int col = bx * kWave + lane;
  const int col0 = bx * kWave;
  const int grp = by * kCompWaves + wave;
  const float4* __restrict__ yt = reinterpret_cast<const float4*>(ytab) + (int64_t)grp * npad;
  const int ntiles = npad / kTile;
  constexpr int kColsPerWave = kWave / kCompWaves;
  const __amdgpu_buffer_rsrc_t xtab_rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(xtab), 0, TAB ? (int)((int64_t)gridDim.x * kWave * npad * 4) : 0,
      0x00020000);

  // Registers holding the next tile: lane l of wave w has point l's x-phases
  // of the wave's kColsPerWave columns (or its record), its row phases, and
  // (wave 0) its amplitude.
  float xv[kColsPerWave];
  float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), yv;
  float r1 = 0.f, av = 0.f;
  auto load_tile = [&](int t) {
    const int j = t * kTile + lane;
    if (TAB) {
#pragma unroll
      for (int k = 0; k < kColsPerWave; ++k) {
        const int c = col0 + wave * kColsPerWave + k;
        xv[k] = __builtin_bit_cast(
            float, __builtin_amdgcn_raw_buffer_load_b32(
                       xtab_rsrc, (unsigned)lane * 4u,
                       (int)(((int64_t)c * npad + (int64_t)t * kTile) * 4), 0));
      }
    } else {
      const float* r = xrec + (int64_t)j * kAxisRec;
      r0 = *reinterpret_cast<const float4*>(r);
      r1 = r[4];
    }
    yv = yt[j];
    if (wave == 0) av = amp[j];
  };
  auto store_tile = [&]() {
#pragma unroll
    for (int k = 0; k < kColsPerWave; ++k) {
      const int c = wave * kColsPerWave + k;
      xs[lane * kTilePitch + c] =
          TAB ? xv[k] : axis_phase((float)(col0 + c), r0.x, r0.y, r0.z, r0.w, r1);
    }
    ys[wave][lane] = yv;
    if (wave == 0) reinterpret_cast<float*>(as4)[lane] = av;
  };

  float acc[kCompRows];
#pragma unroll
  for (int i = 0; i < kCompRows; ++i) acc[i] = 0.0f;
  load_tile(0);
  priority_start();
  for (int t = 0; t < ntiles; ++t) {
    priority_step(t, ntiles);
    if (t > 0) __syncthreads();  // every wave is done with the previous tile
    store_tile();
    __syncthreads();
    if (t + 1 < ntiles) load_tile(t + 1);
#pragma unroll 2
    for (int p = 0; p < kTile; p += 8) {
#pragma unroll
      for (int q = 0; q < 8; q += 4) {
        const float4 a4 = as4[(p + q) / 4];
        const float A[4] = {a4.x, a4.y, a4.z, a4.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float X = xs[(p + q + u) * kTilePitch + lane];
          const float4 y4 = ys[wave][p + q + u];
          acc[0] = __builtin_fmaf(A[u], cos_rev(X + y4.x), acc[0]);
          acc[1] = __builtin_fmaf(A[u], cos_rev(X + y4.y), acc[1]);
          acc[2] = __builtin_fmaf(A[u], cos_rev(X + y4.z), acc[2]);
          acc[3] = __builtin_fmaf(A[u], cos_rev(X + y4.w), acc[3]);
        }
      }
    }
  }
  // The hologram, and in the RES instances the residual I - T (the upstream
  // gradient of 0.5 ||I - T||^2) in the same pass.  The two instances keep
  // the forward without a target at its own code: with the residual store
  // behind a run-time test, the same kernel ran about 1% slower at N >= 8192.
  const int y0 = grp * kCompRows;
  if (col < nx) {
#pragma unroll
    for (int i = 0; i < kCompRows; ++i) {
      if (y0 + i >= ny) continue;
      const int64_t idx = (int64_t)(y0 + i) * nx + col;
      out[idx] = acc[i];
      if constexpr (RES) res[idx] = acc[i] - tgt[idx];
    }
  }
}

__global__ __launch_bounds__(kCompThreads) void fwd_comp_kernel(
    const float* __restrict__ xtab, const float* __restrict__ amp, const float* __restrict__ ytab,
    int npad, int nx, int ny, float* __restrict__ out) {
  fwd_comp_body<true, false>(nullptr, xtab, amp, ytab, npad, nx, ny, out, nullptr, nullptr);
}

__global__ __launch_bounds__(kCompThreads) void fwd_comp_residual_kernel(
    const float* __restrict__ xtab, const float* __restrict__ amp, const float* __restrict__ ytab,
    int npad, int nx, int ny, float* __restrict__ out, const float* __restrict__ tgt,
    float* __restrict__ res) {
  fwd_comp_body<true, true>(nullptr, xtab, amp, ytab, npad, nx, ny, out, tgt, res);
}

__global__ __launch_bounds__(kCompThreads) void fwd_comp_inline_kernel(
    const float* __restrict__ xrec, const float* __restrict__ amp, const float* __restrict__ ytab,
    int npad, int nx, int ny, float* __restrict__ out) {
  fwd_comp_body<false, false>(xrec, nullptr, amp, ytab, npad, nx, ny, out, nullptr, nullptr);
}

__global__ __launch_bounds__(kCompThreads) void fwd_comp_inline_residual_kernel(
    const float* __restrict__ xrec, const float* __restrict__ amp, const float* __restrict__ ytab,
    int npad, int nx, int ny, float* __restrict__ out, const float* __restrict__ tgt,
    float* __restrict__ res) {
  fwd_comp_body<false, true>(xrec, nullptr, amp, ytab, npad, nx, ny, out, tgt, res);
}

// The residual G = I - T of a finished hologram, for the forwards without a
// fused one.
__global__ __launch_bounds__(256) void residual_kernel(const float* __restrict__ I,
                                                       const float* __restrict__ T,
                                                       float* __restrict__ G, int64_t count) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) G[t] = I[t] - T[t];
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

namespace {

template <int K, int R>
hipError_t launch_rec(const Plan& p, const Workspace& w, float* out, hipStream_t s) {
  if (p.rec_s == 2)
    hipLaunchKernelGGL((fwd_rec_kernel<K, R, 2>), dim3(p.rec_gy, p.rec_gx), dim3(kRecThreads * 2),
                       0, s, (const float4*)w.plain, (int)p.npad, p.nx, p.ny, out);
  else
    hipLaunchKernelGGL((fwd_rec_kernel<K, R, 1>), dim3(p.rec_gy, p.rec_gx), dim3(kRecThreads), 0,
                       s, (const float4*)w.plain, (int)p.npad, p.nx, p.ny, out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fwd_rec(const Plan& p, const Workspace& w, float* out, hipStream_t s) {
  switch (p.rec_k * 10 + p.rec_r) {
    case 41: return launch_rec<4, 1>(p, w, out, s);
    case 42: return launch_rec<4, 2>(p, w, out, s);
    case 44: return launch_rec<4, 4>(p, w, out, s);
    case 61: return launch_rec<6, 1>(p, w, out, s);
    case 62: return launch_rec<6, 2>(p, w, out, s);
    case 64: return launch_rec<6, 4>(p, w, out, s);
    case 81: return launch_rec<8, 1>(p, w, out, s);
    case 82: return launch_rec<8, 2>(p, w, out, s);
    case 84: return launch_rec<8, 4>(p, w, out, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fwd_comp(const Plan& p, const Workspace& w, float* out, hipStream_t s,
                           const float* target, float* residual) {
  if ((target == nullptr) != (residual == nullptr)) return hipErrorInvalidValue;
  const dim3 grid(p.fwd_gx, p.comp_gy), block(kCompThreads);
  const float *xtab = w.xtab, *xrec = w.xrec, *amp = w.amp, *ytab = w.ytab;
  const int npad = (int)p.npad;
  if (w.xtab && residual)
    hipLaunchKernelGGL(fwd_comp_residual_kernel, grid, block, 0, s, xtab, amp, ytab, npad, p.nx,
                       p.ny, out, target, residual);
  else if (w.xtab)
    hipLaunchKernelGGL(fwd_comp_kernel, grid, block, 0, s, xtab, amp, ytab, npad, p.nx, p.ny,
                       out);
  else if (residual)
    hipLaunchKernelGGL(fwd_comp_inline_residual_kernel, grid, block, 0, s, xrec, amp, ytab, npad,
                       p.nx, p.ny, out, target, residual);
  else
    hipLaunchKernelGGL(fwd_comp_inline_kernel, grid, block, 0, s, xrec, amp, ytab, npad, p.nx,
                       p.ny, out);
  return hipGetLastError();
}

hipError_t launch_residual(const float* hologram, const float* target, float* residual,
                           int64_t count, hipStream_t s) {
  const unsigned blocks = grid_blocks(count, 256);
  if (!blocks) return hipErrorInvalidValue;
  hipLaunchKernelGGL(residual_kernel, dim3(blocks), dim3(256), 0, s, hologram, target, residual,
                     count);
  return hipGetLastError();
}

hipError_t launch_fwd_f64(const Plan& p, const Workspace& w, double* out, hipStream_t s) {
  const int64_t npix = (int64_t)p.nx * p.ny;
  const unsigned blocks = grid_blocks(npix, 256);
  if (!blocks) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fwd_f64_kernel, dim3(blocks), dim3(256), 0, s,
                     (const double4*)w.rec64, (int)p.npad, p.nx, npix, out);
  return hipGetLastError();
}

}  // namespace cgh
