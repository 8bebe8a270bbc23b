// Adjoint kernels: gradients of a loss through Eq. (1) (Section 1).
//
// For theta = P_j r^2 (the chain rule on Eq. (1)) every point j needs four
// sums over all pixels h of the upstream gradient G = dL/dI:
//   Sc = sum G cos(theta)        Sx = sum G sin(theta) (x_h - x_j)
//   Sr = sum G sin(theta) r^2    Sy = sum G sin(theta) (y_h - y_j)
//
// Work mapping: the transpose of the forward.  Lane = point, so each of the
// four per-point reductions over pixels runs inside one lane and no
// cross-lane reduction is needed at all.  A wave takes 64 points and an equal
// share (a run) of the strip-rows of the hologram, where a strip is kAdjCols
// columns wide; kAdjRounds rounds of resident waves cover everything (in the
// compensated kinds each wave's priority steps down at the quarters of its
// run, so the waves sharing a SIMD finish close together).  G is
// wave-uniform and reaches the lanes through scalar loads, one strip row
// (kAdjCols floats) at a time.  The pixel-dependent factors separate by axis,
// r^2 = dx^2 + dy^2, so per strip the lane keeps the column phases (or dx, or
// the recurrence steps) and the column sums of G sin(theta) in registers, and
// per row it takes the row phase (or dy^2) once and folds the row sum of
// G sin(theta) with dy and dy^2.
// The compensated kinds split the phase by axis, theta = X + Y (the
// compensated column and row phases), and take sin(theta) and cos(theta) from
// the per-axis cosines and sines by the addition theorem,
//   sin(X + Y) = sX cY + cX sY,   cos(X + Y) = cX cY - sX sY,
// an exact identity: per strip the lane keeps cX, sX of its columns, per row
// cY, sY, and per interaction that leaves two products and two fused
// multiply-adds for sin and cos (no transcendental) and three fused
// multiply-adds with G taken straight from an SGPR.  The compensated kind
// reads cY and sY from a row table (one 8-byte load per row and lane) and the
// strip's column phases from a column table (one 4-byte load per column and
// lane per strip segment), both built once per call, instead of forming them
// in every strip.  The plain and recurrence kinds take sin and cos of each
// interaction's phase on the transcendental unit.
//
// Second pass: kAdjFinSlices threads per point add interleaved subsets of
// the region partials in region order, then one thread adds the slice sums in
// slice order (a fixed tree, so the result is bitwise reproducible), in FP64,
// and applies the per-point factors 2 A_j P_j and A_j P_j / z_j.
#include <map>
#include <mutex>
#include <utility>

#include "cgh_internal.h"
#include "phase.h"
#include "records.h"

namespace cgh {

#ifdef CGH_WAVE_TRACE
// Wave trace of a diagnostic build (compiled only with -DCGH_WAVE_TRACE, never
// into the library that build() makes): per wave of the last adjoint launch,
// indexed by its linear workgroup id, the 100 MHz constant clock at its start
// and end, its hardware ids (HW_ID in the low word, XCC_ID in the high word)
// and the shader-clock cycles between start and end.
constexpr unsigned kWaveTraceMax = 65536;
__device__ ulonglong4 g_wave_trace[kWaveTraceMax];
#endif

namespace {

// KIND: kAdjPlain, kAdjCompensated (the rows' cY, sY from the row table,
// column phases from the column table), kAdjCompensatedInline (the same
// values formed here) or kAdjRecurrence.  With the recurrence
// (Eq. (2), Section 2.1) each strip row starts from the plain phase
// Gamma_0 = fract(Prev r^2) at the strip's first column and steps
// Gamma += delta_c, delta_c = Prev (2 (x_c - x_j) + 1) reduced mod 1, the
// same for every row (so the strip keeps delta_c where the plain path keeps
// dx); |Gamma| stays below 1 + kAdjCols revolutions.
template <int KIND>
__global__ __launch_bounds__(kAdjThreads) void adj_partial_kernel(
    const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ z,
    const float* __restrict__ a, int64_t n, double pitch, double wavelength,
    const float* __restrict__ g, int64_t ldg, int ny, int64_t strip_rows, AdjOrder order,
    int npad, const float2* __restrict__ rtab, const float* __restrict__ ctab,
    float4* __restrict__ partial) {
  constexpr bool kComp = KIND == kAdjCompensated || KIND == kAdjCompensatedInline;
#ifdef CGH_WAVE_TRACE
  const unsigned long long trace_t0 = __builtin_amdgcn_s_memrealtime();
  const unsigned long long trace_c0 = __builtin_amdgcn_s_memtime();
#endif
  // Neighbouring runs and all point groups of a run share G and the tables:
  // keep them on one XCD.
  const unsigned tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int run = (int)(tile / gridDim.y);
  const int j = (int)(tile % gridDim.y) * kWave + threadIdx.x;
  const int runs = (int)gridDim.x;
  // Run lengths.  xcd_tile hands each XCD a block of consecutive runs, whose
  // workgroups it dispatches in run order.  When every block holds a whole
  // number of runs per round of resident waves (runs a multiple of
  // kAdjRounds * kXcds), the last 1/kAdjRounds of a block's runs are the
  // last round; those runs are made 2/5 as long as the others (weights 2
  // and 5, the block's total unchanged), and the dispatcher gives the short
  // waves to the slots that free first, which evens out when the SIMDs
  // finish.  Otherwise (few runs of many point groups) a round ends inside a
  // run, and all runs keep one length.  Every run is a range of the
  // strip-row order, [pos(run), pos(run + 1)), and the sums are reduced in
  // run order.
  const int64_t w_short = runs % (kAdjRounds * kXcds) == 0 ? 2 : 5;
  auto weight_before = [&](int r) -> int64_t {
    int64_t acc = 0;
#pragma unroll
    for (int b = 0; b < kXcds; ++b) {
      const int lo = (int)((int64_t)runs * b / kXcds), hi = (int)((int64_t)runs * (b + 1) / kXcds);
      const int t = hi - lo - (hi - lo) / kAdjRounds;  // runs before the last round
      const int upto = min(max(r - lo, 0), hi - lo);
      acc += 5 * (int64_t)min(upto, t) + w_short * (int64_t)max(upto - t, 0);
    }
    return acc;
  };
  const int64_t wsum = weight_before(runs);
  const int64_t q0 = strip_rows * weight_before(run) / wsum;
  const int64_t q1 = strip_rows * weight_before(run + 1) / wsum;

  // This lane's point (j >= n: a zero-amplitude padding point).
  const PointRecord rec = point_record(x, y, z, a, j, n, pitch, wavelength);
  const float px = rec.x, py = rec.y, prev = rec.ph;
  const float xc = rec.xc, xph = rec.ph, xpl = rec.pl, xb = rec.xb, xd = rec.xd;
  const float yc = rec.yc, yph = rec.ph, ypl = rec.pl, yb = rec.yb, yd = rec.yd;

  float Sc0 = 0.f, Sc1 = 0.f, Sx = 0.f, Sy = 0.f, Sr = 0.f;
  // CX: the strip's column terms (compensated kinds: the cosine of the
  // column phase, SX its sine); SgC: column sums of G sin(theta).
  float CX[kAdjCols], SX[kAdjCols], SgC[kAdjCols];
  int col0 = 0, row1 = 0;
  float dx0sq = 0.f;  // recurrence: (x_h - x_j)^2 at the strip's first column

  // G of one strip row lives in SGPRs.  Rows are software-pipelined with two
  // ping-pong buffers: the scalar loads of the next row are issued right
  // after the first use of the current row (which waits for it), so the rest
  // of the row's arithmetic covers their latency.  The last row of a segment
  // re-reads itself, so every load stays in bounds.
  auto load_row = [&](int row, float* dst) {
    const float* src = g + (int64_t)row * ldg + col0;
#pragma unroll
    for (int k = 0; k < kAdjCols; ++k) dst[k] = src[k];
  };
  // The compensated kind's {cY, sY} of a row, from the row table (one 8-byte
  // load per lane, issued a row ahead like G).
  // A buffer load: the row's byte offset (at most kAdjRowTabMaxBytes) is a
  // scalar operand and the lane's offset a 32-bit vector one, so forming the
  // address costs no vector instruction; the descriptor bounds the table.
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  const __amdgpu_buffer_rsrc_t rtab_rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float2*>(rtab), 0, KIND == kAdjCompensated ? (int)((int64_t)ny * npad * 8) : 0,
      0x00020000);
  // The compensated kind's column phases of a strip, from the column table
  // [nsx * kAdjCols][npad] (one 4-byte buffer load per column and lane).
  const __amdgpu_buffer_rsrc_t ctab_rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(ctab), 0,
      KIND == kAdjCompensated ? (int)((int64_t)(strip_rows / ny) * kAdjCols * npad * 4) : 0,
      0x00020000);
  auto load_rtab = [&](int row) {
    const f32x2 v = __builtin_bit_cast(
        f32x2, __builtin_amdgcn_raw_buffer_load_b64(rtab_rsrc, (unsigned)j * 8u,
                                                    (int)((int64_t)row * npad * 8), 0));
    return make_float2(v.x, v.y);
  };
  auto do_row = [&](int row, const float* gc, float* gn, float2 rc, float2& rn) {
    const float dy = (float)row - py;
    const float dy2 = dy * dy;
    // Plain: dy^2; recurrence: the row's starting phase.
    const float RY = KIND == kAdjPlain ? dy2 : 0.f;
    float gam = KIND == kAdjRecurrence ? fract(prev * (dx0sq + dy2)) : 0.f;
    // Compensated kinds: the cosine and sine of the row phase.
    float cY = 0.f, sY = 0.f;
    if (KIND == kAdjCompensated) {
      cY = rc.x;
      sY = rc.y;
    } else if (KIND == kAdjCompensatedInline) {
      const float ry = axis_phase((float)row, yc, yph, ypl, yb, yd);
      cY = cos_rev(ry);
      sY = sin_rev(ry);
    }
    float sr0 = 0.f, sr1 = 0.f;
#pragma unroll
    for (int c = 0; c < kAdjCols; ++c) {
      if (c == 1) {
        __builtin_amdgcn_sched_barrier(0);
        const int next = min(row + 1, row1 - 1);
        load_row(next, gn);
        if (KIND == kAdjCompensated) rn = load_rtab(next);
        __builtin_amdgcn_sched_barrier(0);
      }
      const float G = gc[c];
      float s, co;
      if (kComp) {
        // sin and cos of X + Y by the addition theorem
        s = __builtin_fmaf(SX[c], cY, CX[c] * sY);
        co = __builtin_fmaf(CX[c], cY, -(SX[c] * sY));
      } else {
        float t;
        if (KIND == kAdjRecurrence) {
          t = gam;
          gam += CX[c];
        } else {
          t = fract(prev * __builtin_fmaf(CX[c], CX[c], RY));
        }
        s = sin_rev(t);
        co = cos_rev(t);
      }
      if (c & 1) {
        Sc1 = __builtin_fmaf(G, co, Sc1);
        sr1 = __builtin_fmaf(G, s, sr1);
      } else {
        Sc0 = __builtin_fmaf(G, co, Sc0);
        sr0 = __builtin_fmaf(G, s, sr0);
      }
      SgC[c] = __builtin_fmaf(G, s, SgC[c]);
    }
    const float sr = sr0 + sr1;
    Sy = __builtin_fmaf(dy, sr, Sy);
    Sr = __builtin_fmaf(dy2, sr, Sr);
  };

  // Wave priority by progress (as in the forward), in the compensated kinds:
  // 3 through the first quarter of the run's strip-rows, then 2, 1 and 0.
  // The SIMD arbiter issues the oldest ready wave first, so without the steps
  // the waves that share a SIMD finish far apart and the last runs alone;
  // with them a wave that is behind takes the issue slots first.  Scheduling
  // only: the sums do not change.  (The plain kind, at 4 waves per SIMD, was
  // slower with the steps at 1920x1024; it and the recurrence keep the
  // arbiter's order.)
  int quarter = 0;
  if (kComp) __builtin_amdgcn_s_setprio(3);
  // The run, one strip segment at a time: the strip-rows of one strip within
  // one block of the order (a run crosses at most a few).
  for (int64_t q = q0; q < q1;) {
    int beta = 0;
    while (beta + 1 < kXcds && q >= order.off[beta + 1]) ++beta;
    const int h = beta / order.B, b = beta - h * order.B;
    const int r_lo = b * order.br;
    const int rows_b = min(ny, r_lo + order.br) - r_lo;
    const int64_t local = q - order.off[beta];
    const int strip = h * order.sh + (int)(local / rows_b);
    const int row0 = r_lo + (int)(local - (local / rows_b) * rows_b);
    row1 = (int)min((int64_t)(r_lo + rows_b), row0 + (q1 - q));
    col0 = strip * kAdjCols;
    // Column terms: the compensated x-phase of each strip column, the
    // recurrence step delta_c, or dx.
#pragma unroll
    for (int c = 0; c < kAdjCols; ++c) {
      const float h = (float)(col0 + c);
      if (KIND == kAdjCompensated)
        CX[c] = __builtin_bit_cast(
            float, __builtin_amdgcn_raw_buffer_load_b32(
                       ctab_rsrc, (unsigned)j * 4u, (int)((int64_t)(col0 + c) * npad * 4), 0));
      else if (kComp)
        CX[c] = axis_phase(h, xc, xph, xpl, xb, xd);
      else if (KIND == kAdjRecurrence)
        CX[c] = fract(prev * __builtin_fmaf(2.0f, h - px, 1.0f));
      else
        CX[c] = h - px;
      SgC[c] = 0.f;
    }
    if (kComp) {
#pragma unroll
      for (int c = 0; c < kAdjCols; ++c) {
        SX[c] = sin_rev(CX[c]);
        CX[c] = cos_rev(CX[c]);
      }
    }
    if (KIND == kAdjRecurrence) {
      const float dx0 = (float)col0 - px;
      dx0sq = dx0 * dx0;
    }
    float gA[kAdjCols], gB[kAdjCols];
    float2 rA = make_float2(0.f, 0.f), rB = rA;
    load_row(row0, gA);
    if (KIND == kAdjCompensated) rA = load_rtab(row0);
    int row = row0;
    auto pairs = [&](int rend) {
      for (; row + 1 < rend; row += 2) {
        do_row(row, gA, gB, rA, rB);
        do_row(row + 1, gB, gA, rB, rA);
      }
    };
    if constexpr (kComp) {
      // Row pairs up to the next quarter boundary of the run (rounded up to
      // an even row offset, so the ping-pong buffers keep their parity), then
      // one priority step, until the segment ends.
      const int64_t done = q - q0;
      for (;;) {
        int rend = row1;
        if (quarter < 3) {
          const int64_t nb = (int64_t)(quarter + 1) * (q1 - q0) / 4;
          // nb - done < row1 - row0 here, so the offset fits an int.
          if (nb < done + (row1 - row0)) rend = min(row1, row0 + (int)((nb - done + 1) & ~int64_t(1)));
        }
        pairs(rend);
        if (rend == row1) break;
        ++quarter;
        if (quarter == 1)
          __builtin_amdgcn_s_setprio(2);
        else if (quarter == 2)
          __builtin_amdgcn_s_setprio(1);
        else
          __builtin_amdgcn_s_setprio(0);
      }
    } else {
      pairs(row1);
    }
    if (row < row1) do_row(row, gA, gB, rA, rB);
#pragma unroll
    for (int c = 0; c < kAdjCols; ++c) {
      const float dx = (float)(col0 + c) - px;
      Sx = __builtin_fmaf(dx, SgC[c], Sx);
      Sr = __builtin_fmaf(dx * dx, SgC[c], Sr);
    }
    q += row1 - row0;
  }
  partial[(int64_t)run * npad + j] = make_float4(Sc0 + Sc1, Sx, Sy, Sr);
#ifdef CGH_WAVE_TRACE
  const unsigned long long trace_c1 = __builtin_amdgcn_s_memtime();
  const unsigned long long trace_t1 = __builtin_amdgcn_s_memrealtime();
  const unsigned hw_id = __builtin_amdgcn_s_getreg((31 << 11) | 4);   // HW_ID
  const unsigned xcc_id = __builtin_amdgcn_s_getreg((31 << 11) | 20);  // XCC_ID
  const unsigned wl = blockIdx.y * gridDim.x + blockIdx.x;
  if (threadIdx.x == 0 && wl < kWaveTraceMax)
    g_wave_trace[wl] = make_ulonglong4(trace_t0, trace_t1,
                                       ((unsigned long long)xcc_id << 32) | hw_id,
                                       trace_c1 - trace_c0);
#endif
}

__global__ __launch_bounds__(kAdjFinPoints* kAdjFinSlices) void adj_finalize_kernel(
    const float4* __restrict__ partial, int regions, int64_t npad, int64_t n,
    const float* __restrict__ z, const float* __restrict__ a, double pitch, double wavelength,
    float* __restrict__ gx, float* __restrict__ gy, float* __restrict__ gz,
    float* __restrict__ ga) {
  __shared__ double part[kAdjFinSlices][4][kAdjFinPoints];
  const int pt = threadIdx.x;
  const int slice = threadIdx.y;
  const int64_t j = (int64_t)blockIdx.x * kAdjFinPoints + pt;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (j < npad) {
    // Regions slice, slice + kAdjFinSlices, ... in increasing order.  The
    // loads of kFinBatch regions are issued together, then added in order.
    constexpr int kFinBatch = 8;
    int r = slice;
    for (; r + (kFinBatch - 1) * kAdjFinSlices < regions; r += kFinBatch * kAdjFinSlices) {
      float4 v[kFinBatch];
#pragma unroll
      for (int q = 0; q < kFinBatch; ++q)
        v[q] = partial[(int64_t)(r + q * kAdjFinSlices) * npad + j];
#pragma unroll
      for (int q = 0; q < kFinBatch; ++q) {
        s0 += (double)v[q].x;
        s1 += (double)v[q].y;
        s2 += (double)v[q].z;
        s3 += (double)v[q].w;
      }
    }
    for (; r < regions; r += kAdjFinSlices) {
      const float4 v = partial[(int64_t)r * npad + j];
      s0 += (double)v.x;
      s1 += (double)v.y;
      s2 += (double)v.z;
      s3 += (double)v.w;
    }
  }
  part[slice][0][pt] = s0;
  part[slice][1][pt] = s1;
  part[slice][2][pt] = s2;
  part[slice][3][pt] = s3;
  __syncthreads();
  if (slice != 0 || j >= n) return;
  double Sc = 0.0, Sx = 0.0, Sy = 0.0, Sr = 0.0;
  for (int k = 0; k < kAdjFinSlices; ++k) {
    Sc += part[k][0][pt];
    Sx += part[k][1][pt];
    Sy += part[k][2][pt];
    Sr += part[k][3][pt];
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

#ifdef CGH_WAVE_TRACE
extern "C" int cgh_wave_trace_read(void* host, size_t bytes) {
  if (!host || bytes > sizeof(g_wave_trace)) return 1;
  return hipMemcpyFromSymbol(host, HIP_SYMBOL(g_wave_trace), bytes, 0,
                             hipMemcpyDeviceToHost) == hipSuccess ? 0 : 1;
}
#endif

hipError_t launch_pad_g(const Plan& p, const float* g, float* gpad, hipStream_t s) {
  const int ldp = p.nsx * kAdjCols;
  const int64_t total = (int64_t)ldp * p.ny;
  const unsigned blocks = grid_blocks(total, 256);
  if (!blocks) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pad_g_kernel, dim3(blocks), dim3(256), 0, s, g,
                     p.nx, p.ny, ldp, total, gpad);
  return hipGetLastError();
}

int adj_runs(const Plan& p) {
  // Resident single-wave workgroups per CU of each adjoint kind, per device.
  static std::mutex mu;
  static std::map<std::pair<int, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  int resident = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({dev, p.adj_kind});
    if (it != cache.end()) resident = it->second;
  }
  if (resident == 0) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return -1;
    hipError_t e;
    if (p.adj_kind == kAdjCompensated)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, adj_partial_kernel<kAdjCompensated>, kAdjThreads, 0);
    else if (p.adj_kind == kAdjCompensatedInline)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, adj_partial_kernel<kAdjCompensatedInline>, kAdjThreads, 0);
    else if (p.adj_kind == kAdjRecurrence)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, adj_partial_kernel<kAdjRecurrence>, kAdjThreads, 0);
    else
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, adj_partial_kernel<kAdjPlain>,
                                                       kAdjThreads, 0);
    if (e != hipSuccess || cus < 1 || per_cu < 1) return -1;
    resident = cus * per_cu;
    std::lock_guard<std::mutex> lk(mu);
    cache[{dev, p.adj_kind}] = resident;
  }
  int runs = (kAdjRounds * resident + p.ngroups - 1) / p.ngroups;
  if (runs > p.regions) runs = p.regions;
  return runs < 1 ? 1 : runs;
}

hipError_t launch_adj_partial(const Plan& p, const Workspace& w, const float* x, const float* y,
                              const float* z, const float* a, double pitch, double wavelength,
                              const float* g, int64_t ldg, int runs, hipStream_t s) {
  const dim3 grid(runs, p.ngroups);
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, grid, dim3(kAdjThreads), 0, s, x, y, z, a, p.n, pitch, wavelength,
                       g, ldg, p.ny, p.strip_rows, p.adj_order, (int)p.npad, (const float2*)w.rtab,
                       (const float*)w.ctab, (float4*)w.partial);
  };
  if (p.adj_kind == kAdjCompensated) {
    if (!w.rtab || !w.ctab) return hipErrorInvalidValue;
    go(adj_partial_kernel<kAdjCompensated>);
  } else if (p.adj_kind == kAdjCompensatedInline)
    go(adj_partial_kernel<kAdjCompensatedInline>);
  else if (p.adj_kind == kAdjRecurrence)
    go(adj_partial_kernel<kAdjRecurrence>);
  else
    go(adj_partial_kernel<kAdjPlain>);
  return hipGetLastError();
}

hipError_t launch_adj_finalize(const Plan& p, const Workspace& w, const float* z, const float* a,
                               double pitch, double wavelength, int runs, float* gx, float* gy,
                               float* gz, float* ga, hipStream_t s) {
  hipLaunchKernelGGL(adj_finalize_kernel,
                     dim3((unsigned)((p.n + kAdjFinPoints - 1) / kAdjFinPoints)),
                     dim3(kAdjFinPoints, kAdjFinSlices), 0, s, (const float4*)w.partial, runs,
                     p.npad, p.n, z, a, pitch, wavelength, gx, gy, gz, ga);
  return hipGetLastError();
}

}  // namespace cgh
