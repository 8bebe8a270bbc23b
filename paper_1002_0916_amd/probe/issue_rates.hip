// Machine constants behind the roofline model (a standalone gfx950 program,
// not part of the library): the issue cost of FP32 VALU instructions by kind
// (all operands in VGPRs, or one read from an SGPR), of v_cos_f32,
// v_sin_f32 and v_fract_f32, and of the per-interaction instruction mix of
// each hot kernel, in cycles per 64-lane instruction per CU; and the
// accuracy of v_cos_f32 / v_sin_f32 (cos and sin of 2 pi t) against the
// host's FP64 libm.
//
// Rates: workgroups of 256 threads (one wave per SIMD each), 16, 8, 4, 3 or 2
// of them per CU, each thread running 8 independent dependency chains for
// 4096 steps, so the measurement is issue-bound, not latency-bound; the last
// column is the most waves per SIMD that a mode's register use lets be
// resident (a launch of more runs in rounds).  Cycles are counted at the
// device's nominal clock (hipDeviceProp_t::clockRate); the GHz@16 column is
// the shader clock measured in the 16-wave launch (median over workgroups of
// the s_memtime count over the 100 MHz s_memrealtime count), which falls
// below the nominal clock under a sustained VALU load.  A step of a mixed mode
// issues one instruction of each listed kind per chain.  Values that are
// wave-uniform in the kernels (a, b) are SGPR operands; av, bv hold the same
// values in VGPRs (0 * t is not folded under strict FP).  Best of 4 launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#define CK(x)                                                                        \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) {                                                          \
      printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);          \
      return 1;                                                                      \
    }                                                                                \
  } while (0)

constexpr int kChains = 8;
constexpr int kModes = 22;
const char* const kNames[kModes] = {
    "fma (v, s, s)",  "fma (v, v, v)",   "add (v, s)",        "add (v, v)",
    "fract",          "cos",             "sin",               "cos + sin",
    "cos + fma(v,s,s)", "cos + 4 fma(v,s,s)",
    "fwd compensated: add, cos, fma (A, Y in VGPRs)",
    "fwd compensated: add, cos, fma (A, Y in SGPRs)",
    "fwd plain: sub, fma, mul, fract, cos, fma (point in SGPRs)",
    "adj compensated: add, sin, cos, 3 fma (G in SGPR)",
    "adj compensated: add, sin, cos, 3 fma (G in VGPR)",
    "adj plain: fma, mul, fract, sin, cos, 3 fma (G in SGPR)",
    "adj addition: 2 mul, 2 fma, 3 fma (G in SGPR)",
    "adj factored sums: 4 fma (G in SGPR)",
    "adj factored sums: 4 fma (G in VGPR)",
    "fwd addition: mul, fma, fma (cY, sY, A in VGPRs)",
    "fwd addition: mul, fma, fma (cY, sY, A in SGPRs)",
    "fwd recurrence: add, cos, fma (A in SGPR) + 1/4 add"};

// Eight distinct wave-uniform values (SGPRs, from the kernel arguments).
struct Uniform {
  float g[kChains];
};

// Shader clock during a launch: thread 0 of each workgroup stores the
// shader-clock counter (s_memtime) and the constant 100 MHz counter
// (s_memrealtime) at its start and replaces them by their increments at its
// end; clock = ratio x 100 MHz.  The start values go through memory (the
// barrier forces the reload), so they hold no register across the loop.
__device__ __forceinline__ void clock_start(unsigned long long* clk) {
  const unsigned long long c0 = __builtin_amdgcn_s_memtime();
  const unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
  if (threadIdx.x == 0) {
    clk[2 * blockIdx.x] = c0;
    clk[2 * blockIdx.x + 1] = r0;
  }
}
__device__ __forceinline__ void clock_end(unsigned long long* clk) {
  __asm__ volatile("" ::: "memory");
  const unsigned long long c1 = __builtin_amdgcn_s_memtime();
  const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
  if (threadIdx.x == 0) {
    clk[2 * blockIdx.x] = c1 - clk[2 * blockIdx.x];
    clk[2 * blockIdx.x + 1] = r1 - clk[2 * blockIdx.x + 1];
  }
}

template <int MODE>
__global__ void rate(float* out, int iters, float a, float b, Uniform u,
                     const float* __restrict__ tab, unsigned long long* clk) {
  clock_start(clk);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const float av = __builtin_fmaf(0.0f, (float)t, a), bv = __builtin_fmaf(0.0f, (float)t, b);
  float x[kChains], y[kChains], s0[kChains], s1[kChains], s2[kChains], s3[kChains], gv[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) {
    x[k] = 0.001f * (t + k);
    y[k] = 0.002f * (t - k);
    s0[k] = s1[k] = s2[k] = s3[k] = 0.0f;
    gv[k] = __builtin_fmaf(0.0f, (float)t, u.g[k]);
  }
  // Per-step values of modes 16-18 (a row's cosine and sine), so their
  // products stay in the loop.
  float bw = bv, cw = av;
  for (int it = 0; it < iters; ++it) {
    if (MODE >= 16 && MODE <= 20) bw = bw + a;
    if (MODE >= 17 && MODE <= 20) cw = cw + b;
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
      if (MODE == 0) x[k] = __builtin_fmaf(x[k], a, b);
      if (MODE == 1) x[k] = __builtin_fmaf(x[k], av, bv);
      if (MODE == 2) x[k] = x[k] + a;
      if (MODE == 3) x[k] = x[k] + bv;
      if (MODE == 4) x[k] = __builtin_amdgcn_fractf(x[k]);
      if (MODE == 5) x[k] = __builtin_amdgcn_cosf(x[k]);
      if (MODE == 6) x[k] = __builtin_amdgcn_sinf(x[k]);
      if (MODE == 7) {
        x[k] = __builtin_amdgcn_cosf(x[k]);
        y[k] = __builtin_amdgcn_sinf(y[k]);
      }
      if (MODE == 8) {
        x[k] = __builtin_amdgcn_cosf(x[k]);
        y[k] = __builtin_fmaf(y[k], a, b);
      }
      if (MODE == 9) {
        x[k] = __builtin_amdgcn_cosf(x[k]);
#pragma unroll
        for (int f = 0; f < 4; ++f) y[k] = __builtin_fmaf(y[k], a, b);
      }
      if (MODE == 10 || MODE == 11) {  // X + Y, cos, A * c + acc
        const float c = __builtin_amdgcn_cosf(x[k] + (MODE == 10 ? bv : b));
        s0[k] = __builtin_fmaf(MODE == 10 ? av : a, c, s0[k]);
        x[k] = x[k] + (MODE == 10 ? bv : b);
      }
      if (MODE == 12) {  // dy, r2, Prev r2, fract, cos, acc
        const float dy = x[k] - b;
        const float r2 = __builtin_fmaf(dy, dy, y[k]);
        const float c = __builtin_amdgcn_cosf(__builtin_amdgcn_fractf(a * r2));
        s0[k] = __builtin_fmaf(a, c, s0[k]);
        x[k] = dy;
      }
      if (MODE == 13 || MODE == 14) {  // t = CX + RY, sin, cos, Sc, row sum, column sum
        const float g = MODE == 13 ? a : av;
        const float tt = x[k] + bv;
        const float sn = __builtin_amdgcn_sinf(tt), cs = __builtin_amdgcn_cosf(tt);
        s0[k] = __builtin_fmaf(g, cs, s0[k]);
        s1[k] = __builtin_fmaf(g, sn, s1[k]);
        s2[k] = __builtin_fmaf(g, sn, s2[k]);
        x[k] = tt;
      }
      if (MODE == 16) {  // sin, cos of X + Y from per-axis (cX, sX), (cY, sY); 3 sums
        const float sn = __builtin_fmaf(y[k], av, x[k] * bw);
        const float cs = __builtin_fmaf(x[k], av, -(y[k] * bw));
        s0[k] = __builtin_fmaf(a, cs, s0[k]);
        s1[k] = __builtin_fmaf(a, sn, s1[k]);
        s2[k] = __builtin_fmaf(a, sn, s2[k]);
      }
      if (MODE == 17 || MODE == 18) {  // row sums of G cX, G sX; column sums of G cY, G sY
        const float g = MODE == 17 ? u.g[k] : gv[k];
        s0[k] = __builtin_fmaf(g, x[k], s0[k]);
        s1[k] = __builtin_fmaf(g, y[k], s1[k]);
        s2[k] = __builtin_fmaf(g, cw, s2[k]);
        s3[k] = __builtin_fmaf(g, bw, s3[k]);
      }
      if (MODE == 19 || MODE == 20) {  // cos(X + Y) = cX cY - sX sY, acc += A cos
        // x, y: the lane's (cX, sX), fixed per chain; the row's (cY, sY) change
        // per step, in VGPRs (bw, cw) or SGPRs (from the table); A in a VGPR
        // (av) or an SGPR (a)
        // (mode 20: one row of a 64-row table per step, read by scalar loads)
        const float* row = tab + (it & 63) * 16;
        const float cy = MODE == 19 ? cw : row[k], sy = MODE == 19 ? bw : row[8 + k];
        const float ct = __builtin_fmaf(x[k], cy, -(y[k] * sy));
        s0[k] = __builtin_fmaf(MODE == 19 ? av : a, ct, s0[k]);
      }
      if (MODE == 21) {  // Gamma += delta, cos, A * c + acc (A in an SGPR)
        // chains k = 4c + i: column c of the lane's pair, row i; the rows of
        // a column share delta, which steps by Delta once per column
        s0[k] = __builtin_fmaf(a, __builtin_amdgcn_cosf(x[k]), s0[k]);
        x[k] = x[k] + y[k & ~3];
        if ((k & 3) == 3) y[k & ~3] = y[k & ~3] + bv;
      }
      if (MODE == 15) {  // fract(Prev (dx^2 + RY)), sin, cos, 3 sums
        const float tt = __builtin_amdgcn_fractf(bv * __builtin_fmaf(x[k], x[k], y[k]));
        const float sn = __builtin_amdgcn_sinf(tt), cs = __builtin_amdgcn_cosf(tt);
        s0[k] = __builtin_fmaf(a, cs, s0[k]);
        s1[k] = __builtin_fmaf(a, sn, s1[k]);
        s2[k] = __builtin_fmaf(a, sn, s2[k]);
        x[k] = tt;
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += x[k] + y[k] + s0[k] + s1[k] + s2[k] + s3[k];
  out[t] = s;  // keeps every chain live
  clock_end(clk);
}

// The compensated adjoint's row body as the kernel runs it: 32 columns, each
// taking sin and cos of X + Y by the addition theorem from the column's (cX,
// sX) and the row's (cY, sY), then three sums with G from SGPRs (the point's
// two row-sum chains, its row sum of G sin split in two, and the column sum).
// LOADG = false: G of every row from the kernel arguments; true: G of row r
// from a 64-row table in memory through two scalar loads per row, issued a
// row ahead into ping-pong buffers as the kernel does.
// The compensated forward's addition-theorem step for a lane holding two
// columns and two rows, with the row values (cos, sin of the row phases, A)
// broadcast across the wave by DPP row_newbcast from a VGPR that holds them
// once per 16-lane row: per point two moves (cY of each row) and one (A),
// four products (sX sY, the broadcast folded into the product), four FMAs for
// cos(X + Y) and four for the sums, i.e. 15 instructions per 4 interactions.
// Cycles per interaction; 8 independent lane states per thread.
template <int N>
__device__ __forceinline__ float bcast(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x150 + N, 0xf, 0xf, true));
}
__global__ void fwd_dpp(float* out, int iters, const float* __restrict__ tab) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  float cx[8][2], sx[8][2], acc[8][2][2];
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      cx[k][c] = 0.001f * (t + k + c);
      sx[k][c] = 0.002f * (t - k + c);
      acc[k][c][0] = acc[k][c][1] = 0.f;
    }
  // lane l of each 16-lane row holds value l of the current point's row data
  float v = tab[threadIdx.x & 15];
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float a = bcast<4>(v);
      const float cy[2] = {bcast<0>(v), bcast<1>(v)};
#pragma unroll
      for (int r = 0; r < 2; ++r) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const float m = sx[k][c] * (r ? bcast<3>(v) : bcast<2>(v));
          const float ct = __builtin_fmaf(cx[k][c], cy[r], -m);
          acc[k][c][r] = __builtin_fmaf(a, ct, acc[k][c][r]);
        }
      }
      v = v + 1.0f;  // the next point's row data (one add per 4 interactions)
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int c = 0; c < 2; ++c) s += acc[k][c][0] + acc[k][c][1];
  out[t] = s;
}

constexpr int kRowCols = 32;
struct RowG {
  float g[kRowCols];
};
template <bool LOADG>
__global__ void adj_row(float* out, int iters, float a, float b, RowG u, const float* gtab) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  float CX[kRowCols], SX[kRowCols], SgC[kRowCols];
#pragma unroll
  for (int c = 0; c < kRowCols; ++c) {
    CX[c] = 0.001f * (t + c);
    SX[c] = 0.002f * (t - c);
    SgC[c] = 0.0f;
  }
  float cY = __builtin_fmaf(0.0f, (float)t, a), sY = __builtin_fmaf(0.0f, (float)t, b);
  float Sc0 = 0.f, Sc1 = 0.f, Sy = 0.f, Sr = 0.f;
  float gA[kRowCols], gB[kRowCols];
#pragma unroll
  for (int c = 0; c < kRowCols; ++c) gA[c] = LOADG ? gtab[c] : u.g[c];
  auto row = [&](int it, const float* gc, float* gn) {
    cY = cY + a;
    sY = sY + b;
    float sr0 = 0.f, sr1 = 0.f;
#pragma unroll
    for (int c = 0; c < kRowCols; ++c) {
      if (LOADG && c == 1) {
        __builtin_amdgcn_sched_barrier(0);
        const float* src = gtab + ((it + 1) & 63) * kRowCols;
#pragma unroll
        for (int k = 0; k < kRowCols; ++k) gn[k] = src[k];
        __builtin_amdgcn_sched_barrier(0);
      }
      const float G = LOADG ? gc[c] : u.g[c];
      const float sn = __builtin_fmaf(SX[c], cY, CX[c] * sY);
      const float cs = __builtin_fmaf(CX[c], cY, -(SX[c] * sY));
      if (c & 1) {
        Sc1 = __builtin_fmaf(G, cs, Sc1);
        sr1 = __builtin_fmaf(G, sn, sr1);
      } else {
        Sc0 = __builtin_fmaf(G, cs, Sc0);
        sr0 = __builtin_fmaf(G, sn, sr0);
      }
      SgC[c] = __builtin_fmaf(G, sn, SgC[c]);
    }
    const float sr = sr0 + sr1;
    Sy = __builtin_fmaf(cY, sr, Sy);
    Sr = __builtin_fmaf(sY, sr, Sr);
  };
  for (int it = 0; it < iters; it += 2) {
    row(it, gA, gB);
    row(it + 1, gB, gA);
  }
  float s = Sc0 + Sc1 + Sy + Sr;
#pragma unroll
  for (int c = 0; c < kRowCols; ++c) s += SgC[c];
  out[t] = s;
}

// A 64-row table of 16 floats per row on the device (mode 20), set by main.
const float* g_rowtab = nullptr;
// Per-workgroup clock records (two counters each), sized by main for the
// largest launch.
unsigned long long* g_clk = nullptr;

// Median shader clock in GHz over the workgroups of the last launch.
double median_clock(int blocks) {
  std::vector<unsigned long long> h(2 * (size_t)blocks);
  if (hipMemcpy(h.data(), g_clk, h.size() * sizeof(h[0]), hipMemcpyDeviceToHost) != hipSuccess)
    return -1.0;
  std::vector<double> f(blocks);
  for (int i = 0; i < blocks; ++i) f[i] = h[2 * i + 1] ? 0.1 * (double)h[2 * i] / h[2 * i + 1] : 0.0;
  std::sort(f.begin(), f.end());
  return f[blocks / 2];
}

template <int M>
void launch(int blocks, float* d, int iters) {
  Uniform u;
  for (int k = 0; k < kChains; ++k) u.g[k] = 0.25f + 0.125f * k;
  rate<M><<<blocks, 256>>>(d, iters, 1.0001f, 0.5f, u, g_rowtab, g_clk);
}

template <int M>
int resident(void) {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, rate<M>, 256, 0) != hipSuccess) return -1;
  return blocks;
}

typedef void (*Launch)(int, float*, int);
typedef int (*Resident)(void);
template <int... M>
struct Table {
  static constexpr Launch fns[] = {launch<M>...};
  static constexpr Resident res[] = {resident<M>...};
};

__global__ void trig(const float* in, float* oc, float* os, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) {
    oc[t] = __builtin_amdgcn_cosf(in[t]);
    os[t] = __builtin_amdgcn_sinf(in[t]);
  }
}

int main() {
  hipDeviceProp_t p;
  CK(hipGetDeviceProperties(&p, 0));
  printf("device %s, %d CUs, clock %d kHz, %s\n", p.name, p.multiProcessorCount, p.clockRate,
         p.gcnArchName);
  const int iters = 4096;
  float* d;
  CK(hipMalloc(&d, sizeof(float) * 16 * p.multiProcessorCount * 256));
  {
    float* t;
    CK(hipMalloc(&t, sizeof(float) * 64 * 16));
    std::vector<float> ht(64 * 16);
    for (size_t i = 0; i < ht.size(); ++i) ht[i] = 0.5f + 0.001f * (float)i;
    CK(hipMemcpy(t, ht.data(), sizeof(float) * ht.size(), hipMemcpyHostToDevice));
    g_rowtab = t;
  }
  // One record per workgroup of the largest rate launch.
  CK(hipMalloc(&g_clk, sizeof(unsigned long long) * 2 * 16 * p.multiProcessorCount));
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  typedef Table<0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21>
      Modes;
  const Launch* fns = Modes::fns;
  // One 64-lane instruction per CU per clock.
  const double per_cycle = (double)p.multiProcessorCount * 64 * (p.clockRate * 1e3);
  printf("\ncycles per step (one 64-lane instruction per CU per clock = 1)\n");
  // Workgroups of 4 waves, one per SIMD: 4096 of them give 16 waves per SIMD.
  const int kWaves[] = {16, 8, 4, 3, 2};
  constexpr int kCols = sizeof(kWaves) / sizeof(kWaves[0]);
  printf("%-56s", "step (waves per SIMD)");
  for (int w = 0; w < kCols; ++w) printf(" %7d", kWaves[w]);
  printf(" %7s %7s\n", "max", "GHz@16");
  for (int mode = 0; mode < kModes; ++mode) {
    double cyc[kCols], ghz = 0.0;
    for (int w = 0; w < kCols; ++w) {
      const int blocks = kWaves[w] * p.multiProcessorCount;
      float best = 1e30f;
      for (int rep = 0; rep < 4; ++rep) {
        CK(hipEventRecord(e0));
        fns[mode](blocks, d, iters);
        CK(hipGetLastError());
        CK(hipEventRecord(e1));
        CK(hipEventSynchronize(e1));
        float ms;
        CK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) best = ms;
      }
      const double steps = (double)blocks * 256 * iters * kChains;
      cyc[w] = per_cycle * best * 1e-3 / steps;
      if (w == 0) ghz = median_clock(blocks);
    }
    printf("%-56s", kNames[mode]);
    for (int w = 0; w < kCols; ++w) printf(" %7.3f", cyc[w]);
    printf(" %7d %7.3f\n", Modes::res[mode](), ghz);
  }

  // The adjoint's row body: cycles per interaction (per column of a row).
  {
    RowG u;
    for (int c = 0; c < kRowCols; ++c) u.g[c] = 0.25f + 0.0625f * c;
    float* gtab;
    CK(hipMalloc(&gtab, sizeof(float) * 64 * kRowCols));
    std::vector<float> hg(64 * kRowCols);
    for (size_t i = 0; i < hg.size(); ++i) hg[i] = 0.25f + 0.001f * (float)i;
    CK(hipMemcpy(gtab, hg.data(), sizeof(float) * hg.size(), hipMemcpyHostToDevice));
    // Configurations: G from the kernel arguments or by scalar loads, in
    // workgroups of 4 waves or of one wave (as the adjoint launches them).
    for (int cfg = 0; cfg < 3; ++cfg) {
      const int load = cfg > 0, threads = cfg == 2 ? 64 : 256;
      double cyc[kCols];
      for (int w = 0; w < kCols; ++w) {
        const int blocks = kWaves[w] * p.multiProcessorCount * (256 / threads);
        float best = 1e30f;
        for (int rep = 0; rep < 4; ++rep) {
          CK(hipEventRecord(e0));
          if (load)
            adj_row<true><<<blocks, threads>>>(d, iters / 4, 1e-7f, 2e-7f, u, gtab);
          else
            adj_row<false><<<blocks, threads>>>(d, iters / 4, 1e-7f, 2e-7f, u, gtab);
          CK(hipGetLastError());
          CK(hipEventRecord(e1));
          CK(hipEventSynchronize(e1));
          float ms;
          CK(hipEventElapsedTime(&ms, e0, e1));
          if (ms < best) best = ms;
        }
        const double steps = (double)blocks * threads * (iters / 4) * kRowCols;
        cyc[w] = per_cycle * best * 1e-3 / steps;
      }
      int res = 0;
      if (load)
        CK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&res, adj_row<true>, threads, 0));
      else
        CK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&res, adj_row<false>, threads, 0));
      res = res * threads / 256;
      printf("%-56s", cfg == 0   ? "adj addition row, 32 columns (G in kernel args)"
                      : cfg == 1 ? "adj addition row, 32 columns (G by scalar loads)"
                                 : "  the same, one-wave workgroups");
      for (int w = 0; w < kCols; ++w) printf(" %7.3f", cyc[w]);
      printf(" %7d %7s\n", res, "-");
    }
    CK(hipFree(gtab));
  }

  // The forward's addition-theorem step with DPP row broadcasts.
  {
    double cyc[kCols];
    for (int w = 0; w < kCols; ++w) {
      const int blocks = kWaves[w] * p.multiProcessorCount;
      float best = 1e30f;
      for (int rep = 0; rep < 4; ++rep) {
        CK(hipEventRecord(e0));
        fwd_dpp<<<blocks, 256>>>(d, iters / 4, g_rowtab);
        CK(hipGetLastError());
        CK(hipEventRecord(e1));
        CK(hipEventSynchronize(e1));
        float ms;
        CK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) best = ms;
      }
      const double steps = (double)blocks * 256 * (iters / 4) * 8 * 4;
      cyc[w] = per_cycle * best * 1e-3 / steps;
    }
    int res = 0;
    CK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&res, fwd_dpp, 256, 0));
    printf("%-56s", "fwd addition, 2x2 per lane, DPP row broadcasts");
    for (int w = 0; w < kCols; ++w) printf(" %7.3f", cyc[w]);
    printf(" %7d\n", res);
  }

  // Accuracy of cos(2 pi t) and sin(2 pi t) over 2^24 points of each range.
  const int n = 1 << 24;
  float *din, *dc, *ds;
  CK(hipMalloc(&din, 4ull * n));
  CK(hipMalloc(&dc, 4ull * n));
  CK(hipMalloc(&ds, 4ull * n));
  std::vector<float> hin(n), hc(n), hs(n);
  const double ranges[][2] = {{0.0, 1.0}, {-1.0, 0.0}, {-4.0, 4.0}, {-256.0, 256.0}, {0.0, 0.001},
                              {0.249, 0.251}};
  printf("\n%-18s %12s %12s %12s %12s\n", "t range", "cos max abs", "cos rms", "sin max abs",
         "sin rms");
  for (const auto& r : ranges) {
    for (int i = 0; i < n; ++i) hin[i] = (float)(r[0] + (r[1] - r[0]) * ((double)i / n));
    CK(hipMemcpy(din, hin.data(), 4ull * n, hipMemcpyHostToDevice));
    trig<<<n / 256, 256>>>(din, dc, ds, n);
    CK(hipGetLastError());
    CK(hipDeviceSynchronize());
    CK(hipMemcpy(hc.data(), dc, 4ull * n, hipMemcpyDeviceToHost));
    CK(hipMemcpy(hs.data(), ds, 4ull * n, hipMemcpyDeviceToHost));
    double mc = 0, msn = 0, sc = 0, ss = 0;
    for (int i = 0; i < n; ++i) {
      const double x = hin[i];
      const double ec = fabs(hc[i] - cos(2 * M_PI * x)), es = fabs(hs[i] - sin(2 * M_PI * x));
      sc += ec * ec;
      ss += es * es;
      if (ec > mc) mc = ec;
      if (es > msn) msn = es;
    }
    char label[48];
    snprintf(label, sizeof label, "[%g, %g)", r[0], r[1]);
    printf("%-18s %12.3e %12.3e %12.3e %12.3e\n", label, mc, sqrt(sc / n), msn, sqrt(ss / n));
  }
  return 0;
}
