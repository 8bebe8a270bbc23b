// Machine constants behind the roofline model (a standalone gfx950 program,
// not part of the library): the issue rate of FP32 FMA, v_cos_f32, v_sin_f32
// and v_fract_f32, alone and mixed, in issue slots relative to an FMA, and the
// accuracy of v_cos_f32 / v_sin_f32 (cos and sin of 2 pi t) against the host's
// FP64 libm.
//
// Rates: 4096 workgroups of 256 threads (16 waves per SIMD), each thread
// running 8 independent dependency chains for 4096 steps, so the measurement
// is issue-bound, not latency-bound.  A step of a mixed mode issues one
// instruction of each listed kind per chain.  Best of 4 launches.
#include <hip/hip_runtime.h>

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

template <int MODE>
__global__ void rate(float* out, int iters, float a, float b) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  float x[kChains], y[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) {
    x[k] = 0.001f * (t + k);
    y[k] = 0.002f * (t - k);
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
      if (MODE == 0) x[k] = __builtin_amdgcn_cosf(x[k]);
      if (MODE == 1) x[k] = __builtin_amdgcn_sinf(x[k]);
      if (MODE == 2) x[k] = __builtin_amdgcn_fractf(x[k] + a);
      if (MODE == 3) x[k] = __builtin_fmaf(x[k], a, b);
      if (MODE == 4) {
        x[k] = __builtin_amdgcn_cosf(x[k]);
        y[k] = __builtin_fmaf(y[k], a, b);
      }
      if (MODE == 5) {
        x[k] = __builtin_amdgcn_cosf(x[k]);
#pragma unroll
        for (int f = 0; f < 4; ++f) y[k] = __builtin_fmaf(y[k], a, b);
      }
      if (MODE == 6) {
        x[k] = __builtin_amdgcn_cosf(x[k]);
        y[k] = __builtin_amdgcn_sinf(y[k]);
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += x[k] + y[k];
  out[t] = s;  // keeps every chain live
}

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
  const int blocks = 4096, threads = 256, iters = 4096;
  float* d;
  CK(hipMalloc(&d, sizeof(float) * blocks * threads));
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  const char* names[] = {"cos", "sin", "add+fract", "fma", "cos+fma", "cos+4fma", "cos+sin"};
  double rate_of[7];
  for (int mode = 0; mode < 7; ++mode) {
    float best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
      CK(hipEventRecord(e0));
      switch (mode) {
        case 0: rate<0><<<blocks, threads>>>(d, iters, 1.0001f, 0.5f); break;
        case 1: rate<1><<<blocks, threads>>>(d, iters, 1.0001f, 0.5f); break;
        case 2: rate<2><<<blocks, threads>>>(d, iters, 1.0001f, 0.5f); break;
        case 3: rate<3><<<blocks, threads>>>(d, iters, 1.0001f, 0.5f); break;
        case 4: rate<4><<<blocks, threads>>>(d, iters, 1.0001f, 0.5f); break;
        case 5: rate<5><<<blocks, threads>>>(d, iters, 1.0001f, 0.5f); break;
        default: rate<6><<<blocks, threads>>>(d, iters, 1.0001f, 0.5f); break;
      }
      CK(hipGetLastError());
      CK(hipEventRecord(e1));
      CK(hipEventSynchronize(e1));
      float ms;
      CK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) best = ms;
    }
    rate_of[mode] = (double)blocks * threads * iters * kChains / (best * 1e-3);
  }
  const double fma = rate_of[3];
  const double peak = (double)p.multiProcessorCount * 64 * (p.clockRate * 1e3);
  printf("\n%-10s %16s %22s\n", "step", "steps/s (lanes)", "issue slots (FMA = 1)");
  for (int mode = 0; mode < 7; ++mode)
    printf("%-10s %16.4e %22.2f\n", names[mode], rate_of[mode], fma / rate_of[mode]);
  printf("\nFMA rate %.4e lane-ops/s = %.1f%% of %d CUs x 64 lanes x %.2f GHz\n", fma,
         100.0 * fma / peak, p.multiProcessorCount, p.clockRate * 1e-6);

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
