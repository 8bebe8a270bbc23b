// Separable form with half-precision contractions: operand preparation.
//
// The tables and the gradient grid of the separable form (separable.hip) are
// rounded to 16-bit planes for the fp16 / bf16 matrix cores (gemm_half.hip),
// which accumulate in FP32:
//
//   kHalfF16    v ~ fp16(v)
//   kHalfBF16   v ~ bf16(v)
//   kHalfF16x3  v ~ hi + lo, hi = fp16(v), lo = fp16(v - hi); the GEMM forms
//               hi*hi + hi*lo + lo*hi, dropping only lo*lo (about 2^-24
//               relative), so the products keep FP32-level accuracy.
//
// fp16 has a narrow exponent range, so operands whose scale is not fixed
// (the amplitudes A_j in the forward, the upstream gradient G in the adjoint)
// are first divided by a power of two 2^e >= max |v| (exact: only the
// exponent changes), which maps them into (-1, 1); the GEMM multiplies its
// FP32 result by 2^e again.  The cosine/sine tables are already in [-1, 1].
//
// Layouts (k2 = 2 npad, columns 2j and 2j + 1 of point j hold its cosine and
// sine terms):
//   forward  X [nxp][k2], Y [nyp][k2] (with A_j / 2^e)   GEMM I = Y X^T
//   adjoint  Xt [k2][nxp], Yt [k2][nyp], G [nyp][nxp], Gt [nxp][nyp]
//            U = Yt Gt^T, Pm = Xt G^T (both operands K-contiguous)
#include <stdint.h>

#include "cgh_internal.h"
#include "phase.h"

namespace cgh {

namespace {

inline unsigned blocks_for(int64_t count, int threads) {
  return (unsigned)((count + threads - 1) / threads);
}

// Rounds v (|v| <= 1) to the 16-bit format of MODE; lo is the fp16 residual
// in kHalfF16x3 mode and 0 otherwise.
template <int MODE>
__device__ __forceinline__ void to_half(float v, uint16_t& hi, uint16_t& lo) {
  if (MODE == kHalfBF16) {
    hi = __builtin_bit_cast(uint16_t, (__bf16)v);
    lo = 0;
  } else {
    const _Float16 h = (_Float16)v;
    hi = __builtin_bit_cast(uint16_t, h);
    lo = MODE == kHalfF16x3 ? __builtin_bit_cast(uint16_t, (_Float16)(v - (float)h)) : 0;
  }
}

// 1 / 2^e for the recorded maximum (exact), or 1 without one.
__device__ __forceinline__ float inv_scale(const unsigned* max_bits) {
  return max_bits ? 1.0f / pow2_scale(*max_bits) : 1.0f;
}

__global__ __launch_bounds__(256) void absmax_kernel(const float* __restrict__ v, int64_t count,
                                                     unsigned* __restrict__ out) {
  // |v| as float bits: for non-negative floats the unsigned order is the
  // numeric order (NaN sorts above inf, and pow2_scale treats both as 1).
  unsigned m = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    m = max(m, __float_as_uint(fabsf(v[i])));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, off, 64));
  if ((threadIdx.x & 63) == 0 && m != 0) atomicMax(out, m);
}

// Forward tables [rows_pad][k2]: thread t -> row h = t / npad, point j =
// t % npad; the (cos, sin) pair of 16-bit values is one 32-bit store.
template <int MODE>
__global__ __launch_bounds__(256) void sep_table_half_kernel(
    const float* __restrict__ rec, const float* __restrict__ amp, const unsigned* amp_max,
    int64_t npad, int rows_valid, int64_t total, uint32_t* __restrict__ hi,
    uint32_t* __restrict__ lo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int64_t j = t % npad;
  const int h = (int)(t / npad);
  float c = 0.0f, s = 0.0f;
  if (h < rows_valid) {
    const float* r = rec + j * kAxisRec;
    const float phi = axis_phase((float)h, r[0], r[1], r[2], r[3], r[4]);
    c = cos_rev(phi);
    s = sin_rev(phi);
    if (amp) {
      const float A = amp[j] * inv_scale(amp_max);
      c = A * c;
      s = -(A * s);
    }
  }
  uint16_t ch, cl, sh, sl;
  to_half<MODE>(c, ch, cl);
  to_half<MODE>(s, sh, sl);
  hi[t] = (uint32_t)ch | ((uint32_t)sh << 16);
  if (MODE == kHalfF16x3) lo[t] = (uint32_t)cl | ((uint32_t)sl << 16);
}

// Adjoint tables [k2][rows_pad]: thread t -> row h = t % rows_pad, point
// j = t / rows_pad; rows 2j (cos) and 2j + 1 (sin) of column h.
template <int MODE>
__global__ __launch_bounds__(256) void sep_table_half_t_kernel(const float* __restrict__ rec,
                                                               int rows_valid, int rows_pad,
                                                               int64_t total,
                                                               uint16_t* __restrict__ hi,
                                                               uint16_t* __restrict__ lo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int64_t j = t / rows_pad;
  const int h = (int)(t - j * rows_pad);
  float c = 0.0f, s = 0.0f;
  if (h < rows_valid) {
    const float* r = rec + j * kAxisRec;
    const float phi = axis_phase((float)h, r[0], r[1], r[2], r[3], r[4]);
    c = cos_rev(phi);
    s = sin_rev(phi);
  }
  uint16_t ch, cl, sh, sl;
  to_half<MODE>(c, ch, cl);
  to_half<MODE>(s, sh, sl);
  const int64_t oc = (2 * j) * rows_pad + h, os = oc + rows_pad;
  hi[oc] = ch;
  hi[os] = sh;
  if (MODE == kHalfF16x3) {
    lo[oc] = cl;
    lo[os] = sl;
  }
}

// G / 2^e as 16-bit planes, zero-padded to [nyp][nxp], and its transpose
// [nxp][nyp].  One workgroup per 64 x 64 tile; the transpose goes through LDS
// (row pitch 65 words, so the column reads of 64 lanes hit distinct banks).
template <int MODE>
__global__ __launch_bounds__(256) void sep_pad_half_kernel(
    const float* __restrict__ g, int nx, int ny, int nyp, int nxp, const unsigned* g_max,
    uint16_t* __restrict__ gh, uint16_t* __restrict__ gl, uint16_t* __restrict__ gth,
    uint16_t* __restrict__ gtl) {
  __shared__ uint32_t tile[64][65];
  const float inv = inv_scale(g_max);
  const int x0 = blockIdx.x * 64, y0 = blockIdx.y * 64;
  const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;
#pragma unroll 4
  for (int i = 0; i < 16; ++i) {
    const int r = r0 + 4 * i;
    const int yy = y0 + r, xx = x0 + c;
    const float v = (xx < nx && yy < ny) ? g[(int64_t)yy * nx + xx] * inv : 0.0f;
    uint16_t h, l;
    to_half<MODE>(v, h, l);
    const int64_t o = (int64_t)yy * nxp + xx;
    gh[o] = h;
    if (MODE == kHalfF16x3) gl[o] = l;
    tile[r][c] = (uint32_t)h | ((uint32_t)l << 16);
  }
  __syncthreads();
#pragma unroll 4
  for (int i = 0; i < 16; ++i) {
    const int r = r0 + 4 * i;       // column x0 + r of G
    const uint32_t v = tile[c][r];  // G(y0 + c, x0 + r)
    const int64_t o = (int64_t)(x0 + r) * nyp + y0 + c;
    gth[o] = (uint16_t)(v & 0xffffu);
    if (MODE == kHalfF16x3) gtl[o] = (uint16_t)(v >> 16);
  }
}

}  // namespace

hipError_t launch_absmax(const float* v, int64_t count, unsigned* out, hipStream_t s) {
  hipError_t e = launch_fill_zero_f32((float*)out, 1, s);  // 0.0f has all-zero bits
  if (e != hipSuccess || count <= 0) return e;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)blocks), dim3(256), 0, s, v, count, out);
  return hipGetLastError();
}

hipError_t launch_sep_table_half(int mode, const float* rec, const float* amp,
                                 const unsigned* amp_max, int64_t npad, int rows_valid,
                                 int rows_pad, bool transposed, uint16_t* hi, uint16_t* lo,
                                 hipStream_t s) {
  const int64_t total = (int64_t)rows_pad * npad;
  const dim3 grid(blocks_for(total, 256)), block(256);
  if (transposed) {
    if (mode == kHalfF16x3)
      hipLaunchKernelGGL(sep_table_half_t_kernel<kHalfF16x3>, grid, block, 0, s, rec, rows_valid,
                         rows_pad, total, hi, lo);
    else if (mode == kHalfBF16)
      hipLaunchKernelGGL(sep_table_half_t_kernel<kHalfBF16>, grid, block, 0, s, rec, rows_valid,
                         rows_pad, total, hi, lo);
    else
      hipLaunchKernelGGL(sep_table_half_t_kernel<kHalfF16>, grid, block, 0, s, rec, rows_valid,
                         rows_pad, total, hi, lo);
  } else {
    uint32_t* h32 = (uint32_t*)hi;
    uint32_t* l32 = (uint32_t*)lo;
    if (mode == kHalfF16x3)
      hipLaunchKernelGGL(sep_table_half_kernel<kHalfF16x3>, grid, block, 0, s, rec, amp, amp_max,
                         npad, rows_valid, total, h32, l32);
    else if (mode == kHalfBF16)
      hipLaunchKernelGGL(sep_table_half_kernel<kHalfBF16>, grid, block, 0, s, rec, amp, amp_max,
                         npad, rows_valid, total, h32, l32);
    else
      hipLaunchKernelGGL(sep_table_half_kernel<kHalfF16>, grid, block, 0, s, rec, amp, amp_max,
                         npad, rows_valid, total, h32, l32);
  }
  return hipGetLastError();
}

hipError_t launch_sep_pad_half(int mode, const float* g, int nx, int ny, int nyp, int nxp,
                               const unsigned* g_max, uint16_t* gh, uint16_t* gl, uint16_t* gth,
                               uint16_t* gtl, hipStream_t s) {
  const dim3 grid((unsigned)(nxp / 64), (unsigned)(nyp / 64)), block(256);
  if (mode == kHalfF16x3)
    hipLaunchKernelGGL(sep_pad_half_kernel<kHalfF16x3>, grid, block, 0, s, g, nx, ny, nyp, nxp,
                       g_max, gh, gl, gth, gtl);
  else if (mode == kHalfBF16)
    hipLaunchKernelGGL(sep_pad_half_kernel<kHalfBF16>, grid, block, 0, s, g, nx, ny, nyp, nxp,
                       g_max, gh, gl, gth, gtl);
  else
    hipLaunchKernelGGL(sep_pad_half_kernel<kHalfF16>, grid, block, 0, s, g, nx, ny, nyp, nxp,
                       g_max, gh, gl, gth, gtl);
  return hipGetLastError();
}

}  // namespace cgh
