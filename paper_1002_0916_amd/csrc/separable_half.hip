// Separable form with half-precision contractions: operand preparation.
//
// The tables and the gradient grid of the separable form (separable.hip) are
// rounded to 16-bit planes for the fp16 / bf16 matrix cores (gemm_half.hip),
// which accumulate in FP32:
//
//   kHalfF16    v ~ fp16(v)
//   kHalfBF16   v ~ bf16(v)
//   kHalfF16x3  v ~ hi + lo, hi = fp16(v), lo = fp16(v - hi); the GEMM forms
//               hi*hi + hi*lo + lo*hi, dropping only lo*lo (at most 2^-22 of
//               the product), so the products keep near-FP32 accuracy.
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

// Block-level max of |v| (float bits: for non-negative floats the unsigned
// order is the numeric order; NaN sorts above inf and pow2_scale treats both
// as 1), then one atomic per workgroup.
__global__ __launch_bounds__(256) void absmax_kernel(const float* __restrict__ v, int64_t count,
                                                     unsigned* __restrict__ out) {
  __shared__ unsigned wave_max[4];
  unsigned m = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (((uintptr_t)v & 15u) == 0) {
    const int64_t n4 = count / 4;
    const float4* v4 = reinterpret_cast<const float4*>(v);
    auto take = [&](const float4& q) {
      m = max(m, max(max(__float_as_uint(fabsf(q.x)), __float_as_uint(fabsf(q.y))),
                     max(__float_as_uint(fabsf(q.z)), __float_as_uint(fabsf(q.w)))));
    };
    // Eight loads in flight per thread before their maxima are taken: the
    // pass is bound by memory latency, not by the max operations.
    int64_t i = first;
    for (; i + 7 * stride < n4; i += 8 * stride) {
      float4 q[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) q[k] = v4[i + k * stride];
#pragma unroll
      for (int k = 0; k < 8; ++k) take(q[k]);
    }
    for (; i < n4; i += stride) take(v4[i]);
    for (int64_t i = 4 * n4 + first; i < count; i += stride)
      m = max(m, __float_as_uint(fabsf(v[i])));
  } else {
    for (int64_t i = first; i < count; i += stride) m = max(m, __float_as_uint(fabsf(v[i])));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, off, 64));
  if ((threadIdx.x & 63) == 0) wave_max[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = max(max(wave_max[0], wave_max[1]), max(wave_max[2], wave_max[3]));
    if (m != 0) atomicMax(out, m);
  }
}

// (cos, sin) of the axis phase of point j at coordinate h (zero for h beyond
// the hologram).
__device__ __forceinline__ void axis_cs(const float* __restrict__ rec, int64_t j, int h,
                                        int rows_valid, float& c, float& s) {
  c = 0.0f;
  s = 0.0f;
  if (h < rows_valid) {
    const float* r = rec + j * kAxisRec;
    const float phi = axis_phase((float)h, r[0], r[1], r[2], r[3], r[4]);
    c = cos_rev(phi);
    s = sin_rev(phi);
  }
}

// Forward operands, one launch: table rows r in [0, nxp) are X [nxp][k2],
// rows [nxp, nxp + nyp) are Y [nyp][k2] with (A_j cY, -A_j sY) / 2^e.  Lane
// -> point j = blockIdx.x * 256 + threadIdx.x, the workgroups of one x index
// stride over the rows; each (cos, sin) pair of 16-bit values is one 32-bit
// store at [h][j].
template <int MODE>
__global__ __launch_bounds__(256) void sep_tables_half_kernel(
    const float* __restrict__ xrec, const float* __restrict__ yrec,
    const float* __restrict__ amp, const unsigned* __restrict__ amp_max, int64_t npad, int nx,
    int nxp, int ny, int nyp, uint32_t* __restrict__ xh, uint32_t* __restrict__ xl,
    uint32_t* __restrict__ yh, uint32_t* __restrict__ yl) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= npad) return;
  float xr[5], yr[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    xr[i] = xrec[j * kAxisRec + i];
    yr[i] = yrec[j * kAxisRec + i];
  }
  const float A = amp[j] * inv_scale(amp_max);
  for (int r = blockIdx.y; r < nxp + nyp; r += gridDim.y) {
    const bool is_x = r < nxp;
    const int h = is_x ? r : r - nxp;
    float c = 0.0f, s = 0.0f;
    if (h < (is_x ? nx : ny)) {
      const float* q = is_x ? xr : yr;
      const float phi = axis_phase((float)h, q[0], q[1], q[2], q[3], q[4]);
      c = cos_rev(phi);
      s = sin_rev(phi);
      if (!is_x) {
        c = A * c;
        s = -(A * s);
      }
    }
    uint16_t ch, cl, sh, sl;
    to_half<MODE>(c, ch, cl);
    to_half<MODE>(s, sh, sl);
    const int64_t o = (int64_t)h * npad + j;
    (is_x ? xh : yh)[o] = (uint32_t)ch | ((uint32_t)sh << 16);
    if (MODE == kHalfF16x3) (is_x ? xl : yl)[o] = (uint32_t)cl | ((uint32_t)sl << 16);
  }
}

// Adjoint operands, one launch (1-D grid).  The first tab_blocks * tab_rows
// workgroups fill the transposed tables Xt [k2][nxp] then Yt [k2][nyp]:
// workgroup b takes coordinates h = (b % tab_blocks) * 256 + lane of the
// concatenated [nxp + nyp] range and the points j = b / tab_blocks + k *
// tab_rows (rows 2j (cos) and 2j + 1 (sin)).  Each remaining workgroup takes
// one 64 x 64 tile of G / 2^e, zero-padded, into G [nyp][nxp] and, through
// LDS (row pitch 65 words, so the column reads of 64 lanes hit distinct
// banks), into Gt [nxp][nyp].
template <int MODE>
__global__ __launch_bounds__(256) void sep_adj_operands_half_kernel(
    const float* __restrict__ xrec, const float* __restrict__ yrec, int64_t npad, int nx, int nxp,
    int ny, int nyp, int tab_blocks, int tab_rows, const float* __restrict__ g,
    const unsigned* __restrict__ g_max, uint16_t* __restrict__ xh, uint16_t* __restrict__ xl,
    uint16_t* __restrict__ yh, uint16_t* __restrict__ yl, uint16_t* __restrict__ gh,
    uint16_t* __restrict__ gl, uint16_t* __restrict__ gth, uint16_t* __restrict__ gtl) {
  __shared__ uint32_t tile[64][65];
  const int bid = (int)blockIdx.x;
  if (bid < tab_blocks * tab_rows) {
    const int u = (bid % tab_blocks) * 256 + (int)threadIdx.x;
    if (u >= nxp + nyp) return;
    const bool is_x = u < nxp;
    const int h = is_x ? u : u - nxp;
    const int rows_pad = is_x ? nxp : nyp;
    const float* rec = is_x ? xrec : yrec;
    const int valid = is_x ? nx : ny;
    uint16_t* hi = is_x ? xh : yh;
    uint16_t* lo = is_x ? xl : yl;
    for (int64_t j = bid / tab_blocks; j < npad; j += tab_rows) {
      float c, s;
      axis_cs(rec, j, h, valid, c, s);
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
    return;
  }
  const int b = bid - tab_blocks * tab_rows;
  const int tiles_x = nxp / 64;
  const int x0 = (int)(b % tiles_x) * 64, y0 = (int)(b / tiles_x) * 64;
  const float inv = inv_scale(g_max);
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
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 256 * 16 - 1) / (256 * 16);
  if (blocks > 256) blocks = 256;
  hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)blocks), dim3(256), 0, s, v, count, out);
  return hipGetLastError();
}

hipError_t launch_sep_tables_half(int mode, const Plan& p, const Workspace& w, hipStream_t s) {
  const dim3 grid = table_grid(p.npad, p.nxp + p.nyp), block(256);
  uint32_t *xh = (uint32_t*)w.hx_hi, *xl = (uint32_t*)w.hx_lo;
  uint32_t *yh = (uint32_t*)w.hy_hi, *yl = (uint32_t*)w.hy_lo;
  if (mode == kHalfF16x3)
    hipLaunchKernelGGL(sep_tables_half_kernel<kHalfF16x3>, grid, block, 0, s, w.xrec, w.yrec,
                       w.amp, w.hmax, p.npad, p.nx, p.nxp, p.ny, p.nyp, xh, xl, yh, yl);
  else if (mode == kHalfBF16)
    hipLaunchKernelGGL(sep_tables_half_kernel<kHalfBF16>, grid, block, 0, s, w.xrec, w.yrec,
                       w.amp, w.hmax, p.npad, p.nx, p.nxp, p.ny, p.nyp, xh, xl, yh, yl);
  else
    hipLaunchKernelGGL(sep_tables_half_kernel<kHalfF16>, grid, block, 0, s, w.xrec, w.yrec,
                       w.amp, w.hmax, p.npad, p.nx, p.nxp, p.ny, p.nyp, xh, xl, yh, yl);
  return hipGetLastError();
}

// About 1024 table workgroups (point strides of tab_rows), then the tiles.
hipError_t launch_sep_adj_operands_half(int mode, const Plan& p, const Workspace& w,
                                        const float* g, hipStream_t s) {
  const int tab_blocks = (int)grid_blocks(p.nxp + p.nyp, 256);
  int tab_rows = tab_blocks >= 1024 ? 1 : 1024 / tab_blocks;
  if (tab_rows > p.npad) tab_rows = (int)p.npad;
  const int tiles = (p.nxp / 64) * (p.nyp / 64);
  const dim3 grid((unsigned)(tab_blocks * tab_rows + tiles)), block(256);
  if (mode == kHalfF16x3)
    hipLaunchKernelGGL(sep_adj_operands_half_kernel<kHalfF16x3>, grid, block, 0, s, w.xrec,
                       w.yrec, p.npad, p.nx, p.nxp, p.ny, p.nyp, tab_blocks, tab_rows, g, w.hmax, w.hx_hi,
                       w.hx_lo, w.hy_hi, w.hy_lo, w.hg_hi, w.hg_lo, w.hgt_hi, w.hgt_lo);
  else if (mode == kHalfBF16)
    hipLaunchKernelGGL(sep_adj_operands_half_kernel<kHalfBF16>, grid, block, 0, s, w.xrec,
                       w.yrec, p.npad, p.nx, p.nxp, p.ny, p.nyp, tab_blocks, tab_rows, g, w.hmax, w.hx_hi,
                       w.hx_lo, w.hy_hi, w.hy_lo, w.hg_hi, w.hg_lo, w.hgt_hi, w.hgt_lo);
  else
    hipLaunchKernelGGL(sep_adj_operands_half_kernel<kHalfF16>, grid, block, 0, s, w.xrec,
                       w.yrec, p.npad, p.nx, p.nxp, p.ny, p.nyp, tab_blocks, tab_rows, g, w.hmax, w.hx_hi,
                       w.hx_lo, w.hy_hi, w.hy_lo, w.hg_hi, w.hg_lo, w.hgt_hi, w.hgt_lo);
  return hipGetLastError();
}

}  // namespace cgh
