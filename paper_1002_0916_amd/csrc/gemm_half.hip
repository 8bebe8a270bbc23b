// Half-precision matrix-core GEMM for the separable form (FP32 accumulate).
//
//   C[m][n] = sum_k A(m, k) B(n, k),  A and B stored K-contiguous as 16-bit
//   planes [rows][ld] (element (m, k) at m * ld + k).
//
// Formats (template MODE):
//   kHalfF16    one fp16 plane per operand, one MFMA per product;
//   kHalfBF16   one bf16 plane per operand;
//   kHalfF16x3  hi and lo fp16 planes per operand (value = hi + lo) and three
//               MFMAs per product, hi*hi + hi*lo + lo*hi: about 22 significant
//               bits, close to FP32, at the fp16 matrix-core rate.
//
// v_mfma_f32_32x32x16_{f16,bf16}: lane l holds A[l % 32][(l / 32) * 8 + i]
// and B[(l / 32) * 8 + i][l % 32] (i = 0..7, one 16-byte register quad), and
// accumulator register r of lane l is C[(r / 4) * 8 + (l / 32) * 4 + r % 4]
// [l % 32] (layout checked on the device).  The workgroup computes a 128 x 128
// tile with 4 waves (64 x 64 each = 2 x 2 blocks); K advances 32 per stage
// through double-buffered LDS tiles [row][k] (64-byte rows, chunk-swizzled:
// lds_at).  Split-K over the grid's z extent as in the FP32 kernel.  M, N
// multiples of 128; K a multiple of 32 (the last K slice may be shorter);
// stores masked to m < m_valid, n < n_valid.
#include <stdint.h>

#include "cgh_internal.h"
#include "fold.h"

namespace cgh {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kHBM = 128, kHBN = 128, kHBK = 32, kHPitch = kHBK;

// LDS tiles are [row][k] with 64-byte rows (no padding) and the four 16-byte
// chunks of a row permuted by chunk ^ ((row / 4) % 4).  Both access patterns
// then spread over all 64 banks: a fragment read (16 lanes: 16 consecutive
// rows, one chunk) and a tile store (16 lanes: 4 consecutive rows, all four
// chunks).
__device__ __forceinline__ int lds_at(int row, int chunk) {
  return row * kHPitch + ((chunk ^ ((row >> 2) & 3)) << 3);
}
constexpr int kHThreads = 256;

// This thread's share of a 128 x 32 plane tile: 16-byte chunks c = t and
// t + 256 of the tile's 512, chunk c holding k = 8 (c % 4) .. 8 (c % 4) + 7 of
// row c / 4.  Each wave instruction thus reads 16 whole 64-byte row
// segments.
struct Half16 {
  uint4 lo8, hi8;  // chunks t and t + 256
};

__device__ __forceinline__ Half16 load_plane(const uint16_t* __restrict__ src, int64_t ld, int row0,
                                             int k0) {
  const int t = threadIdx.x;
  const uint16_t* p = src + (int64_t)(row0 + t / 4) * ld + k0 + (t & 3) * 8;
  Half16 r;
  r.lo8 = *reinterpret_cast<const uint4*>(p);
  r.hi8 = *reinterpret_cast<const uint4*>(p + 64 * ld);
  return r;
}

__device__ __forceinline__ void store_plane(uint16_t* __restrict__ lds, const Half16& r) {
  const int t = threadIdx.x;
  *reinterpret_cast<uint4*>(lds + lds_at(t / 4, t & 3)) = r.lo8;
  *reinterpret_cast<uint4*>(lds + lds_at(t / 4 + 64, t & 3)) = r.hi8;
}

template <int MODE>
__device__ __forceinline__ floatx16 mma(uint4 a, uint4 b, floatx16 c) {
  if (MODE == kHalfBF16)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(halfx8, a),
                                                __builtin_bit_cast(halfx8, b), c, 0, 0, 0);
}

template <int MODE, int FOLD>
__global__ __launch_bounds__(kHThreads, 2) void gemm_half_kernel(
    const uint16_t* __restrict__ Ah, const uint16_t* __restrict__ Al, int64_t lda,
    const uint16_t* __restrict__ Bh, const uint16_t* __restrict__ Bl, int64_t ldb,
    float* __restrict__ C, int64_t ldc, int64_t slice_stride, int k_slice, int k_total, int m_valid,
    int n_valid, const unsigned* __restrict__ scale_max, FoldSpec fold) {
  constexpr bool kSplit = MODE == kHalfF16x3;
  constexpr int kPlane = kHBM * kHPitch;
  // [buffer][plane]: A hi, B hi, and (split) A lo, B lo
  __shared__ uint16_t smem[2][kSplit ? 4 : 2][kPlane];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // XCD-aware order over (slice, tile row, tile column), slice-major: each
  // XCD takes a contiguous range, i.e. a compact block of tiles of one K
  // slice, whose operand rows and columns fit its L2.
  const unsigned per_slice = gridDim.x * gridDim.y;
  const unsigned tile = xcd_tile(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                 per_slice * gridDim.z);
  const int slice = (int)(tile / per_slice);
  const int m0 = (int)((tile % per_slice) / gridDim.x) * kHBM;
  const int n0 = (int)(tile % gridDim.x) * kHBN;
  const int kbeg = slice * k_slice;
  // the last slice may be shorter (never empty: checked at launch)
  const int nstages = (min(kbeg + k_slice, k_total) - kbeg) / kHBK;

  floatx16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  Half16 rah = load_plane(Ah, lda, m0, kbeg);
  Half16 rbh = load_plane(Bh, ldb, n0, kbeg);
  Half16 ral, rbl;
  if (kSplit) {
    ral = load_plane(Al, lda, m0, kbeg);
    rbl = load_plane(Bl, ldb, n0, kbeg);
  }
  store_plane(smem[0][0], rah);
  store_plane(smem[0][1], rbh);
  if (kSplit) {
    store_plane(smem[0][2], ral);
    store_plane(smem[0][3], rbl);
  }
  __syncthreads();

  for (int s = 0; s < nstages; ++s) {
    const int buf = s & 1;
    if (s + 1 < nstages) {
      const int kn = kbeg + (s + 1) * kHBK;
      rah = load_plane(Ah, lda, m0, kn);
      rbh = load_plane(Bh, ldb, n0, kn);
      if (kSplit) {
        ral = load_plane(Al, lda, m0, kn);
        rbl = load_plane(Bl, ldb, n0, kn);
      }
    }
#pragma unroll
    for (int t = 0; t < kHBK / 16; ++t) {
      uint4 fah[2], fbh[2], fal[2], fbl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int ra = lds_at(wm * 64 + i * 32 + (lane & 31), 2 * t + (lane >> 5));
        const int rb = lds_at(wn * 64 + i * 32 + (lane & 31), 2 * t + (lane >> 5));
        fah[i] = *reinterpret_cast<const uint4*>(&smem[buf][0][ra]);
        fbh[i] = *reinterpret_cast<const uint4*>(&smem[buf][1][rb]);
        if (kSplit) {
          fal[i] = *reinterpret_cast<const uint4*>(&smem[buf][2][ra]);
          fbl[i] = *reinterpret_cast<const uint4*>(&smem[buf][3][rb]);
        }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = mma<MODE>(fah[i], fbh[j], acc[i][j]);
          if (kSplit) {
            acc[i][j] = mma<MODE>(fah[i], fbl[j], acc[i][j]);
            acc[i][j] = mma<MODE>(fal[i], fbh[j], acc[i][j]);
          }
        }
    }
    if (s + 1 < nstages) {
      store_plane(smem[buf ^ 1][0], rah);
      store_plane(smem[buf ^ 1][1], rbh);
      if (kSplit) {
        store_plane(smem[buf ^ 1][2], ral);
        store_plane(smem[buf ^ 1][3], rbl);
      }
    }
    __syncthreads();
  }

  // Undo the power-of-two operand scaling (exact).
  const float alpha = scale_max ? pow2_scale(*scale_max) : 1.0f;
  if (FOLD) {
    const int64_t npts = (int64_t)gridDim.y * (kHBM / 2);
    float4* dst = fold.out + ((int64_t)slice * gridDim.x + n0 / kHBN) * npts + m0 / 2;
    fold_tile<FOLD>(acc, m0, n0, fold.rec, fold.plain, fold.n_valid, alpha, dst,
                    reinterpret_cast<float4*>(&smem[0][0][0]));
    return;
  }
  float* Cz = C + (int64_t)slice * slice_stride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn * 64 + j * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm * 64 + i * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        if (m < m_valid && n < n_valid) Cz[(int64_t)m * ldc + n] = alpha * acc[i][j][r];
      }
    }
}

template <int MODE>
hipError_t launch_mode(const uint16_t* Ah, const uint16_t* Al, int64_t lda, const uint16_t* Bh,
                       const uint16_t* Bl, int64_t ldb, float* C, int64_t ldc,
                       int64_t slice_stride, int M, int N, int K, int splits, int m_valid,
                       int n_valid, const unsigned* scale_max, const FoldSpec* fold,
                       hipStream_t s) {
  const dim3 grid(N / kHBN, M / kHBM, splits);
  // Slices of k_slice (a multiple of the stage depth), the last one shorter
  // but never empty.
  if (splits < 1 || K < kHBK || K % kHBK != 0) return hipErrorInvalidValue;
  const int k_slice = (K / kHBK + splits - 1) / splits * kHBK;
  if ((int64_t)(splits - 1) * k_slice >= K) return hipErrorInvalidValue;
  const FoldSpec f = fold ? *fold : FoldSpec{0, nullptr, nullptr, 0, nullptr};
  if (f.part == 1)
    hipLaunchKernelGGL((gemm_half_kernel<MODE, 1>), grid, dim3(kHThreads), 0, s, Ah, Al, lda, Bh,
                       Bl, ldb, C, ldc, slice_stride, k_slice, K, m_valid, n_valid, scale_max, f);
  else if (f.part == 2)
    hipLaunchKernelGGL((gemm_half_kernel<MODE, 2>), grid, dim3(kHThreads), 0, s, Ah, Al, lda, Bh,
                       Bl, ldb, C, ldc, slice_stride, k_slice, K, m_valid, n_valid, scale_max, f);
  else
    hipLaunchKernelGGL((gemm_half_kernel<MODE, 0>), grid, dim3(kHThreads), 0, s, Ah, Al, lda, Bh,
                       Bl, ldb, C, ldc, slice_stride, k_slice, K, m_valid, n_valid, scale_max, f);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_half(int mode, const uint16_t* Ah, const uint16_t* Al, int64_t lda,
                            const uint16_t* Bh, const uint16_t* Bl, int64_t ldb, float* C,
                            int64_t ldc, int64_t slice_stride, int M, int N, int K, int splits,
                            int m_valid, int n_valid, const unsigned* scale_max,
                            const FoldSpec* fold, hipStream_t s) {
  if (mode == kHalfF16x3)
    return launch_mode<kHalfF16x3>(Ah, Al, lda, Bh, Bl, ldb, C, ldc, slice_stride, M, N, K,
                                   splits, m_valid, n_valid, scale_max, fold, s);
  if (mode == kHalfBF16)
    return launch_mode<kHalfBF16>(Ah, Al, lda, Bh, Bl, ldb, C, ldc, slice_stride, M, N, K, splits,
                                  m_valid, n_valid, scale_max, fold, s);
  return launch_mode<kHalfF16>(Ah, Al, lda, Bh, Bl, ldb, C, ldc, slice_stride, M, N, K, splits,
                               m_valid, n_valid, scale_max, fold, s);
}

}  // namespace cgh
