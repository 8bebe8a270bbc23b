// FP32 matrix-core GEMM for the separable form of the hologram sum.
//
//   C[m][n] (+)= sum_k A(m, k) B(n, k)
//
// Each operand is stored either K-contiguous (element (m, k) at m * ld + k)
// or M/N-contiguous (element (m, k) at k * ld + m).  The workgroup computes a
// 128 x 128 tile of C with 4 waves, each a 64 x 64 quadrant made of 2 x 2
// blocks of v_mfma_f32_32x32x2_f32 (lane l holds A[l % 32][l / 32] and
// B[l / 32][l % 32]; accumulator register r of lane l is C[(r / 4) * 8 +
// (l / 32) * 4 + r % 4][l % 32]).  K advances 32 at a time through
// double-buffered LDS tiles stored [row][k] with rows padded to 36 floats;
// within a stage, the MFMA at substep t takes k = t on lanes 0-31 and
// k = 16 + t on lanes 32-63, so each lane reads 16 consecutive floats per
// block (four 16-byte LDS reads).  Global loads of the next stage are issued
// before the current stage's MFMAs.
//
// Split-K: the grid's z extent counts the K slices; slice z writes its own
// C plane (C + z * slice_stride), summed afterwards in a fixed order.
//
// Shapes: M, N multiples of 128 and K a multiple of 32 (the last K slice may
// be shorter), with the operands zero-padded to those sizes; the store is
// masked to m < m_valid, n < n_valid.
#include "cgh_internal.h"
#include "fold.h"

namespace cgh {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kBM = 128, kBN = 128, kBK = 32, kPitch = kBK + 4;
constexpr int kGemmThreads = 256;

// This thread's share of a 128 x 32 operand tile (16 floats), kept in named
// registers (no array, so nothing is ever placed in scratch memory).
struct Frag16 {
  float4 q0, q1, q2, q3;
};

template <bool KCONTIG>
__device__ __forceinline__ Frag16 load_tile(const float* __restrict__ src, int64_t ld, int row0,
                                            int k0) {
  const int t = threadIdx.x;
  Frag16 r;
  if (KCONTIG) {
    // 16-byte chunks c = t + 256 i (i = 0..3) of the tile's 1024, chunk c
    // holding k = 4 (c % 8) .. 4 (c % 8) + 3 of row c / 8: each wave
    // instruction reads 8 whole 128-byte row segments.
    const float* p = src + (int64_t)(row0 + t / 8) * ld + k0 + (t & 7) * 4;
    r.q0 = *reinterpret_cast<const float4*>(p);
    r.q1 = *reinterpret_cast<const float4*>(p + 32 * ld);
    r.q2 = *reinterpret_cast<const float4*>(p + 64 * ld);
    r.q3 = *reinterpret_cast<const float4*>(p + 96 * ld);
  } else {
    // M/N-contiguous: k = t % 32 and 16 consecutive rows from (t / 32) * 16
    // (k fastest across lanes keeps the transposing LDS stores conflict-free).
    const float* p = src + (int64_t)(k0 + (t & 31)) * ld + row0 + (t >> 5) * 16;
    r.q0 = *reinterpret_cast<const float4*>(p + 0);
    r.q1 = *reinterpret_cast<const float4*>(p + 4);
    r.q2 = *reinterpret_cast<const float4*>(p + 8);
    r.q3 = *reinterpret_cast<const float4*>(p + 12);
  }
  return r;
}

__device__ __forceinline__ void store_col(float* lds, int m, int k, float4 v) {
  lds[(m + 0) * kPitch + k] = v.x;
  lds[(m + 1) * kPitch + k] = v.y;
  lds[(m + 2) * kPitch + k] = v.z;
  lds[(m + 3) * kPitch + k] = v.w;
}

template <bool KCONTIG>
__device__ __forceinline__ void store_tile(float* __restrict__ lds, const Frag16& r) {
  const int t = threadIdx.x;
  if (KCONTIG) {
    float* p = lds + (t / 8) * kPitch + (t & 7) * 4;
    *reinterpret_cast<float4*>(p) = r.q0;
    *reinterpret_cast<float4*>(p + 32 * kPitch) = r.q1;
    *reinterpret_cast<float4*>(p + 64 * kPitch) = r.q2;
    *reinterpret_cast<float4*>(p + 96 * kPitch) = r.q3;
  } else {
    const int k = t & 31, m0 = (t >> 5) * 16;
    store_col(lds, m0 + 0, k, r.q0);
    store_col(lds, m0 + 4, k, r.q1);
    store_col(lds, m0 + 8, k, r.q2);
    store_col(lds, m0 + 12, k, r.q3);
  }
}

template <bool AK, bool BK, int FOLD>
__global__ __launch_bounds__(kGemmThreads, 2) void gemm_f32_kernel(
    const float* __restrict__ A, int64_t lda, const float* __restrict__ B, int64_t ldb,
    float* __restrict__ C, int64_t ldc, int64_t slice_stride, int k_slice, int k_total, int m_valid,
    int n_valid, FoldSpec fold) {
  __shared__ float As[2][kBM * kPitch];
  __shared__ float Bs[2][kBN * kPitch];
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
  const int m0 = (int)((tile % per_slice) / gridDim.x) * kBM;
  const int n0 = (int)(tile % gridDim.x) * kBN;
  const int kbeg = slice * k_slice;
  // the last slice may be shorter (never empty: checked at launch)
  const int nstages = (min(kbeg + k_slice, k_total) - kbeg) / kBK;

  floatx16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  Frag16 ra = load_tile<AK>(A, lda, m0, kbeg);
  Frag16 rb = load_tile<BK>(B, ldb, n0, kbeg);
  store_tile<AK>(As[0], ra);
  store_tile<BK>(Bs[0], rb);
  __syncthreads();

  const int kk = (lane >> 5) * 16;
  for (int s = 0; s < nstages; ++s) {
    const int buf = s & 1;
    if (s + 1 < nstages) {
      ra = load_tile<AK>(A, lda, m0, kbeg + (s + 1) * kBK);
      rb = load_tile<BK>(B, ldb, n0, kbeg + (s + 1) * kBK);
    }
    float fa[2][16], fb[2][16];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const float* pa = As[buf] + (wm * 64 + i * 32 + (lane & 31)) * kPitch + kk;
      const float* pb = Bs[buf] + (wn * 64 + i * 32 + (lane & 31)) * kPitch + kk;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 va = *reinterpret_cast<const float4*>(pa + 4 * q);
        const float4 vb = *reinterpret_cast<const float4*>(pb + 4 * q);
        fa[i][4 * q + 0] = va.x; fa[i][4 * q + 1] = va.y;
        fa[i][4 * q + 2] = va.z; fa[i][4 * q + 3] = va.w;
        fb[i][4 * q + 0] = vb.x; fb[i][4 * q + 1] = vb.y;
        fb[i][4 * q + 2] = vb.z; fb[i][4 * q + 3] = vb.w;
      }
    }
#pragma unroll
    for (int t = 0; t < 16; ++t)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[i][t], fb[j][t], acc[i][j], 0, 0, 0);
    if (s + 1 < nstages) {
      store_tile<AK>(As[buf ^ 1], ra);
      store_tile<BK>(Bs[buf ^ 1], rb);
    }
    __syncthreads();
  }

  if (FOLD) {
    const int64_t npts = (int64_t)gridDim.y * (kBM / 2);
    float4* dst = fold.out + ((int64_t)slice * gridDim.x + n0 / kBN) * npts + m0 / 2;
    fold_tile<FOLD>(acc, m0, n0, fold.rec, fold.plain, fold.n_valid, 1.0f, dst,
                    reinterpret_cast<float4*>(&As[0][0]));
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
        if (m < m_valid && n < n_valid) Cz[(int64_t)m * ldc + n] = acc[i][j][r];
      }
    }
}

}  // namespace

hipError_t launch_gemm_f32(bool a_kcontig, bool b_kcontig, const float* A, int64_t lda,
                           const float* B, int64_t ldb, float* C, int64_t ldc,
                           int64_t slice_stride, int M, int N, int K, int splits, int m_valid,
                           int n_valid, const FoldSpec* fold, hipStream_t s) {
  const dim3 grid(N / kBN, M / kBM, splits);
  // Slices of k_slice (a multiple of the stage depth), the last one shorter
  // but never empty.
  if (splits < 1 || K < kBK || K % kBK != 0) return hipErrorInvalidValue;
  const int k_slice = (K / kBK + splits - 1) / splits * kBK;
  if ((int64_t)(splits - 1) * k_slice >= K) return hipErrorInvalidValue;
  const FoldSpec f = fold ? *fold : FoldSpec{0, nullptr, nullptr, 0, nullptr};
  if (f.part != 0) {
    // The adjoint contractions: A M-contiguous; B N-contiguous (U) or
    // K-contiguous (Pm).
    if (a_kcontig) return hipErrorInvalidValue;
    if (f.part == 1 && !b_kcontig)
      hipLaunchKernelGGL((gemm_f32_kernel<false, false, 1>), grid, dim3(kGemmThreads), 0, s, A,
                         lda, B, ldb, C, ldc, slice_stride, k_slice, K, m_valid, n_valid, f);
    else if (f.part == 2 && b_kcontig)
      hipLaunchKernelGGL((gemm_f32_kernel<false, true, 2>), grid, dim3(kGemmThreads), 0, s, A,
                         lda, B, ldb, C, ldc, slice_stride, k_slice, K, m_valid, n_valid, f);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (a_kcontig && b_kcontig)
    hipLaunchKernelGGL((gemm_f32_kernel<true, true, 0>), grid, dim3(kGemmThreads), 0, s, A, lda,
                       B, ldb, C, ldc, slice_stride, k_slice, K, m_valid, n_valid, f);
  else if (!a_kcontig && !b_kcontig)
    hipLaunchKernelGGL((gemm_f32_kernel<false, false, 0>), grid, dim3(kGemmThreads), 0, s, A,
                       lda, B, ldb, C, ldc, slice_stride, k_slice, K, m_valid, n_valid, f);
  else if (!a_kcontig && b_kcontig)
    hipLaunchKernelGGL((gemm_f32_kernel<false, true, 0>), grid, dim3(kGemmThreads), 0, s, A, lda,
                       B, ldb, C, ldc, slice_stride, k_slice, K, m_valid, n_valid, f);
  else
    hipLaunchKernelGGL((gemm_f32_kernel<true, false, 0>), grid, dim3(kGemmThreads), 0, s, A, lda,
                       B, ldb, C, ldc, slice_stride, k_slice, K, m_valid, n_valid, f);
  return hipGetLastError();
}

}  // namespace cgh
