// Per-point fold of the separable adjoint, applied by a GEMM block to its own
// 128 x 128 accumulator tile (the contractions of separable.hip):
//
//   x part (tile of U: row 2j = U_j(x) = sum_y G cY, row 2j + 1 = V_j(x) =
//   sum_y G sY; columns x):
//     s0 = sum_x cX U - sX V                  (the Sc term)
//     s1 = sum_x dx (sX U + cX V),  s2 = sum_x dx^2 (sX U + cX V)
//   y part (tile of Pm: row 2j = sum_x G cX, row 2j + 1 = sum_x G sX;
//   columns y):
//     s1 = sum_y dy (cY Psin + sY Pcos),  s2 = sum_y dy^2 (cY Psin + sY Pcos)
//
// with (c, s) the cosine and sine of the compensated axis phase of point j at
// the column and d = column - x_j (or y_j).  Each fold is linear in the tile,
// so every split-K slice folds its own partial contraction.
//
// Accumulator layout (v_mfma_f32_32x32x*): register r of lane l in block
// (i, jb) is row wm * 64 + i * 32 + (r / 4) * 8 + (l / 32) * 4 + r % 4 and
// column wn * 64 + jb * 32 + l % 32 of the tile, so registers r, r + 1 (r
// even) of a lane hold the cosine and sine rows of one point at one column.
// A wave sums its 64 columns per point (the lane's two columns, then a
// butterfly over the 32 lanes of each half-wave); the two waves that share
// rows (wn = 0, 1) are added in that order through LDS, and the block writes
// one float4 {s0, s1, s2, 0} per point of the tile to fold_out[point - m0 /
// 2] (the caller points fold_out at this block's (slice, column tile) plane,
// offset by the tile's first point).  Deterministic.
#pragma once

#include "cgh_internal.h"
#include "phase.h"

namespace cgh {

typedef float foldx16 __attribute__((ext_vector_type(16)));

// FOLD: 1 = x part, 2 = y part.  m0: first row of the tile (twice its first
// point); n0: first column; rec: the axis records of the folded axis
// (xrec for the x part, yrec for the y part); plain: point records (x_j,
// y_j); n_valid: columns from it on (padding) add nothing and are skipped;
// alpha: scale applied to the accumulators first; sums: 128 float4 of LDS
// that no wave reads or writes any more (the GEMM's tile buffers after its
// last barrier), used as [wm][wn][point of the wave's 32].
template <int FOLD>
__device__ __forceinline__ void fold_tile(const foldx16 (&acc)[2][2], int m0, int n0,
                                          const float* __restrict__ rec,
                                          const float4* __restrict__ plain, int n_valid,
                                          float alpha, float4* __restrict__ fold_out,
                                          float4* __restrict__ sums) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int half = lane >> 5;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int r = 0; r < 16; r += 2) {
      // this lane's point: local index p of the wave's 32, global j
      const int p = i * 16 + (r >> 2) * 4 + half * 2 + ((r & 3) >> 1);
      const int j = m0 / 2 + wm * 32 + p;
      const float* q = rec + (int64_t)j * kAxisRec;
      const float4 pj = plain[j];
      const float pc = FOLD == 1 ? pj.x : pj.y;
      float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) {
        const int h = n0 + wn * 64 + jb * 32 + (lane & 31);
        if (h < n_valid) {
          const float even = alpha * acc[i][jb][r], odd = alpha * acc[i][jb][r + 1];
          const float phi = axis_phase((float)h, q[0], q[1], q[2], q[3], q[4]);
          const float c = cos_rev(phi), s = sin_rev(phi);
          const float d = (float)h - pc;
          float w;
          if (FOLD == 1) {
            s0 = __builtin_fmaf(c, even, s0);
            s0 = __builtin_fmaf(-s, odd, s0);
            w = __builtin_fmaf(s, even, c * odd);
          } else {
            w = __builtin_fmaf(c, odd, s * even);
          }
          s1 = __builtin_fmaf(d, w, s1);
          s2 = __builtin_fmaf(d * d, w, s2);
        }
      }
#pragma unroll
      for (int off = 1; off < 32; off <<= 1) {
        s0 += __shfl_xor(s0, off, 64);
        s1 += __shfl_xor(s1, off, 64);
        s2 += __shfl_xor(s2, off, 64);
      }
      if ((lane & 31) == 0) sums[(wm * 2 + wn) * 32 + p] = make_float4(s0, s1, s2, 0.f);
    }
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int w = threadIdx.x >> 5, p = threadIdx.x & 31;
    const float4 a = sums[(w * 2) * 32 + p], b = sums[(w * 2 + 1) * 32 + p];
    fold_out[w * 32 + p] = make_float4(a.x + b.x, a.y + b.y, a.z + b.z, 0.f);
  }
}

}  // namespace cgh
