// Internal declarations shared by the library's HIP sources (not installed).
//
// Workspace layout, point-record formats and the launch wrappers of every
// kernel.  All kernels target gfx950 (CDNA4, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cgh {

constexpr int kWave = 64;
constexpr int kXcds = 8;

// MI355X dispatches workgroups round-robin over its 8 XCDs (linear id i runs
// on XCD i % 8), each with its own L2.  xcd_tile renumbers linear id i of n
// so that every XCD receives one contiguous range of tile indices: tiles
// that are neighbours in tile order (and share input data) then share an L2.
// A bijection on [0, n) for any n.
__device__ __forceinline__ unsigned xcd_tile(unsigned i, unsigned n) {
  const unsigned per = n / kXcds, rem = n % kXcds;
  const unsigned x = i % kXcds, k = i / kXcds;
  return x < rem ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

// Wave priority by progress.  The SIMD arbiter issues the oldest ready wave
// first, so the workgroups that share a CU from the launch on do not advance
// together: the first finishes long before the last, which then runs with few
// waves per SIMD.  A wave that starts at priority 3 and drops to 2, 1 and 0 as
// it passes each quarter of its loop yields to the waves behind it, so the
// workgroups of a CU finish close together.  Scheduling only: results do not
// change.  priority_step(i, n) is called at step i of a loop whose counter
// steps by one through [0, n).
__device__ __forceinline__ void priority_start() { __builtin_amdgcn_s_setprio(3); }
__device__ __forceinline__ void priority_step(int i, int n) {
  if (i == n / 4) __builtin_amdgcn_s_setprio(2);
  if (i == n / 2) __builtin_amdgcn_s_setprio(1);
  if (i == 3 * n / 4) __builtin_amdgcn_s_setprio(0);
}

// Workgroups of `threads` covering `count` items on a 1-D grid, or 0 when
// that exceeds the grid's x limit (2^31 - 1); launchers then return
// hipErrorInvalidValue instead of launching a truncated grid.
inline unsigned grid_blocks(int64_t count, int threads) {
  const int64_t b = (count + threads - 1) / threads;
  return (b < 1 || b > 0x7fffffff) ? 0u : (unsigned)b;
}

// ---------------------------------------------------------------- forward --
// Plain forward: a workgroup is 4 waves.  Lane l of every wave owns hologram
// column x0 + l; wave w owns kRows consecutive rows, so a workgroup covers 64
// columns x (4 * kRows) rows and every lane produces kRows pixels of one
// column.
constexpr int kFwdWaves = 4;
constexpr int kRows = 8;
constexpr int kFwdThreads = kFwdWaves * kWave;
constexpr int kFwdRowsPerWG = kFwdWaves * kRows;
// Points are processed in unrolled groups of kUnroll; the compensated
// forward stages kTile points at a time in LDS.  The point arrays in the
// workspace are padded to a multiple of kPointPad with zero-amplitude
// points.
constexpr int kUnroll = 4;
constexpr int kTile = 64;
constexpr int kTilePitch = kWave + 1;

// Compensated forward: a workgroup of kCompWaves waves covers 64 columns x
// (kCompWaves * kCompRows) rows; each wave owns kCompRows rows.  Its x-phases,
// row phases and amplitudes are staged in LDS a tile of kTile points at a
// time (x-phase rows padded to kTilePitch floats, so that lane-per-point
// writes hit distinct banks).  Overridable at build time for tuning
// experiments.
#ifndef CGH_COMP_WAVES
#define CGH_COMP_WAVES 8
#endif
#ifndef CGH_COMP_ROWS
#define CGH_COMP_ROWS 4
#endif
constexpr int kCompWaves = CGH_COMP_WAVES;
constexpr int kCompRows = CGH_COMP_ROWS;
constexpr int kCompThreads = kCompWaves * kWave;
constexpr int kCompRowsPerWG = kCompWaves * kCompRows;
static_assert(kWave % kCompWaves == 0, "x-phase fill splits the 64 columns over the waves");
static_assert(kTile % 16 == 0, "the inner loop takes 16 points per iteration");
// The compensated forward reads its x-phases from a column table
// [fwd_gx * 64][npad] while that takes at most kCompColTabMaxBytes, else it
// forms them per workgroup (the same values).  Every row block of
// workgroups reads the whole table again, so it pays only while the table
// stays in the 256 MB Infinity Cache (measured: 252 MB faster, 503 MB 10%
// slower than forming the values).
constexpr int64_t kCompColTabMaxBytes = int64_t(256) << 20;
constexpr int kPointPad = 64;

// Recurrence forward (Eq. (2)): lane l of a wave covers K consecutive pixels
// of R rows, a group of kRecWaves waves is stacked in y, and a workgroup holds
// S such groups that split the points between them; points are taken
// kRecUnroll at a time (scalar loads one group ahead).  (K, R) comes from a
// small set of instantiations chosen per shape by rec_shape().
constexpr int kRecWaves = 4;
constexpr int kRecThreads = kRecWaves * kWave;
constexpr int kRecUnroll = 4;
static_assert(kPointPad % (2 * kRecUnroll) == 0, "point padding holds whole group pairs");

// ---------------------------------------------------------------- adjoint --
// An adjoint wave holds 64 points (one per lane) and sweeps a run of
// strip-rows: the hologram is cut into strips of kAdjCols columns, and the
// strip-rows (strip-major: strip s, row r -> s * ny + r) of every point group
// are split into equal contiguous runs, one per wave.  G is broadcast to the
// wave through scalar loads, one strip row at a time.
constexpr int kAdjCols = 32;
// Phase arithmetic of the adjoint kernel (Plan::adj_kind): the plain FP32
// phase, the compensated axis phases, or the recurrence of Eq. (2) along the
// strip row.  The compensated kind reads the cosine and sine of each row's
// y-phase from a table [ny][npad] and each strip column's x-phase from a table
// [nsx * kAdjCols][npad], both built by one precompute launch (the same
// values it would form itself, once per row or column and point instead of
// once per strip and point); when either table would exceed
// kAdjRowTabMaxBytes the kernel forms them inline instead
// (kAdjCompensatedInline: the same values, so the same result whenever the
// launch takes the same run count; its lower occupancy can give it another).
constexpr int kAdjPlain = 0;
constexpr int kAdjCompensated = 1;
constexpr int kAdjRecurrence = 2;
constexpr int kAdjCompensatedInline = 3;
constexpr int64_t kAdjRowTabMaxBytes = int64_t(512) << 20;
constexpr int kAdjThreads = kWave;
// At launch the number of runs is chosen so that kAdjRounds rounds of
// resident waves (CUs x resident waves per CU, from the occupancy query)
// cover the whole hologram with equal work per wave, and runs hold at least
// kAdjMinRun strip-rows.  The partial-sum buffer is sized for kAdjRounds
// rounds at up to 8 resident waves per SIMD on 256 CUs (kAdjMaxWaves), so
// the last round is never cut short at any occupancy a kernel reaches.
#ifndef CGH_ADJ_ROUNDS
#define CGH_ADJ_ROUNDS 3
#endif
constexpr int kAdjRounds = CGH_ADJ_ROUNDS;
constexpr int kAdjMaxWaves = kAdjRounds * 256 * 4 * 8;
constexpr int kAdjMinRun = 8;
// Second passes: kFinSlices threads per point add interleaved subsets of the
// partial planes (the separable finalize), and the direct adjoint's finalize
// spreads its many run partials over kAdjFinSlices threads for each of
// kAdjFinPoints points per workgroup.
constexpr int kFinSlices = 16;
constexpr int kAdjFinPoints = 16;
constexpr int kAdjFinSlices = 64;

// The adjoint's order of strip-rows.  The (strip, row) space is cut into
// kXcds blocks, H strip groups x B row bands (H B = kXcds): block
// beta = h B + b covers strips [h sh, min(nsx, (h + 1) sh)) and rows
// [b br, min(ny, (b + 1) br)), strip-major inside, and off[beta] is its first
// index in the order (off[kXcds] = nsx ny).  Runs are equal ranges of this
// order and xcd_tile places consecutive runs on one XCD, so each XCD works
// through about one block: it reads only its band of the row table and its
// strips' share of the column table.  H is chosen to minimise the bytes the
// XCDs read between them: H row tables and B column tables.
struct AdjOrder {
  int64_t off[kXcds + 1];
  int sh, br, B;
};

// Point records, all produced on the device by the prep kernel from the FP32
// inputs with FP64 arithmetic.
//
//  plain   float4 {x, y, Prev, A}         Prev = fl32(p^2 / (2 lambda z)),
//                                           the phase coefficient in
//                                           revolutions per pixel^2.
//  axis    float[8] {c, Ph, Pl, b, d, A, v, 0} per axis (x then y arrays):
//          c = rint(v) (v = x_j or y_j), f = v - c (exact),
//          Ph = fl32(Prev), Pl = fl32(Prev - Ph),
//          b = fl32(-2 Prev f), d = fl32(Prev f^2),
//          so that Prev (h - v)^2 = (Ph + Pl) m^2 + b m + d with m = h - c,
//          an integer: m^2 is exact in FP32 for |m| < 4096.
//  f64     double4 {x, y, Prev, A}.
constexpr int kAxisRec = 8;

struct Workspace {
  float4* plain;   // [npad]
  float* amp;      // [npad] amplitudes A_j (contiguous, for scalar loads)
  float* xrec;     // [npad][8]
  float* yrec;     // [npad][8]
  double4* rec64;  // [npad]
  float* ytab;     // forward, compensated: [groups][npad][kCompRows]
  float* xtab;     // forward, compensated (optional): [fwd_gx * 64][npad] x-phases
  float2* rtab;    // adjoint, compensated: [ny][npad] {cos, sin of the y-phase}
  float* ctab;     // adjoint, compensated: [nsx * kAdjCols][npad] x-phases
  float* partial;  // adjoint: [regions][npad][4]
  float* gpad;     // adjoint: G copied to a [ny][nsx*kAdjCols] zero-padded grid
  // separable variant (tables of k2 = 2 * npad floats per row / column)
  float* sep_x;    // [nxp][k2]  (cX, sX) per point
  float* sep_y;    // [nyp][k2]  forward: (A cY, -A sY); adjoint: (cY, sY)
  float* sep_c;    // forward split-K planes [splits][nyp][nxp]
  float* sep_g;    // adjoint: G zero-padded to [nyp][nxp]
  float4* fold_x;  // adjoint: x-part fold planes [splits_u][nxp / 128][npad]
  float4* fold_y;  // adjoint: y-part fold planes [splits_p][nyp / 128][npad]
  // half-precision separable variants: 16-bit planes (hi, lo) and scales
  uint16_t *hx_hi, *hx_lo;   // forward [nxp][k2]; adjoint transposed [k2][nxp]
  uint16_t *hy_hi, *hy_lo;   // forward [nyp][k2] (with A); adjoint [k2][nyp]
  uint16_t *hg_hi, *hg_lo;   // adjoint: G [nyp][nxp]
  uint16_t *hgt_hi, *hgt_lo; // adjoint: G^T [nxp][nyp]
  unsigned* hmax;            // largest |A| (forward) or |G| (adjoint), as float bits
};

struct Plan {
  int64_t n, npad;
  int32_t nx, ny;
  int32_t variant, op;
  // forward
  int32_t fwd_gx, fwd_gy, comp_gy, groups;
  bool comp_xtab;  // the compensated forward has its column table
  int32_t rec_k, rec_r, rec_s, rec_gx, rec_gy;  // recurrence forward shape, split, grid
  // adjoint: runs of strip-rows per point group (regions = the most runs the
  // partial buffer holds; the launch may use fewer)
  int32_t nsx, regions, ngroups, adj_kind;
  int64_t strip_rows;
  AdjOrder adj_order;
  bool need_gpad;
  // separable variant
  int32_t nxp, nyp, sep_splits, sep_splits_u, sep_splits_p;
  int64_t k2;
  size_t off_sep_x, off_sep_y, off_sep_c, off_sep_g, off_fold_x, off_fold_y;
  size_t off_hx, off_hy, off_hg, off_hgt, off_hmax;  // half variants (hi plane; lo follows)
  size_t off_plain, off_amp, off_xrec, off_yrec, off_rec64, off_ytab, off_xtab, off_rtab,
      off_ctab, off_partial, off_gpad, total;
};

// col_table = false plans the compensated forward without its column table
// (the kernel then forms the x-phases itself: the same bits, less scratch).
Plan make_plan(int64_t n, int32_t nx, int32_t ny, int32_t variant, int32_t op,
               bool col_table = true);
Workspace carve(const Plan& p, void* base);

// Launch wrappers (return the hipError_t of the launch).
// The prep kernel also clears w.hmax (when the plan has one) for the
// abs-max reduction that follows it on the stream.
hipError_t launch_prep(const float* x, const float* y, const float* z, const float* a, int64_t n,
                       int64_t npad, double pitch, double wavelength, const Workspace& w,
                       bool want64, hipStream_t s);
hipError_t launch_fill_zero_f32(float* p, int64_t count, hipStream_t s);
hipError_t launch_fill_zero_f64(double* p, int64_t count, hipStream_t s);
// The compensated forward's precompute: the point records (as launch_prep),
// the per-row y-phase table and (when planned) the column x-phase table, in
// one launch.
hipError_t launch_prep_ytab(const float* x, const float* y, const float* z, const float* a,
                            double pitch, double wavelength, const Plan& p, const Workspace& w,
                            hipStream_t s);
// The compensated adjoint's tables, from the FP32 inputs in one launch: for
// every row y_h and point j the cosine and sine of the compensated y-phase of
// y_h, and for every strip column x_h and point j the compensated x-phase of
// x_h.
hipError_t launch_prep_rtab(const float* x, const float* y, const float* z, const float* a,
                            double pitch, double wavelength, const Plan& p, const Workspace& w,
                            hipStream_t s);
hipError_t launch_fwd_plain(const Plan& p, const Workspace& w, float* out, hipStream_t s);
// With target and residual (both or neither) the compensated forward also
// writes residual = out - target in its store.
hipError_t launch_fwd_comp(const Plan& p, const Workspace& w, float* out, hipStream_t s,
                           const float* target = nullptr, float* residual = nullptr);
// residual = hologram - target over count elements (the other forwards).
hipError_t launch_residual(const float* hologram, const float* target, float* residual,
                           int64_t count, hipStream_t s);
hipError_t launch_fwd_rec(const Plan& p, const Workspace& w, float* out, hipStream_t s);
hipError_t launch_fwd_f64(const Plan& p, const Workspace& w, double* out, hipStream_t s);
hipError_t launch_pad_g(const Plan& p, const float* g, float* gpad, hipStream_t s);
// Optional epilogue of the adjoint GEMMs (fold.h): instead of storing its
// tile, each block folds it into per-point sums, written as float4 planes
// out[(z * (N / 128) + column tile) * (M / 2) + point] for K slice z.
struct FoldSpec {
  int part;             // 1: x part (U), 2: y part (Pm)
  const float* rec;     // axis records of the folded axis (xrec or yrec)
  const float4* plain;  // point records {x, y, Prev, A}
  int n_valid;          // nx or ny
  float4* out;
};
// FP32 matrix-core GEMM (gemm.hip): C[m][n] = sum_k A(m, k) B(n, k), split
// over `splits` K slices written to C + z * slice_stride (or folded, when
// fold is given: then A must be M-contiguous, as in the adjoint).  M, N
// multiples of 128; K a multiple of 32; slices of ceil(K / 32 / splits)
// chunks of 32, the last one shorter and never empty (else an error).
hipError_t launch_gemm_f32(bool a_kcontig, bool b_kcontig, const float* A, int64_t lda,
                           const float* B, int64_t ldb, float* C, int64_t ldc,
                           int64_t slice_stride, int M, int N, int K, int splits, int m_valid,
                           int n_valid, const FoldSpec* fold, hipStream_t s);
// Separable variant (separable.hip).
// Grid of the per-axis table kernels: x over points (256 per workgroup), y a
// few workgroup rows that stride over the table rows.
dim3 table_grid(int64_t npad, int rows);
// Both axis tables (x: (cX, sX) [nxp][k2]; y: (A cY, -A sY) with amp, else
// (cY, sY), [nyp][k2]) in one launch.
hipError_t launch_sep_tables(const float* xrec, const float* yrec, const float* amp, int64_t npad,
                             int nx, int nxp, int ny, int nyp, float* tab_x, float* tab_y,
                             hipStream_t s);
hipError_t launch_sep_sum_slices(const float* C, int splits, int64_t slice_stride, int64_t ldc,
                                 int nx, int ny, float* out, hipStream_t s);
hipError_t launch_sep_pad(const float* g, int nx, int ny, int rows_pad, int cols_pad, float* gp,
                          hipStream_t s);
// Sums the fold planes of both adjoint GEMMs per point in a fixed order
// (FP64) and scales them into the gradients.
hipError_t launch_sep_finalize(const Plan& p, const Workspace& w, const float* z, const float* a,
                               double pitch, double wavelength, float* gx, float* gy, float* gz,
                               float* ga, hipStream_t s);
// Half-precision matrix-core GEMM (gemm_half.hip), K-contiguous 16-bit
// planes; formats:
constexpr int kHalfF16 = 0;    // one fp16 plane per operand
constexpr int kHalfBF16 = 1;   // one bf16 plane per operand
constexpr int kHalfF16x3 = 2;  // fp16 hi + lo planes, hi*hi + hi*lo + lo*hi
hipError_t launch_gemm_half(int mode, const uint16_t* Ah, const uint16_t* Al, int64_t lda,
                            const uint16_t* Bh, const uint16_t* Bl, int64_t ldb, float* C,
                            int64_t ldc, int64_t slice_stride, int M, int N, int K, int splits,
                            int m_valid, int n_valid, const unsigned* scale_max,
                            const FoldSpec* fold, hipStream_t s);

// Power-of-two scale 2^e >= m for the largest magnitude m, given as the bits
// of the non-negative float m (1 when m is 0 or not finite).  Dividing an
// operand by it maps it into [-1, 1] exactly (only the exponent changes).
__device__ __forceinline__ float pow2_scale(unsigned max_bits) {
  const float m = __uint_as_float(max_bits);
  if (!(m > 0.0f) || !(m < 3.0e38f)) return 1.0f;
  int e;
  const float f = frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
  (void)f;
  return ldexpf(1.0f, e);
}

// Separable variants with half-precision contractions (separable_half.hip).
// launch_absmax raises *out (cleared beforehand, by the prep kernel) to the
// float bits of max |v|.
hipError_t launch_absmax(const float* v, int64_t count, unsigned* out, hipStream_t s);
// Forward operands: X [nxp][k2] and Y [nyp][k2] (with A_j / 2^e) planes.
hipError_t launch_sep_tables_half(int mode, const Plan& p, const Workspace& w, hipStream_t s);
// Adjoint operands: Xt [k2][nxp], Yt [k2][nyp], and G / 2^e as G [nyp][nxp]
// and Gt [nxp][nyp] planes, in one launch.
hipError_t launch_sep_adj_operands_half(int mode, const Plan& p, const Workspace& w,
                                        const float* g, hipStream_t s);
// Runs per point group for this launch (<= p.regions), from the occupancy of
// the adjoint kernel on the current device.
int adj_runs(const Plan& p);
hipError_t launch_adj_partial(const Plan& p, const Workspace& w, const float* x, const float* y,
                              const float* z, const float* a, double pitch, double wavelength,
                              const float* g, int64_t ldg, int runs, hipStream_t s);
hipError_t launch_adj_finalize(const Plan& p, const Workspace& w, const float* z, const float* a,
                               double pitch, double wavelength, int runs, float* gx, float* gy,
                               float* gz, float* ga, hipStream_t s);

}  // namespace cgh
