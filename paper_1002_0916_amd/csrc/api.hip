// C ABI of the library (declared in include/cgh.h): argument checks,
// workspace planning, kernel sequencing on the caller's stream, and optional
// HIP-event timing of the main kernels.
#include <math.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/cgh.h"
#include "cgh_internal.h"

namespace cgh {

namespace {

// 4,000,000 points pad to 62,500 waves of 64, within the 65,535 limit of the
// adjoint grid's y dimension (the regions go in x).
constexpr int64_t kMaxPoints = 4000000;
constexpr int32_t kMaxSide = 1 << 20;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Split-K count for a GEMM of `tiles` 128 x 128 output tiles and contraction
// length k (a multiple of 32).  A slice holds ceil(k / 32 / splits) stages of
// 32 (the last slice fewer, never none) and at least 8 stages.  The count
// minimises a simple time model in units of one workgroup stage: rounds of
// 512 resident GEMM workgroups (two per CU on 256 CUs) times the stages per
// slice, plus the partial planes (each tile of each slice costs about six
// stages of traffic, spread over the 512 slots).
inline int gemm_splits(int64_t tiles, int64_t k) {
  const int64_t chunks = k / 32;
  int best = 1;
  double best_time = 0.0;
  for (int s = 1; s <= 512; ++s) {
    const int64_t per = (chunks + s - 1) / s;
    if (s > 1 && per < 8) break;
    if ((chunks + per - 1) / per != s) continue;  // some slice would be empty
    const int64_t rounds = (tiles * s + 511) / 512;
    const double time = (double)(rounds * per) + 6.0 * (double)(s * tiles) / 512.0;
    if (s == 1 || time < best_time) {
      best_time = time;
      best = s;
    }
  }
  return best;
}

// Shape of the recurrence forward: K pixels x R rows per lane, from the
// instantiated set K in {4, 6, 8}, R in {1, 2, 4}.  The choice minimises a
// time model in issue slots per SIMD: the workgroups each of the 256 CUs runs
// (ceil(workgroups / 256); a workgroup is one wave per SIMD) times the
// interactions per lane per point (K R) times the slots per interaction,
//   4 + 1/R + (4 R + 7) / (K R)
// (cosine 2, the Gamma add and the accumulate per interaction; delta's add
// once per column step for R rows; dx, dx^2, delta_0 and Delta once per point
// and lane; Gamma_0 once per row).  CGH_REC_SHAPE = 10 K + R forces a shape
// (tuning builds only).
inline void rec_shape(int32_t nx, int32_t ny, int32_t& k_out, int32_t& r_out) {
#ifdef CGH_REC_SHAPE
  (void)nx;
  (void)ny;
  k_out = CGH_REC_SHAPE / 10;
  r_out = CGH_REC_SHAPE % 10;
#else
  static const int kShapes[][2] = {{8, 4}, {8, 2}, {8, 1}, {6, 4}, {6, 2},
                                   {6, 1}, {4, 4}, {4, 2}, {4, 1}};
  double best = 0.0;
  for (const auto& sh : kShapes) {
    const int K = sh[0], R = sh[1];
    const int64_t wgs = ceil_div(nx, (int64_t)kWave * K) * ceil_div(ny, (int64_t)kRecWaves * R);
    const double slots = 4.0 + 1.0 / R + (4.0 * R + 7.0) / (K * R);
    const double t = (double)ceil_div(wgs, 256) * K * R * slots;
    if (best == 0.0 || t < best) {
      best = t;
      k_out = K;
      r_out = R;
    }
  }
#endif
}

inline bool valid_variant(int32_t v) { return v >= CGH_PLAIN && v <= CGH_RECURRENCE; }

// The 16-bit GEMM format of a half-precision separable variant, or -1.
inline int half_mode(int32_t v) {
  switch (v) {
    case CGH_SEPARABLE_F16X3:
      return kHalfF16x3;
    case CGH_SEPARABLE_F16:
      return kHalfF16;
    case CGH_SEPARABLE_BF16:
      return kHalfBF16;
    default:
      return -1;
  }
}

inline bool is_separable(int32_t v) { return v == CGH_SEPARABLE || half_mode(v) >= 0; }

}  // namespace

Plan make_plan(int64_t n, int32_t nx, int32_t ny, int32_t variant, int32_t op,
               bool col_table) {
  Plan p{};
  p.n = n;
  p.nx = nx;
  p.ny = ny;
  p.variant = variant;
  p.op = op;
  p.npad = ceil_div(n > 0 ? n : 1, kPointPad) * kPointPad;
  p.fwd_gx = (int32_t)ceil_div(nx, kWave);
  p.fwd_gy = (int32_t)ceil_div(ny, kFwdRowsPerWG);
  p.comp_gy = (int32_t)ceil_div(ny, kCompRowsPerWG);
  p.groups = p.comp_gy * kCompWaves;
  p.comp_xtab = col_table && (int64_t)p.fwd_gx * kWave * p.npad <=
                                 kCompColTabMaxBytes / (int64_t)sizeof(float);
  rec_shape(nx, ny, p.rec_k, p.rec_r);
  p.rec_gx = (int32_t)ceil_div(nx, (int64_t)kWave * p.rec_k);
  p.rec_gy = (int32_t)ceil_div(ny, (int64_t)kRecWaves * p.rec_r);
  // Points split over two wave groups per workgroup: measured 1-3% faster
  // (more waves per SIMD) at every workload shape, never slower.
  // CGH_REC_SPLIT = 1 or 2 forces it (tuning builds only).
#ifdef CGH_REC_SPLIT
  p.rec_s = CGH_REC_SPLIT;
#else
  p.rec_s = 2;
#endif
  p.ngroups = (int32_t)(p.npad / kWave);
  const bool rtab_fits =
      (int64_t)ny * p.npad <= kAdjRowTabMaxBytes / (int64_t)sizeof(float2) &&
      ceil_div(nx, kAdjCols) * kAdjCols * p.npad <= kAdjRowTabMaxBytes / (int64_t)sizeof(float);
  p.adj_kind = variant == CGH_COMPENSATED  ? (rtab_fits ? kAdjCompensated : kAdjCompensatedInline)
               : variant == CGH_RECURRENCE ? kAdjRecurrence
                                           : kAdjPlain;
  p.nsx = (int32_t)ceil_div(nx, kAdjCols);
  p.strip_rows = (int64_t)p.nsx * ny;
  {
    int best_h = 1;
    double best = 0.0;
    for (int h = 1; h <= kXcds; h *= 2) {
      const double bytes = (double)h * ny * 8.0 + (double)(kXcds / h) * p.nsx * kAdjCols * 4.0;
      if (h == 1 || bytes < best) {
        best = bytes;
        best_h = h;
      }
    }
    AdjOrder& o = p.adj_order;
    o.B = kXcds / best_h;
    o.sh = (int)ceil_div(p.nsx, best_h);
    o.br = (int)ceil_div(ny, o.B);
    o.off[0] = 0;
    for (int beta = 0; beta < kXcds; ++beta) {
      const int h = beta / o.B, b = beta % o.B;
      const int64_t strips = std::max<int64_t>(0, std::min<int64_t>(p.nsx, (int64_t)(h + 1) * o.sh) - (int64_t)h * o.sh);
      const int64_t rows = std::max<int64_t>(0, std::min<int64_t>(ny, (int64_t)(b + 1) * o.br) - (int64_t)b * o.br);
      o.off[beta + 1] = o.off[beta] + strips * rows;
    }
  }
  int64_t runs = ceil_div(kAdjMaxWaves, p.ngroups);
  const int64_t max_runs = ceil_div(p.strip_rows, kAdjMinRun);
  if (runs > max_runs) runs = max_runs;
  if (runs < 1) runs = 1;
  p.regions = (int32_t)runs;
  p.need_gpad = (nx % kAdjCols) != 0;

  // Separable variant: padded GEMM shapes and split-K counts.
  p.nxp = (int32_t)ceil_div(nx, 128) * 128;
  p.nyp = (int32_t)ceil_div(ny, 128) * 128;
  p.k2 = 2 * p.npad;
  p.sep_splits = gemm_splits((int64_t)(p.nyp / 128) * (p.nxp / 128), p.k2);
  p.sep_splits_u = gemm_splits((p.k2 / 128) * (p.nxp / 128), p.nyp);
  p.sep_splits_p = gemm_splits((p.k2 / 128) * (p.nyp / 128), p.nxp);

  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t np = (size_t)p.npad;
  p.off_plain = take(np * sizeof(float4));
  p.off_amp = take(np * sizeof(float));
  p.off_xrec = take(np * kAxisRec * sizeof(float));
  p.off_yrec = take(np * kAxisRec * sizeof(float));
  p.off_rec64 = op == CGH_OP_FORWARD_F64 ? take(np * sizeof(double4)) : 0;
  p.off_ytab = (op == CGH_OP_FORWARD && variant == CGH_COMPENSATED)
                   ? take((size_t)p.groups * np * kCompRows * sizeof(float))
                   : 0;
  p.off_xtab = (op == CGH_OP_FORWARD && variant == CGH_COMPENSATED && p.comp_xtab)
                   ? take((size_t)p.fwd_gx * kWave * np * sizeof(float))
                   : 0;
  const bool direct_adj = op == CGH_OP_BACKWARD && !is_separable(variant);
  p.off_rtab = (direct_adj && p.adj_kind == kAdjCompensated)
                   ? take((size_t)ny * np * sizeof(float2))
                   : 0;
  p.off_ctab = (direct_adj && p.adj_kind == kAdjCompensated)
                   ? take((size_t)p.nsx * kAdjCols * np * sizeof(float))
                   : 0;
  p.off_partial = direct_adj ? take((size_t)p.regions * np * sizeof(float4)) : 0;
  p.off_gpad = (direct_adj && p.need_gpad)
                   ? take((size_t)p.nsx * kAdjCols * (size_t)ny * sizeof(float))
                   : 0;
  const bool sep = is_separable(variant) && op != CGH_OP_FORWARD_F64;
  const bool f32 = sep && variant == CGH_SEPARABLE;
  const int hm = sep ? half_mode(variant) : -1;
  const bool fwd = op == CGH_OP_FORWARD, bwd = op == CGH_OP_BACKWARD;
  const size_t k2 = (size_t)p.k2;
  const size_t nxp = (size_t)p.nxp, nyp = (size_t)p.nyp;
  p.off_sep_x = f32 ? take(nxp * k2 * sizeof(float)) : 0;
  p.off_sep_y = f32 ? take(nyp * k2 * sizeof(float)) : 0;
  p.off_sep_g = (f32 && bwd) ? take(nyp * nxp * sizeof(float)) : 0;
  p.off_sep_c = (sep && fwd && p.sep_splits > 1)
                    ? take((size_t)p.sep_splits * nyp * nxp * sizeof(float))
                    : 0;
  p.off_fold_x =
      (sep && bwd) ? take((size_t)p.sep_splits_u * (nxp / 128) * np * sizeof(float4)) : 0;
  p.off_fold_y =
      (sep && bwd) ? take((size_t)p.sep_splits_p * (nyp / 128) * np * sizeof(float4)) : 0;
  // 16-bit planes: hi, then (f16x3) lo at the next 256-byte boundary.
  const size_t planes = hm == kHalfF16x3 ? 2 : 1;
  auto take_planes = [&](size_t elems) { return take(planes * align256(elems * 2)); };
  p.off_hx = hm >= 0 ? take_planes(nxp * k2) : 0;
  p.off_hy = hm >= 0 ? take_planes(nyp * k2) : 0;
  p.off_hg = (hm >= 0 && bwd) ? take_planes(nyp * nxp) : 0;
  p.off_hgt = (hm >= 0 && bwd) ? take_planes(nyp * nxp) : 0;
  p.off_hmax = hm >= 0 ? take(sizeof(unsigned)) : 0;
  p.total = off;
  return p;
}

Workspace carve(const Plan& p, void* base) {
  char* b = (char*)base;
  Workspace w{};
  w.plain = (float4*)(b + p.off_plain);
  w.amp = (float*)(b + p.off_amp);
  w.xrec = (float*)(b + p.off_xrec);
  w.yrec = (float*)(b + p.off_yrec);
  w.rec64 = p.op == CGH_OP_FORWARD_F64 ? (double4*)(b + p.off_rec64) : nullptr;
  w.ytab = (p.op == CGH_OP_FORWARD && p.variant == CGH_COMPENSATED) ? (float*)(b + p.off_ytab)
                                                                     : nullptr;
  w.xtab = (p.op == CGH_OP_FORWARD && p.variant == CGH_COMPENSATED && p.comp_xtab)
               ? (float*)(b + p.off_xtab)
               : nullptr;
  const bool direct_adj = p.op == CGH_OP_BACKWARD && !is_separable(p.variant);
  w.rtab = (direct_adj && p.adj_kind == kAdjCompensated) ? (float2*)(b + p.off_rtab) : nullptr;
  w.ctab = (direct_adj && p.adj_kind == kAdjCompensated) ? (float*)(b + p.off_ctab) : nullptr;
  w.partial = direct_adj ? (float*)(b + p.off_partial) : nullptr;
  w.gpad = (direct_adj && p.need_gpad) ? (float*)(b + p.off_gpad) : nullptr;
  const bool sep = is_separable(p.variant) && p.op != CGH_OP_FORWARD_F64;
  const bool f32 = sep && p.variant == CGH_SEPARABLE;
  const int hm = sep ? half_mode(p.variant) : -1;
  const bool fwd = p.op == CGH_OP_FORWARD, bwd = p.op == CGH_OP_BACKWARD;
  w.sep_x = f32 ? (float*)(b + p.off_sep_x) : nullptr;
  w.sep_y = f32 ? (float*)(b + p.off_sep_y) : nullptr;
  w.sep_g = (f32 && bwd) ? (float*)(b + p.off_sep_g) : nullptr;
  w.sep_c = (sep && fwd && p.sep_splits > 1) ? (float*)(b + p.off_sep_c) : nullptr;
  w.fold_x = (sep && bwd) ? (float4*)(b + p.off_fold_x) : nullptr;
  w.fold_y = (sep && bwd) ? (float4*)(b + p.off_fold_y) : nullptr;
  if (hm >= 0) {
    const size_t k2 = (size_t)p.k2, nxp = (size_t)p.nxp, nyp = (size_t)p.nyp;
    const bool split = hm == kHalfF16x3;
    auto planes = [&](size_t off, size_t elems, uint16_t*& hi, uint16_t*& lo) {
      hi = (uint16_t*)(b + off);
      lo = split ? (uint16_t*)(b + off + align256(elems * 2)) : nullptr;
    };
    planes(p.off_hx, nxp * k2, w.hx_hi, w.hx_lo);
    planes(p.off_hy, nyp * k2, w.hy_hi, w.hy_lo);
    if (bwd) {
      planes(p.off_hg, nyp * nxp, w.hg_hi, w.hg_lo);
      planes(p.off_hgt, nyp * nxp, w.hgt_hi, w.hgt_lo);
    }
    w.hmax = (unsigned*)(b + p.off_hmax);
  }
  return w;
}

// ------------------------------------------------------------ profiling --

namespace {

struct EventPair {
  hipEvent_t start, stop;
};

struct Profiler {
  std::mutex mu;
  std::atomic<bool> on{false};
  std::vector<EventPair> pool;                      // idle, reusable
  std::vector<EventPair> pending[CGH_KERNEL_COUNT];  // recorded, unread
};

Profiler& profiler() {
  static Profiler P;
  return P;
}

constexpr size_t kMaxPending = 4096;

// Records the start event of a timed launch; returns the pair to close, or a
// pair of nulls when timing is off (or not possible).
EventPair profile_begin(int kernel, hipStream_t s, bool timed = true) {
  Profiler& P = profiler();
  EventPair e{nullptr, nullptr};
  if (!timed || !P.on.load(std::memory_order_relaxed)) return e;  // no lock, no event
  std::lock_guard<std::mutex> lk(P.mu);
  if (!P.on || P.pending[kernel].size() >= kMaxPending) return e;
  if (!P.pool.empty()) {
    e = P.pool.back();
    P.pool.pop_back();
  } else {
    // Timing-only events: no system-scope fence at record, so recording them
    // neither writes back nor invalidates the caches between the kernels they
    // bracket (their times are read after the stream has synchronised).
    if (hipEventCreateWithFlags(&e.start, hipEventDisableSystemFence) != hipSuccess)
      return EventPair{nullptr, nullptr};
    if (hipEventCreateWithFlags(&e.stop, hipEventDisableSystemFence) != hipSuccess) {
      (void)hipEventDestroy(e.start);
      return EventPair{nullptr, nullptr};
    }
  }
  if (hipEventRecord(e.start, s) != hipSuccess) {
    P.pool.push_back(e);
    return EventPair{nullptr, nullptr};
  }
  return e;
}

void profile_end(int kernel, EventPair e, hipStream_t s) {
  if (!e.start) return;
  Profiler& P = profiler();
  std::lock_guard<std::mutex> lk(P.mu);
  if (hipEventRecord(e.stop, s) != hipSuccess) {
    P.pool.push_back(e);
    return;
  }
  P.pending[kernel].push_back(e);
}

// ------------------------------------------------------------ validation --

bool finite_positive(double v) { return isfinite(v) && v > 0.0; }

int check_common(const float* x, const float* y, const float* z, const float* a, int64_t n,
                 int32_t nx, int32_t ny, double pitch, double wavelength) {
  if (n < 0 || n > kMaxPoints) return CGH_EINVAL;
  if (nx < 1 || ny < 1 || nx > kMaxSide || ny > kMaxSide) return CGH_EINVAL;
  if (n > 0 && (!x || !y || !z || !a)) return CGH_EINVAL;
  if (!finite_positive(pitch) || !finite_positive(wavelength)) return CGH_EINVAL;
  return CGH_OK;
}

int check_workspace(const Plan& p, void* ws, size_t bytes) {
  if (p.total == 0) return CGH_OK;
  if (!ws || bytes < p.total) return CGH_EWORKSPACE;
  if (((uintptr_t)ws & 255u) != 0) return CGH_EWORKSPACE;
  return CGH_OK;
}

inline int hip_status(hipError_t e) { return e == hipSuccess ? CGH_OK : CGH_EHIP; }

}  // namespace

// ------------------------------------------------------------- separable --

// I = P Q^T with P = (A cY, -A sY) [nyp][k2], Q = (cX, sX) [nxp][k2].
int forward_separable(const Plan& p, const Workspace& w, float* hologram, hipStream_t s,
                      bool timed) {
  hipError_t e =
      launch_sep_tables(w.xrec, w.yrec, w.amp, p.npad, p.nx, p.nxp, p.ny, p.nyp, w.sep_x, w.sep_y, s);
  if (e != hipSuccess) return CGH_EHIP;
  const EventPair ev = profile_begin(CGH_KERNEL_FWD_SEPARABLE, s, timed);
  if (p.sep_splits == 1) {
    e = launch_gemm_f32(true, true, w.sep_y, p.k2, w.sep_x, p.k2, hologram, p.nx, 0, p.nyp,
                        p.nxp, (int)p.k2, 1, p.ny, p.nx, nullptr, s);
  } else {
    const int64_t plane = (int64_t)p.nyp * p.nxp;
    e = launch_gemm_f32(true, true, w.sep_y, p.k2, w.sep_x, p.k2, w.sep_c, p.nxp, plane, p.nyp,
                        p.nxp, (int)p.k2, p.sep_splits, p.nyp, p.nxp, nullptr, s);
  }
  profile_end(CGH_KERNEL_FWD_SEPARABLE, ev, s);
  if (e != hipSuccess) return CGH_EHIP;
  if (p.sep_splits > 1)
    e = launch_sep_sum_slices(w.sep_c, p.sep_splits, (int64_t)p.nyp * p.nxp, p.nxp, p.nx, p.ny,
                              hologram, s);
  return hip_status(e);
}

// U = Y^T G (Y = (cY, sY) [nyp][k2]), Pm = X^T G^T (X = (cX, sX) [nxp][k2]),
// each folded per point in its GEMM epilogue, then the per-point sums.
int backward_separable(const Plan& p, const Workspace& w, const float* z, const float* a,
                       double pitch, double wavelength, const float* g, float* gx, float* gy,
                       float* gz, float* ga, hipStream_t s) {
  hipError_t e = launch_sep_tables(w.xrec, w.yrec, nullptr, p.npad, p.nx, p.nxp, p.ny, p.nyp,
                                   w.sep_x, w.sep_y, s);
  if (e == hipSuccess) e = launch_sep_pad(g, p.nx, p.ny, p.nyp, p.nxp, w.sep_g, s);
  if (e != hipSuccess) return CGH_EHIP;
  const FoldSpec fx{1, w.xrec, w.plain, p.nx, w.fold_x};
  const FoldSpec fy{2, w.yrec, w.plain, p.ny, w.fold_y};
  const EventPair ev = profile_begin(CGH_KERNEL_ADJ_SEPARABLE, s);
  // U[k][x] = sum_y Y[y][k] G[y][x]: A = Y stored [y][k], B = G stored [y][x];
  // folded in the epilogue.
  e = launch_gemm_f32(false, false, w.sep_y, p.k2, w.sep_g, p.nxp, nullptr, 0, 0, (int)p.k2,
                      p.nxp, p.nyp, p.sep_splits_u, (int)p.k2, p.nxp, &fx, s);
  // Pm[k][y] = sum_x X[x][k] G[y][x]: A = X stored [x][k], B = G stored [y][x].
  if (e == hipSuccess)
    e = launch_gemm_f32(false, true, w.sep_x, p.k2, w.sep_g, p.nxp, nullptr, 0, 0, (int)p.k2,
                        p.nyp, p.nxp, p.sep_splits_p, (int)p.k2, p.nyp, &fy, s);
  profile_end(CGH_KERNEL_ADJ_SEPARABLE, ev, s);
  if (e != hipSuccess) return CGH_EHIP;
  e = launch_sep_finalize(p, w, z, a, pitch, wavelength, gx, gy, gz, ga, s);
  return hip_status(e);
}

// Half-precision separable variants: the same contractions on 16-bit planes
// (A_j, resp. G, divided by a power of two recorded in w.hmax).
int forward_separable_half(const Plan& p, const Workspace& w, float* hologram, hipStream_t s,
                           bool timed) {
  const int hm = half_mode(p.variant);
  hipError_t e = launch_absmax(w.amp, p.npad, w.hmax, s);  // w.hmax cleared by prep
  if (e == hipSuccess) e = launch_sep_tables_half(hm, p, w, s);
  if (e != hipSuccess) return CGH_EHIP;
  const EventPair ev = profile_begin(CGH_KERNEL_FWD_SEPARABLE, s, timed);
  if (p.sep_splits == 1) {
    e = launch_gemm_half(hm, w.hy_hi, w.hy_lo, p.k2, w.hx_hi, w.hx_lo, p.k2, hologram, p.nx, 0,
                         p.nyp, p.nxp, (int)p.k2, 1, p.ny, p.nx, w.hmax, nullptr, s);
  } else {
    const int64_t plane = (int64_t)p.nyp * p.nxp;
    e = launch_gemm_half(hm, w.hy_hi, w.hy_lo, p.k2, w.hx_hi, w.hx_lo, p.k2, w.sep_c, p.nxp,
                         plane, p.nyp, p.nxp, (int)p.k2, p.sep_splits, p.nyp, p.nxp, w.hmax, nullptr,
                         s);
  }
  profile_end(CGH_KERNEL_FWD_SEPARABLE, ev, s);
  if (e != hipSuccess) return CGH_EHIP;
  if (p.sep_splits > 1)
    e = launch_sep_sum_slices(w.sep_c, p.sep_splits, (int64_t)p.nyp * p.nxp, p.nxp, p.nx, p.ny,
                              hologram, s);
  return hip_status(e);
}

int backward_separable_half(const Plan& p, const Workspace& w, const float* z, const float* a,
                            double pitch, double wavelength, const float* g, float* gx, float* gy,
                            float* gz, float* ga, hipStream_t s) {
  const int hm = half_mode(p.variant);
  hipError_t e = launch_absmax(g, (int64_t)p.nx * p.ny, w.hmax, s);  // w.hmax cleared by prep
  if (e == hipSuccess) e = launch_sep_adj_operands_half(hm, p, w, g, s);
  if (e != hipSuccess) return CGH_EHIP;
  const FoldSpec fx{1, w.xrec, w.plain, p.nx, w.fold_x};
  const FoldSpec fy{2, w.yrec, w.plain, p.ny, w.fold_y};
  const EventPair ev = profile_begin(CGH_KERNEL_ADJ_SEPARABLE, s);
  // U[k][x] = sum_y Yt[k][y] Gt[x][y], folded in the epilogue
  e = launch_gemm_half(hm, w.hy_hi, w.hy_lo, p.nyp, w.hgt_hi, w.hgt_lo, p.nyp, nullptr, 0, 0,
                       (int)p.k2, p.nxp, p.nyp, p.sep_splits_u, (int)p.k2, p.nxp, w.hmax, &fx, s);
  // Pm[k][y] = sum_x Xt[k][x] G[y][x], folded in the epilogue
  if (e == hipSuccess)
    e = launch_gemm_half(hm, w.hx_hi, w.hx_lo, p.nxp, w.hg_hi, w.hg_lo, p.nxp, nullptr, 0, 0,
                         (int)p.k2, p.nyp, p.nxp, p.sep_splits_p, (int)p.k2, p.nyp, w.hmax, &fy,
                         s);
  profile_end(CGH_KERNEL_ADJ_SEPARABLE, ev, s);
  if (e != hipSuccess) return CGH_EHIP;
  e = launch_sep_finalize(p, w, z, a, pitch, wavelength, gx, gy, gz, ga, s);
  return hip_status(e);
}

// ------------------------------------------------------ static scratch --
//
// Scratch of cgh_forward_noalloc: a file-scope device array, one copy per GPU
// the library is loaded on, held until the process ends.  In host code its
// name is a host-side stand-in, not a device address, so it is never passed
// to a kernel or a copy: the entry point takes the array's address on the
// current device from hipGetSymbolAddress, once per device (the first call
// there), and uses that.  Every call on a GPU shares that GPU's array.
constexpr size_t kScratchBytes = CGH_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex scratch_mu;
std::map<int, void*> scratch_ptr;  // device -> the array's address there

int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CGH_EHIP;
  std::lock_guard<std::mutex> lk(scratch_mu);
  auto it = scratch_ptr.find(dev);
  if (it != scratch_ptr.end()) {
    *out = it->second;
    return CGH_OK;
  }
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return CGH_EHIP;
  if (((uintptr_t)ptr & 255u) != 0) return CGH_EHIP;
  scratch_ptr[dev] = ptr;
  *out = ptr;
  return CGH_OK;
}

}  // namespace

// Enqueues the forward for plan p with its scratch at `workspace` (the
// caller's workspace, or the static scratch), after the argument checks.
// timed = false skips the event timing (which creates events), for the
// allocation-free entry point.  With target and residual it also writes
// residual = hologram - target: fused into the compensated forward's store,
// a separate elementwise launch after the other forwards.
int forward_run(const Plan& p, void* workspace, const float* x, const float* y, const float* z,
                const float* a, double pitch, double wavelength, float* hologram,
                hipStream_t s, bool timed = true, const float* target = nullptr,
                float* residual = nullptr);

}  // namespace cgh

using namespace cgh;

extern "C" {

size_t cgh_workspace_bytes(int64_t n, int32_t nx, int32_t ny, int32_t variant, int32_t op) {
  if (op != CGH_OP_FORWARD && op != CGH_OP_FORWARD_F64 && op != CGH_OP_BACKWARD) return 0;
  if (op != CGH_OP_FORWARD_F64 && !valid_variant(variant)) return 0;
  if (n < 0 || n > kMaxPoints || nx < 1 || ny < 1 || nx > kMaxSide || ny > kMaxSide) return 0;
  if (n == 0) return 0;
  return make_plan(n, nx, ny, variant, op).total;
}

int cgh_forward(const float* x, const float* y, const float* z, const float* a, int64_t n,
                int32_t nx, int32_t ny, double pitch, double wavelength, int32_t variant,
                float* hologram, void* workspace, size_t workspace_bytes, void* stream) {
  int rc = check_common(x, y, z, a, n, nx, ny, pitch, wavelength);
  if (rc) return rc;
  if (!valid_variant(variant)) return CGH_EINVAL;
  if (!hologram) return CGH_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (n == 0) return hip_status(launch_fill_zero_f32(hologram, (int64_t)nx * ny, s));
  const Plan p = make_plan(n, nx, ny, variant, CGH_OP_FORWARD);
  rc = check_workspace(p, workspace, workspace_bytes);
  if (rc) return rc;
  return forward_run(p, workspace, x, y, z, a, pitch, wavelength, hologram, s, true);
}

int cgh_forward_residual(const float* x, const float* y, const float* z, const float* a,
                         int64_t n, int32_t nx, int32_t ny, double pitch, double wavelength,
                         int32_t variant, const float* target, float* hologram, float* residual,
                         void* workspace, size_t workspace_bytes, void* stream) {
  int rc = check_common(x, y, z, a, n, nx, ny, pitch, wavelength);
  if (rc) return rc;
  if (!valid_variant(variant)) return CGH_EINVAL;
  if (!hologram || !target || !residual) return CGH_EINVAL;
  if (residual == hologram || residual == target || hologram == target) return CGH_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int64_t count = (int64_t)nx * ny;
  if (n == 0) {
    hipError_t e = launch_fill_zero_f32(hologram, count, s);
    if (e == hipSuccess) e = launch_residual(hologram, target, residual, count, s);
    return hip_status(e);
  }
  const Plan p = make_plan(n, nx, ny, variant, CGH_OP_FORWARD);
  rc = check_workspace(p, workspace, workspace_bytes);
  if (rc) return rc;
  return forward_run(p, workspace, x, y, z, a, pitch, wavelength, hologram, s, true, target,
                     residual);
}

int cgh_forward_noalloc(const float* x, const float* y, const float* z, const float* a,
                        int64_t n, int32_t nx, int32_t ny, double pitch, double wavelength,
                        int32_t variant, float* hologram, void* stream) {
  int rc = check_common(x, y, z, a, n, nx, ny, pitch, wavelength);
  if (rc) return rc;
  if (!valid_variant(variant)) return CGH_EINVAL;
  if (!hologram) return CGH_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (n == 0) return hip_status(launch_fill_zero_f32(hologram, (int64_t)nx * ny, s));
  Plan p = make_plan(n, nx, ny, variant, CGH_OP_FORWARD);
  // Without its column table the compensated forward needs less scratch and
  // gives the same bits.
  if (p.total > kScratchBytes && p.comp_xtab)
    p = make_plan(n, nx, ny, variant, CGH_OP_FORWARD, false);
  if (p.total > kScratchBytes) return CGH_ETOOBIG;
  void* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc) return rc;
  return forward_run(p, ws, x, y, z, a, pitch, wavelength, hologram, s, false);
}

}  // extern "C"

namespace cgh {

int forward_run(const Plan& p, void* workspace, const float* x, const float* y, const float* z,
                const float* a, double pitch, double wavelength, float* hologram,
                hipStream_t s, bool timed, const float* target, float* residual) {
  const int32_t variant = p.variant;
  const int64_t n = p.n;
  const Workspace w = carve(p, workspace);
  // The compensated forward forms the records with its row-phase table.
  hipError_t e = variant == CGH_COMPENSATED
                     ? launch_prep_ytab(x, y, z, a, pitch, wavelength, p, w, s)
                     : launch_prep(x, y, z, a, n, p.npad, pitch, wavelength, w, false, s);
  if (e != hipSuccess) return CGH_EHIP;
  auto separate_residual = [&](int rc) {
    if (rc != CGH_OK || !residual) return rc;
    return hip_status(launch_residual(hologram, target, residual, (int64_t)p.nx * p.ny, s));
  };
  if (variant == CGH_SEPARABLE)
    return separate_residual(forward_separable(p, w, hologram, s, timed));
  if (half_mode(variant) >= 0)
    return separate_residual(forward_separable_half(p, w, hologram, s, timed));
  if (variant == CGH_COMPENSATED) {
    const EventPair ev = profile_begin(CGH_KERNEL_FWD_COMPENSATED, s, timed);
    e = launch_fwd_comp(p, w, hologram, s, target, residual);
    profile_end(CGH_KERNEL_FWD_COMPENSATED, ev, s);
    return hip_status(e);
  } else if (variant == CGH_RECURRENCE) {
    const EventPair ev = profile_begin(CGH_KERNEL_FWD_RECURRENCE, s, timed);
    e = launch_fwd_rec(p, w, hologram, s);
    profile_end(CGH_KERNEL_FWD_RECURRENCE, ev, s);
  } else {
    const EventPair ev = profile_begin(CGH_KERNEL_FWD_PLAIN, s, timed);
    e = launch_fwd_plain(p, w, hologram, s);
    profile_end(CGH_KERNEL_FWD_PLAIN, ev, s);
  }
  return separate_residual(hip_status(e));
}

}  // namespace cgh

extern "C" {

int cgh_forward_f64(const float* x, const float* y, const float* z, const float* a, int64_t n,
                    int32_t nx, int32_t ny, double pitch, double wavelength, double* hologram,
                    void* workspace, size_t workspace_bytes, void* stream) {
  int rc = check_common(x, y, z, a, n, nx, ny, pitch, wavelength);
  if (rc) return rc;
  if (!hologram) return CGH_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (n == 0) return hip_status(launch_fill_zero_f64(hologram, (int64_t)nx * ny, s));
  const Plan p = make_plan(n, nx, ny, CGH_PLAIN, CGH_OP_FORWARD_F64);
  rc = check_workspace(p, workspace, workspace_bytes);
  if (rc) return rc;
  const Workspace w = carve(p, workspace);
  hipError_t e = launch_prep(x, y, z, a, n, p.npad, pitch, wavelength, w, true, s);
  if (e != hipSuccess) return CGH_EHIP;
  const EventPair ev = profile_begin(CGH_KERNEL_FWD_F64, s);
  e = launch_fwd_f64(p, w, hologram, s);
  profile_end(CGH_KERNEL_FWD_F64, ev, s);
  return hip_status(e);
}

int cgh_backward(const float* x, const float* y, const float* z, const float* a, int64_t n,
                 int32_t nx, int32_t ny, double pitch, double wavelength, int32_t variant,
                 const float* grad_hologram, float* grad_x, float* grad_y, float* grad_z,
                 float* grad_a, void* workspace, size_t workspace_bytes, void* stream) {
  int rc = check_common(x, y, z, a, n, nx, ny, pitch, wavelength);
  if (rc) return rc;
  if (!valid_variant(variant)) return CGH_EINVAL;
  if (!grad_hologram) return CGH_EINVAL;
  if (n > 0 && (!grad_x || !grad_y || !grad_z || !grad_a)) return CGH_EINVAL;
  if (n == 0) return CGH_OK;
  hipStream_t s = (hipStream_t)stream;
  const Plan p = make_plan(n, nx, ny, variant, CGH_OP_BACKWARD);
  rc = check_workspace(p, workspace, workspace_bytes);
  if (rc) return rc;
  const Workspace w = carve(p, workspace);
  hipError_t e;
  if (is_separable(variant)) {
    e = launch_prep(x, y, z, a, n, p.npad, pitch, wavelength, w, false, s);
    if (e != hipSuccess) return CGH_EHIP;
    if (variant == CGH_SEPARABLE)
      return backward_separable(p, w, z, a, pitch, wavelength, grad_hologram, grad_x, grad_y,
                                grad_z, grad_a, s);
    return backward_separable_half(p, w, z, a, pitch, wavelength, grad_hologram, grad_x, grad_y,
                                   grad_z, grad_a, s);
  }
  // The direct adjoint forms each point's records itself (one point per
  // lane); the compensated one takes its row phases from a table built here.
  if (p.adj_kind == kAdjCompensated) {
    e = launch_prep_rtab(x, y, z, a, pitch, wavelength, p, w, s);
    if (e != hipSuccess) return CGH_EHIP;
  }
  const float* g = grad_hologram;
  int64_t ldg = nx;
  if (p.need_gpad) {
    e = launch_pad_g(p, grad_hologram, w.gpad, s);
    if (e != hipSuccess) return CGH_EHIP;
    g = w.gpad;
    ldg = (int64_t)p.nsx * kAdjCols;
  }
  const int runs = adj_runs(p);
  if (runs < 1) return CGH_EHIP;
  const int kid = variant == CGH_COMPENSATED  ? CGH_KERNEL_ADJ_COMPENSATED
                  : variant == CGH_RECURRENCE ? CGH_KERNEL_ADJ_RECURRENCE
                                              : CGH_KERNEL_ADJ_PLAIN;
  const EventPair ev = profile_begin(kid, s);
  e = launch_adj_partial(p, w, x, y, z, a, pitch, wavelength, g, ldg, runs, s);
  profile_end(kid, ev, s);
  if (e != hipSuccess) return CGH_EHIP;
  e = launch_adj_finalize(p, w, z, a, pitch, wavelength, runs, grad_x, grad_y, grad_z, grad_a, s);
  return hip_status(e);
}

const char* cgh_strerror(int status) {
  switch (status) {
    case CGH_OK:
      return "success";
    case CGH_EINVAL:
      return "invalid argument";
    case CGH_EWORKSPACE:
      return "workspace missing, misaligned or too small";
    case CGH_EHIP:
      return "HIP launch or runtime error";
    case CGH_ETOOBIG:
      return "problem needs more scratch than the allocation-free entry point's static buffer "
             "holds";
    default:
      return "unknown status";
  }
}

int cgh_version(void) { return 103; }

int cgh_profile_enable(int32_t on) {
  Profiler& P = profiler();
  std::lock_guard<std::mutex> lk(P.mu);
  P.on = on != 0;
  return CGH_OK;
}

int cgh_profile_read_each(int32_t kernel, int64_t* launches, double* total_ms, float* each_ms,
                          int64_t capacity) {
  if (kernel < 0 || kernel >= CGH_KERNEL_COUNT || !launches || !total_ms) return CGH_EINVAL;
  if (capacity < 0 || (capacity > 0 && !each_ms)) return CGH_EINVAL;
  Profiler& P = profiler();
  std::vector<EventPair> mine;
  {
    std::lock_guard<std::mutex> lk(P.mu);
    mine.swap(P.pending[kernel]);
  }
  int rc = CGH_OK;
  double sum = 0.0;
  int64_t count = 0;
  for (const EventPair& e : mine) {
    float ms = 0.0f;
    if (hipEventSynchronize(e.stop) != hipSuccess ||
        hipEventElapsedTime(&ms, e.start, e.stop) != hipSuccess) {
      rc = CGH_EHIP;
      continue;
    }
    if (count < capacity) each_ms[count] = ms;
    sum += ms;
    ++count;
  }
  {
    std::lock_guard<std::mutex> lk(P.mu);
    for (const EventPair& e : mine) P.pool.push_back(e);
  }
  *launches = count;
  *total_ms = sum;
  return rc;
}

int cgh_profile_read(int32_t kernel, int64_t* launches, double* total_ms) {
  return cgh_profile_read_each(kernel, launches, total_ms, nullptr, 0);
}

}  // extern "C"
