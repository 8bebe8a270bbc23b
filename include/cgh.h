/*
 * cgh.h -- C ABI of the MI355X (gfx950) direct point-source hologram library.
 *
 * The library computes the computer-generated hologram of N point light
 * sources, Eq. (1) of Shimobaba et al., "Fast calculation of
 * computer-generated-hologram on AMD HD5000 series GPU and OpenCL",
 * Section 1:
 *
 *     I(x_h, y_h) = sum_j A_j cos( P_j ((x_h - x_j)^2 + (y_h - y_j)^2) ),
 *     P_j = pi p^2 / (lambda z_j),
 *
 * and the adjoint of that map (gradients of a scalar loss with respect to
 * every point's x, y, z and A).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Coordinates: x_j, y_j and the pixel coordinates are in units of the
 *    sampling pitch p, as in Section 1 (the paper normalises them by p).
 *    Pixel (i, k) of an nx x ny hologram sits at x_h = i, y_h = k.
 *    z_j, pitch and wavelength are in metres.
 *  - Layout: point arrays are device float32[n] (structure of arrays); the
 *    hologram and its gradient are device arrays [ny][nx], row-major, x
 *    fastest, densely packed (row stride nx).
 *  - Ownership: every pointer is device memory owned by the caller.  The
 *    library never allocates, frees or retains device memory on these calls;
 *    all scratch comes from the caller's `workspace` (see
 *    cgh_workspace_bytes).  Nothing is kept between calls.
 *  - Streams: `stream` is a hipStream_t (passed as void*, NULL = the default
 *    stream).  All work is enqueued on it asynchronously; no call
 *    synchronises the host.  Calls that share a workspace must be ordered on
 *    one stream.
 *  - Limits: 0 <= n <= 4,000,000 points; 1 <= nx, ny <= 1,048,576 pixels.
 *  - Errors: argument checks run on the host before anything is enqueued and
 *    return CGH_EINVAL (null pointer with n > 0, nx or ny outside the limits,
 *    n < 0 or above the limit, non-finite or non-positive pitch/wavelength,
 *    unknown variant, null output) or
 *    CGH_EWORKSPACE (workspace missing or smaller than required).  A failed
 *    launch returns CGH_EHIP.  Device-resident values are not inspected: a
 *    z_j <= 0 gives inf/NaN outputs, not an error code.
 *  - Variants (the phase arithmetic, all FP32 in the bulk):
 *      CGH_PLAIN        the phase P_j r^2 formed directly in FP32, reduced
 *                       with fract, then the native revolution-domain cosine.
 *      CGH_COMPENSATED  r^2 formed exactly on the integer pixel grid and
 *                       P_j r^2 taken as a compensated split product reduced
 *                       mod 1 revolution, per axis: the square of each grid
 *                       offset m = x_h - rint(x_j) (and the same in y) is an
 *                       exact FP32 pair for |m| < 2^24, so the phase error
 *                       per axis is at most about 2^-24 (1 + 1.5 Prev |m|)
 *                       + 2^-46 Prev m^2 revolutions (Prev = P_j / 2 pi):
 *                       below 5e-7 rev for |m| <= 16384 at pitch 8 um,
 *                       633 nm and z_j >= 0.2 m.  The cosine's argument stays within a
 *                       few revolutions for every accepted input.
 *      CGH_SEPARABLE    not the per-interaction cosine: the phase separates
 *                       exactly into x and y parts (each formed as in
 *                       CGH_COMPENSATED), cos(X + Y) = cXcY - sXsY turns the sum
 *                       into a dense real contraction of per-axis tables, and
 *                       the forward and adjoint run as FP32 matrix-core GEMMs.
 *                       Needs a larger workspace (tables of 2N floats per row
 *                       and per column, plus split-K partial planes).
 *      CGH_SEPARABLE_F16X3, CGH_SEPARABLE_F16, CGH_SEPARABLE_BF16
 *                       CGH_SEPARABLE with the contractions on the fp16 / bf16
 *                       matrix cores (FP32 accumulation).  The tables and G are
 *                       rounded to 16 bits after dividing A_j (forward) or G
 *                       (adjoint) by a power of two >= their largest
 *                       magnitude (undone exactly on the FP32 result).  F16X3
 *                       splits each operand into fp16 hi + lo and forms
 *                       hi*hi + hi*lo + lo*hi (near-FP32 accuracy); F16 and
 *                       BF16 round each operand once (unit roundoff 2^-11 and
 *                       2^-8), so the forward error stays below about
 *                       2 u sum |A_j| (u = 2^-11, 2^-8).
 *      CGH_RECURRENCE   the forward by the two recurrence formulas of Eq. (2)
 *                       (Section 2.1): along a row Gamma_n = Gamma_{n-1} +
 *                       delta_{n-1}, delta_n = delta_{n-1} + Delta, each lane
 *                       producing a few consecutive pixels from the plain
 *                       FP32 phase Gamma_0 of the first (same accuracy class
 *                       as CGH_PLAIN).  Its backward steps the phase the same
 *                       way along each 32-pixel run of a row.
 *    FP64 appears only in the per-point precompute of P_j / (2 pi) and its
 *    hi/lo split (and in cgh_forward_f64).
 */
#ifndef CGH_H
#define CGH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define CGH_OK 0
#define CGH_EINVAL 1
#define CGH_EWORKSPACE 2
#define CGH_EHIP 3
#define CGH_ETOOBIG 4

/* Phase-arithmetic variants. */
#define CGH_PLAIN 0
#define CGH_COMPENSATED 1
#define CGH_SEPARABLE 2
#define CGH_SEPARABLE_F16X3 3
#define CGH_SEPARABLE_F16 4
#define CGH_SEPARABLE_BF16 5
#define CGH_RECURRENCE 6

/* Operations, for cgh_workspace_bytes. */
#define CGH_OP_FORWARD 0
#define CGH_OP_FORWARD_F64 1
#define CGH_OP_BACKWARD 2

/* Kernels that cgh_profile_read reports on. */
#define CGH_KERNEL_FWD_PLAIN 0
#define CGH_KERNEL_FWD_COMPENSATED 1
#define CGH_KERNEL_FWD_F64 2
#define CGH_KERNEL_ADJ_PLAIN 3
#define CGH_KERNEL_ADJ_COMPENSATED 4
#define CGH_KERNEL_FWD_SEPARABLE 5 /* the forward GEMM (every separable variant) */
#define CGH_KERNEL_ADJ_SEPARABLE 6 /* both adjoint GEMMs, one event pair */
#define CGH_KERNEL_FWD_RECURRENCE 7
#define CGH_KERNEL_ADJ_RECURRENCE 8
#define CGH_KERNEL_COUNT 9

/*
 * Bytes of device workspace that `op` (CGH_OP_*) needs for n points on an
 * nx x ny hologram with `variant` (ignored for CGH_OP_FORWARD_F64).  Returns 0
 * when the arguments are invalid (and also when no workspace is needed,
 * which does not happen for n > 0).  The workspace must be 256-byte aligned
 * (any hipMalloc/torch allocation is).
 */
size_t cgh_workspace_bytes(int64_t n, int32_t nx, int32_t ny, int32_t variant, int32_t op);

/*
 * Forward, Eq. (1) (Section 1), FP32 output.
 *   x, y, z, a   device float32[n]: point coordinates (pixels, pixels, metres)
 *                and amplitudes A_j.
 *   hologram     device float32[ny][nx], overwritten with I.  n = 0 writes
 *                zeros.
 *   variant      CGH_PLAIN, CGH_COMPENSATED, CGH_SEPARABLE, one of the
 *                half-precision separable variants, or CGH_RECURRENCE.
 */
int cgh_forward(const float* x, const float* y, const float* z, const float* a, int64_t n,
                int32_t nx, int32_t ny, double pitch, double wavelength, int32_t variant,
                float* hologram, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Forward with the residual of a target, for a loss L = 0.5 ||I - T||^2 whose
 * upstream gradient dL/dI = I - T feeds cgh_backward (the chain rule on
 * Eq. (1), Section 1).  Writes I exactly as cgh_forward (the same bits) and
 *   residual[h] = hologram[h] - target[h]   (one FP32 subtraction each),
 * in the compensated forward's own store pass, after the other forwards as
 * one more kernel on the same stream.
 *   target       device float32[ny][nx], read only.
 *   hologram     device float32[ny][nx], overwritten with I.
 *   residual     device float32[ny][nx], overwritten with I - T.
 * The three arrays must not overlap (the same pointer twice returns
 * CGH_EINVAL; partial overlaps are not detected).  Workspace as cgh_forward
 * (cgh_workspace_bytes with CGH_OP_FORWARD).  n = 0 writes I = 0 and
 * residual = -target.  Other errors as cgh_forward.
 */
int cgh_forward_residual(const float* x, const float* y, const float* z, const float* a,
                         int64_t n, int32_t nx, int32_t ny, double pitch, double wavelength,
                         int32_t variant, const float* target, float* hologram, float* residual,
                         void* workspace, size_t workspace_bytes, void* stream);

/*
 * Forward, Eq. (1), with FP64 phase arithmetic and FP64 output: the
 * on-device reference used to measure the FP32 variants at full size.
 *   hologram     device float64[ny][nx], overwritten.
 */
int cgh_forward_f64(const float* x, const float* y, const float* z, const float* a, int64_t n,
                    int32_t nx, int32_t ny, double pitch, double wavelength, double* hologram,
                    void* workspace, size_t workspace_bytes, void* stream);

/*
 * Adjoint of Eq. (1).  Given G = dL/dI (device float32[ny][nx]) it writes,
 * for every point j (device float32[n] each, overwritten, not accumulated):
 *   grad_a[j] = sum_h G cos(theta)
 *   grad_x[j] = 2 A_j P_j sum_h G sin(theta) (x_h - x_j)
 *   grad_y[j] = 2 A_j P_j sum_h G sin(theta) (y_h - y_j)
 *   grad_z[j] = (A_j P_j / z_j) sum_h G sin(theta) r^2      (per metre)
 * with theta = P_j r^2, the chain rule applied to Eq. (1).  The per-point
 * sums over pixels are reduced in a fixed order, so results are
 * bitwise reproducible run to run.  n = 0 does nothing.
 */
int cgh_backward(const float* x, const float* y, const float* z, const float* a, int64_t n,
                 int32_t nx, int32_t ny, double pitch, double wavelength, int32_t variant,
                 const float* grad_hologram, float* grad_x, float* grad_y, float* grad_z,
                 float* grad_a, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Forward as cgh_forward, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  It takes no workspace and calls no allocator: its scratch is a
 * static device buffer of CGH_NOALLOC_SCRATCH_BYTES (64 MiB) on each GPU the
 * library is loaded on, held until the process ends.  The caller still
 * passes the inputs and the output (`hologram`, device float32[ny][nx]).
 * Same kernels, same results (bitwise) as cgh_forward for every variant.
 *   Returns CGH_ETOOBIG (before anything is enqueued) when the problem needs
 * more scratch than the buffer holds: about 84 bytes per point plus the
 * variant's tables (the compensated forward: 4 bytes per point and row, and
 * 4 per point and column unless dropped to fit, since the kernel can form
 * those values itself; the separable forms: their GEMM tables and split-K
 * planes).  At 1920 x 1024 with 1,024 points every variant fits.
 *   Every call on a GPU shares that GPU's buffer, which keeps the last call's
 * contents (each call rewrites what it reads): calls that overlap on one GPU
 * (on different streams, or from several threads without ordering) race.
 * Order them on one stream.  The first call on each device looks up the
 * buffer's device address (not a stream operation).  Other errors as
 * cgh_forward.
 */
#define CGH_NOALLOC_SCRATCH_BYTES 67108864
int cgh_forward_noalloc(const float* x, const float* y, const float* z, const float* a,
                        int64_t n, int32_t nx, int32_t ny, double pitch, double wavelength,
                        int32_t variant, float* hologram, void* stream);

/* Human-readable text for a status code (static storage, never NULL). */
const char* cgh_strerror(int status);

/* Library ABI version (major * 100 + minor): 101 adds the half-precision
 * separable variants, 102 CGH_RECURRENCE, 103 cgh_forward_noalloc. */
int cgh_version(void);

/*
 * Kernel timing with HIP events, for measurement.  cgh_profile_enable(1)
 * makes every later entry-point call record an event pair on its stream
 * immediately around its main compute kernel (at most 4096 pairs per kernel
 * until read); cgh_profile_enable(0) stops recording.  cgh_profile_read
 * waits for the recorded events of `kernel` (CGH_KERNEL_*), returns how many
 * launches were recorded and their summed duration in milliseconds, and
 * clears that kernel's record.  Returns CGH_EINVAL for an unknown kernel id
 * or null outputs, CGH_EHIP if an event call fails.
 */
int cgh_profile_enable(int32_t on);
int cgh_profile_read(int32_t kernel, int64_t* launches, double* total_ms);

/*
 * As cgh_profile_read, and also copies the first `capacity` per-launch
 * durations (milliseconds, in launch order) into the host array `each_ms`
 * (caller-owned, may be NULL when capacity is 0).  *launches counts all
 * recorded launches, also those beyond `capacity`.  CGH_EINVAL for a negative
 * capacity or a NULL array with capacity > 0.
 */
int cgh_profile_read_each(int32_t kernel, int64_t* launches, double* total_ms, float* each_ms,
                          int64_t capacity);

#ifdef __cplusplus
}
#endif

#endif /* CGH_H */
