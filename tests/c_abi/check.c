/*
 * A plain-C consumer of the library (test program): device buffers from the
 * HIP runtime, every call through include/cgh.h, no Python.
 *
 * One point at (x0, y0) on a pixel node, depth z0, amplitude A.  Eq. (1)
 * (Section 1) then fixes I(x0, y0) = A (cos 0 = 1) and
 * I(x0 + u, y0 + v) = A cos(P (u^2 + v^2)), P = pi p^2 / (lambda z0); the
 * adjoint with G = 1 at pixel (x0 + u, y0 + v) and 0 elsewhere gives
 * dL/dA = cos(P (u^2 + v^2)).  Checked for the compensated, separable
 * (f16 hi/lo) and recurrence variants; also the status codes of a bad call.
 * Prints "c abi ok" and exits 0 on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "cgh.h"

#define CHECK_HIP(call)                                                   \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess) {                                               \
      fprintf(stderr, "%s:%d HIP error %d\n", __FILE__, __LINE__, (int)e_); \
      return 2;                                                           \
    }                                                                     \
  } while (0)

static int fail(const char* what, double got, double want) {
  fprintf(stderr, "c abi check failed: %s: got %.9g want %.9g\n", what, got, want);
  return 1;
}

static int run(int32_t variant) {
  const int32_t nx = 96, ny = 80;
  const double pitch = 8e-6, wavelength = 633e-9;
  const float hx = 40.0f, hy = 33.0f, hz = 0.45f, ha = 0.75f;
  const int u = 7, v = -5;
  const double P = M_PI * pitch * pitch / (wavelength * (double)hz);
  const double want_far = (double)ha * cos(P * (double)(u * u + v * v));

  float *x, *y, *z, *a, *img, *g, *gx, *gy, *gz, *ga;
  CHECK_HIP(hipMalloc((void**)&x, sizeof(float)));
  CHECK_HIP(hipMalloc((void**)&y, sizeof(float)));
  CHECK_HIP(hipMalloc((void**)&z, sizeof(float)));
  CHECK_HIP(hipMalloc((void**)&a, sizeof(float)));
  CHECK_HIP(hipMalloc((void**)&gx, sizeof(float)));
  CHECK_HIP(hipMalloc((void**)&gy, sizeof(float)));
  CHECK_HIP(hipMalloc((void**)&gz, sizeof(float)));
  CHECK_HIP(hipMalloc((void**)&ga, sizeof(float)));
  CHECK_HIP(hipMalloc((void**)&img, sizeof(float) * nx * ny));
  CHECK_HIP(hipMalloc((void**)&g, sizeof(float) * nx * ny));
  CHECK_HIP(hipMemcpy(x, &hx, sizeof(float), hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(y, &hy, sizeof(float), hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(z, &hz, sizeof(float), hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(a, &ha, sizeof(float), hipMemcpyHostToDevice));

  size_t wf = cgh_workspace_bytes(1, nx, ny, variant, CGH_OP_FORWARD);
  size_t wb = cgh_workspace_bytes(1, nx, ny, variant, CGH_OP_BACKWARD);
  size_t wbytes = wf > wb ? wf : wb;
  void* ws = NULL;
  CHECK_HIP(hipMalloc(&ws, wbytes));

  /* A short workspace is refused before anything is enqueued. */
  int rc = cgh_forward(x, y, z, a, 1, nx, ny, pitch, wavelength, variant, img, ws, wf - 1, NULL);
  if (rc != CGH_EWORKSPACE) return fail("short workspace status", rc, CGH_EWORKSPACE);

  rc = cgh_forward(x, y, z, a, 1, nx, ny, pitch, wavelength, variant, img, ws, wbytes, NULL);
  if (rc != CGH_OK) return fail(cgh_strerror(rc), rc, CGH_OK);
  float* host = (float*)malloc(sizeof(float) * nx * ny);
  CHECK_HIP(hipMemcpy(host, img, sizeof(float) * nx * ny, hipMemcpyDeviceToHost));
  const double at_point = host[(int)hy * nx + (int)hx];
  const double far = host[((int)hy + v) * nx + (int)hx + u];
  if (fabs(at_point - ha) > 1e-5) return fail("I at the point", at_point, ha);
  if (fabs(far - want_far) > 1e-4 * ha) return fail("I off the point", far, want_far);

  /* Adjoint of the impulse at (x0 + u, y0 + v): dL/dA = cos(P r^2). */
  for (int k = 0; k < nx * ny; ++k) host[k] = 0.0f;
  host[((int)hy + v) * nx + (int)hx + u] = 1.0f;
  CHECK_HIP(hipMemcpy(g, host, sizeof(float) * nx * ny, hipMemcpyHostToDevice));
  rc = cgh_backward(x, y, z, a, 1, nx, ny, pitch, wavelength, variant, g, gx, gy, gz, ga, ws,
                    wbytes, NULL);
  if (rc != CGH_OK) return fail(cgh_strerror(rc), rc, CGH_OK);
  float dA;
  CHECK_HIP(hipMemcpy(&dA, ga, sizeof(float), hipMemcpyDeviceToHost));
  if (fabs((double)dA - want_far / ha) > 1e-4) return fail("dL/dA", dA, want_far / ha);

  free(host);
  CHECK_HIP(hipFree(ws));
  CHECK_HIP(hipFree(g));
  CHECK_HIP(hipFree(img));
  CHECK_HIP(hipFree(ga));
  CHECK_HIP(hipFree(gz));
  CHECK_HIP(hipFree(gy));
  CHECK_HIP(hipFree(gx));
  CHECK_HIP(hipFree(a));
  CHECK_HIP(hipFree(z));
  CHECK_HIP(hipFree(y));
  CHECK_HIP(hipFree(x));
  return 0;
}

int main(void) {
  if (cgh_version() < 102) return fail("version", cgh_version(), 102);
  const int32_t variants[] = {CGH_COMPENSATED, CGH_SEPARABLE_F16X3, CGH_RECURRENCE};
  for (int i = 0; i < 3; ++i) {
    const int rc = run(variants[i]);
    if (rc) return rc;
  }
  printf("c abi ok\n");
  return 0;
}
