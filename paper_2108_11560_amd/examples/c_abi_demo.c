/*
 * c_abi_demo.c -- libbessel from C, with no Python and no torch: device
 * buffers from the HIP runtime, one call per entry point, results checked
 * against closed forms.
 *
 *   K_{1/2}(x) = sqrt(pi / (2x)) e^{-x}   (DLMF 10.39.2), so
 *   log K_{1/2}(x) = 0.5 log(pi / (2x)) - x,  d/dx log K = -1/(2x) - 1,
 *   d2/dx2 log K = 1 / (2 x^2),
 *   d2K/dx2 = sqrt(pi / 2) e^{-x} (x^{-1/2} + x^{-3/2} + (3/4) x^{-5/2}).
 *
 * Prints one line per check and exits non-zero if any check fails.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "bessel.h"

#define N 1000

static const double kPi = 3.14159265358979323846;

static int failures = 0;

static void check(int ok, const char* what, double err) {
  printf("%-52s %s (max error %.3g)\n", what, ok ? "ok" : "FAILED", err);
  if (!ok) ++failures;
}

static int hip_ok(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return 0;
  }
  return 1;
}

int main(void) {
  double hv[N], hx[N], hlk[N], hdx[N], hdxx[N];
  for (int i = 0; i < N; ++i) {
    hv[i] = (i % 2) ? 0.5 : -0.5; /* K_{-v} = K_v */
    hx[i] = pow(10.0, -3.0 + 6.0 * i / (N - 1));
  }
  double *v = NULL, *x = NULL, *lk = NULL, *dv = NULL, *dx = NULL, *dxx = NULL;
  const size_t bytes = N * sizeof(double);
  if (!hip_ok(hipMalloc((void**)&v, bytes), "hipMalloc") || !hip_ok(hipMalloc((void**)&x, bytes), "hipMalloc") ||
      !hip_ok(hipMalloc((void**)&lk, bytes), "hipMalloc") || !hip_ok(hipMalloc((void**)&dv, bytes), "hipMalloc") ||
      !hip_ok(hipMalloc((void**)&dx, bytes), "hipMalloc") || !hip_ok(hipMalloc((void**)&dxx, bytes), "hipMalloc"))
    return 2;
  if (!hip_ok(hipMemcpy(v, hv, bytes, hipMemcpyHostToDevice), "copy") ||
      !hip_ok(hipMemcpy(x, hx, bytes, hipMemcpyHostToDevice), "copy"))
    return 2;

  printf("%s\n", bessel_version());

  /* log K on the default stream (NULL), FP64, Newton bracket, 128 bins */
  int rc = bessel_logk(BESSEL_F64, N, v, x, lk, 128, BESSEL_RANGE_NEWTON, NULL, NULL);
  if (rc != BESSEL_OK || !hip_ok(hipMemcpy(hlk, lk, bytes, hipMemcpyDeviceToHost), "copy")) {
    fprintf(stderr, "bessel_logk: %d %s\n", rc, bessel_last_error());
    return 1;
  }
  double e = 0.0;
  for (int i = 0; i < N; ++i) {
    const double ref = 0.5 * log(kPi / (2.0 * hx[i])) - hx[i];
    const double m = fabs(hlk[i] - ref) / fmax(1.0, fabs(ref));
    if (m > e) e = m;
  }
  check(e <= 1e-12, "bessel_logk, K_{1/2} closed form", e);

  /* first and second derivatives in one pass */
  rc = bessel_logk_hess(BESSEL_F64, N, v, x, NULL, dv, dx, NULL, dxx, NULL, 128, NULL);
  if (rc != BESSEL_OK || !hip_ok(hipMemcpy(hdx, dx, bytes, hipMemcpyDeviceToHost), "copy") ||
      !hip_ok(hipMemcpy(hdxx, dxx, bytes, hipMemcpyDeviceToHost), "copy")) {
    fprintf(stderr, "bessel_logk_hess: %d %s\n", rc, bessel_last_error());
    return 1;
  }
  double e1 = 0.0, e2 = 0.0;
  for (int i = 0; i < N; ++i) {
    const double r1 = -0.5 / hx[i] - 1.0, r2 = 0.5 / (hx[i] * hx[i]);
    const double m1 = fabs(hdx[i] - r1) / fmax(1.0, fabs(r1));
    const double m2 = fabs(hdxx[i] - r2) / fmax(1.0, fabs(r2));
    if (m1 > e1) e1 = m1;
    if (m2 > e2) e2 = m2;
  }
  check(e1 <= 1e-12, "bessel_logk_hess, d/dx log K_{1/2}", e1);
  check(e2 <= 1e-10, "bessel_logk_hess, d2/dx2 log K_{1/2}", e2);

  /* d2K/dx2 itself, its integrand over its own bracket, as log |D| and sign */
  double *ld = NULL, *sg = NULL, hld[N], hsg[N];
  if (!hip_ok(hipMalloc((void**)&ld, bytes), "hipMalloc") || !hip_ok(hipMalloc((void**)&sg, bytes), "hipMalloc"))
    return 2;
  rc = bessel_logdk(BESSEL_F64, N, v, x, 0, 2, ld, sg, 128, NULL);
  if (rc != BESSEL_OK || !hip_ok(hipMemcpy(hld, ld, bytes, hipMemcpyDeviceToHost), "copy") ||
      !hip_ok(hipMemcpy(hsg, sg, bytes, hipMemcpyDeviceToHost), "copy")) {
    fprintf(stderr, "bessel_logdk: %d %s\n", rc, bessel_last_error());
    return 1;
  }
  double e3 = 0.0;
  int signs_ok = 1;
  for (int i = 0; i < N; ++i) {
    const double xi = hx[i];
    const double ref = 0.5 * log(kPi / 2.0) - xi + log(pow(xi, -0.5) + pow(xi, -1.5) + 0.75 * pow(xi, -2.5));
    const double m = fabs(hld[i] - ref) / fmax(1.0, fabs(ref));
    if (m > e3) e3 = m;
    if (hsg[i] != 1.0) signs_ok = 0;
  }
  check(e3 <= 1e-12 && signs_ok, "bessel_logdk, log d2K/dx2 of K_{1/2}", e3);

  /* an invalid argument comes back as a status with a message, before any GPU work */
  rc = bessel_logk(BESSEL_F64, N, v, x, lk, 1, BESSEL_RANGE_NEWTON, NULL, NULL);
  check(rc == BESSEL_ERR_NBINS, "nbins = 1 rejected with BESSEL_ERR_NBINS", 0.0);
  printf("  message: %s\n", bessel_last_error());

  (void)hipFree(v);
  (void)hipFree(x);
  (void)hipFree(lk);
  (void)hipFree(dv);
  (void)hipFree(dx);
  (void)hipFree(dxx);
  (void)hipFree(ld);
  (void)hipFree(sg);
  return failures ? 1 : 0;
}
