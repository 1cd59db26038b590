/*
 * sanitize_driver.c -- test infrastructure: calls every entry point of
 * oracle.c on a few inputs (ordinary, extreme and special values) with
 * several threads, so that the test suite can run the oracle under the
 * address, undefined-behaviour and thread sanitizers.  Prints one checksum
 * per entry point; exits non-zero if an entry point rejects valid arguments.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>

int oracle_logk_batch(int64_t n, const double* v, const double* x, double* logk, double* dv, double* dx,
                      int nthreads);
int oracle_logk_hess_batch(int64_t n, const double* v, const double* x, double* out, int nthreads);
int oracle_range_exact(int64_t n, const double* v, const double* x, double log_eps, double* tp, double* G,
                       double* t0, double* t1, int nthreads);
int oracle_method_batch(int64_t n, const double* v, const double* x, int nbins, double log_eps, int halve_ok,
                        double tol, int max_iter, double* out, double* tp, double* t0, double* t1, int nthreads);
int oracle_trapezoid_brute(double vin, double xin, double lo, double hi, int64_t nbins, double out[3]);
int oracle_logdk_batch(int64_t n, const double* v, const double* x, int a, int b, double* out, double* sign,
                       int nthreads);

#define N 12

static double checksum(const double* a, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i)
    if (isfinite(a[i])) s += a[i];
  return s;
}

int main(void) {
  const double v[N] = {0.0, 0.5, -1.5, 3.0, 10.0, 35.0, 49.0, 0.25, 2.0, NAN, 1.0, 7.0};
  const double x[N] = {1.0, 0.01, 2.0, 1e-3, 1e3, 22.0, 0.05, 5.0, 0.0, 1.0, INFINITY, 40.0};
  double a[N], b[N], c[N], d[N], h[6 * N], r3[3];
  int bad = 0;
  bad |= oracle_logk_batch(N, v, x, a, b, c, 4) != 0;
  printf("logk %.17g %.17g %.17g\n", checksum(a, N), checksum(b, N), checksum(c, N));
  bad |= oracle_logk_hess_batch(N, v, x, h, 4) != 0;
  printf("hess %.17g\n", checksum(h, 6 * N));
  bad |= oracle_range_exact(N, v, x, -36.04, a, b, c, d, 4) != 0;
  printf("range %.17g %.17g %.17g %.17g\n", checksum(a, N), checksum(b, N), checksum(c, N), checksum(d, N));
  bad |= oracle_method_batch(N, v, x, 64, -36.04, 1, 1.0, 10, a, b, c, d, 4) != 0;
  printf("method %.17g\n", checksum(a, N));
  bad |= oracle_trapezoid_brute(1.3, 0.7, 0.0, 6.0, 4096, r3) != 0;
  printf("brute %.17g %.17g %.17g\n", r3[0], r3[1], r3[2]);
  for (int o = 0; o < 4; ++o) {
    bad |= oracle_logdk_batch(N, v, x, o, 3 - o, a, b, 4) != 0;
    printf("logdk(%d,%d) %.17g %.17g\n", o, 3 - o, checksum(a, N), checksum(b, N));
  }
  return bad;
}
