/*
 * abi_errors_driver.c -- test infrastructure: exercises the host side of
 * every entry point of include/bessel.h that can run without a GPU (the
 * argument checks, error statuses and messages, the batch-size policy, the
 * version string), so that the test suite can run the library's host code
 * under the address and undefined-behaviour sanitizers.  Exits non-zero on
 * the first unexpected status.
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "bessel.h"

static int failures = 0;

static void expect(int got, int want, const char* what) {
  if (got != want) {
    printf("FAIL %s: got %d want %d (%s)\n", what, got, want, bessel_last_error());
    ++failures;
  }
}

int main(void) {
  void* A = (void*)0x10000;
  void* B = (void*)0x20000;
  void* C = (void*)0x30000;
  void* inside = (void*)(0x10000 + 16);
  printf("%s\n", bessel_version());

  expect(bessel_logk(7, 4, A, B, C, 128, 0, NULL, NULL), BESSEL_ERR_DTYPE, "logk dtype");
  expect(bessel_logk(1, -1, A, B, C, 128, 0, NULL, NULL), BESSEL_ERR_ARG, "logk n");
  expect(bessel_logk(1, 4, NULL, B, C, 128, 0, NULL, NULL), BESSEL_ERR_ARG, "logk null v");
  expect(bessel_logk(1, 4, A, B, C, 1, 0, NULL, NULL), BESSEL_ERR_NBINS, "logk nbins");
  expect(bessel_logk(1, 4, A, B, C, 128, 9, NULL, NULL), BESSEL_ERR_RANGE_MODE, "logk range");
  expect(bessel_logk(0, 4, A, B, C, 128, BESSEL_RANGE_MLP, NULL, NULL), BESSEL_ERR_RANGE_MODE, "logk mlp null");
  expect(bessel_logk(1, 4, A, B, C, 128, BESSEL_RANGE_MLP_TABLE, (const bessel_mlp*)A, NULL),
         BESSEL_ERR_UNSUPPORTED, "logk table f64");
  expect(bessel_logk(1, 4, A, B, inside, 128, 0, NULL, NULL), BESSEL_ERR_ALIAS, "logk alias");
  expect(bessel_logk(1, 0, NULL, NULL, NULL, 128, 0, NULL, NULL), BESSEL_OK, "logk empty");
  expect(bessel_logk_dv_dx(1, 4, A, B, NULL, NULL, C, C, 128, 0, NULL, NULL), BESSEL_ERR_ALIAS, "dv_dx alias");
  expect(bessel_logk_dv_dx(1, 4, A, B, NULL, NULL, NULL, C, 128, 0, NULL, NULL), BESSEL_ERR_ARG, "dv_dx null");
  expect(bessel_range(1, 4, A, B, C, C, NULL, NULL, 0, NULL, NULL, NULL), BESSEL_ERR_ALIAS, "range alias");
  expect(bessel_range(1, 4, A, B, NULL, C, NULL, NULL, 0, NULL, NULL, NULL), BESSEL_ERR_ARG, "range null");
  expect(bessel_logk_backward(1, 4, A, B, C, A, NULL, NULL), BESSEL_ERR_ALIAS, "backward alias");
  expect(bessel_logk_hess(1, 4, A, B, NULL, NULL, NULL, NULL, NULL, NULL, 128, NULL), BESSEL_ERR_ARG, "hess none");
  expect(bessel_logk_hess(1, 4, A, B, C, C, NULL, NULL, NULL, NULL, 128, NULL), BESSEL_ERR_ALIAS, "hess alias");
  expect(bessel_hess_vjp(1, 4, A, NULL, B, NULL, B, A, NULL, NULL), BESSEL_ERR_ALIAS, "vjp alias");
  expect(bessel_logdk(1, 4, A, B, 9, 0, C, NULL, 128, NULL), BESSEL_ERR_ORDER, "logdk order");
  expect(bessel_logdk(1, 4, A, B, 1, 0, C, C, 128, NULL), BESSEL_ERR_ALIAS, "logdk alias");
  expect(bessel_logdk(1, 4, A, B, 1, 0, NULL, NULL, 128, NULL), BESSEL_ERR_ARG, "logdk null");
  expect(bessel_gh_logk_sum(4, A, A, A, A, 4, B, NULL, C, NULL, NULL, NULL, NULL, 128, 1, NULL, NULL),
         BESSEL_ERR_UNSUPPORTED, "gh learned");
  expect(bessel_gh_logk_sum(-1, A, A, A, A, 4, B, NULL, C, NULL, NULL, NULL, NULL, 128, 0, NULL, NULL), BESSEL_ERR_ARG,
         "gh n");
  expect(bessel_mlp_create(A, 7, NULL), BESSEL_ERR_ARG, "mlp create");
  expect(bessel_mlp_destroy(NULL), BESSEL_OK, "mlp destroy null");
  expect(bessel_mlp_set_params(NULL, NULL, 0), BESSEL_ERR_ARG, "mlp set null");
  expect(bessel_mlp_forward(NULL, 4, A, B, C, 1, NULL), BESSEL_ERR_ARG, "mlp forward null");
  int64_t prev = 0;
  expect(bessel_set_split_threshold(-1, &prev), BESSEL_ERR_ARG, "split negative");
  expect(bessel_set_split_threshold(77, &prev), BESSEL_OK, "split set");
  expect(bessel_set_split_threshold(prev, &prev), BESSEL_OK, "split restore");
  expect(prev == 77 ? BESSEL_OK : -100, BESSEL_OK, "split previous");
  if (strlen(bessel_last_error()) == 0) {
    printf("FAIL: empty error message after a failed call\n");
    ++failures;
  }
  printf("%d failures\n", failures);
  return failures ? 1 : 0;
}
