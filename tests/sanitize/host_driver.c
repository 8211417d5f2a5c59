/* Host-only driver of libsfrde's argument validation and host helpers, built
 * with AddressSanitizer and UndefinedBehaviorSanitizer on the host code (see
 * tests/test_sanitize_host.py). Every call below returns before any device
 * call: bad plan arguments (SFRDE_EINVAL), NULL handles, the host eigenvalue
 * and coefficient evaluators over their whole range. Exit status 0 when
 * every return code is the expected one. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "sfrde.h"

static int failures = 0;

static void expect(int got, int want, const char* what) {
  if (got != want) {
    fprintf(stderr, "%s: got %d, want %d (%s)\n", what, got, want, sfrde_last_error());
    ++failures;
  }
}

int main(void) {
  const int64_t n2[2] = {8, 6};
  const double h2[2] = {0.1, 0.1};
  const double alpha[2] = {1.5, 1.5}, kappa[2] = {0.01, 0.02};
  const double prm[3] = {1.0, 0.1, 0.9};
  sfrde_plan_t p = NULL;

  /* one bad argument at a time */
  const int64_t bad_n[2] = {1, 6}, big_n[2] = {8, 4096};
  const double bad_h[2] = {0.0, 0.1}, nan_h[2] = {NAN, 0.1};
  const double bad_alpha[2] = {2.5, 1.5}, bad_kappa[2] = {-1.0, 0.1};
  const double nan_prm[3] = {1.0, NAN, 0.9};
  expect(sfrde_plan(&p, 4, n2, 2, h2, 2, alpha, kappa, 0.1, 3, 3, prm, 1, 0, NULL), SFRDE_EINVAL, "ndim");
  expect(sfrde_plan(&p, 2, bad_n, 2, h2, 2, alpha, kappa, 0.1, 3, 3, prm, 1, 0, NULL), SFRDE_EINVAL, "n < 2");
  expect(sfrde_plan(&p, 2, big_n, 2, h2, 2, alpha, kappa, 0.1, 3, 3, prm, 1, 0, NULL), SFRDE_EINVAL, "n > max");
  expect(sfrde_plan(&p, 2, n2, 3, h2, 2, alpha, kappa, 0.1, 3, 3, prm, 1, 0, NULL), SFRDE_EINVAL, "bc");
  expect(sfrde_plan(&p, 2, n2, 2, bad_h, 2, alpha, kappa, 0.1, 3, 3, prm, 1, 0, NULL), SFRDE_EINVAL, "h 0");
  expect(sfrde_plan(&p, 2, n2, 2, nan_h, 2, alpha, kappa, 0.1, 3, 3, prm, 1, 0, NULL), SFRDE_EINVAL, "h nan");
  expect(sfrde_plan(&p, 2, n2, 2, h2, 5, alpha, kappa, 0.1, 3, 3, prm, 1, 0, NULL), SFRDE_EINVAL, "species");
  expect(sfrde_plan(&p, 2, n2, 2, h2, 2, bad_alpha, kappa, 0.1, 3, 3, prm, 1, 0, NULL), SFRDE_EINVAL, "alpha");
  expect(sfrde_plan(&p, 2, n2, 2, h2, 2, alpha, bad_kappa, 0.1, 3, 3, prm, 1, 0, NULL), SFRDE_EINVAL, "kappa");
  expect(sfrde_plan(&p, 2, n2, 2, h2, 2, alpha, kappa, 0.0, 3, 3, prm, 1, 0, NULL), SFRDE_EINVAL, "dt");
  expect(sfrde_plan(&p, 2, n2, 2, h2, 2, alpha, kappa, 0.1, 9, 3, prm, 1, 0, NULL), SFRDE_EINVAL, "reaction");
  expect(sfrde_plan(&p, 2, n2, 2, h2, 2, alpha, kappa, 0.1, 3, 2, prm, 1, 0, NULL), SFRDE_EINVAL, "nparams");
  expect(sfrde_plan(&p, 2, n2, 2, h2, 2, alpha, kappa, 0.1, 3, 3, nan_prm, 1, 0, NULL), SFRDE_EINVAL, "params");
  expect(sfrde_plan(&p, 2, n2, 2, h2, 2, alpha, kappa, 0.1, 3, 3, NULL, 1, 0, NULL), SFRDE_EINVAL, "params NULL");
  expect(sfrde_plan(&p, 2, n2, 2, h2, 2, alpha, kappa, 0.1, 3, 3, prm, 2, 0, NULL), SFRDE_EINVAL, "dtype");
  expect(sfrde_plan(&p, 2, n2, 2, h2, 2, alpha, kappa, 0.1, 3, 3, prm, 1, 7, NULL), SFRDE_EINVAL, "scheme");
  expect(sfrde_plan(NULL, 2, n2, 2, h2, 2, alpha, kappa, 0.1, 3, 3, prm, 1, 0, NULL), SFRDE_EINVAL, "out NULL");
  expect(sfrde_plan(&p, 2, NULL, 2, h2, 2, alpha, kappa, 0.1, 3, 3, prm, 1, 0, NULL), SFRDE_EINVAL, "n NULL");
  if (p != NULL) {
    fprintf(stderr, "a plan was returned for bad arguments\n");
    ++failures;
  }
  /* an ensemble whose third member is bad: the message names it */
  double ab[6] = {1.5, 1.5, 1.2, 1.8, 1.5, 2.5}, kb[6] = {0.1, 0.1, 0.1, 0.1, 0.1, 0.1};
  double pb[9] = {1, 0.1, 0.9, 1, 0.1, 0.9, 1, 0.1, 0.9};
  expect(sfrde_plan_batch(&p, 3, 2, n2, 2, h2, 2, ab, kb, 0.1, 3, 3, pb, 1, 0, NULL), SFRDE_EINVAL, "member");
  if (!strstr(sfrde_last_error(), "member 2")) {
    fprintf(stderr, "ensemble message: %s\n", sfrde_last_error());
    ++failures;
  }
  expect(sfrde_plan_batch(&p, 0, 2, n2, 2, h2, 2, ab, kb, 0.1, 3, 3, pb, 1, 0, NULL), SFRDE_EINVAL, "batch 0");

  /* NULL handles on every call that takes a plan */
  double g[8];
  int64_t cnt[8];
  expect(sfrde_step(NULL, NULL, 0.0), SFRDE_EINVAL, "step");
  expect(sfrde_integrate(NULL, NULL, 1, 0.0, 0, NULL), SFRDE_EINVAL, "integrate");
  expect((int)sfrde_ckpt_bytes(NULL, 4, 2), SFRDE_EINVAL, "ckpt_bytes");
  expect(sfrde_resume(NULL, NULL, 0, NULL, 1, 0.0, 0, NULL), SFRDE_EINVAL, "resume");
  expect(sfrde_backward(NULL, NULL, 1, 1, 0.0, NULL, NULL, g, g, g), SFRDE_EINVAL, "backward");
  expect(sfrde_backward_noalloc(NULL, NULL, 1, 1, 0.0, NULL, NULL, g, g, g), SFRDE_EINVAL, "noalloc");
  expect(sfrde_destroy(NULL), SFRDE_EINVAL, "destroy");
  expect((int)sfrde_workspace_bytes(NULL), SFRDE_EINVAL, "workspace");
  expect(sfrde_profile(NULL, 1), SFRDE_EINVAL, "profile");
  expect(sfrde_profile_read(NULL, g, cnt), SFRDE_EINVAL, "profile_read");
  expect(sfrde_amplification(5, 1, NULL, NULL, NULL, NULL), SFRDE_EINVAL, "amplification");
  expect(sfrde_stability_boundary(0, -1, NULL, 4, NULL, NULL, NULL), SFRDE_EINVAL, "boundary");

  /* host helpers over their range: every boundary condition and size */
  static double lam[1024];
  for (int bc = 0; bc < 3; ++bc)
    for (int64_t n = 2; n <= 1024; n = n < 64 ? n + 1 : n * 2) {
      expect(sfrde_axis_eigenvalues(bc, n, 1.0 / (double)n, lam), SFRDE_OK, "eigenvalues");
      for (int64_t k = 0; k < n; ++k)
        if (!(lam[k] >= 0.0) || !isfinite(lam[k])) {
          fprintf(stderr, "eigenvalue bc %d n %lld k %lld = %g\n", bc, (long long)n,
                  (long long)k, lam[k]);
          ++failures;
        }
    }
  expect(sfrde_axis_eigenvalues(0, 1, 0.1, lam), SFRDE_EINVAL, "eigenvalues n 1");
  double c[6];
  for (int scheme = 0; scheme < 2; ++scheme)
    for (int deriv = 0; deriv < 2; ++deriv)
      for (double L = 0.0; L < 1e6; L = L < 1e-8 ? 1e-8 : L * 1.7) {
        expect(sfrde_eval_coefficients(scheme, L, 0.01, deriv, c), SFRDE_OK, "coefficients");
        for (int q = 0; q < 6; ++q)
          if (!isfinite(c[q])) {
            fprintf(stderr, "coefficient %d of L = %g not finite\n", q, L);
            ++failures;
          }
      }
  expect(sfrde_eval_coefficients(0, -1.0, 0.01, 0, c), SFRDE_EINVAL, "coefficients L < 0");
  printf("host driver: %d failures\n", failures);
  return failures == 0 ? 0 : 1;
}
