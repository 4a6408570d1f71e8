/* Host-side checks of the C ABI, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer against a host-only build of the library
 * (tests/test_host_sanitizers.py).  Every call here is answered by the
 * library's argument validation or host arithmetic before any HIP call, so
 * no GPU is needed; the sanitizers watch the host code on those paths. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "cssar.h"

static int failures = 0;

#define CHECK(cond)                                                \
  do {                                                             \
    if (!(cond)) {                                                 \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                  \
    }                                                              \
  } while (0)

static cssar_params stripmap(void) {
  cssar_params p;
  memset(&p, 0, sizeof p);
  p.fc = 5.3e9;
  p.Kr = 3e12;
  p.Tp = 1e-5;
  p.fs = 3.6e7;
  p.prf = 1700.0;
  p.v = 7100.0;
  p.r_ref = 8.5e5;
  p.ba = 1360.0;
  p.f_dc = 0.0;
  p.src = 1;
  return p;
}

int main(void) {
  /* plan inspection */
  static const int lengths[] = {64, 128, 256, 512, 768, 1024, 1536, 2048, 3072, 4096, 8192};
  for (size_t i = 0; i < sizeof lengths / sizeof lengths[0]; ++i) {
    int e = 0, np = 0, radices[8] = {0};
    CHECK(cssar_supported_length(lengths[i]) == 1);
    CHECK(cssar_plan_info(lengths[i], &e, &np, radices) == CSSAR_OK);
    int prod = 1;
    for (int s = 0; s < np; ++s) prod *= radices[s];
    CHECK(prod == lengths[i] && e > 0 && np > 0 && np <= 8);
  }
  static const int bad[] = {0, -4, 3, 100, 1000, 16384, 1 << 30};
  for (size_t i = 0; i < sizeof bad / sizeof bad[0]; ++i) {
    int e = 0, np = 0, radices[8] = {0};
    CHECK(cssar_supported_length(bad[i]) == 0);
    CHECK(cssar_plan_info(bad[i], &e, &np, radices) != CSSAR_OK);
  }

  /* the (K_a, K_r) parameterisation */
  cssar_params p = stripmap(), q;
  const double ka = cssar_azimuth_fm_rate(&p);
  CHECK(ka > 0.0 && isfinite(ka));
  CHECK(cssar_params_with_rates(&p, 1.5 * ka, 2.0 * p.Kr, &q) == CSSAR_OK);
  CHECK(fabs(cssar_azimuth_fm_rate(&q) / (1.5 * ka) - 1.0) < 1e-12 && q.Kr == 2.0 * p.Kr);
  CHECK(cssar_params_with_rates(&p, -1.0, p.Kr, &q) == CSSAR_EINVAL);
  CHECK(cssar_params_with_rates(&p, ka, NAN, &q) == CSSAR_EINVAL);
  CHECK(cssar_params_with_rates(NULL, ka, p.Kr, &q) == CSSAR_EINVAL);
  CHECK(cssar_azimuth_fm_rate(NULL) == 0.0);

  /* operator construction: invalid arguments, rejected before any HIP call */
  cssar_op* op = NULL;
  CHECK(cssar_make_operator(NULL, 256, 256, &op) == CSSAR_EINVAL && op == NULL);
  CHECK(cssar_make_operator(&p, 256, 256, NULL) == CSSAR_EINVAL);
  CHECK(cssar_make_operator(&p, 0, 256, &op) != CSSAR_OK && op == NULL);
  CHECK(cssar_make_operator(&p, 256, 100, &op) == CSSAR_EUNSUPPORTED && op == NULL);
  q = p;
  q.f_dc = 10.0;
  CHECK(cssar_make_operator(&q, 256, 256, &op) == CSSAR_EUNSUPPORTED && op == NULL);
  q = p;
  q.fs = -1.0;
  CHECK(cssar_make_operator(&q, 256, 256, &op) == CSSAR_EINVAL && op == NULL);
  q = p;
  q.prf = 1e9; /* beyond the migration singularity */
  CHECK(cssar_make_operator(&q, 256, 256, &op) == CSSAR_EINVAL && op == NULL);
  CHECK(cssar_make_operator_rda(&p, 256, 256, 7, &op) == CSSAR_EINVAL && op == NULL);
  CHECK(cssar_make_operator_rda(&p, 256, 256, 0, &op) == CSSAR_EINVAL && op == NULL);
  CHECK(strlen(cssar_last_error()) > 0);

  /* NULL handles */
  CHECK(cssar_destroy_operator(NULL) == CSSAR_OK);
  CHECK(cssar_workspace_size(NULL, 1) == 0);
  CHECK(cssar_operator_chain(NULL) == CSSAR_EINVAL);
  CHECK(cssar_ita_solve(NULL, NULL, NULL, 0.1f, 1, NULL, NULL, NULL, NULL) == CSSAR_EINVAL);
  CHECK(cssar_ita_solve_ex(NULL, NULL, NULL, 0.1f, 1, NULL, NULL, NULL, NULL) == CSSAR_EINVAL);
  CHECK(cssar_apply_G(NULL, NULL, NULL, NULL, NULL) == CSSAR_EINVAL);
  CHECK(cssar_apply_GH(NULL, NULL, NULL, NULL, NULL) == CSSAR_EINVAL);
  CHECK(cssar_sync_status(NULL, NULL) == CSSAR_EINVAL);
  CHECK(cssar_profile_enable(NULL, 1) == CSSAR_EINVAL);
  CHECK(cssar_make_batch(NULL, 0, NULL) == CSSAR_EINVAL);
  cssar_batch* b = NULL;
  cssar_op* ops[2] = {NULL, NULL};
  CHECK(cssar_make_batch(ops, 2, &b) == CSSAR_EINVAL && b == NULL);
  CHECK(cssar_destroy_batch(NULL) == CSSAR_OK);
  CHECK(cssar_batch_workspace_size(NULL) == 0);
  CHECK(cssar_batch_describe(NULL, NULL, 0) == CSSAR_EINVAL);
  CHECK(cssar_batch_set_graph(NULL, 1) == CSSAR_EINVAL);
  int scene = 7;
  CHECK(cssar_batch_sync_status(NULL, NULL, &scene) == CSSAR_EINVAL && scene == -1);
  CHECK(cssar_checkpoint_size(NULL, 20, 5) == 0);

  /* a long message is truncated, not overrun */
  char small[4];
  memset(small, 'x', sizeof small);
  CHECK(cssar_batch_describe(NULL, small, (int)sizeof small) == CSSAR_EINVAL);

  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("abi driver: all checks passed\n");
  return 0;
}
