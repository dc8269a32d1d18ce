/* Plain C99 client of include/lbm.h: host-only entry points (no GPU work),
 * to check that the header compiles as C and the library links and answers
 * from C.  Prints one line per check; exit status 0 when all pass. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "lbm.h"

static int failures = 0;

static void check(int ok, const char *what) {
  printf("%s %s\n", ok ? "ok" : "FAIL", what);
  if (!ok) ++failures;
}

int main(void) {
  lbm_config cfg;
  check(lbm_config_default(&cfg, 64, 128) == LBM_OK, "lbm_config_default");
  check(cfg.layout == LBM_LAYOUT_COLUMN && cfg.storage == LBM_FP64 && cfg.path == LBM_PATH_FUSED,
        "defaults: column layout, FP64, fused path");
  size_t n64 = lbm_required_bytes(&cfg);
  cfg.storage = LBM_FP32;
  size_t n32 = lbm_required_bytes(&cfg);
  check(n64 > 0 && n32 > 0 && n64 == 2 * n32, "lbm_required_bytes halves for FP32");

  cfg.tau = 0.4; /* invalid: tau must exceed 1/2 */
  check(lbm_required_bytes(&cfg) == 0, "invalid tau rejected");
  const char *msg = lbm_last_error(NULL);
  check(msg != NULL && strstr(msg, "tau") != NULL, "lbm_last_error names the field");

  int32_t e[2 * LBM_NPOP], opp[LBM_NPOP];
  double w[LBM_NPOP], r = 0.0, sum = 0.0;
  check(lbm_tables(e, opp, w, &r) == LBM_OK, "lbm_tables");
  for (int l = 0; l < LBM_NPOP; ++l) sum += w[l];
  check(fabs(sum - 1.0) < 1e-15 && r > 1.19 && r < 1.20, "weights sum to 1, r ~ 1.197");
  int pairs = 1;
  for (int l = 0; l < LBM_NPOP; ++l)
    pairs &= e[2 * opp[l]] == -e[2 * l] && e[2 * opp[l] + 1] == -e[2 * l + 1];
  check(pairs, "opposite populations have opposite hops");

  double k[LBM_NPOP];
  check(lbm_wall_factors(1.0, k) == LBM_OK, "lbm_wall_factors");
  int same = 1;
  for (int l = 0; l < LBM_NPOP; ++l) same &= k[l] == w[l];
  check(same, "K_l(1) equals w_l");

  lbm_handle *h = (lbm_handle *)0;
  check(lbm_create(&cfg, NULL, 0, NULL, &h) == LBM_EINVAL && h == NULL, "lbm_create rejects NULL memory");
  lbm_destroy(NULL);
  return failures == 0 ? 0 : 1;
}
