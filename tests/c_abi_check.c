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

  /* every storage type and layout sizes; FP16 deviations add the reference rows */
  {
    size_t sz[3][2];
    int all = 1;
    for (int st = 0; st < 3; ++st)
      for (int lay = 0; lay < 2; ++lay) {
        lbm_config c;
        lbm_config_default(&c, 130, 257);
        c.storage = (lbm_storage)st;
        c.layout = (lbm_layout_kind)lay;
        sz[st][lay] = lbm_required_bytes(&c);
        all &= sz[st][lay] > 0;
      }
    check(all, "lbm_required_bytes for every storage type and layout");
    check(sz[0][0] > sz[1][0] && sz[1][0] > sz[2][0], "bytes shrink with the storage type");
    lbm_config c;
    lbm_config_default(&c, 130, 257);
    size_t plain = lbm_required_bytes(&c);
    c.stride_pad = 4096;
    check(lbm_required_bytes(&c) > plain, "stride padding adds bytes");
  }

  /* each validation branch, with the field named in the message */
  {
    struct {
      const char *field;
      int which;
    } bad[] = {{"lx", 0}, {"ly", 1}, {"tau", 2}, {"gravity", 3}, {"temperatures", 4},
               {"storage", 5}, {"layout", 6}, {"path", 7}, {"block", 8}, {"too large", 9}};
    for (unsigned i = 0; i < sizeof(bad) / sizeof(bad[0]); ++i) {
      lbm_config c;
      lbm_config_default(&c, 64, 128);
      switch (bad[i].which) {
        case 0: c.lx = 2; break;
        case 1: c.ly = 5; break;
        case 2: c.tau = 0.5; break;
        case 3: c.gy = NAN; break;
        case 4: c.t_top = 0.0; break;
        case 5: c.storage = (lbm_storage)7; break;
        case 6: c.layout = (lbm_layout_kind)5; break;
        case 7: c.path = (lbm_path)9; break;
        case 8: c.block = 96; break;
        default: c.lx = 1 << 20; c.ly = 1 << 20; break;
      }
      const size_t n = lbm_required_bytes(&c);
      const char *why = lbm_last_error(NULL);
      char line[96];
      snprintf(line, sizeof line, "invalid config rejected: %s", bad[i].field);
      check(n == 0 && why != NULL && strstr(why, bad[i].field) != NULL, line);
    }
    check(lbm_required_bytes(NULL) == 0, "NULL config rejected");
  }

  /* every entry point taking a handle rejects NULL */
  {
    double d[LBM_NPHASES];
    int64_t cnt[LBM_NPHASES], lay[6];
    int32_t xy = 0;
    int ok = 1;
    ok &= lbm_set_stream(NULL, NULL) == LBM_EINVAL;
    ok &= lbm_init_rt(NULL, NULL) == LBM_EINVAL;
    ok &= lbm_step(NULL, 1) == LBM_EINVAL;
    ok &= lbm_step_captured(NULL, 1) == LBM_EINVAL;
    ok &= lbm_run_phase(NULL, 0) == LBM_EINVAL;
    ok &= lbm_moments(NULL, d, d, d, d) == LBM_EINVAL;
    ok &= lbm_conservation(NULL, d) == LBM_EINVAL;
    ok &= lbm_get_populations(NULL, d) == LBM_EINVAL;
    ok &= lbm_set_populations(NULL, d) == LBM_EINVAL;
    ok &= lbm_get_sites(NULL, 1, &xy, &xy, d) == LBM_EINVAL;
    ok &= lbm_get_sites_noalloc(NULL, 1, &xy, &xy, d) == LBM_EINVAL;
    ok &= lbm_set_reference(NULL, d, 1.0, 1.0, 0) == LBM_EINVAL;
    ok &= lbm_get_reference(NULL, d, d, NULL) == LBM_EINVAL;
    ok &= lbm_set_timing(NULL, 1) == LBM_EINVAL;
    ok &= lbm_read_timing(NULL, d, cnt) == LBM_EINVAL;
    ok &= lbm_layout(NULL, lay) == LBM_EINVAL;
    check(ok, "NULL handle rejected by every entry point");
    check(lbm_last_error(NULL) != NULL, "lbm_last_error(NULL) is a message");
    check(lbm_probe_bandwidth(3, NULL, NULL, 4096, 0, NULL) == LBM_EINVAL, "probe rejects a bad mode");
  }

  /* engine host checks */
  {
    lbm_engine *e = (lbm_engine *)0;
    int32_t slot = 0, left = 0, til[3];
    double ms = 0.0;
    check(lbm_engine_required_bytes(16) > 0 && lbm_engine_required_bytes(0) == 0 &&
              lbm_engine_required_bytes((1 << 20) + 1) == 0,
          "lbm_engine_required_bytes bounds");
    check(lbm_engine_create(16, NULL, 0, NULL, &e) == LBM_EINVAL && e == NULL,
          "lbm_engine_create rejects NULL memory");
    int ok = 1;
    ok &= lbm_engine_add(NULL, NULL, 1, &slot) == LBM_EINVAL;
    ok &= lbm_engine_remove(NULL, 0) == LBM_EINVAL;
    ok &= lbm_engine_step(NULL, 1) == LBM_EINVAL;
    ok &= lbm_engine_status(NULL, &left) == LBM_EINVAL;
    ok &= lbm_engine_set_tiling(NULL, 0, 0, 0) == LBM_EINVAL;
    ok &= lbm_engine_get_tiling(NULL, til) == LBM_EINVAL;
    ok &= lbm_engine_tune(NULL, 1, til, &ms) == LBM_EINVAL;
    check(ok, "NULL engine rejected by every entry point");
    check(lbm_engine_last_error(NULL) != NULL, "lbm_engine_last_error(NULL) is a message");
    lbm_engine_destroy(NULL);
  }
  return failures == 0 ? 0 : 1;
}
