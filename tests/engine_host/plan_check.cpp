// Host check of the two-step kernel's strip and segment plan
// (fused2_plan.hpp), on the CPU stand-in of the HIP runtime.  For every
// shape: the strips' output rows partition [0, ly); each strip's 64 rows
// lie inside the lattice and hold every row its outputs' second pull
// reaches inside the lattice; the interior launch's strips hold no wall
// row; the two launches take every strip once; the segments cover every
// column; and the lattices the plan refuses are exactly those below 64
// rows or not stored in binary64.
#include <cstdio>
#include <vector>

#include "fused2_plan.hpp"

using namespace d2q37;

static int failures = 0;
#define CHECK(c, ...)                       \
  do {                                      \
    if (!(c)) {                             \
      if (failures++ < 20) {                \
        std::printf("FAIL %s: ", #c);       \
        std::printf(__VA_ARGS__);           \
        std::printf("\n");                  \
      }                                     \
    }                                       \
  } while (0)

static void check(int lx, int ly, int simds) {
  Geometry g{};
  g.lx = lx;
  g.ly = ly;
  g.storage = STORAGE_F64;
  const Fused2Plan p = fused2_plan(g, simds);
  CHECK(p.ok == (ly >= F2_ROWS), "lx %d ly %d ok %d", lx, ly, p.ok);
  g.storage = STORAGE_F32;
  CHECK(!fused2_plan(g, simds).ok, "binary32 lattice %d x %d accepted", lx, ly);
  if (!p.ok) return;
  const int nstrip = fused2_strips(ly);
  CHECK(p.interior.nstrip == nstrip && p.wall.nstrip == nstrip, "nstrip %d x %d", lx, ly);
  int next = 0;
  for (int k = 0; k < nstrip; ++k) {
    const Fused2Rows r = fused2_rows(k, nstrip, ly);
    CHECK(r.out_lo == next, "%d x %d strip %d starts at %d, not %d", lx, ly, k, r.out_lo, next);
    CHECK(r.out_hi > r.out_lo, "%d x %d strip %d empty", lx, ly, k);
    CHECK(r.base >= 0 && r.base + F2_ROWS <= ly, "%d x %d strip %d base %d", lx, ly, k, r.base);
    for (int y = r.out_lo; y < r.out_hi; ++y) {
      const int lo = std::max(y - HALO, 0), hi = std::min(y + HALO, ly - 1);
      CHECK(lo >= r.base && hi < r.base + F2_ROWS, "%d x %d strip %d row %d pulls outside", lx, ly, k, y);
    }
    next = r.out_hi;
  }
  CHECK(next == ly, "%d x %d outputs end at %d", lx, ly, next);
  std::vector<int> taken(nstrip, 0);
  for (int i = 0; i < p.interior.count; ++i) {
    const int k = fused2_strip_of(p.interior, false, i);
    CHECK(k >= 0 && k < nstrip, "%d x %d interior strip %d", lx, ly, k);
    if (k < 0 || k >= nstrip) continue;
    ++taken[k];
    const Fused2Rows r = fused2_rows(k, nstrip, ly);
    CHECK(r.base >= WALL_ROWS && r.base + F2_ROWS <= ly - WALL_ROWS, "%d x %d interior strip %d holds a wall row",
          lx, ly, k);
  }
  for (int i = 0; i < p.wall.count; ++i) {
    const int k = fused2_strip_of(p.wall, true, i);
    CHECK(k >= 0 && k < nstrip, "%d x %d wall strip %d", lx, ly, k);
    if (k >= 0 && k < nstrip) ++taken[k];
  }
  for (int k = 0; k < nstrip; ++k) CHECK(taken[k] == 1, "%d x %d strip %d taken %d times", lx, ly, k, taken[k]);
  for (const Fused2Strips* s : {&p.interior, &p.wall}) {
    CHECK(s->seg_w >= 1 && s->seg_w <= lx, "%d x %d segment width %d", lx, ly, s->seg_w);
    const int nseg = (lx + s->seg_w - 1) / s->seg_w;
    CHECK((nseg - 1) * s->seg_w < lx && nseg * s->seg_w >= lx, "%d x %d segments", lx, ly);
  }
}

int main() {
  const int lxs[] = {1, 3, 7, 16, 33, 130, 515, 1024, 2048, 4096};
  for (int simds : {1024, 256, 40, 1})
    for (int lx : lxs)
      for (int ly = 1; ly <= 1300; ++ly) check(lx, ly, simds);
  for (int ly : {4096, 8192, 8193, 16384, 65536, 131072})
    for (int lx : {3, 2048, 8192}) check(lx, ly, 1024);
  // the benchmark lattice on one MI355X: one round, 7 interior segments of
  // 293 columns and 21 wall segments of 98
  Geometry g{};
  g.lx = 2048;
  g.ly = 8192;
  g.storage = STORAGE_F64;
  const Fused2Plan p = fused2_plan(g, 1024);
  CHECK(p.interior.count == 140 && p.interior.seg_w == 293 && p.wall.count == 2 && p.wall.seg_w == 98,
        "2048 x 8192: %d strips of %d, %d of %d", p.interior.count, p.interior.seg_w, p.wall.count,
        p.wall.seg_w);
  const long long waves = 140LL * 7 + 2LL * 21;
  CHECK(waves <= 1024, "2048 x 8192 waves %lld", waves);
  if (failures) {
    std::printf("%d failures\n", failures);
    return 1;
  }
  std::printf("two-step plan: ok\n");
  return 0;
}
