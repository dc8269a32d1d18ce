// Drives the ensemble engine's host code through the C ABI, on the CPU
// stand-in of the HIP runtime, with the call sequences of the GPU engine
// tests: lattices of several sizes and storage types joining an engine,
// stepping under several tilings, a lattice leaving mid-run and its slot
// being reused, status and population read-back of members and former
// members, a member refused a direct step, and teardown in the order the
// Python owners use (engine first, then lattices, then their memory).
// Every asynchronous copy and launch runs only at the synchronisation that
// covers it, so a source, destination or lattice buffer that dies before
// then is a sanitizer report.  Exit status 0: the sequences completed and
// every checked value was as expected.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "lbm.h"

namespace {

int g_fail = 0;
#define CHECK(cond)                                                           \
  do {                                                                        \
    if (!(cond)) {                                                            \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
      g_fail = 1;                                                             \
    }                                                                         \
  } while (0)

struct Lat {
  lbm_handle* h = nullptr;
  void* mem = nullptr;
  int lx = 0, ly = 0;
};

Lat make(int lx, int ly, lbm_storage st, lbm_layout_kind layout) {
  Lat L;
  lbm_config c;
  lbm_config_default(&c, lx, ly);
  c.storage = st;
  c.layout = layout;
  const size_t n = lbm_required_bytes(&c);
  CHECK(n > 0);
  L.mem = std::aligned_alloc(256, (n + 255) / 256 * 256);
  CHECK(lbm_create(&c, L.mem, n, nullptr, &L.h) == LBM_OK);
  const double amp[2] = {0.5, 0.25}, phase[2] = {0.1, 0.2};
  lbm_rt_params rt{2.0, 0.5 * (ly - 1), 2, amp, phase};
  CHECK(lbm_init_rt(L.h, &rt) == LBM_OK);
  L.lx = lx;
  L.ly = ly;
  return L;
}

void close(Lat& L) {
  lbm_destroy(L.h);
  std::free(L.mem);
  L = Lat{};
}

std::vector<double> get(Lat& L) {
  std::vector<double> out(static_cast<size_t>(LBM_NPOP) * L.lx * L.ly);
  CHECK(lbm_get_populations(L.h, out.data()) == LBM_OK);
  return out;
}

struct Eng {
  lbm_engine* e = nullptr;
  void* mem = nullptr;
  int max_slots = 0;
};

Eng engine(int max_slots) {
  Eng E;
  const size_t n = lbm_engine_required_bytes(max_slots);
  E.mem = std::aligned_alloc(256, (n + 255) / 256 * 256);
  CHECK(lbm_engine_create(max_slots, E.mem, n, nullptr, &E.e) == LBM_OK);
  E.max_slots = max_slots;
  return E;
}

void close(Eng& E) {
  lbm_engine_destroy(E.e);
  std::free(E.mem);
  E = Eng{};
}

std::vector<int32_t> status(Eng& E) {
  std::vector<int32_t> left(E.max_slots);
  CHECK(lbm_engine_status(E.e, left.data()) == LBM_OK);
  return left;
}

// A mix of lattices stepped together, then read back (the mix test).
void mix(int block, int groups, int sched) {
  struct Spec { int lx, ly; lbm_storage st; int steps; lbm_layout_kind lay; };
  const Spec specs[] = {{64, 128, LBM_FP64, 9, LBM_LAYOUT_COLUMN}, {37, 70, LBM_FP32, 5, LBM_LAYOUT_PLANAR},
                        {130, 257, LBM_FP64, 12, LBM_LAYOUT_PLANAR}, {3, 6, LBM_FP64, 4, LBM_LAYOUT_COLUMN},
                        {9, 1100, LBM_FP32, 7, LBM_LAYOUT_COLUMN}, {16, 32, LBM_FP64, 0, LBM_LAYOUT_PLANAR},
                        {256, 64, LBM_FP32, 3, LBM_LAYOUT_COLUMN}};
  std::vector<Lat> lats;
  for (const Spec& s : specs) lats.push_back(make(s.lx, s.ly, s.st, s.lay));
  Eng E = engine(16);
  if (block) CHECK(lbm_engine_set_tiling(E.e, block, groups, sched) == LBM_OK);
  std::vector<int32_t> slots;
  for (size_t i = 0; i < lats.size(); ++i) {
    int32_t s = -1;
    CHECK(lbm_engine_add(E.e, lats[i].h, specs[i].steps, &s) == LBM_OK);
    slots.push_back(s);
  }
  CHECK(lbm_engine_step(E.e, 14) == LBM_OK);
  const std::vector<int32_t> left = status(E);
  for (int32_t s : slots) CHECK(left[s] == 0);
  for (Lat& L : lats) (void)get(L);
  close(E);
  for (Lat& L : lats) close(L);
}

// Lattices join and leave between engine steps (the join/leave test).
void join_and_leave() {
  Lat a = make(64, 128, LBM_FP64, LBM_LAYOUT_COLUMN);
  Lat b = make(37, 70, LBM_FP32, LBM_LAYOUT_PLANAR);
  Lat c = make(130, 257, LBM_FP64, LBM_LAYOUT_PLANAR);
  Eng E = engine(4);
  int32_t sa = -1, sb = -1, sc = -1;
  CHECK(lbm_engine_add(E.e, a.h, 10, &sa) == LBM_OK);
  CHECK(lbm_engine_step(E.e, 3) == LBM_OK);
  CHECK(lbm_engine_add(E.e, b.h, 6, &sb) == LBM_OK);
  CHECK(lbm_engine_step(E.e, 2) == LBM_OK);
  CHECK(lbm_engine_remove(E.e, sa) == LBM_OK);
  CHECK(lbm_engine_add(E.e, c.h, 4, &sc) == LBM_OK);
  CHECK(lbm_engine_step(E.e, 8) == LBM_OK);
  const std::vector<int32_t> left = status(E);
  CHECK(sc == sa);
  CHECK(left[sb] == 0 && left[sc] == 0);
  for (int s = 0; s < 4; ++s)
    if (s != sb && s != sc) CHECK(left[s] == -1);
  (void)get(a);
  (void)get(b);
  (void)get(c);
  CHECK(lbm_step(b.h, 1) == LBM_ESTATE);
  CHECK(lbm_step(a.h, 1) == LBM_OK);
  (void)get(a);
  close(E);
  close(a);
  close(b);
  close(c);
}

// A serving-like churn: members finish at different times, are read back
// and removed, and their lattices and memory are freed while the engine
// keeps stepping the others; new lattices take the freed slots.
void churn() {
  Eng E = engine(3);
  std::vector<Lat> active(3);
  std::vector<int> left_of(3, 0);
  int next = 0;
  for (int round = 0; round < 40; ++round) {
    for (int s = 0; s < 3; ++s)
      if (!active[s].h) {
        const int k = next++;
        active[s] = make(8 + 5 * (k % 7), 16 + 9 * (k % 5), k % 2 ? LBM_FP32 : LBM_FP64,
                         k % 3 ? LBM_LAYOUT_COLUMN : LBM_LAYOUT_PLANAR);
        int32_t slot = -1;
        left_of[s] = 1 + k % 4;
        CHECK(lbm_engine_add(E.e, active[s].h, left_of[s], &slot) == LBM_OK);
        CHECK(slot == s);
      }
    int n = 1000;
    for (int s = 0; s < 3; ++s) n = left_of[s] < n ? left_of[s] : n;
    CHECK(lbm_engine_step(E.e, n) == LBM_OK);
    (void)status(E);
    for (int s = 0; s < 3; ++s) {
      left_of[s] -= n;
      if (left_of[s] == 0) {
        (void)get(active[s]);
        CHECK(lbm_engine_remove(E.e, s) == LBM_OK);
        close(active[s]);
      }
    }
  }
  close(E);
  for (Lat& L : active)
    if (L.h) close(L);
}

}  // namespace

int main() {
  mix(0, 0, 0);
  mix(64, 3, 0);
  mix(128, 1024, 1);
  join_and_leave();
  join_and_leave();
  churn();
  // a lattice destroyed while it is still in an engine leaves it first
  Lat a = make(16, 32, LBM_FP64, LBM_LAYOUT_COLUMN);
  Eng E = engine(2);
  int32_t s = -1;
  CHECK(lbm_engine_add(E.e, a.h, 5, &s) == LBM_OK);
  CHECK(lbm_engine_step(E.e, 2) == LBM_OK);
  close(a);
  CHECK(status(E)[s] == -1);
  close(E);
  std::printf("engine host sequences: %s\n", g_fail ? "FAILED" : "ok");
  return g_fail;
}
