// Kernel launchers of the library (kernels.hpp, engine.hpp) for the CPU
// stand-in of the HIP runtime: each launch is queued on its stream and, when
// the stream runs it, touches the memory the real kernel would read and
// write (first and last element of each lattice copy it uses, every element
// of staging buffers), so that a launch that runs after its memory was freed
// is reported by the sanitizer.  The engine's step kernel walks its tile
// table as on the GPU and aborts if a tile would fall outside its slot's
// lattice; the advance kernel is simulated exactly (it is the state the
// host reads back).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "engine.hpp"
#include "kernels.hpp"

namespace d2q37 {
namespace {

size_t elem(int storage) { return storage == STORAGE_F64 ? 8 : storage == STORAGE_F32 ? 4 : 2; }

// Last element of a lattice copy: (l, X, y) = (36, lx + 5, ly - 1).
size_t last_byte(long long pstride, long long cstride, int lx, int ly, int storage) {
  const long long idx = 36 * pstride + static_cast<long long>(lx + 5) * cstride + (ly - 1);
  return static_cast<size_t>(idx) * elem(storage);
}

volatile unsigned char g_sink;

void touch_read(const void* p, size_t last) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  g_sink = b[0];
  g_sink = b[last];
}
void touch_write(void* p, size_t last) {
  unsigned char* b = static_cast<unsigned char*>(p);
  b[0] = 0;
  b[last] = 0;
}

void enqueue(hipStream_t s, std::function<void()> op) { hipstub::of(s).ops.push_back(std::move(op)); }

size_t last_of(const Geometry& g) { return last_byte(g.pstride, g.cstride, g.lx, g.ly, g.storage); }

// Engine kernels.  The step kernel walks the tile table as the GPU kernel
// does and checks what its indexing relies on: the active slots of its
// storage type in table order, prefix sums from 0 to the total, and for
// every slot with steps left a tile count of lx * ceil(ly / 64), so that
// every tile's column and row block lie inside that slot's lattice; it
// touches each column's first and last element in both copies of every
// slot it steps.  The advance kernel flips and counts as on the GPU.
void sim_check(bool ok, const char* what) {
  if (ok) return;
  std::fprintf(stderr, "engine step kernel stand-in: %s\n", what);
  std::abort();
}
template <int STORAGE>
void engine_step_sim(const std::vector<std::vector<unsigned char>>& a) {
  const SlotDesc* slots;
  const int* table;
  int m;
  std::memcpy(&slots, a[0].data(), sizeof slots);
  std::memcpy(&table, a[1].data(), sizeof table);
  std::memcpy(&m, a[2].data(), sizeof m);
  const int n = table[0];
  const int total = table[1];
  if (n <= 0 || total <= 0) return;
  const int* order = table + 2;
  const int* start = table + 2 + m;
  sim_check(n <= m, "more active slots than slots");
  sim_check(start[0] == 0 && start[n] == total, "prefix sums do not run from 0 to the tile total");
  for (int k = 0; k < n; ++k) {
    sim_check(start[k] <= start[k + 1], "prefix sums decrease");
    sim_check(order[k] >= 0 && order[k] < m, "slot id out of range");
    const SlotDesc& d = slots[order[k]];
    sim_check(d.storage == STORAGE, "slot of another storage type in this kernel's table");
    if (d.steps_left <= 0) continue;  // the kernel skips it
    sim_check(d.ny_waves == (d.ly + 63) / 64, "row blocks per column do not match ly");
    sim_check(static_cast<long long>(start[k + 1]) - start[k] == static_cast<long long>(d.lx) * d.ny_waves,
              "tile count of a stepped slot does not match its lattice");
    const size_t e = elem(d.storage);
    for (int x = 0; x < d.lx; ++x) {
      const long long col = static_cast<long long>(x + 3) * d.cstride;
      const size_t first = static_cast<size_t>(col) * e;
      const size_t last = static_cast<size_t>(col + 36 * d.pstride + (d.ly - 1)) * e;
      const unsigned char* src = reinterpret_cast<const unsigned char*>(d.buf[d.cur]);
      unsigned char* dst = reinterpret_cast<unsigned char*>(d.buf[d.cur ^ 1]);
      g_sink = src[first];
      g_sink = src[last];
      dst[first] = 0;
      dst[last] = 0;
    }
  }
}
void engine_advance_sim(const std::vector<std::vector<unsigned char>>& a) {
  SlotDesc* slots;
  int m;
  int* status;
  std::memcpy(&slots, a[0].data(), sizeof slots);
  std::memcpy(&m, a[1].data(), sizeof m);
  std::memcpy(&status, a[2].data(), sizeof status);
  for (int s = 0; s < m; ++s) {
    SlotDesc& d = slots[s];
    if (d.steps_left > 0) {
      d.cur ^= 1;
      d.steps_left -= 1;
    }
    status[2 * s] = d.steps_left;
    status[2 * s + 1] = d.cur;
  }
}
char g_step_f64, g_step_f32, g_advance;  // stand-in kernel "functions"

struct Register {
  Register() {
    hipstub::sims().push_back({&g_step_f64, engine_step_sim<STORAGE_F64>});
    hipstub::sims().push_back({&g_step_f32, engine_step_sim<STORAGE_F32>});
    for (const void* f : {static_cast<const void*>(&g_step_f64), static_cast<const void*>(&g_step_f32)})
      hipstub::arg_sizes().push_back({f, {sizeof(void*), sizeof(void*), sizeof(int)}});
    hipstub::sims().push_back({&g_advance, engine_advance_sim});
    hipstub::arg_sizes().push_back({&g_advance, {sizeof(void*), sizeof(int), sizeof(void*)}});
  }
} g_register;

}  // namespace

hipError_t launch_pbc(const Geometry& g, void* f, hipStream_t s) {
  const size_t last = last_of(g);
  enqueue(s, [=] { touch_write(f, last); });
  return hipSuccess;
}
hipError_t launch_propagate(const Geometry& g, const void* src, void* dst, hipStream_t s) {
  const size_t last = last_of(g);
  enqueue(s, [=] { touch_read(src, last); touch_write(dst, last); });
  return hipSuccess;
}
hipError_t launch_bc(const Geometry& g, void* f, const WallParams&, hipStream_t s) { return launch_pbc(g, f, s); }
hipError_t launch_collide(const Geometry& g, const void* src, void* dst, const CollideParams&, hipStream_t s) {
  return launch_propagate(g, src, dst, s);
}
hipError_t launch_fused(const Geometry& g, const void* src, void* dst, const CollideParams&, const WallParams&,
                        hipStream_t s, const ColumnSet*, bool) {
  return launch_propagate(g, src, dst, s);
}
hipError_t launch_fused2(const Geometry& g, const void* src, void* dst, const CollideParams&, const WallParams&,
                         const Fused2Strips&, bool, hipStream_t s) {
  return launch_propagate(g, src, dst, s);
}
hipError_t launch_moments(const Geometry& g, const void* f, double* out, hipStream_t s) {
  const size_t last = last_of(g);
  const size_t n = 4 * static_cast<size_t>(g.lx) * g.ly;
  enqueue(s, [=] { touch_read(f, last); for (size_t i = 0; i < n; ++i) out[i] = 1.0; });
  return hipSuccess;
}
hipError_t launch_conservation(const Geometry& g, const void* f, double* partials, double* result, hipStream_t s) {
  const size_t last = last_of(g);
  enqueue(s, [=] {
    touch_read(f, last);
    for (int i = 0; i < CONS_BLOCKS * CONS_FIELDS; ++i) partials[i] = 0.0;
    for (int k = 0; k < CONS_FIELDS; ++k) result[k] = 0.0;
  });
  return hipSuccess;
}
hipError_t launch_get_sites(const Geometry& g, const void* f, const int* xs, const int* ys, int n, double* out,
                            hipStream_t s) {
  const size_t last = last_of(g);
  enqueue(s, [=] {
    touch_read(f, last);
    for (int i = 0; i < n; ++i)
      for (int l = 0; l < 37; ++l) out[static_cast<size_t>(l) * n + i] = xs[i] + ys[i];
  });
  return hipSuccess;
}
hipError_t launch_init_rt(const Geometry& g, void* f, const RtParams&, hipStream_t s) { return launch_pbc(g, f, s); }
hipError_t launch_rt_reference(const Geometry& g, double* ref, double* inv_ref, const RtParams&, hipStream_t s) {
  const int ly = g.ly;
  enqueue(s, [=] { for (int y = 0; y < ly; ++y) { ref[y] = 1.0; inv_ref[y] = 1.0; } });
  return hipSuccess;
}
hipError_t launch_encode_population(const Geometry& g, const double* in, void* f, int, hipStream_t s) {
  const size_t last = last_of(g);
  const size_t n = static_cast<size_t>(g.lx) * g.ly;
  enqueue(s, [=] { double acc = 0; for (size_t i = 0; i < n; ++i) acc += in[i]; g_sink = acc > 0; touch_write(f, last); });
  return hipSuccess;
}
hipError_t launch_decode_population(const Geometry& g, const void* f, double* out, int l, hipStream_t s) {
  const size_t last = last_of(g);
  const size_t n = static_cast<size_t>(g.lx) * g.ly;
  enqueue(s, [=] { touch_read(f, last); for (size_t i = 0; i < n; ++i) out[i] = l; });
  return hipSuccess;
}
hipError_t launch_probe(int, const void*, void*, size_t, int, hipStream_t) { return hipSuccess; }

hipError_t launch_engine_step(int storage, const SlotDesc* slots, const int* table, int max_slots, int, int, int,
                              hipStream_t s) {
  const void* f = storage == STORAGE_F32 ? &g_step_f32 : &g_step_f64;
  void* args[] = {&slots, &table, &max_slots};
  return hipLaunchKernel(f, dim3(1), dim3(64), args, 0, s);
}
hipError_t launch_engine_advance(SlotDesc* slots, int max_slots, int* status, hipStream_t s) {
  void* args[] = {&slots, &max_slots, &status};
  return hipLaunchKernel(&g_advance, dim3(1), dim3(64), args, 0, s);
}
hipError_t engine_step_node(int storage, int block, int groups, int, void** func, dim3* grid, dim3* threads) {
  if (groups <= 0) return hipErrorInvalidValue;
  *func = storage == STORAGE_F32 ? static_cast<void*>(&g_step_f32) : static_cast<void*>(&g_step_f64);
  *grid = dim3(groups);
  *threads = dim3(block);
  return hipSuccess;
}
hipError_t engine_advance_node(int, void** func, dim3* grid, dim3* threads) {
  *func = &g_advance;
  *grid = dim3(1);
  *threads = dim3(256);
  return hipSuccess;
}

}  // namespace d2q37
