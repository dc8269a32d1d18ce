// C ABI of the ensemble engine (declared in include/lbm.h): slots over
// existing lattice handles, the active-slot table, the per-step graph and
// the tile autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "engine.hpp"
#include "internal.hpp"
#include "lbm.h"

using namespace d2q37;
using namespace d2q37::host;

struct lbm_engine {
  int max_slots = 0;
  int block = 256;
  int groups = 0;
  int schedule = SCHED_CHUNKED;
  int device = 0;
  int cus = 256;
  hipStream_t stream = nullptr;
  SlotDesc* d_slots = nullptr;
  int* d_table[2] = {nullptr, nullptr};  // per storage type: STORAGE_F64, STORAGE_F32
  int* d_status = nullptr;
  std::vector<SlotDesc> slots;        // host copies, as uploaded
  std::vector<lbm_handle*> handles;   // nullptr: free slot
  std::vector<int> steps_left;        // last known (from status)
  std::vector<int> status_init;       // (steps_left, cur) per slot as uploaded on add
  std::vector<int> table[2];
  int graph_classes = 0;              // storage types with a step node in the graph (bit mask)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string err;
};

namespace {

thread_local std::string g_engine_err;

int efail(lbm_engine* e, int code, const std::string& msg) {
  if (e)
    e->err = msg;
  else
    g_engine_err = msg;
  return code;
}

#define ENG_HIP(e, expr)                                                                 \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return efail((e), LBM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t v) { return (v + 255) / 256 * 256; }
size_t slots_bytes(int m) { return align256(sizeof(SlotDesc) * static_cast<size_t>(m)); }
size_t table_bytes(int m) { return align256(sizeof(int) * engine_table_ints(m)); }
size_t status_bytes(int m) { return align256(sizeof(int) * 2 * static_cast<size_t>(m)); }
int classes_present(const lbm_engine* e) {
  return (e->table[0].empty() || e->table[0][0] == 0 ? 0 : 1) | (e->table[1].empty() || e->table[1][0] == 0 ? 0 : 2);
}

void drop_graph(lbm_engine* e) {
  if (e->exec) (void)hipGraphExecDestroy(e->exec);
  if (e->graph) (void)hipGraphDestroy(e->graph);
  e->exec = nullptr;
  e->graph = nullptr;
}

// Rebuild and upload the active-slot tables: occupied slots with steps
// left, in slot order, one table per storage type, with the prefix sums of
// their tile counts.  The step graph is rebuilt when the set of storage
// types present changes.
int upload_table(lbm_engine* e) {
  const int m = e->max_slots;
  for (int c = 0; c < 2; ++c) {
    std::vector<int>& t = e->table[c];
    t.assign(engine_table_ints(m), 0);
    const int storage = c == 0 ? STORAGE_F64 : STORAGE_F32;
    int n = 0;
    long long total = 0;
    for (int s = 0; s < m; ++s) {
      if (!e->handles[s] || e->steps_left[s] <= 0 || e->slots[s].storage != storage) continue;
      t[2 + n] = s;
      t[2 + m + n] = static_cast<int>(total);
      total += static_cast<long long>(e->slots[s].lx) * e->slots[s].ny_waves;
      ++n;
    }
    // < 2^30 keeps every tile index plus a grid stride (< 2^23) inside int
    if (total >= (1LL << 30)) return efail(e, LBM_EINVAL, "too many tiles in the engine");
    t[0] = n;
    t[1] = static_cast<int>(total);
    t[2 + m + n] = static_cast<int>(total);
    ENG_HIP(e, hipMemcpyAsync(e->d_table[c], t.data(), t.size() * sizeof(int), hipMemcpyHostToDevice,
                              e->stream));
  }
  if (classes_present(e) != e->graph_classes) drop_graph(e);
  return LBM_OK;
}

// Upload every occupied slot (cur and steps_left as last known).
int upload_slots(lbm_engine* e) {
  for (int s = 0; s < e->max_slots; ++s) {
    if (!e->handles[s]) continue;
    SlotDesc& d = e->slots[s];
    d.steps_left = e->steps_left[s];
    d.cur = e->handles[s]->cur;
    ENG_HIP(e, hipMemcpyAsync(e->d_slots + s, &d, sizeof(SlotDesc), hipMemcpyHostToDevice, e->stream));
  }
  return LBM_OK;
}

// One engine step as a graph: a step kernel per storage type present (no
// dependency between them, so they may run concurrently), then the
// advance kernel after both.
int build_graph(lbm_engine* e) {
  drop_graph(e);
  const int classes = classes_present(e);
  ENG_HIP(e, hipGraphCreate(&e->graph, 0));
  std::vector<hipGraphNode_t> steps;
  int m = e->max_slots;
  const SlotDesc* cs = e->d_slots;
  const int* tables[2] = {e->d_table[0], e->d_table[1]};
  for (int c = 0; c < 2; ++c) {
    if (!(classes & (1 << c))) continue;
    void* f;
    dim3 g, t;
    ENG_HIP(e, engine_step_node(c == 0 ? STORAGE_F64 : STORAGE_F32, e->block, e->groups, e->schedule,
                                &f, &g, &t));
    void* args[] = {&cs, &tables[c], &m};
    hipKernelNodeParams p{};
    p.func = f;
    p.gridDim = g;
    p.blockDim = t;
    p.kernelParams = args;
    hipGraphNode_t node;
    ENG_HIP(e, hipGraphAddKernelNode(&node, e->graph, nullptr, 0, &p));
    steps.push_back(node);
  }
  void* fa;
  dim3 ga, ta;
  ENG_HIP(e, engine_advance_node(e->max_slots, &fa, &ga, &ta));
  SlotDesc* ms = e->d_slots;
  int* st = e->d_status;
  void* aargs[] = {&ms, &m, &st};
  hipKernelNodeParams pa{};
  pa.func = fa;
  pa.gridDim = ga;
  pa.blockDim = ta;
  pa.kernelParams = aargs;
  hipGraphNode_t adv;
  ENG_HIP(e, hipGraphAddKernelNode(&adv, e->graph, steps.data(), steps.size(), &pa));
  ENG_HIP(e, hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0));
  e->graph_classes = classes;
  return LBM_OK;
}

// Read (steps_left, cur) of every slot; write cur back to the handles.
int read_status(lbm_engine* e) {
  std::vector<int> st(2 * static_cast<size_t>(e->max_slots));
  ENG_HIP(e, hipMemcpyAsync(st.data(), e->d_status, st.size() * sizeof(int), hipMemcpyDeviceToHost,
                            e->stream));
  ENG_HIP(e, hipStreamSynchronize(e->stream));
  bool finished = false;
  for (int s = 0; s < e->max_slots; ++s) {
    if (!e->handles[s]) continue;
    if (st[2 * s] != e->steps_left[s] && st[2 * s] == 0) finished = true;
    e->steps_left[s] = st[2 * s];
    e->handles[s]->cur = st[2 * s + 1];
    e->slots[s].cur = st[2 * s + 1];
    e->slots[s].steps_left = st[2 * s];
  }
  if (finished) return upload_table(e);
  return LBM_OK;
}

bool valid_block(int b) { return b == 64 || b == 128 || b == 256 || b == 512; }

}  // namespace

namespace d2q37 {
namespace host {

int engine_refresh(lbm_engine* e) {
  DeviceGuard dg(e->device);
  return read_status(e);
}

void engine_detach(lbm_engine* e, int slot) { (void)lbm_engine_remove(e, slot); }

}  // namespace host
}  // namespace d2q37

extern "C" {

size_t lbm_engine_required_bytes(int32_t max_slots) {
  if (max_slots <= 0 || max_slots > (1 << 20)) {
    g_engine_err = "max_slots must be in [1, 2^20]";
    return 0;
  }
  return slots_bytes(max_slots) + 2 * table_bytes(max_slots) + status_bytes(max_slots);
}

int lbm_engine_create(int32_t max_slots, void* dev_mem, size_t dev_bytes, void* stream,
                      lbm_engine** out) {
  if (!out) return efail(nullptr, LBM_EINVAL, "out is NULL");
  *out = nullptr;
  const size_t need = lbm_engine_required_bytes(max_slots);
  if (need == 0) return efail(nullptr, LBM_EINVAL, g_engine_err);
  if (!dev_mem) return efail(nullptr, LBM_EINVAL, "dev_mem is NULL");
  if (reinterpret_cast<uintptr_t>(dev_mem) % 256) return efail(nullptr, LBM_ENOMEM, "dev_mem must be 256-byte aligned");
  if (dev_bytes < need) return efail(nullptr, LBM_ENOMEM, "dev_bytes < lbm_engine_required_bytes");
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, dev_mem) != hipSuccess) {
    (void)hipGetLastError();
    return efail(nullptr, LBM_EINVAL, "dev_mem is not device memory");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return efail(nullptr, LBM_EINVAL, "dev_mem is not device memory");
  auto* e = new lbm_engine();
  e->max_slots = max_slots;
  e->device = attr.device;
  e->stream = static_cast<hipStream_t>(stream);
  char* p = static_cast<char*>(dev_mem);
  e->d_slots = reinterpret_cast<SlotDesc*>(p);
  e->d_table[0] = reinterpret_cast<int*>(p + slots_bytes(max_slots));
  e->d_table[1] = reinterpret_cast<int*>(p + slots_bytes(max_slots) + table_bytes(max_slots));
  e->d_status = reinterpret_cast<int*>(p + slots_bytes(max_slots) + 2 * table_bytes(max_slots));
  e->slots.assign(max_slots, SlotDesc{});
  e->handles.assign(max_slots, nullptr);
  e->steps_left.assign(max_slots, 0);
  e->status_init.assign(2 * static_cast<size_t>(max_slots), 0);
  int cus = 0;
  DeviceGuard dg(e->device);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, e->device) != hipSuccess || cus <= 0)
    cus = 256;
  e->cus = cus;
  // default: a large strided grid (about one tile per work-group on big
  // lattices), which measured faster than a persistent chunked grid
  e->groups = 256 * cus;
  e->schedule = SCHED_STRIDED;
  // every slot starts free: zeroed descriptors (steps_left 0) and status
  std::vector<SlotDesc> zero(max_slots, SlotDesc{});
  std::vector<int> zst(2 * static_cast<size_t>(max_slots), 0);
  int rc = LBM_OK;
  if (hipMemcpyAsync(e->d_slots, zero.data(), zero.size() * sizeof(SlotDesc), hipMemcpyHostToDevice,
                     e->stream) != hipSuccess ||
      hipMemcpyAsync(e->d_status, zst.data(), zst.size() * sizeof(int), hipMemcpyHostToDevice,
                     e->stream) != hipSuccess)
    rc = efail(e, LBM_EDEVICE, "engine table upload failed");
  if (rc == LBM_OK) rc = upload_table(e);
  if (rc == LBM_OK && hipStreamSynchronize(e->stream) != hipSuccess) rc = LBM_EDEVICE;
  if (rc != LBM_OK) {
    g_engine_err = e->err;
    delete e;
    return rc;
  }
  *out = e;
  return LBM_OK;
}

int lbm_engine_set_tiling(lbm_engine* e, int32_t block, int32_t groups, int32_t schedule) {
  if (!e) return efail(nullptr, LBM_EINVAL, "engine is NULL");
  if (!valid_block(block)) return efail(e, LBM_EINVAL, "block must be 64, 128, 256 or 512");
  if (groups <= 0 || groups > (1 << 20)) return efail(e, LBM_EINVAL, "groups must be in [1, 2^20]");
  if (schedule != SCHED_CHUNKED && schedule != SCHED_STRIDED) return efail(e, LBM_EINVAL, "bad schedule");
  DeviceGuard dg(e->device);
  const int rc0 = read_status(e);
  if (rc0 != LBM_OK) return rc0;
  e->block = block;
  e->groups = groups;
  e->schedule = schedule;
  drop_graph(e);
  int rc = upload_slots(e);
  if (rc == LBM_OK) rc = upload_table(e);
  return rc;
}

int lbm_engine_get_tiling(const lbm_engine* e, int32_t out[3]) {
  if (!e || !out) return efail(nullptr, LBM_EINVAL, "engine/out is NULL");
  out[0] = e->block;
  out[1] = e->groups;
  out[2] = e->schedule;
  return LBM_OK;
}

int lbm_engine_add(lbm_engine* e, lbm_handle* h, int32_t steps, int32_t* slot) {
  if (!e) return efail(nullptr, LBM_EINVAL, "engine is NULL");
  if (!h || !slot) return efail(e, LBM_EINVAL, "handle/slot is NULL");
  if (steps < 0) return efail(e, LBM_EINVAL, "steps must be >= 0");
  if (!h->ready) return efail(e, LBM_ESTATE, "lattice not initialised");
  if (h->engine_slot >= 0) return efail(e, LBM_ESTATE, "lattice already in an engine");
  if (h->geo.storage != STORAGE_F64 && h->geo.storage != STORAGE_F32)
    return efail(e, LBM_EINVAL, "the engine steps LBM_FP64 and LBM_FP32 lattices");
  if (h->device != e->device) return efail(e, LBM_EINVAL, "lattice lives on another device");
  int s = 0;
  while (s < e->max_slots && e->handles[s]) ++s;
  if (s == e->max_slots) return efail(e, LBM_ENOMEM, "no free slot");
  DeviceGuard dg(e->device);
  ENG_HIP(e, hipStreamSynchronize(h->stream));  // the lattice's own pending work
  SlotDesc& d = e->slots[s];
  d = SlotDesc{};
  d.buf[0] = h->buf[0];
  d.buf[1] = h->buf[1];
  d.pstride = h->geo.pstride;
  d.cstride = h->geo.cstride;
  d.storage = h->geo.storage;
  d.lx = h->geo.lx;
  d.ly = h->geo.ly;
  d.ny_waves = (d.ly + 63) / 64;
  d.cur = h->cur;
  d.steps_left = steps;
  d.cp = h->cp;
  d.wp = h->wp;
  e->handles[s] = h;
  e->steps_left[s] = steps;
  // copies only from engine-owned host memory, which outlives them
  e->status_init[2 * s] = steps;
  e->status_init[2 * s + 1] = h->cur;
  ENG_HIP(e, hipMemcpyAsync(e->d_slots + s, &d, sizeof(SlotDesc), hipMemcpyHostToDevice, e->stream));
  ENG_HIP(e, hipMemcpyAsync(e->d_status + 2 * s, &e->status_init[2 * s], 2 * sizeof(int),
                            hipMemcpyHostToDevice, e->stream));
  const int rc = upload_table(e);
  if (rc != LBM_OK) {
    e->handles[s] = nullptr;
    e->steps_left[s] = 0;
    (void)hipStreamSynchronize(e->stream);
    return rc;
  }
  ENG_HIP(e, hipStreamSynchronize(e->stream));
  h->engine_slot = s;
  h->engine = e;
  h->home_stream = h->stream;
  h->stream = e->stream;
  *slot = s;
  return LBM_OK;
}

int lbm_engine_remove(lbm_engine* e, int32_t slot) {
  if (!e) return efail(nullptr, LBM_EINVAL, "engine is NULL");
  if (slot < 0 || slot >= e->max_slots || !e->handles[slot]) return efail(e, LBM_EINVAL, "no such slot");
  DeviceGuard dg(e->device);
  int rc = read_status(e);
  if (rc != LBM_OK) return rc;
  lbm_handle* h = e->handles[slot];
  h->engine_slot = -1;
  h->engine = nullptr;
  h->stream = h->home_stream;  // ordered: the engine stream is synchronised below
  e->handles[slot] = nullptr;
  e->steps_left[slot] = 0;
  e->slots[slot] = SlotDesc{};
  ENG_HIP(e, hipMemcpyAsync(e->d_slots + slot, &e->slots[slot], sizeof(SlotDesc), hipMemcpyHostToDevice,
                            e->stream));
  rc = upload_table(e);
  if (rc == LBM_OK) ENG_HIP(e, hipStreamSynchronize(e->stream));
  return rc;
}

int lbm_engine_step(lbm_engine* e, int32_t n) {
  if (!e) return efail(nullptr, LBM_EINVAL, "engine is NULL");
  if (n < 0) return efail(e, LBM_EINVAL, "n must be >= 0");
  if (n == 0 || classes_present(e) == 0) return LBM_OK;
  DeviceGuard dg(e->device);
  if (!e->exec) {
    const int rc = build_graph(e);
    if (rc != LBM_OK) return rc;
  }
  for (int32_t i = 0; i < n; ++i) ENG_HIP(e, hipGraphLaunch(e->exec, e->stream));
  return LBM_OK;
}

int lbm_engine_status(lbm_engine* e, int32_t* steps_left) {
  if (!e) return efail(nullptr, LBM_EINVAL, "engine is NULL");
  DeviceGuard dg(e->device);
  const int rc = read_status(e);
  if (rc != LBM_OK) return rc;
  if (steps_left)
    for (int s = 0; s < e->max_slots; ++s) steps_left[s] = e->handles[s] ? e->steps_left[s] : -1;
  return LBM_OK;
}

int lbm_engine_tune(lbm_engine* e, int32_t reps, int32_t out[3], double* best_ms) {
  if (!e) return efail(nullptr, LBM_EINVAL, "engine is NULL");
  if (reps <= 0) return efail(e, LBM_EINVAL, "reps must be > 0");
  if (classes_present(e) == 0) return efail(e, LBM_ESTATE, "no active lattice to tune on");
  DeviceGuard dg(e->device);
  int rc = read_status(e);
  if (rc != LBM_OK) return rc;
  hipEvent_t a, b;
  ENG_HIP(e, hipEventCreate(&a));
  ENG_HIP(e, hipEventCreate(&b));
  int best[3] = {e->block, e->groups, e->schedule};
  float best_t = 1e30f;
  const int blocks[] = {64, 128, 256, 512};
  const int per_cu[] = {2, 4, 8, 16, 32, 64, 128, 256, 512, 1024};
  for (int blk : blocks) {
    e->block = blk;
    rc = upload_slots(e);
    if (rc == LBM_OK) rc = upload_table(e);
    if (rc != LBM_OK) break;
    for (int k : per_cu) {
      for (int sch = SCHED_CHUNKED; sch <= SCHED_STRIDED; ++sch) {
        const int groups = k * e->cus;
        // step launches only: each reads the current buffer and writes the
        // other, so repeating them leaves the lattices' state unchanged
        const int classes = classes_present(e);
        auto launch_all = [&]() -> hipError_t {
          for (int c = 0; c < 2; ++c) {
            if (!(classes & (1 << c))) continue;
            hipError_t err = launch_engine_step(c == 0 ? STORAGE_F64 : STORAGE_F32, e->d_slots,
                                                e->d_table[c], e->max_slots, blk, groups, sch, e->stream);
            if (err != hipSuccess) return err;
          }
          return hipSuccess;
        };
        ENG_HIP(e, launch_all());
        ENG_HIP(e, hipEventRecord(a, e->stream));
        for (int r = 0; r < reps; ++r) ENG_HIP(e, launch_all());
        ENG_HIP(e, hipEventRecord(b, e->stream));
        ENG_HIP(e, hipEventSynchronize(b));
        float ms = 0.0f;
        ENG_HIP(e, hipEventElapsedTime(&ms, a, b));
        ms /= static_cast<float>(reps);
        if (ms < best_t) {
          best_t = ms;
          best[0] = blk;
          best[1] = groups;
          best[2] = sch;
        }
      }
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc != LBM_OK) return rc;
  e->block = best[0];
  e->groups = best[1];
  e->schedule = best[2];
  drop_graph(e);
  rc = upload_slots(e);
  if (rc == LBM_OK) rc = upload_table(e);
  if (rc == LBM_OK) ENG_HIP(e, hipStreamSynchronize(e->stream));
  if (out) {
    out[0] = best[0];
    out[1] = best[1];
    out[2] = best[2];
  }
  if (best_ms) *best_ms = best_t;
  return rc;
}

const char* lbm_engine_last_error(const lbm_engine* e) { return e ? e->err.c_str() : g_engine_err.c_str(); }

void lbm_engine_destroy(lbm_engine* e) {
  if (!e) return;
  {
    DeviceGuard dg(e->device);
    (void)read_status(e);
    // read_status may have queued a table upload from e's host memory
    (void)hipStreamSynchronize(e->stream);
    for (int s = 0; s < e->max_slots; ++s)
      if (e->handles[s]) {
        e->handles[s]->engine_slot = -1;
        e->handles[s]->engine = nullptr;
        e->handles[s]->stream = e->handles[s]->home_stream;
      }
    drop_graph(e);
  }
  delete e;
}

}  // extern "C"
