// Internal host-side definitions shared by the C-ABI translation units:
// the lattice handle, error reporting and small helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "kernels.hpp"
#include "lbm.h"

// A lattice bound to caller memory (see lbm_create).
struct lbm_handle {
  lbm_config cfg{};
  d2q37::Geometry geo{};
  size_t buf_bytes = 0;
  char* buf[2] = {nullptr, nullptr};
  int cur = 0;  // buffer holding the current populations
  int engine_slot = -1;          // slot while an ensemble engine steps this lattice
  lbm_engine* engine = nullptr;  // that engine
  hipStream_t home_stream = nullptr;  // the handle's stream before it joined the engine
  hipStream_t stream = nullptr;
  int device = 0;
  bool ready = false;
  bool has_ref = false;  // deviation storage: reference state set
  std::vector<double> rho_ref;          // that state (host copies): density per row,
  double t_layers[2] = {1.0, 1.0};      // temperatures below / from geo.ysplit
  d2q37::CollideParams cp{};
  d2q37::WallParams wp{};
  std::string err;
  // region path: a second stream for pbc and the border columns, and the
  // events that order it against the bulk launches on the caller's stream
  hipStream_t side = nullptr;
  hipEvent_t ev_ready = nullptr;   // caller's stream at the start of a step call
  hipEvent_t ev_border = nullptr;  // last border launch
  hipEvent_t ev_bulk = nullptr;    // last bulk launch
  // captured step sequences: (n, starting buffer) -> instantiated graph
  struct Captured {
    int n, cur, cur_after;  // steps, buffer at start and at the end
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<Captured> captured;
  hipStream_t cap = nullptr;  // private stream the step sequences are captured on
  // per-launch timing
  bool timing = false;
  std::vector<hipEvent_t> events;
  size_t ev_used = 0;
  struct Rec {
    int phase;
    size_t ev;
  };  // events ev, ev + 1 recorded on the launch's stream
  std::vector<Rec> recs;
};

namespace d2q37 {
namespace host {

// Engine hooks used by the lattice calls (defined with the engine): bring
// the handle's current-buffer index up to date, or take it out of its
// engine before the handle goes away.
int engine_refresh(lbm_engine* e);
void engine_detach(lbm_engine* e, int slot);

inline thread_local std::string g_err;

// Record a failure (on the handle, or per thread when there is none).
inline int fail(lbm_handle* h, int code, const std::string& msg) {
  if (h)
    h->err = msg;
  else
    g_err = msg;
  return code;
}

#define LBM_HIP(h, expr)                                                              \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail((h), LBM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)


// Make the handle's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1, want;
  explicit DeviceGuard(int d) : want(d) {
    if (hipGetDevice(&prev) == hipSuccess && prev != want) (void)hipSetDevice(want);
  }
  ~DeviceGuard() {
    if (prev >= 0 && prev != want) (void)hipSetDevice(prev);
  }
};

inline char* other(lbm_handle* h) { return h->buf[h->cur ^ 1]; }
inline char* current(lbm_handle* h) { return h->buf[h->cur]; }
inline double* scratch(lbm_handle* h) { return reinterpret_cast<double*>(other(h)); }

inline int elem_bytes(const Geometry& g) {
  return g.storage == STORAGE_F32 ? 4 : g.storage == STORAGE_F16DEV ? 2 : 8;
}


}  // namespace host
}  // namespace d2q37
