// C ABI of the D2Q37 library (declared in include/lbm.h): argument and
// config validation, the lattice layout in the caller's device memory, the
// double-buffer state machine of the time step, and kernel launches on the
// caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"
#include "fused2_plan.hpp"
#include "kernels.hpp"
#include "lbm.h"

using namespace d2q37;
using namespace d2q37::host;

namespace {

constexpr long long kMaxSites = (1LL << 29);  // (lx + 6) * pitch; row byte offsets fit 32 bits

long long round_up(long long v, long long m) { return (v + m - 1) / m * m; }

struct Layout {
  Geometry geo;
  size_t buf_bytes;
  size_t ref_bytes;  // deviation storage: rho_ref[ly], 1/rho_ref[ly], the layer factors
  size_t total() const { return 2 * buf_bytes + ref_bytes; }
};

// Default work-group size: the fastest measured on the 2048 x 8192 fused
// step per storage type (512 for binary64, 256 for binary32, 64 for
// binary16 deviations), but no more rows than the smallest power of two
// covering ly, so that short columns do not idle most of the lanes.  A
// lattice with fewer wavefronts than an MI355X has SIMDs (256 CUs x 4)
// gets one-wavefront work-groups, spread over as many CUs as possible.
int default_block(int storage, int lx, int ly) {
  const long long waves = static_cast<long long>(lx) * ((ly + 63) / 64);
  if (waves < 1024) return 64;
  const int pref = storage == LBM_FP64 ? 512 : storage == LBM_FP32 ? 256 : 64;
  int b = 64;
  while (b < pref && b < ly) b *= 2;
  return b;
}

// Validate cfg and derive the layout; returns LBM_OK or LBM_EINVAL with *why.
int make_layout(const lbm_config* c, Layout* out, std::string* why) {
  if (!c) return *why = "config is NULL", LBM_EINVAL;
  if (c->lx < 3) return *why = "lx must be >= 3 (three halo columns per side)", LBM_EINVAL;
  if (c->ly < 2 * WALL_ROWS) return *why = "ly must be >= 6 (two bands of 3 wall rows)", LBM_EINVAL;
  if (!std::isfinite(c->tau) || !(c->tau > 0.5)) return *why = "tau must be finite and > 0.5", LBM_EINVAL;
  if (!std::isfinite(c->gx) || !std::isfinite(c->gy)) return *why = "gravity must be finite", LBM_EINVAL;
  if (!std::isfinite(c->t_bottom) || !(c->t_bottom > 0.0) || !std::isfinite(c->t_top) ||
      !(c->t_top > 0.0))
    return *why = "wall temperatures must be finite and > 0", LBM_EINVAL;
  if (c->storage != LBM_FP64 && c->storage != LBM_FP32 && c->storage != LBM_FP16DEV)
    return *why = "storage must be LBM_FP64, LBM_FP32 or LBM_FP16DEV", LBM_EINVAL;
  if (c->layout != LBM_LAYOUT_COLUMN && c->layout != LBM_LAYOUT_PLANAR)
    return *why = "layout must be LBM_LAYOUT_COLUMN or LBM_LAYOUT_PLANAR", LBM_EINVAL;
  if (c->path != LBM_PATH_SEPARATE && c->path != LBM_PATH_FUSED && c->path != LBM_PATH_REGIONS &&
      c->path != LBM_PATH_FUSED2)
    return *why = "path must be LBM_PATH_SEPARATE, LBM_PATH_FUSED, LBM_PATH_REGIONS or LBM_PATH_FUSED2",
           LBM_EINVAL;
  if (c->path == LBM_PATH_FUSED2 && c->storage != LBM_FP64)
    return *why = "LBM_PATH_FUSED2 takes LBM_FP64 storage (its intermediate step is binary64)", LBM_EINVAL;
  const int block = c->block == 0 ? default_block(c->storage, c->lx, c->ly) : c->block;
  if (block != 64 && block != 128 && block != 256 && block != 512 && block != 1024)
    return *why = "block must be 0, 64, 128, 256, 512 or 1024", LBM_EINVAL;
  if (c->ny_pad > (1 << 20)) return *why = "ny_pad too large", LBM_EINVAL;
  if (c->stride_pad > (1LL << 24)) return *why = "stride_pad too large", LBM_EINVAL;

  Geometry g{};
  g.lx = c->lx;
  g.ly = c->ly;
  g.storage = c->storage == LBM_FP32 ? STORAGE_F32
              : c->storage == LBM_FP16DEV ? STORAGE_F16DEV : STORAGE_F64;
  g.layout = c->layout == LBM_LAYOUT_PLANAR ? LAYOUT_PLANAR : LAYOUT_COLUMN;
  g.block = block;
  const long long ny = round_up(c->ly, 64) + (c->ny_pad > 0 ? c->ny_pad : 0);
  const long long nx = static_cast<long long>(c->lx) + 2 * HALO;
  if (nx * ny >= kMaxSites)
    return *why = "lattice too large: (lx + 6) * pitch must stay below 2^29 sites", LBM_EINVAL;
  g.ny = static_cast<int>(ny);
  g.ny_blocks = (c->ly + block - 1) / block;
  if (static_cast<long long>(c->lx) * g.ny_blocks >= (1LL << 31))
    return *why = "too many work-groups", LBM_EINVAL;
  const long long pad = c->stride_pad > 0 ? c->stride_pad : 0;
  long long elems;
  if (g.layout == LAYOUT_PLANAR) {
    g.cstride = ny;
    g.pstride = round_up(nx * ny, 64) + pad;
    elems = NPOP * g.pstride;
  } else {
    g.pstride = ny;
    g.cstride = NPOP * ny + pad;
    elems = nx * g.cstride;
  }
  // byte offsets from a column's start to 3 rows past its last run must
  // fit a buffer descriptor's 31-bit range
  g.run_off = (NPOP * g.pstride + ny + 2 * HALO) * elem_bytes(g) < (1LL << 31) - 1 ? 1 : 0;
  out->geo = g;
  out->buf_bytes = static_cast<size_t>(round_up(elems * elem_bytes(g), 256));
  out->ref_bytes = g.storage == STORAGE_F16DEV
                       ? static_cast<size_t>(2 * round_up(8LL * c->ly, 256) + round_up(8LL * KF_LEN, 256))
                       : 0;
  // host transfers stage one population ([lx][ly] binary64) in the idle copy
  if (static_cast<size_t>(8) * c->lx * c->ly > out->buf_bytes)
    return *why = "internal: staging does not fit", LBM_EINVAL;
  return LBM_OK;
}

// Launch with optional timing events around it.
int run_phase(lbm_handle* h, int phase);

template <class F>
int timed_on(lbm_handle* h, int phase, hipStream_t stream, F&& launch) {
  size_t ev = 0;
  if (h->timing) {
    if (h->ev_used + 2 > h->events.size()) {
      for (int k = 0; k < 256; ++k) {
        hipEvent_t e;
        LBM_HIP(h, hipEventCreate(&e));
        h->events.push_back(e);
      }
    }
    ev = h->ev_used;
    h->ev_used += 2;
    LBM_HIP(h, hipEventRecord(h->events[ev], stream));
  }
  LBM_HIP(h, launch());
  if (h->timing) {
    LBM_HIP(h, hipEventRecord(h->events[ev + 1], stream));
    h->recs.push_back({phase, ev});
  }
  return LBM_OK;
}

template <class F>
int timed(lbm_handle* h, int phase, F&& launch) {
  return timed_on(h, phase, h->stream, launch);
}

// The second stream and events of the region path (created outside any
// stream capture).  The stream is non-blocking: every ordering the region
// schedule needs is an explicit event, and a blocking stream would also be
// ordered against the legacy null stream, serialising the bulk launches
// with the border launches when the caller steps on the null stream.
int ensure_side(lbm_handle* h) {
  if (h->side) return LBM_OK;
  LBM_HIP(h, hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
  LBM_HIP(h, hipEventCreateWithFlags(&h->ev_ready, hipEventDisableTiming));
  LBM_HIP(h, hipEventCreateWithFlags(&h->ev_border, hipEventDisableTiming));
  LBM_HIP(h, hipEventCreateWithFlags(&h->ev_bulk, hipEventDisableTiming));
  return LBM_OK;
}

// One step of the fused path: one launch that wraps x.
int fused_step(lbm_handle* h) { return run_phase(h, LBM_PHASE_FUSED); }

// n steps of the region path.  Step k runs the fused kernel on the bulk
// columns 3..Lx-4 (which pull from no halo) on the caller's stream, and pbc
// followed by the 3 + 3 border columns on the side stream, concurrently.
// Within a step the two write disjoint columns of the destination, so the
// only orderings are across steps:
//   bulk k   after border k-1 (it reads the border columns border k-1 wrote,
//            and overwrites the bulk columns border k-1 read);
//   border k after bulk k-1   (it reads the bulk columns next to the border
//            that bulk k-1 wrote, and overwrites the border columns bulk
//            k-1 read);
//   pbc k    after border k-1 (it copies the border columns into the halo;
//            same stream).
// The first step of a call waits for everything already on the caller's
// stream, and the caller's stream waits for the last border at the end, so
// the call is ordered on the caller's stream as a whole.  Lattices narrower
// than 7 columns have no bulk and take the plain fused step.
int region_steps(lbm_handle* h, int32_t n) {
  const Geometry& g = h->geo;
  if (g.lx < 7) {
    for (int32_t k = 0; k < n; ++k) {
      const int rc = fused_step(h);
      if (rc != LBM_OK) return rc;
    }
    return LBM_OK;
  }
  if (n == 0) return LBM_OK;
  int rc = ensure_side(h);
  if (rc != LBM_OK) return rc;
  const ColumnSet bulk{HALO, g.lx - 2 * HALO, 0};
  const ColumnSet border{0, HALO, g.lx - HALO, HALO};
  LBM_HIP(h, hipEventRecord(h->ev_ready, h->stream));
  LBM_HIP(h, hipStreamWaitEvent(h->side, h->ev_ready, 0));
  for (int32_t k = 0; k < n; ++k) {
    if (k > 0) LBM_HIP(h, hipStreamWaitEvent(h->stream, h->ev_border, 0));
    rc = timed_on(h, LBM_PHASE_PBC, h->side, [&] { return launch_pbc(g, current(h), h->side); });
    if (rc != LBM_OK) return rc;
    if (k > 0) LBM_HIP(h, hipStreamWaitEvent(h->side, h->ev_bulk, 0));
    rc = timed_on(h, LBM_PHASE_FUSED_BORDER, h->side, [&] {
      return launch_fused(g, current(h), other(h), h->cp, h->wp, h->side, &border);
    });
    if (rc != LBM_OK) return rc;
    LBM_HIP(h, hipEventRecord(h->ev_border, h->side));
    rc = timed(h, LBM_PHASE_FUSED_BULK,
               [&] { return launch_fused(g, current(h), other(h), h->cp, h->wp, h->stream, &bulk); });
    if (rc != LBM_OK) return rc;
    LBM_HIP(h, hipEventRecord(h->ev_bulk, h->stream));
    h->cur ^= 1;
  }
  LBM_HIP(h, hipStreamWaitEvent(h->stream, h->ev_border, 0));
  return LBM_OK;
}

// n steps of the two-step path: n / 2 launch pairs, then one fused step
// if n is odd.  A pair steps the interior strips on the caller's stream
// and the wall strips on the side stream concurrently (they write disjoint
// rows of the destination and read only the source); the side stream
// waits for everything before the pair and the caller's stream for the
// wall launch after it, so each pair is ordered on the caller's stream as
// a whole.  Lattices lower than 64 rows take fused steps.
int fused2_steps(lbm_handle* h, int32_t n) {
  const Geometry& g = h->geo;
  int cus = 0;
  LBM_HIP(h, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
  const Fused2Plan plan = fused2_plan(g, 4 * cus);
  int rc = LBM_OK;
  if (plan.ok && n >= 2) {
    rc = ensure_side(h);
    if (rc != LBM_OK) return rc;
    for (; n >= 2; n -= 2) {
      LBM_HIP(h, hipEventRecord(h->ev_ready, h->stream));
      LBM_HIP(h, hipStreamWaitEvent(h->side, h->ev_ready, 0));
      LBM_HIP(h, launch_fused2(g, current(h), other(h), h->cp, h->wp, plan.wall, true, h->side));
      LBM_HIP(h, hipEventRecord(h->ev_border, h->side));
      rc = timed(h, LBM_PHASE_FUSED2, [&] {
        return launch_fused2(g, current(h), other(h), h->cp, h->wp, plan.interior, false, h->stream);
      });
      if (rc != LBM_OK) return rc;
      LBM_HIP(h, hipStreamWaitEvent(h->stream, h->ev_border, 0));
      h->cur ^= 1;
    }
  }
  for (; n > 0; --n) {
    rc = fused_step(h);
    if (rc != LBM_OK) return rc;
  }
  return LBM_OK;
}

int run_phase(lbm_handle* h, int phase) {
  const Geometry& g = h->geo;
  int rc = LBM_OK;
  switch (phase) {
    case LBM_PHASE_PBC:
      rc = timed(h, phase, [&] { return launch_pbc(g, current(h), h->stream); });
      break;
    case LBM_PHASE_PROPAGATE:
      rc = timed(h, phase, [&] { return launch_propagate(g, current(h), other(h), h->stream); });
      if (rc == LBM_OK) h->cur ^= 1;
      break;
    case LBM_PHASE_BC:
      rc = timed(h, phase, [&] { return launch_bc(g, current(h), h->wp, h->stream); });
      break;
    case LBM_PHASE_COLLIDE:
      rc = timed(h, phase, [&] { return launch_collide(g, current(h), other(h), h->cp, h->stream); });
      if (rc == LBM_OK) h->cur ^= 1;
      break;
    case LBM_PHASE_FUSED:  // periodic x by wrapping
      rc = timed(h, phase, [&] {
        return launch_fused(g, current(h), other(h), h->cp, h->wp, h->stream, nullptr, true);
      });
      if (rc == LBM_OK) h->cur ^= 1;
      break;
    default:
      return fail(h, LBM_EINVAL, "unknown phase");
  }
  return rc;
}

// Build and upload the deviation-storage reference from the reference
// state: density rho(y) per row, temperature t_lo on rows y < ysplit and
// t_hi on rows y >= ysplit.  Uploads rho, 1 / rho and the shell factors
// K_s(t_lo), K_s(t_hi) (the wall factor of the first population of shell
// s: the zero-velocity equilibrium per unit density), their reciprocals
// and the shell weights divided by them, each rounded once.  Keeps host copies for
// lbm_get_reference.  Synchronises the handle's stream.
int set_reference_table(lbm_handle* h, const double* rho, double t_lo, double t_hi, int ysplit) {
  const int ly = h->geo.ly;
  if (ysplit < 0 || ysplit > ly) return fail(h, LBM_EINVAL, "y_split must be in [0, Ly]");
  if (!std::isfinite(t_lo) || !(t_lo > 0.0) || !std::isfinite(t_hi) || !(t_hi > 0.0))
    return fail(h, LBM_EINVAL, "layer temperatures must be finite and > 0");
  std::vector<double> rows(2 * static_cast<size_t>(ly));
  for (int y = 0; y < ly; ++y) {
    if (!std::isfinite(rho[y]) || !(rho[y] > 0.0)) return fail(h, LBM_EINVAL, "rho_ref must be finite and > 0");
    rows[y] = rho[y];
    rows[ly + y] = 1.0 / rho[y];
  }
  std::vector<double> kf(KF_LEN);
  for (int sh = 0; sh < NSHELL; ++sh) {
    kf[KF_LO + sh] = wall_factor(SHELL_START[sh], t_lo);
    kf[KF_HI + sh] = wall_factor(SHELL_START[sh], t_hi);
    if (!std::isfinite(kf[KF_LO + sh]) || !(kf[KF_LO + sh] > 0.0) || !std::isfinite(kf[KF_HI + sh]) ||
        !(kf[KF_HI + sh] > 0.0))
      return fail(h, LBM_EINVAL, "the zero-velocity equilibrium is not positive at the layer temperatures");
    kf[KF_INV_LO + sh] = 1.0 / kf[KF_LO + sh];
    kf[KF_INV_HI + sh] = 1.0 / kf[KF_HI + sh];
    kf[KF_WK_LO + sh] = W_SHELL[sh] / kf[KF_LO + sh];
    kf[KF_WK_HI + sh] = W_SHELL[sh] / kf[KF_HI + sh];
  }
  LBM_HIP(h, hipMemcpyAsync(const_cast<double*>(h->geo.ref), rows.data(), ly * sizeof(double),
                            hipMemcpyHostToDevice, h->stream));
  LBM_HIP(h, hipMemcpyAsync(const_cast<double*>(h->geo.inv_ref), rows.data() + ly, ly * sizeof(double),
                            hipMemcpyHostToDevice, h->stream));
  LBM_HIP(h, hipMemcpyAsync(const_cast<double*>(h->geo.kf), kf.data(), KF_LEN * sizeof(double),
                            hipMemcpyHostToDevice, h->stream));
  LBM_HIP(h, hipStreamSynchronize(h->stream));
  h->geo.ysplit = ysplit;
  h->rho_ref.assign(rho, rho + ly);
  h->t_layers[0] = t_lo;
  h->t_layers[1] = t_hi;
  h->has_ref = true;
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_config_default(lbm_config* cfg, int32_t lx, int32_t ly) {
  if (!cfg) return fail(nullptr, LBM_EINVAL, "config is NULL");
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->lx = lx;
  cfg->ly = ly;
  cfg->tau = 0.8;
  cfg->gx = 0.0;
  cfg->gy = -1e-4;
  cfg->t_bottom = 1.05;
  cfg->t_top = 0.95;
  cfg->storage = LBM_FP64;
  cfg->path = LBM_PATH_FUSED;
  cfg->layout = LBM_LAYOUT_COLUMN;
  cfg->block = 0;
  cfg->ny_pad = -1;
  cfg->stride_pad = -1;
  return LBM_OK;
}

size_t lbm_required_bytes(const lbm_config* cfg) {
  Layout L{};
  std::string why;
  if (make_layout(cfg, &L, &why) != LBM_OK) {
    fail(nullptr, LBM_EINVAL, why);
    return 0;
  }
  return L.total();
}

int lbm_create(const lbm_config* cfg, void* dev_mem, size_t dev_bytes, void* stream,
               lbm_handle** out) {
  if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
  *out = nullptr;
  Layout L{};
  std::string why;
  if (make_layout(cfg, &L, &why) != LBM_OK) return fail(nullptr, LBM_EINVAL, why);
  if (!dev_mem) return fail(nullptr, LBM_EINVAL, "dev_mem is NULL");
  if (reinterpret_cast<uintptr_t>(dev_mem) % 256 != 0)
    return fail(nullptr, LBM_ENOMEM, "dev_mem must be 256-byte aligned");
  if (dev_bytes < L.total())
    return fail(nullptr, LBM_ENOMEM,
                "dev_bytes " + std::to_string(dev_bytes) + " < required " + std::to_string(L.total()));
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, dev_mem);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // do not leave the error for the next call
    return fail(nullptr, LBM_EINVAL, std::string("dev_mem is not device memory (") +
                                        hipGetErrorString(e) + ")");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(nullptr, LBM_EINVAL, "dev_mem is not device memory");

  auto* h = new lbm_handle();
  h->cfg = *cfg;
  h->geo = L.geo;
  h->buf_bytes = L.buf_bytes;
  h->buf[0] = static_cast<char*>(dev_mem);
  h->buf[1] = static_cast<char*>(dev_mem) + L.buf_bytes;
  if (L.ref_bytes) {
    char* r = static_cast<char*>(dev_mem) + 2 * L.buf_bytes;
    const size_t row_bytes = static_cast<size_t>(round_up(8LL * cfg->ly, 256));
    h->geo.ref = reinterpret_cast<const double*>(r);
    h->geo.inv_ref = reinterpret_cast<const double*>(r + row_bytes);
    h->geo.kf = reinterpret_cast<const double*>(r + 2 * row_bytes);
  }
  h->stream = static_cast<hipStream_t>(stream);
  h->device = attr.device;
  const double tau = cfg->tau;
  h->cp.omega = 1.0 / tau;
  h->cp.one_minus_omega = 1.0 - h->cp.omega;
  h->cp.tgx = tau * cfg->gx;
  h->cp.tgy = tau * cfg->gy;
  h->cp.dtemp = tau * tau * (cfg->gx * cfg->gx + cfg->gy * cfg->gy) / 2.0;
  for (int l = 0; l < NPOP; ++l) {
    h->wp.kb[l] = wall_factor(l, cfg->t_bottom);
    h->wp.kt[l] = wall_factor(l, cfg->t_top);
  }
  *out = h;
  return LBM_OK;
}

int lbm_set_stream(lbm_handle* h, void* stream) {
  if (!h) return fail(nullptr, LBM_EINVAL, "handle is NULL");
  if (h->engine) return fail(h, LBM_ESTATE, "lattice is stepped by an engine (remove it first)");
  h->stream = static_cast<hipStream_t>(stream);
  return LBM_OK;
}

int lbm_init_rt(lbm_handle* h, const lbm_rt_params* rt) {
  if (!h) return fail(nullptr, LBM_EINVAL, "handle is NULL");
  if (!rt) return fail(h, LBM_EINVAL, "rt params are NULL");
  if (!std::isfinite(rt->width) || !(rt->width > 0.0)) return fail(h, LBM_EINVAL, "width must be > 0");
  if (!std::isfinite(rt->y_center)) return fail(h, LBM_EINVAL, "y_center must be finite");
  if (rt->n_modes < 0 || rt->n_modes > LBM_MAX_MODES)
    return fail(h, LBM_EINVAL, "n_modes must be in [0, 32]");
  if (rt->n_modes > 0 && (!rt->amp || !rt->phase)) return fail(h, LBM_EINVAL, "amp/phase are NULL");
  if (h->engine) return fail(h, LBM_ESTATE, "lattice is stepped by an engine (remove it first)");
  RtParams p{};
  p.tm = 0.5 * (h->cfg.t_bottom + h->cfg.t_top);
  p.a = 0.5 * (h->cfg.t_bottom - h->cfg.t_top);
  p.width = rt->width;
  p.y_center = rt->y_center;
  p.gy = h->cfg.gy;
  p.n_modes = rt->n_modes;
  for (int k = 0; k < rt->n_modes; ++k) {
    if (!std::isfinite(rt->amp[k]) || !std::isfinite(rt->phase[k]))
      return fail(h, LBM_EINVAL, "amp/phase must be finite");
    p.amp[k] = rt->amp[k];
    p.phase[k] = rt->phase[k];
  }
  DeviceGuard dg(h->device);
  if (h->geo.storage == STORAGE_F16DEV) {
    // the reference state: the density of the flat-interface state, on
    // the device with the same closed form as the initial state; the wall
    // temperatures as the layers, split at the first row above the
    // interface
    const int ly = h->geo.ly;
    double* rows = scratch(h);
    std::vector<double> rho(ly);
    LBM_HIP(h, launch_rt_reference(h->geo, rows, rows + ly, p, h->stream));
    LBM_HIP(h, hipMemcpyAsync(rho.data(), rows, ly * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    LBM_HIP(h, hipStreamSynchronize(h->stream));
    const int ysplit = static_cast<int>(std::min<double>(std::max(std::ceil(rt->y_center), 0.0), ly));
    const int rc = set_reference_table(h, rho.data(), h->cfg.t_bottom, h->cfg.t_top, ysplit);
    if (rc != LBM_OK) return rc;
  }
  LBM_HIP(h, launch_init_rt(h->geo, current(h), p, h->stream));
  h->ready = true;
  return LBM_OK;
}

int lbm_step(lbm_handle* h, int32_t n) {
  if (!h) return fail(nullptr, LBM_EINVAL, "handle is NULL");
  if (n < 0) return fail(h, LBM_EINVAL, "n must be >= 0");
  if (!h->ready) return fail(h, LBM_ESTATE, "lattice not initialised");
  if (h->engine) return fail(h, LBM_ESTATE, "lattice is stepped by an engine (remove it first)");
  DeviceGuard dg(h->device);
  if (h->cfg.path == LBM_PATH_REGIONS) return region_steps(h, n);
  if (h->cfg.path == LBM_PATH_FUSED2) return fused2_steps(h, n);
  for (int32_t i = 0; i < n; ++i) {
    int rc;
    if (h->cfg.path == LBM_PATH_FUSED) {
      rc = fused_step(h);
    } else {
      rc = run_phase(h, LBM_PHASE_PBC);
      if (rc == LBM_OK) rc = run_phase(h, LBM_PHASE_PROPAGATE);
      if (rc == LBM_OK) rc = run_phase(h, LBM_PHASE_BC);
      if (rc == LBM_OK) rc = run_phase(h, LBM_PHASE_COLLIDE);
    }
    if (rc != LBM_OK) return rc;
  }
  return LBM_OK;
}

int lbm_step_captured(lbm_handle* h, int32_t n) {
  if (!h) return fail(nullptr, LBM_EINVAL, "handle is NULL");
  if (n < 0) return fail(h, LBM_EINVAL, "n must be >= 0");
  if (!h->ready) return fail(h, LBM_ESTATE, "lattice not initialised");
  if (h->engine) return fail(h, LBM_ESTATE, "lattice is stepped by an engine (remove it first)");
  if (h->timing) return fail(h, LBM_EINVAL, "timing must be off for captured steps");
  if (n == 0) return LBM_OK;
  DeviceGuard dg(h->device);
  const int start = h->cur;
  hipGraphExec_t exec = nullptr;
  int cur_after = start;
  for (const auto& c : h->captured)
    if (c.n == n && c.cur == start) {
      exec = c.exec;
      cur_after = c.cur_after;
    }
  if (!exec) {
    if (h->cfg.path == LBM_PATH_REGIONS || h->cfg.path == LBM_PATH_FUSED2) {
      // create the side stream outside the capture
      const int rs = ensure_side(h);
      if (rs != LBM_OK) return rs;
    }
    // capture on a private stream (the caller's may be the null stream,
    // which cannot be captured); the graph is launched on the caller's
    if (!h->cap) LBM_HIP(h, hipStreamCreate(&h->cap));
    LBM_HIP(h, hipStreamSynchronize(h->stream));
    hipStream_t user = h->stream;
    h->stream = h->cap;
    hipError_t eb = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
    const int rc = eb == hipSuccess ? lbm_step(h, n) : LBM_EDEVICE;
    hipGraph_t graph = nullptr;
    const hipError_t e = eb == hipSuccess ? hipStreamEndCapture(h->cap, &graph) : eb;
    h->stream = user;
    cur_after = h->cur;  // where the recorded steps leave the state
    h->cur = start;      // the capture only recorded them
    if (rc != LBM_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      if (rc != LBM_OK && eb == hipSuccess) return rc;
      return fail(h, LBM_EDEVICE, std::string("stream capture: ") + hipGetErrorString(e));
    }
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return fail(h, LBM_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    h->captured.push_back({n, start, cur_after, graph, exec});
  }
  LBM_HIP(h, hipGraphLaunch(exec, h->stream));
  h->cur = cur_after;
  return LBM_OK;
}

int lbm_run_phase(lbm_handle* h, int32_t phase) {
  if (!h) return fail(nullptr, LBM_EINVAL, "handle is NULL");
  if (phase < 0 || phase > LBM_PHASE_FUSED) return fail(h, LBM_EINVAL, "unknown phase");
  if (!h->ready) return fail(h, LBM_ESTATE, "lattice not initialised");
  if (h->engine) return fail(h, LBM_ESTATE, "lattice is stepped by an engine (remove it first)");
  DeviceGuard dg(h->device);
  return run_phase(h, phase);
}

int lbm_moments(lbm_handle* h, double* rho, double* ux, double* uy, double* T) {
  if (!h) return fail(nullptr, LBM_EINVAL, "handle is NULL");
  if (!h->ready) return fail(h, LBM_ESTATE, "lattice not initialised");
  if (h->engine && engine_refresh(h->engine) != LBM_OK)
    return fail(h, LBM_EDEVICE, "engine status refresh failed");
  DeviceGuard dg(h->device);
  double* tmp = scratch(h);
  LBM_HIP(h, launch_moments(h->geo, current(h), tmp, h->stream));
  const size_t n = static_cast<size_t>(h->geo.lx) * h->geo.ly;
  double* outs[4] = {rho, ux, uy, T};
  for (int k = 0; k < 4; ++k)
    if (outs[k])
      LBM_HIP(h, hipMemcpyAsync(outs[k], tmp + k * n, n * sizeof(double), hipMemcpyDeviceToHost,
                                h->stream));
  LBM_HIP(h, hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_conservation(lbm_handle* h, double out[5]) {
  if (!h) return fail(nullptr, LBM_EINVAL, "handle is NULL");
  if (!out) return fail(h, LBM_EINVAL, "out is NULL");
  if (!h->ready) return fail(h, LBM_ESTATE, "lattice not initialised");
  if (h->engine && engine_refresh(h->engine) != LBM_OK)
    return fail(h, LBM_EDEVICE, "engine status refresh failed");
  DeviceGuard dg(h->device);
  double* partials = scratch(h);
  double* result = partials + CONS_BLOCKS * CONS_FIELDS;
  LBM_HIP(h, launch_conservation(h->geo, current(h), partials, result, h->stream));
  LBM_HIP(h, hipMemcpyAsync(out, result, CONS_FIELDS * sizeof(double), hipMemcpyDeviceToHost,
                            h->stream));
  LBM_HIP(h, hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_get_populations(lbm_handle* h, double* host) {
  if (!h) return fail(nullptr, LBM_EINVAL, "handle is NULL");
  if (!host) return fail(h, LBM_EINVAL, "host is NULL");
  if (!h->ready) return fail(h, LBM_ESTATE, "lattice not initialised");
  if (h->engine && engine_refresh(h->engine) != LBM_OK)
    return fail(h, LBM_EDEVICE, "engine status refresh failed");
  DeviceGuard dg(h->device);
  const Geometry& g = h->geo;
  const size_t n = static_cast<size_t>(g.lx) * g.ly;
  double* stage = scratch(h);
  for (int l = 0; l < NPOP; ++l) {
    LBM_HIP(h, launch_decode_population(g, current(h), stage, l, h->stream));
    LBM_HIP(h, hipMemcpyAsync(host + static_cast<size_t>(l) * n, stage, n * sizeof(double),
                              hipMemcpyDeviceToHost, h->stream));
  }
  LBM_HIP(h, hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_set_populations(lbm_handle* h, const double* host) {
  if (!h) return fail(nullptr, LBM_EINVAL, "handle is NULL");
  if (!host) return fail(h, LBM_EINVAL, "host is NULL");
  if (h->geo.storage == STORAGE_F16DEV && !h->has_ref)
    return fail(h, LBM_ESTATE, "deviation storage: set the reference density first");
  if (h->engine) return fail(h, LBM_ESTATE, "lattice is stepped by an engine (remove it first)");
  DeviceGuard dg(h->device);
  const Geometry& g = h->geo;
  const size_t n = static_cast<size_t>(g.lx) * g.ly;
  double* stage = scratch(h);
  for (int l = 0; l < NPOP; ++l) {
    LBM_HIP(h, hipMemcpyAsync(stage, host + static_cast<size_t>(l) * n, n * sizeof(double),
                              hipMemcpyHostToDevice, h->stream));
    LBM_HIP(h, launch_encode_population(g, stage, current(h), l, h->stream));
  }
  LBM_HIP(h, hipStreamSynchronize(h->stream));
  h->ready = true;
  return LBM_OK;
}

int lbm_set_reference(lbm_handle* h, const double* rho_ref, double t_lo, double t_hi, int32_t y_split) {
  if (!h) return fail(nullptr, LBM_EINVAL, "handle is NULL");
  if (h->engine) return fail(h, LBM_ESTATE, "lattice is stepped by an engine (remove it first)");
  if (!rho_ref) return fail(h, LBM_EINVAL, "rho_ref is NULL");
  if (h->geo.storage != STORAGE_F16DEV)
    return fail(h, LBM_EINVAL, "a reference state exists only for LBM_FP16DEV storage");
  DeviceGuard dg(h->device);
  const int rc = set_reference_table(h, rho_ref, t_lo, t_hi, y_split);
  if (rc != LBM_OK) return rc;
  h->ready = false;  // stored deviations refer to the old reference
  return LBM_OK;
}

int lbm_get_reference(lbm_handle* h, double* rho_ref, double t_layers[2], int32_t* y_split) {
  if (!h) return fail(nullptr, LBM_EINVAL, "handle is NULL");
  if (!rho_ref) return fail(h, LBM_EINVAL, "rho_ref is NULL");
  if (h->geo.storage != STORAGE_F16DEV || !h->has_ref)
    return fail(h, LBM_ESTATE, "no reference state (LBM_FP16DEV only, after init or set)");
  std::copy(h->rho_ref.begin(), h->rho_ref.end(), rho_ref);
  if (t_layers) {
    t_layers[0] = h->t_layers[0];
    t_layers[1] = h->t_layers[1];
  }
  if (y_split) *y_split = h->geo.ysplit;
  return LBM_OK;
}

int lbm_get_sites(lbm_handle* h, int32_t n, const int32_t* xs, const int32_t* ys, double* out) {
  if (!h) return fail(nullptr, LBM_EINVAL, "handle is NULL");
  if (n < 0) return fail(h, LBM_EINVAL, "n must be >= 0");
  if (n == 0) return LBM_OK;
  if (!xs || !ys || !out) return fail(h, LBM_EINVAL, "xs/ys/out are NULL");
  if (!h->ready) return fail(h, LBM_ESTATE, "lattice not initialised");
  if (h->engine && engine_refresh(h->engine) != LBM_OK)
    return fail(h, LBM_EDEVICE, "engine status refresh failed");
  const size_t per_site = NPOP * sizeof(double) + 2 * sizeof(int);  // 304 bytes
  if (static_cast<size_t>(n) > h->buf_bytes / per_site)
    return fail(h, LBM_EINVAL, "too many sites for the scratch copy");
  // x coordinates, then y coordinates
  std::vector<int> xy(2 * static_cast<size_t>(n));
  for (int32_t i = 0; i < n; ++i) {
    if (xs[i] < 0 || xs[i] >= h->geo.lx || ys[i] < 0 || ys[i] >= h->geo.ly)
      return fail(h, LBM_EINVAL, "site " + std::to_string(i) + " outside the lattice");
    xy[i] = xs[i];
    xy[n + i] = ys[i];
  }
  DeviceGuard dg(h->device);
  double* scratch_out = scratch(h);
  int* scratch_xy = reinterpret_cast<int*>(scratch_out + static_cast<size_t>(NPOP) * n);
  LBM_HIP(h, hipMemcpyAsync(scratch_xy, xy.data(), xy.size() * sizeof(int), hipMemcpyHostToDevice,
                            h->stream));
  LBM_HIP(h, launch_get_sites(h->geo, current(h), scratch_xy, scratch_xy + n, n, scratch_out, h->stream));
  LBM_HIP(h, hipMemcpyAsync(out, scratch_out, static_cast<size_t>(NPOP) * n * sizeof(double),
                            hipMemcpyDeviceToHost, h->stream));
  LBM_HIP(h, hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_set_timing(lbm_handle* h, int32_t enable) {
  if (!h) return fail(nullptr, LBM_EINVAL, "handle is NULL");
  h->timing = enable != 0;
  return LBM_OK;
}

int lbm_read_timing(lbm_handle* h, double ms[LBM_NPHASES], int64_t count[LBM_NPHASES]) {
  if (!h) return fail(nullptr, LBM_EINVAL, "handle is NULL");
  if (!ms || !count) return fail(h, LBM_EINVAL, "ms/count are NULL");
  DeviceGuard dg(h->device);
  LBM_HIP(h, hipStreamSynchronize(h->stream));
  if (h->side) LBM_HIP(h, hipStreamSynchronize(h->side));
  for (int p = 0; p < LBM_NPHASES; ++p) {
    ms[p] = 0.0;
    count[p] = 0;
  }
  for (const auto& r : h->recs) {
    float t = 0.0f;
    LBM_HIP(h, hipEventElapsedTime(&t, h->events[r.ev], h->events[r.ev + 1]));
    ms[r.phase] += t;
    count[r.phase] += 1;
  }
  h->recs.clear();
  h->ev_used = 0;
  return LBM_OK;
}

int lbm_layout(const lbm_handle* h, int64_t out[6]) {
  if (!h || !out) return fail(nullptr, LBM_EINVAL, "handle/out is NULL");
  out[0] = h->geo.lx + 2 * HALO;
  out[1] = h->geo.ny;
  out[2] = h->geo.pstride;
  out[3] = h->geo.cstride;
  out[4] = static_cast<int64_t>(h->buf_bytes);
  out[5] = h->geo.block;
  return LBM_OK;
}

int lbm_tables(int32_t* e, int32_t* opp, double* w, double* r) {
  for (int l = 0; l < NPOP; ++l) {
    if (e) {
      e[2 * l] = EX[l];
      e[2 * l + 1] = EY[l];
    }
    if (opp) opp[l] = opp_of(l);
    if (w) w[l] = weight_of(l);
  }
  if (r) *r = R;
  return LBM_OK;
}

int lbm_wall_factors(double t_wall, double out[LBM_NPOP]) {
  if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
  for (int l = 0; l < NPOP; ++l) out[l] = wall_factor(l, t_wall);
  return LBM_OK;
}

int lbm_probe_bandwidth(int32_t mode, const void* src, void* dst, size_t bytes, int32_t shift,
                        void* stream) {
  if (!src || !dst) return fail(nullptr, LBM_EINVAL, "src/dst are NULL");
  if (mode < LBM_PROBE_COPY || mode > LBM_PROBE_ARMW) return fail(nullptr, LBM_EINVAL, "bad probe mode");
  if (bytes % 16 != 0 || bytes < 2048)
    return fail(nullptr, LBM_EINVAL, "bytes must be a multiple of 16 and at least 2048");
  if (reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
    return fail(nullptr, LBM_EINVAL, "src/dst must be 16-byte aligned");
  if (shift < -64 || shift > 64) return fail(nullptr, LBM_EINVAL, "shift must be within [-64, 64]");
  if (mode == LBM_PROBE_COPY && shift != 0) return fail(nullptr, LBM_EINVAL, "COPY takes shift 0");
  LBM_HIP(nullptr, launch_probe(mode, src, dst, bytes / 16, shift, static_cast<hipStream_t>(stream)));
  return LBM_OK;
}

const char* lbm_last_error(const lbm_handle* h) { return h ? h->err.c_str() : g_err.c_str(); }

void lbm_destroy(lbm_handle* h) {
  if (!h) return;
  if (h->engine) engine_detach(h->engine, h->engine_slot);
  {
    DeviceGuard dg(h->device);
    (void)hipStreamSynchronize(h->stream);
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    for (auto& c : h->captured) {
      (void)hipGraphExecDestroy(c.exec);
      (void)hipGraphDestroy(c.graph);
    }
    if (h->cap) (void)hipStreamDestroy(h->cap);
    if (h->side) {
      (void)hipStreamSynchronize(h->side);
      (void)hipStreamDestroy(h->side);
      (void)hipEventDestroy(h->ev_ready);
      (void)hipEventDestroy(h->ev_border);
      (void)hipEventDestroy(h->ev_bulk);
    }
  }
  delete h;
}

}  // extern "C"
