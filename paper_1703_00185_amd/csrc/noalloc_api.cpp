// lbm_get_sites_noalloc: the site gather of lbm_get_sites with its device
// staging (the gathered populations and the uploaded coordinates) in a
// fixed array of this library's code object instead of the lattice's idle
// copy, for callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.hpp"
#include "lbm.h"

using namespace d2q37;
using namespace d2q37::host;

namespace {

constexpr size_t kMaxSites = LBM_NOALLOC_MAX_SITES;
constexpr size_t kOutBytes = static_cast<size_t>(NPOP) * kMaxSites * sizeof(double);
constexpr size_t kScratchBytes = kOutBytes + 2 * kMaxSites * sizeof(int);
static_assert(kOutBytes % 256 == 0, "coordinates start 256-byte aligned");

// One copy per GPU, held until the process ends.  Host code never uses
// this name as an address (on the host it is only a stand-in for the
// symbol): the device address comes from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (current), looked up once per
// device.  nullptr with a message on failure.
void* scratch_address(int dev, std::string* why) {
  if (dev < 0 || dev >= kMaxDevices) {
    *why = "device index out of range for the static staging array";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

int lbm_get_sites_noalloc(lbm_handle* h, int32_t n, const int32_t* xs, const int32_t* ys, double* out) {
  if (!h) return fail(nullptr, LBM_EINVAL, "handle is NULL");
  if (n < 0) return fail(h, LBM_EINVAL, "n must be >= 0");
  if (static_cast<size_t>(n) > kMaxSites)
    return fail(h, LBM_EINVAL,
                "n = " + std::to_string(n) + " exceeds LBM_NOALLOC_MAX_SITES (" + std::to_string(kMaxSites) + ")");
  if (n == 0) return LBM_OK;
  if (!xs || !ys || !out) return fail(h, LBM_EINVAL, "xs/ys/out are NULL");
  if (!h->ready) return fail(h, LBM_ESTATE, "lattice not initialised");
  for (int32_t i = 0; i < n; ++i)
    if (xs[i] < 0 || xs[i] >= h->geo.lx || ys[i] < 0 || ys[i] >= h->geo.ly)
      return fail(h, LBM_EINVAL, "site " + std::to_string(i) + " outside the lattice");
  if (h->engine && engine_refresh(h->engine) != LBM_OK)
    return fail(h, LBM_EDEVICE, "engine status refresh failed");
  DeviceGuard dg(h->device);
  std::string why;
  char* base = static_cast<char*>(scratch_address(h->device, &why));
  if (!base) return fail(h, LBM_EDEVICE, why);
  double* d_out = reinterpret_cast<double*>(base);
  int* d_xs = reinterpret_cast<int*>(base + kOutBytes);
  int* d_ys = d_xs + kMaxSites;
  // every staged element is written before it is read: nothing to clear
  LBM_HIP(h, hipMemcpyAsync(d_xs, xs, static_cast<size_t>(n) * sizeof(int), hipMemcpyHostToDevice, h->stream));
  LBM_HIP(h, hipMemcpyAsync(d_ys, ys, static_cast<size_t>(n) * sizeof(int), hipMemcpyHostToDevice, h->stream));
  LBM_HIP(h, launch_get_sites(h->geo, current(h), d_xs, d_ys, n, d_out, h->stream));
  LBM_HIP(h, hipMemcpyAsync(out, d_out, static_cast<size_t>(NPOP) * n * sizeof(double), hipMemcpyDeviceToHost,
                            h->stream));
  LBM_HIP(h, hipStreamSynchronize(h->stream));
  return LBM_OK;
}

}  // extern "C"
