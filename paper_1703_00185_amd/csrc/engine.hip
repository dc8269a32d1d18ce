// Ensemble engine kernels: one persistent launch steps every active lattice
// (propagate + bc + collide, as the fused kernel, with periodic x done by
// wrapping the source column), and a small kernel advances each lattice's
// double buffer and step count.
//
// Work decomposition: a tile is one wavefront, 64 consecutive rows of one
// column of one lattice, so that lattices of any height waste only the
// lanes of their last, ragged wavefront per column; the tiles of all
// active lattices form one index space, in the order of the active-slot
// table.  Each wavefront of a work-group takes its own tiles.  The grid is
// persistent (a fixed number of work-groups).  CHUNKED gives each
// work-group one contiguous run of tiles, dealt to its wavefronts in turn,
// so neighbouring tiles of a column run on the same CU at the same time and
// share the cache lines the +-3-row pull straddles; the lattice of the next
// tile is found by stepping through the prefix table.  STRIDED deals tiles
// round-robin over all wavefronts of the grid and finds each tile's lattice
// by binary search.  In both, work-group ids are renumbered so that each of
// the 8 XCDs (which the hardware deals ids to round-robin, each with its
// own L2) takes one contiguous share of the tiles.
#pragma clang fp contract(off)

#include "d2q37_device.hpp"
#include "engine.hpp"

namespace d2q37 {
namespace {

// Lattice buffers are read from the slot table, so the compiler cannot
// know they are global memory; these pointers say so, which keeps loads
// and stores in the global (not flat) address mode.
#define GLOBAL_AS __attribute__((address_space(1)))
// The slot table is read through the constant address space: no step
// kernel writes it (the advance kernel and the host do, between launches),
// and with a wavefront-uniform slot index every descriptor field is then a
// scalar load into scalar registers instead of a vector load into VGPRs.
#define CONST_AS __attribute__((address_space(4)))
using SlotView = const CONST_AS SlotDesc;

// Source column of population l for a tile at column x: periodic wrap.
// x is uniform over the work-group, so this is scalar arithmetic.
__device__ __forceinline__ int wrap_col(int x, int ex, int lx) {
  int xs = x - ex;
  if (xs < 0) xs += lx;
  if (xs >= lx) xs -= lx;
  return xs;
}

template <class C>
__device__ __forceinline__ void gather_wrap_interior(SlotView& d, const C& cd,
                                                     const GLOBAL_AS typename C::S* src, int x, int y,
                                                     double (&f)[NPOP]) {
  using S = typename C::S;
  const unsigned uy = static_cast<unsigned>(y);
#pragma unroll
  for (int l = 0; l < NPOP; ++l) {
    const int col = wrap_col(x, EX[l], d.lx) + HALO;
    const GLOBAL_AS S* base =
        src + (static_cast<long long>(l) * d.pstride + static_cast<long long>(col) * d.cstride - EY[l]);
    f[l] = cd.dec(base[uy], l, y - EY[l]);
  }
}

// Wall wavefronts: each population through its uniform run base at the
// lane's row clamped into the lattice; the lanes whose source lies beyond a
// wall (at most three rows) read the opposite population of their own site
// in a second, masked load.
template <class C>
__device__ __forceinline__ void gather_wrap_wall(SlotView& d, const C& cd,
                                                 const GLOBAL_AS typename C::S* src, int x, int y,
                                                 double (&f)[NPOP]) {
  using S = typename C::S;
  const unsigned uy = static_cast<unsigned>(y);
#pragma unroll
  for (int l = 0; l < NPOP; ++l) {
    const int col = wrap_col(x, EX[l], d.lx) + HALO;
    const GLOBAL_AS S* run =
        src + (static_cast<long long>(l) * d.pstride + static_cast<long long>(col) * d.cstride);
    if (EY[l] == 0) {
      f[l] = cd.dec(run[uy], l, y);
      continue;
    }
    const int ys = y - EY[l];
    const bool inside = (ys >= 0) && (ys < d.ly);
    const unsigned yc = static_cast<unsigned>(min(max(ys, 0), d.ly - 1));
    S v = run[yc];
    if (!inside)
      v = src[static_cast<long long>(opp_of(l)) * d.pstride + static_cast<long long>(x + HALO) * d.cstride + uy];
    f[l] = cd.dec(v, l, inside ? ys : y);
  }
}

// One tile: rows yw*64 .. yw*64+63 of column x of lattice d, from buffer
// cur to the other buffer.  Same arithmetic as the single-lattice fused
// kernel.
template <class C>
__device__ __forceinline__ void step_tile(SlotView& d, int x, int yw) {
  using S = typename C::S;
  const C cd{};
  const GLOBAL_AS S* src = (const GLOBAL_AS S*)(d.buf[d.cur]);
  GLOBAL_AS S* dst = (GLOBAL_AS S*)(d.buf[d.cur ^ 1]);
  const int ywave = yw * WAVE;
  const int y = ywave + static_cast<int>(threadIdx.x & (WAVE - 1));
  double f[NPOP];
  const int interior = (ywave >= WALL_ROWS) && (ywave + WAVE <= d.ly - WALL_ROWS);
  if (__builtin_amdgcn_readfirstlane(interior)) {
    gather_wrap_interior(d, cd, src, x, y, f);
  } else {
    const int yc = y < d.ly ? y : d.ly - 1;
    gather_wrap_wall(d, cd, src, x, yc, f);
    if (yc < WALL_ROWS || yc >= d.ly - WALL_ROWS) thermalise(f, yc < WALL_ROWS, d.wp);
  }
  CollideParams cp;  // field by field: no implicit copy out of the constant address space
  cp.omega = d.cp.omega;
  cp.one_minus_omega = d.cp.one_minus_omega;
  cp.tgx = d.cp.tgx;
  cp.tgy = d.cp.tgy;
  cp.dtemp = d.cp.dtemp;
  collide_site(f, cp);
  if (y < d.ly) {
    const unsigned off = static_cast<unsigned>(y) * static_cast<unsigned>(sizeof(S));
    GLOBAL_AS S* col = dst + static_cast<long long>(x + HALO) * d.cstride;
    // streaming stores: every element is written once per step
#pragma unroll
    for (int l = 0; l < NPOP; ++l)
      st_nt((S*)(col + static_cast<long long>(l) * d.pstride), off, cd.enc(f[l], l, y));
  }
}

template <class C>
__device__ __forceinline__ void run_tile(SlotView& d, int local) {
  if (d.steps_left <= 0) return;
  // the tile coordinates are uniform over the wavefront: keep them (and
  // every address derived from them) in scalar registers
  const int x = __builtin_amdgcn_readfirstlane(local / d.ny_waves);
  const int yw = __builtin_amdgcn_readfirstlane(local - x * d.ny_waves);
  step_tile<C>(d, x, yw);
}

// Last k in [0, n) with start[k] <= t (start[0] = 0 <= t).
__device__ __forceinline__ int find_slot(const int* start, int n, int t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// One kernel per storage type (C): each walks the tile table of the
// lattices of its type.  Wavefronts never synchronise with each other.
// Bounded to 128 VGPRs (4 wavefronts per SIMD), which it fits without
// spilling.
template <class C, int BLOCK, int SCHED>
__global__ void __launch_bounds__(BLOCK, 4) engine_step_kernel(const SlotDesc* __restrict__ slots,
                                                            const int* __restrict__ table,
                                                            int max_slots) {
  constexpr int W = BLOCK / WAVE;  // wavefronts per work-group
  SlotView* cslots = (SlotView*)(slots);
  const int n = table[0];
  const int total = table[1];
  const int* order = table + 2;
  const int* start = table + 2 + max_slots;
  if (n <= 0 || total <= 0) return;
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / WAVE);
  if (SCHED == SCHED_CHUNKED) {
    // each XCD takes one contiguous share of the tile runs
    const long long g = gridDim.x;
    const long long b = xcd_tile(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
    const int t0 = static_cast<int>(total * b / g);
    const int t1 = static_cast<int>(total * (b + 1) / g);
    if (t0 + wave >= t1) return;
    int k = find_slot(start, n, t0 + wave);
    for (int t = t0 + wave; t < t1; t += W) {
      while (t >= start[k + 1]) ++k;
      run_tile<C>(cslots[order[k]], t - start[k]);
    }
  } else {
    const int stride = static_cast<int>(gridDim.x) * W;
    // renumber over the work-groups that have tiles in the first sweep, so
    // that each XCD takes a contiguous share of them (all of them when the
    // grid exceeds the tile count)
    const int busy = min(static_cast<int>(gridDim.x), (total + W - 1) / W);
    const int b = static_cast<int>(blockIdx.x) < busy ? xcd_tile(static_cast<int>(blockIdx.x), busy)
                                                    : static_cast<int>(blockIdx.x);
    for (int t = b * W + wave; t < total; t += stride) {
      const int k = find_slot(start, n, t);
      run_tile<C>(cslots[order[k]], t - start[k]);
    }
  }
}

// After a step: flip the buffer and count the step for every slot that
// still had steps to run (free slots hold steps_left = 0); publish
// (steps_left, cur) per slot.
__global__ void __launch_bounds__(256) engine_advance_kernel(SlotDesc* __restrict__ slots,
                                                             int max_slots, int* __restrict__ status) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= max_slots) return;
  SlotDesc& d = slots[s];
  if (d.steps_left > 0) {
    d.cur ^= 1;
    d.steps_left -= 1;
  }
  status[2 * s] = d.steps_left;
  status[2 * s + 1] = d.cur;
}

template <class C, int SCHED>
void* step_func(int block) {
  switch (block) {
    case 64: return reinterpret_cast<void*>(&engine_step_kernel<C, 64, SCHED>);
    case 128: return reinterpret_cast<void*>(&engine_step_kernel<C, 128, SCHED>);
    case 256: return reinterpret_cast<void*>(&engine_step_kernel<C, 256, SCHED>);
    case 512: return reinterpret_cast<void*>(&engine_step_kernel<C, 512, SCHED>);
    default: return nullptr;
  }
}

template <class C>
void* step_func(int block, int schedule) {
  return schedule == SCHED_STRIDED ? step_func<C, SCHED_STRIDED>(block) : step_func<C, SCHED_CHUNKED>(block);
}

}  // namespace

hipError_t engine_step_node(int storage, int block, int groups, int schedule, void** func, dim3* grid,
                            dim3* threads) {
  void* f = storage == STORAGE_F32 ? step_func<CodecF32>(block, schedule) : step_func<CodecF64>(block, schedule);
  if (!f || groups <= 0) return hipErrorInvalidValue;
  *func = f;
  *grid = dim3(groups);
  *threads = dim3(block);
  return hipSuccess;
}

hipError_t engine_advance_node(int max_slots, void** func, dim3* grid, dim3* threads) {
  *func = reinterpret_cast<void*>(&engine_advance_kernel);
  *grid = dim3((max_slots + 255) / 256);
  *threads = dim3(256);
  return hipSuccess;
}

hipError_t launch_engine_step(int storage, const SlotDesc* slots, const int* table, int max_slots,
                              int block, int groups, int schedule, hipStream_t s) {
  void* f;
  dim3 grid, threads;
  hipError_t e = engine_step_node(storage, block, groups, schedule, &f, &grid, &threads);
  if (e != hipSuccess) return e;
  void* args[] = {&slots, &table, &max_slots};
  (void)hipGetLastError();
  return hipLaunchKernel(f, grid, threads, args, 0, s);
}

hipError_t launch_engine_advance(SlotDesc* slots, int max_slots, int* status, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(engine_advance_kernel, dim3((max_slots + 255) / 256), dim3(256), 0, s, slots,
                     max_slots, status);
  return hipGetLastError();
}

}  // namespace d2q37
