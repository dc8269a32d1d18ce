// gfx950 kernels of the D2Q37 thermal lattice Boltzmann step.
//
// One lane per lattice site, lanes of a wavefront along y (the contiguous
// direction of each population run), so that each of the 37 population
// loads and stores of a wavefront is one contiguous segment of 64 elements
// (the structure-of-arrays principle of Sec. 4 "Data Structure Analysis";
// the column and planar layouts differ only in the two strides).
//
// Floating point: the file is compiled without contraction; every fused
// multiply-add below is an explicit fma().  A kernel therefore rounds
// exactly as written, wherever the device functions are inlined: the fused
// kernel and the separate propagate/bc/collide kernels give identical bits,
// and bc is bit-reproducible on any IEEE-754 binary64 machine.
#include <algorithm>
#include <cmath>

#pragma clang fp contract(off)

#include "d2q37_device.hpp"
#include "fused2_plan.hpp"
#include "kernels.hpp"

namespace d2q37 {
namespace {
// ---------------------------------------------------------------------------
// Lattice traversal
// ---------------------------------------------------------------------------

// Site of this lane: column x (physical), row y, first row of its wavefront.
// The grid covers cols.na columns from cols.xa, then columns from cols.xb
// (two ranges, so that the two border strips of a region split are one
// launch); a full-lattice launch uses xa = 0, na = lx.
template <int BLOCK>
__device__ __forceinline__ void lane_site(const Geometry& g, const ColumnSet& cols, int& x, int& y,
                                          int& ywave) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int nyb = cols.nyb > 0 ? cols.nyb : g.ny_blocks;
  const int c = tile / nyb;
  x = c < cols.na ? cols.xa + c : cols.xb + (c - cols.na);
  const int yb = tile - c * nyb;
  y = cols.y0 + yb * BLOCK + threadIdx.x;
  ywave = cols.y0 + yb * BLOCK + (threadIdx.x & ~(WAVE - 1));
}

// True (wavefront-uniform) when every row this wavefront pulls from lies
// inside the lattice and none of its rows is a wall row.
__device__ __forceinline__ bool interior_wave(const Geometry& g, int ywave) {
  const int ok = (ywave >= WALL_ROWS) && (ywave + WAVE <= g.ly - WALL_ROWS);
  return __builtin_amdgcn_readfirstlane(ok) != 0;
}

// Start of the run of population l in column X, elements.
__device__ __forceinline__ long long run_of(const Geometry& g, int l, int X) {
  return static_cast<long long>(l) * g.pstride + static_cast<long long>(X) * g.cstride;
}

// Stored column X of the source of a pull from column x by e_x: with WRAP
// the periodic image inside the lattice (x - e_x taken mod Lx; one
// correction suffices since |e_x| <= 3 <= Lx), else x - e_x itself, whose
// columns beyond the lattice are the halo columns filled by pbc.
template <bool WRAP>
__device__ __forceinline__ int source_column(const Geometry& g, int x, int ex) {
  int xs = x - ex;
  if (WRAP) {
    if (xs < 0) xs += g.lx;
    else if (xs >= g.lx) xs -= g.lx;
  }
  return xs + HALO;
}

// Pull gather of Eq. (10): f_l(x, y) <- f_l(x - e_lx, y - e_ly), periodic
// in x.  Interior form, for a column x uniform over the work-group: the 37
// source runs start at uniform (scalar) addresses and all loads share the
// lane's byte offset.  RUN_OFF: one buffer descriptor per source column
// (7), the lane's offset taken from row y - 3 and the run of population l
// addressed by the scalar offset l * pstride + 3 - e_ly elements (the
// caller guarantees that a column's runs span less than 2^31 bytes); else
// one descriptor per population.
template <bool WRAP, bool RUN_OFF = false, class C>
__device__ __forceinline__ void gather_interior(const Geometry& g, const C& cd,
                                                const typename C::S* __restrict__ src, int x, int y,
                                                double (&f)[NPOP]) {
  using S = typename C::S;
  if constexpr (RUN_OFF) {
    // rows are addressed from y - 3 (>= 0 in an interior wavefront), so
    // that every scalar offset l * pstride + 3 - e_ly is non-negative
    constexpr int kReachY = HALO;              // max |e_y| (the velocity set is symmetric)
    const unsigned off3 = static_cast<unsigned>(y - kReachY) * static_cast<unsigned>(sizeof(S));
    __amdgpu_buffer_rsrc_t col[2 * HALO + 1];  // source column x - e_x, e_x = -3 .. 3
#pragma unroll
    for (int e = -HALO; e <= HALO; ++e)
      col[e + HALO] = buffer_at(src + static_cast<long long>(source_column<WRAP>(g, x, e)) * g.cstride);
    const unsigned ps = static_cast<unsigned>(g.pstride) * static_cast<unsigned>(sizeof(S));
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
      const unsigned so =
          static_cast<unsigned>(l) * ps + static_cast<unsigned>((kReachY - EY[l]) * static_cast<int>(sizeof(S)));
      f[l] = cd.dec(ld_at<S>(col[EX[l] + HALO], off3, so), l, y - EY[l]);
    }
  } else {
    const unsigned off = static_cast<unsigned>(y) * static_cast<unsigned>(sizeof(S));
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
      const S* base = src + (static_cast<long long>(source_column<WRAP>(g, x, EX[l])) * g.cstride +
                             static_cast<long long>(l) * g.pstride - EY[l]);
      f[l] = cd.dec(ld(base, off), l, y - EY[l]);
    }
  }
}

// General form, for wavefronts touching the walls: a source row beyond a
// wall is replaced by the opposite population of the same site.  Each
// population is read through its wavefront-uniform run base at the lane's
// row, clamped into the lattice, and the lanes whose source lies beyond a
// wall (at most three rows) read the opposite population of their own site
// in a second, masked load.  LANE_ADDR: one load per population from a
// per-lane 64-bit index instead (the propagate kernel, whose interior
// wavefronts are so short that the scalar address set-up the uniform form
// shares with them would slow the whole kernel).
template <bool WRAP, bool LANE_ADDR = false, class C>
__device__ __forceinline__ void gather_wall(const Geometry& g, const C& cd,
                                            const typename C::S* __restrict__ src, int x, int y,
                                            double (&f)[NPOP]) {
  using S = typename C::S;
  const int X = x + HALO;
  if constexpr (LANE_ADDR) {
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
      const int ys = y - EY[l];
      const bool inside = (ys >= 0) && (ys < g.ly);
      const long long idx =
          inside ? run_of(g, l, source_column<WRAP>(g, x, EX[l])) + ys : run_of(g, opp_of(l), X) + y;
      f[l] = cd.dec(src[idx], l, inside ? ys : y);  // opp(l) shares w_l
    }
  } else {
    const unsigned off = static_cast<unsigned>(y) * static_cast<unsigned>(sizeof(S));
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
      const S* run = src + run_of(g, l, source_column<WRAP>(g, x, EX[l]));
      if (EY[l] == 0) {
        f[l] = cd.dec(ld(run, off), l, y);
        continue;
      }
      const int ys = y - EY[l];
      const bool inside = (ys >= 0) && (ys < g.ly);
      const int yc = min(max(ys, 0), g.ly - 1);
      S v = ld(run, static_cast<unsigned>(yc) * static_cast<unsigned>(sizeof(S)));
      if (!inside) v = ld(src + run_of(g, opp_of(l), X), off);
      f[l] = cd.dec(v, l, inside ? ys : y);  // opp(l) shares w_l
    }
  }
}

// The 37 populations of site (x, y), x uniform over the work-group.
template <class C>
__device__ __forceinline__ void load_column_site(const Geometry& g, const C& cd,
                                                 const typename C::S* __restrict__ src, int x, int y,
                                                 double (&f)[NPOP]) {
  using S = typename C::S;
  const unsigned off = static_cast<unsigned>(y) * static_cast<unsigned>(sizeof(S));
  const S* col = src + static_cast<long long>(x + HALO) * g.cstride;
#pragma unroll
  for (int l = 0; l < NPOP; ++l) f[l] = cd.dec(ld(col + static_cast<long long>(l) * g.pstride, off), l, y);
}

// Store of site (x, y), x uniform over the work-group.  Non-temporal: the
// step kernels write every element once and nothing reads it back before
// the next launch.  RUN_OFF: one descriptor for the column and scalar run
// offsets, as in gather_interior.
template <bool RUN_OFF = false, class C>
__device__ __forceinline__ void store_column_site(const Geometry& g, const C& cd,
                                                  typename C::S* __restrict__ dst, int x, int y,
                                                  const double (&f)[NPOP]) {
  using S = typename C::S;
  const unsigned off = static_cast<unsigned>(y) * static_cast<unsigned>(sizeof(S));
  S* col = dst + static_cast<long long>(x + HALO) * g.cstride;
  if constexpr (RUN_OFF) {
    const __amdgpu_buffer_rsrc_t r = buffer_at(col);
    const unsigned ps = static_cast<unsigned>(g.pstride) * static_cast<unsigned>(sizeof(S));
#pragma unroll
    for (int l = 0; l < NPOP; ++l) st_nt_at<S>(r, off, static_cast<unsigned>(l) * ps, cd.enc(f[l], l, y));
  } else {
#pragma unroll
    for (int l = 0; l < NPOP; ++l) st_nt(col + static_cast<long long>(l) * g.pstride, off, cd.enc(f[l], l, y));
  }
}

// Any site (x per lane).
template <class C>
__device__ __forceinline__ void load_site(const Geometry& g, const C& cd,
                                          const typename C::S* __restrict__ src, int x, int y,
                                          double (&f)[NPOP]) {
#pragma unroll
  for (int l = 0; l < NPOP; ++l) f[l] = cd.dec(src[run_of(g, l, x + HALO) + y], l, y);
}

template <class C>
__device__ __forceinline__ void store_site(const Geometry& g, const C& cd, typename C::S* __restrict__ dst,
                                           int x, int y, const double (&f)[NPOP]) {
#pragma unroll
  for (int l = 0; l < NPOP; ++l) dst[run_of(g, l, x + HALO) + y] = cd.enc(f[l], l, y);
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Halo columns to refresh: population l with |e_lx| = k needs k columns
// beyond each vertical boundary, 26 (population, distance) pairs per side.
struct HaloCopies {
  int l[52];
  int d[52];
  int right[52];  // 1: e_lx < 0, the copy goes to the right halo
};
constexpr HaloCopies make_halo_copies() {
  HaloCopies h{};
  int n = 0;
  for (int l = 0; l < NPOP; ++l) {
    const int k = EX[l] < 0 ? -EX[l] : EX[l];
    for (int d = 1; d <= k; ++d) {
      h.l[n] = l;
      h.d[n] = d;
      h.right[n] = EX[l] < 0 ? 1 : 0;
      ++n;
    }
  }
  return h;
}
constexpr int count_halo_copies() {
  int n = 0;
  for (int l = 0; l < NPOP; ++l) n += EX[l] < 0 ? -EX[l] : EX[l];
  return n;
}
static_assert(count_halo_copies() == 52, "26 populations cross each vertical boundary");
__constant__ HaloCopies kHalo = make_halo_copies();

// pbc (Sec. 4): periodic x.  A population with e_x = k > 0 pulls from the
// left halo columns X = 3 - d (d = 1..k), copies of physical column
// Lx - d; one with e_x = -k pulls from X = Lx + 2 + d, copies of column d - 1.
template <class S>
__global__ void __launch_bounds__(256) pbc_kernel(S* __restrict__ f, Geometry g) {
  const int y = blockIdx.x * 256 + threadIdx.x;
  if (y >= g.ly) return;
  const int c = blockIdx.y;
  const int l = kHalo.l[c];
  const int d = kHalo.d[c];
  const int dst_col = kHalo.right[c] ? g.lx + HALO - 1 + d : HALO - d;
  const int src_col = kHalo.right[c] ? HALO - 1 + d : g.lx + HALO - d;
  S* fl = f + static_cast<long long>(l) * g.pstride;
  fl[static_cast<long long>(dst_col) * g.cstride + y] = fl[static_cast<long long>(src_col) * g.cstride + y];
}

// propagate (Sec. 4): pull gather into the other lattice copy.
template <class C, int BLOCK>
__global__ void __launch_bounds__(BLOCK) propagate_kernel(const typename C::S* __restrict__ src,
                                                          typename C::S* __restrict__ dst, Geometry g) {
  const C cd = C::of(g);
  int x, y, ywave;
  lane_site<BLOCK>(g, ColumnSet{0, g.lx, 0}, x, y, ywave);
  if (ywave >= g.ly) return;  // whole wavefront beyond the lattice (no barrier follows)
  double f[NPOP];
  if (interior_wave(g, ywave)) {
    gather_interior<false>(g, cd, src, x, y, f);
  } else {
    gather_wall<false, true>(g, cd, src, x, y < g.ly ? y : g.ly - 1, f);
  }
  if (y < g.ly) store_column_site(g, cd, dst, x, y, f);
}

// bc (Sec. 4): thermal walls, in place, on the 3 bottom and 3 top rows.
template <class C>
__global__ void __launch_bounds__(256) bc_kernel(typename C::S* __restrict__ f, Geometry g, WallParams w) {
  const C cd = C::of(g);
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= g.lx * 2 * WALL_ROWS) return;
  const int x = t / (2 * WALL_ROWS);
  const int r = t - x * (2 * WALL_ROWS);
  const bool bottom = r < WALL_ROWS;
  const int y = bottom ? r : g.ly - 2 * WALL_ROWS + r;
  double v[NPOP];
  load_site(g, cd, f, x, y, v);
  thermalise(v, bottom, w);
  store_site(g, cd, f, x, y, v);
}

// collide (Sec. 4): site-local collision into the other lattice copy.
template <class C, int BLOCK>
__global__ void __launch_bounds__(BLOCK) collide_kernel(const typename C::S* __restrict__ src,
                                                        typename C::S* __restrict__ dst, Geometry g,
                                                        CollideParams c) {
  const C cd = C::of(g);
  int x, y, ywave;
  lane_site<BLOCK>(g, ColumnSet{0, g.lx, 0}, x, y, ywave);
  if (y >= g.ly) return;
  double f[NPOP];
  load_column_site(g, cd, src, x, y, f);
  collide_site(f, c);
  store_column_site(g, cd, dst, x, y, f);
}

// Interior wavefront of one temperature layer, binary16 deviations, in
// units of the destination's reference c_l = K_s rho_ref(y): the stored
// d_l widen to g_l = (rho_ref(y - e_ly) / rho_ref(y)) (1 + d_l), so that
// f_l / c_l = g_l and f_l = K_s rho_ref(y) g_l.  The moment sums apply K_s
// once per shell (density in units of rho_ref(y); velocity and
// temperature are ratios and come out unscaled), the equilibrium takes the
// weights W_s / K_s from the reference table (wk), and the stored
// q_l = f_new,l / c_l - 1 = (1 - omega) g_l + (omega f^eq_l / c_l - 1) is
// one multiply-add, the -1 folded into each shell's constant term.
template <bool WRAP, bool RUN_OFF>
__device__ __forceinline__ void fused_layer_interior(const Geometry& g, const CodecF16DevLayer& lc, ConstD* wk,
                                                     const _Float16* __restrict__ src, _Float16* __restrict__ dst,
                                                     const CollideParams& p, int x, int y) {
  using S = _Float16;
  double gv[NPOP];
  gather_interior<WRAP, RUN_OFF>(g, CodecF16DevRatio{lc.ref, lc.inv_ref[y]}, src, x, y, gv);
  const MomentSums m = moment_sums_of(gv, ShellFactor{lc.k});
  const unsigned off = static_cast<unsigned>(y) * static_cast<unsigned>(sizeof(S));
  const unsigned ps = static_cast<unsigned>(g.pstride) * static_cast<unsigned>(sizeof(S));
  S* col = dst + static_cast<long long>(x + HALO) * g.cstride;
  const __amdgpu_buffer_rsrc_t r = buffer_at(col);
  auto put = [&](int l, double q) {
    const S v = static_cast<S>(static_cast<float>(q));
    if constexpr (RUN_OFF) st_nt_at<S>(r, off, static_cast<unsigned>(l) * ps, v);
    else st_nt(col + static_cast<long long>(l) * g.pstride, off, v);
  };
  const double om1 = p.one_minus_omega;
  collide_by<true>(
      m, p, [&](double eq) { put(0, fma(om1, gv[0], eq)); },
      [&](int a, double ea, int b, double eb) {
        put(a, fma(om1, gv[a], ea));
        put(b, fma(om1, gv[b], eb));
      },
      [](int) { return 1.0; }, ShellFactor{wk});
}

// One site of the fused step (below), with the codec cd.
template <class C, int BLOCK, bool WRAP, bool BAND, bool RUN_OFF>
__device__ __forceinline__ void fused_site(const Geometry& g, const C& cd, const typename C::S* __restrict__ src,
                                           typename C::S* __restrict__ dst, const CollideParams& c,
                                           const WallParams& w, const ColumnSet& cols, int x, int y,
                                           int ywave) {
  if (ywave >= g.ly) return;  // whole wavefront beyond the lattice (no barrier follows)
  double f[NPOP];
  if constexpr (C::kLayered) {
    // The layer of the reference is uniform over a wavefront unless its
    // rows or its pull sources (3 rows beyond) reach both layers: those
    // wavefronts (at most two per column) are left to the band launch,
    // which takes the general codec; every other one takes the codec of
    // its layer, whose shell factors are wavefront-uniform.
    const int yw = __builtin_amdgcn_readfirstlane(ywave);  // uniform: scalar branches and loads
    const int lowest = max(yw - WALL_ROWS, 0);
    const int highest = min(yw + WAVE + WALL_ROWS - 1, g.ly - 1);
    const bool straddles = lowest < g.ysplit && highest >= g.ysplit;
    if constexpr (BAND) {
      if (!straddles) return;
      const int yc = y < g.ly ? y : g.ly - 1;
      gather_wall<WRAP>(g, cd, src, x, yc, f);
      if (yc < WALL_ROWS || yc >= g.ly - WALL_ROWS) thermalise(f, yc < WALL_ROWS, w);
      collide_site(f, c);
      if (y < g.ly) store_column_site(g, cd, dst, x, y, f);
      return;
    }
    if (straddles) return;
    const bool hi = yw >= g.ysplit;
    const ConstD* kf = (ConstD*)(g.kf);
    const CodecF16DevLayer lc{g.ref, g.inv_ref, kf + (hi ? KF_HI : KF_LO), kf + (hi ? KF_INV_HI : KF_INV_LO)};
    if (interior_wave(g, ywave)) {
      fused_layer_interior<WRAP, RUN_OFF>(g, lc, kf + (hi ? KF_WK_HI : KF_WK_LO), src, dst, c, x, y);
      return;
    } else {
      const int yc = y < g.ly ? y : g.ly - 1;
      gather_wall<WRAP>(g, lc, src, x, yc, f);
      if (yc < WALL_ROWS || yc >= g.ly - WALL_ROWS) thermalise(f, yc < WALL_ROWS, w);
    }
    collide_site(f, c);
    if (y < g.ly) store_column_site<RUN_OFF>(g, lc, dst, x, y, f);
    return;
  }
  if constexpr (C::kWrapAlways) {
    // every column wraps its 7 source columns (scalar arithmetic: the
    // column is uniform over the work-group), one gather code path
    if (interior_wave(g, ywave)) {
      gather_interior<WRAP>(g, cd, src, x, y, f);
    } else {
      const int yc = y < g.ly ? y : g.ly - 1;
      gather_wall<WRAP>(g, cd, src, x, yc, f);
      if (yc < WALL_ROWS || yc >= g.ly - WALL_ROWS) thermalise(f, yc < WALL_ROWS, w);
    }
  } else {
    // only the 3 + 3 edge columns pull across the periodic boundary; the
    // column is uniform over the work-group, so this is one scalar branch
    // and every other column runs the plain gather
    const bool edge = WRAP && (x < HALO || x >= g.lx - HALO);
    if (interior_wave(g, ywave)) {
      if (edge) gather_interior<true>(g, cd, src, x, y, f);
      else gather_interior<false>(g, cd, src, x, y, f);
    } else {
      const int yc = y < g.ly ? y : g.ly - 1;
      if (edge) gather_wall<true>(g, cd, src, x, yc, f);
      else gather_wall<false>(g, cd, src, x, yc, f);
      if (yc < WALL_ROWS || yc >= g.ly - WALL_ROWS) thermalise(f, yc < WALL_ROWS, w);
    }
  }
  collide_site(f, c);
  if (y < g.ly) store_column_site(g, cd, dst, x, y, f);
}

// propagate + bc + collide in registers: one read and one write of every
// population per step (the fusion the paper applies in Sec. 5, here on
// every row, walls included, since bc is site-local).  WRAP: periodic x by
// wrapping source columns (no halo read, so no pbc launch is needed);
// else the halo columns are read.
// BAND: the launch over the wavefronts that straddle the layers of the
// binary16 deviation reference (see fused_site); a few wavefronts per
// column, so it takes no register bound.
// RUN_OFF: scalar run offsets in the interior gather and the store (one
// buffer descriptor per column); the launcher takes it for binary16
// deviation lattices whose column runs span less than 2^31 bytes, where
// it removes most of the scalar address arithmetic that otherwise
// precedes each of the 74 accesses.
template <class C, int BLOCK, bool WRAP, bool BAND = false, bool RUN_OFF = false>
__global__ void __launch_bounds__(BLOCK, BAND ? 1 : C::kMinWaves) fused_kernel(const typename C::S* __restrict__ src,
                                                      typename C::S* __restrict__ dst, Geometry g,
                                                      CollideParams c, WallParams w, ColumnSet cols) {
  int x, y, ywave;
  lane_site<BLOCK>(g, cols, x, y, ywave);
  const C cd = C::of(g);
  fused_site<C, BLOCK, WRAP, BAND, RUN_OFF>(g, cd, src, dst, c, w, cols, x, y, ywave);
}

// ---------------------------------------------------------------------------
// Two steps per launch (temporal blocking on chip), binary64 storage
// ---------------------------------------------------------------------------
// One wavefront takes a strip of 64 consecutive rows (row base + lane) and
// marches along x over a segment of columns.  At column x1 it does the
// first step of that column (the pull of Eq. (10), the walls, the
// collision) and then the second step of column x1 - 3: the second pull
// of population l reads the first step's output at column x1 - 3 - e_lx,
// stepped 3 + e_lx columns ago, and at row y - e_ly, held by lane
// lane - e_ly (a cross-lane permute).  Each population of the first step's
// output is kept exactly 3 + e_lx columns (111 binary64 values per lane in
// all, in registers and LDS, below), so the intermediate lattice never
// reaches memory: per site and two steps, 296 bytes are read and 296
// written, instead of twice that.  The price is overlap: a strip's edge
// lanes are not outputs unless they lie at a wall (their second pull would
// need rows of the neighbouring strip), so a strip yields 58 rows (61 at a
// wall), and a segment of n output columns steps n + 6 columns once.
//
// Strips: strip k has base = min(58 k, ly - 64) and outputs rows
// [k == 0 ? 0 : 58 k + 3, k == last ? ly : 58 k + 61); ly >= 64.  Rows
// beyond a wall are replaced as in gather_wall: in the first step from
// the source lattice, in the second from the first step's output at the
// site itself, population opp(l), which the wall lanes (lanes 0-2 and
// 61-63) keep in a small LDS stash, the whole site four columns deep.
//
// The second step of a column is collided one iteration later, in the same
// block as the next column's first step: the two collisions are
// independent, and a lone wavefront per SIMD needs that instruction-level
// parallelism to cover the FP64 latencies (+5 % on 2048 x 8192).
//
// Arithmetic is that of the fused kernel, operation for operation
// (gather_interior / gather_wall, thermalise, collide_site), so two steps
// of this kernel equal two launches of the fused kernel bit for bit.
static_assert(F2_ROWS == WAVE, "a strip is one wavefront");

// Population l waits lag_of(l) = 3 + e_lx columns between its first and its
// second step.  The short waits (at most 3 columns, 40 values) are shift
// registers; the long ones (4-6 columns, 71 values) are circular buffers
// in LDS, one 64-lane row of binary64 per slot and each lane touching only
// its own column of it, so no barrier is needed.  Both together would not
// fit the 512 registers of a lane without spilling.
constexpr int lag_of(int l) { return HALO + EX[l]; }
constexpr int LDS_LAG = 4;  // lags from 4 up live in LDS
constexpr bool in_lds(int l) { return lag_of(l) >= LDS_LAG; }
constexpr int ring_off(int l) {
  int o = 0;
  for (int k = 0; k < l; ++k) o += in_lds(k) ? 0 : lag_of(k);
  return o;
}
constexpr int lds_off(int l) {
  int o = 0;
  for (int k = 0; k < l; ++k) o += in_lds(k) ? lag_of(k) : 0;
  return o;
}
constexpr int RING_LEN = ring_off(NPOP);
constexpr int LDS_SLOTS = lds_off(NPOP);
static_assert(RING_LEN + LDS_SLOTS == 3 * NPOP, "the e_x of the velocity set sum to zero");
constexpr int STASH_COLS = 4;   // columns x1 - 3 .. x1
constexpr int STASH_LANES = 6;  // lanes 0-2 and 61-63

__device__ __forceinline__ double lane_fetch(double v, int src_lane) {
  const int addr = src_lane << 2;  // ds_bpermute takes lane * 4, modulo 64 lanes
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_ds_bpermute(addr, static_cast<int>(b));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, static_cast<int>(b >> 32));
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// Column position j mod L of the circular buffer of lag L (L = 4, 5, 6).
__device__ __forceinline__ int lds_pos(int l, int r4, int r5, int r6) {
  return lag_of(l) == 4 ? r4 : lag_of(l) == 5 ? r5 : r6;
}

template <bool WALL>
__global__ void __launch_bounds__(WAVE, 1) fused2_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                       Geometry g, CollideParams c, WallParams w,
                                                       Fused2Strips st) {
  __shared__ double lring[LDS_SLOTS][WAVE];
  __shared__ double stash[WALL ? STASH_COLS : 1][WALL ? NPOP : 1][STASH_LANES];
  const CodecF64 cd{};
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int i = tile % st.count;
  const int seg = tile / st.count;
  const int strip = fused2_strip_of(st, WALL, i);
  const int lane = static_cast<int>(threadIdx.x);
  const Fused2Rows rows = fused2_rows(strip, st.nstrip, g.ly);
  const int y = rows.base + lane;
  const bool out = y >= rows.out_lo && y < rows.out_hi;
  const bool wall_row = y < WALL_ROWS || y >= g.ly - WALL_ROWS;
  const int slot = lane < WALL_ROWS ? lane : lane - (WAVE - 2 * WALL_ROWS);
  const int x_first = seg * st.seg_w;
  const int nout = min(st.seg_w, g.lx - x_first);
  int x1 = x_first - HALO;
  if (x1 < 0) x1 += g.lx;
  double ring[RING_LEN];
#pragma unroll
  for (int r = 0; r < RING_LEN; ++r) ring[r] = 0.0;
  int r4 = 0, r5 = 0, r6 = 0;  // j mod 4, 5, 6
  // the loads of each column are issued one column ahead (a lone
  // wavefront per SIMD hides no memory latency by switching)
  auto gather = [&](int x, double(&v)[NPOP]) {
    if constexpr (WALL) gather_wall<true>(g, cd, src, x, y, v);
    else gather_interior<true>(g, cd, src, x, y, v);
  };
  double next[NPOP];
  gather(x1, next);
  const int ncol = nout + 2 * HALO;
  // qp: the second step's pulled site of the previous iteration (column
  // xq), collided in the same block as this iteration's first step, so
  // that the two independent collisions can interleave
  double qp[NPOP];
#pragma unroll
  for (int l = 0; l < NPOP; ++l) qp[l] = 0.0;
  int xq = 0;
  for (int j = 0; j <= ncol; ++j) {
    double f[NPOP];
#pragma unroll
    for (int l = 0; l < NPOP; ++l) f[l] = next[l];
    if (j + 1 < ncol) gather(x1 + 1 == g.lx ? 0 : x1 + 1, next);
    if (WALL && wall_row) thermalise(f, y < WALL_ROWS, w);
    collide_site(f, c);
    collide_site(qp, c);
    if (j > 2 * HALO && out) store_column_site(g, cd, dst, xq, y, qp);
    if (j == ncol) break;
    if (WALL && wall_row) {
#pragma unroll
      for (int k = 0; k < NPOP; ++k) stash[j % STASH_COLS][k][slot] = f[k];
    }
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
      if (lag_of(l) == 0) {
        qp[l] = f[l];
      } else if (in_lds(l)) {
        double* cell = &lring[lds_off(l) + lds_pos(l, r4, r5, r6)][lane];
        qp[l] = *cell;
        *cell = f[l];
      } else {
        qp[l] = ring[ring_off(l)];
#pragma unroll
        for (int r = 0; r + 1 < lag_of(l); ++r) ring[ring_off(l) + r] = ring[ring_off(l) + r + 1];
        ring[ring_off(l) + lag_of(l) - 1] = f[l];
      }
    }
#pragma unroll
    for (int l = 0; l < NPOP; ++l)
      if (EY[l] != 0) qp[l] = lane_fetch(qp[l], lane - EY[l]);
    if (WALL && wall_row) {
#pragma unroll
      for (int l = 0; l < NPOP; ++l) {
        if (EY[l] == 0) continue;
        const int ys = y - EY[l];
        if (ys < 0 || ys >= g.ly) qp[l] = stash[(j + 1) % STASH_COLS][opp_of(l)][slot];
      }
      thermalise(qp, y < WALL_ROWS, w);
    }
    r4 = r4 == 3 ? 0 : r4 + 1;
    r5 = r5 == 4 ? 0 : r5 + 1;
    r6 = r6 == 5 ? 0 : r6 + 1;
    xq = x1 - HALO;
    if (xq < 0) xq += g.lx;
    x1 = x1 + 1 == g.lx ? 0 : x1 + 1;
  }
}

// Per-site rho, ux, uy, T into out[4][lx][ly] (Sec. 2 moment definitions;
// D rho T = sum |c|^2 f - rho |u|^2).
template <class C>
__global__ void __launch_bounds__(256) moments_kernel(const typename C::S* __restrict__ src,
                                                      double* __restrict__ out, Geometry g) {
  const C cd = C::of(g);
  const long long n = static_cast<long long>(g.lx) * g.ly;
  const long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const int x = static_cast<int>(i / g.ly);
  const int y = static_cast<int>(i - static_cast<long long>(x) * g.ly);
  double f[NPOP];
  load_site(g, cd, src, x, y, f);
  const MomentSums m = moment_sums(f);
  const double inv_rho = 1.0 / m.rho;
  const double ux = R * m.jx * inv_rho;
  const double uy = R * m.jy * inv_rho;
  out[i] = m.rho;
  out[n + i] = ux;
  out[2 * n + i] = uy;
  out[3 * n + i] = 0.5 * (R2 * m.eps * inv_rho - (ux * ux + uy * uy));
}

// Sum of a work-group's values in a fixed order: butterfly inside each
// wavefront, then wavefront totals in index order.
template <int THREADS>
__device__ __forceinline__ double block_sum(double v, double* lds) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v = v + __shfl_xor(v, o, WAVE);
  const int wave = threadIdx.x / WAVE;
  __syncthreads();
  if ((threadIdx.x & (WAVE - 1)) == 0) lds[wave] = v;
  __syncthreads();
  double s = lds[0];
#pragma unroll
  for (int k = 1; k < THREADS / WAVE; ++k) s = s + lds[k];
  return s;
}

// Conservation sums, pass 1: each work-group walks a fixed strided set of
// sites and writes its 5 partial sums.
template <class C>
__global__ void __launch_bounds__(CONS_THREADS) conservation_partial_kernel(
    const typename C::S* __restrict__ src, Geometry g, double* __restrict__ partials) {
  const C cd = C::of(g);
  __shared__ double lds[CONS_THREADS / WAVE];
  const long long n = static_cast<long long>(g.lx) * g.ly;
  double acc[CONS_FIELDS] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (long long i = static_cast<long long>(blockIdx.x) * CONS_THREADS + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * CONS_THREADS) {
    const int x = static_cast<int>(i / g.ly);
    const int y = static_cast<int>(i - static_cast<long long>(x) * g.ly);
    double f[NPOP];
    load_site(g, cd, src, x, y, f);
    int bad = 0;
#pragma unroll
    for (int l = 0; l < NPOP; ++l) bad += isfinite(f[l]) ? 0 : 1;
    const MomentSums m = moment_sums(f);
    acc[0] = acc[0] + m.rho;
    acc[1] = acc[1] + R * m.jx;
    acc[2] = acc[2] + R * m.jy;
    acc[3] = acc[3] + 0.5 * (R2 * m.eps);
    acc[4] = acc[4] + static_cast<double>(bad);
  }
#pragma unroll
  for (int k = 0; k < CONS_FIELDS; ++k) {
    const double s = block_sum<CONS_THREADS>(acc[k], lds);
    if (threadIdx.x == 0) partials[blockIdx.x * CONS_FIELDS + k] = s;
  }
}

// Pass 2: one work-group adds the partials in a fixed order.
__global__ void __launch_bounds__(CONS_THREADS) conservation_final_kernel(
    const double* __restrict__ partials, int nparts, double* __restrict__ result) {
  __shared__ double lds[CONS_THREADS / WAVE];
#pragma unroll
  for (int k = 0; k < CONS_FIELDS; ++k) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += CONS_THREADS) acc = acc + partials[i * CONS_FIELDS + k];
    const double s = block_sum<CONS_THREADS>(acc, lds);
    if (threadIdx.x == 0) result[k] = s;
  }
}

// Gather the populations of n listed sites (coordinates checked on the
// host): out[l * n + i] = f_l(xs[i], ys[i]).
template <class C>
__global__ void __launch_bounds__(256) get_sites_kernel(const typename C::S* __restrict__ f, Geometry g,
                                                        const int* __restrict__ xs,
                                                        const int* __restrict__ ys, int n,
                                                        double* __restrict__ out) {
  const C cd = C::of(g);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int x = xs[i];
  const int y = ys[i];
  double v[NPOP];
  load_site(g, cd, f, x, y, v);
#pragma unroll
  for (int l = 0; l < NPOP; ++l) out[static_cast<long long>(l) * n + i] = v[l];
}

__device__ __forceinline__ double log_cosh(double z) {
  const double a = fabs(z);
  return (a + log1p(exp(-2.0 * a))) - 0.6931471805599453094172321;
}

// Rayleigh-Taylor fields at row y of a column whose interface is displaced
// by h: tanh temperature interface, pressure in hydrostatic balance
// d ln p / dy = r gy / T (closed-form integral from the interface, where
// p = 1), rho = p / T.
__device__ __forceinline__ void rt_fields(const RtParams& p, int y, double h, double& rho,
                                          double& temp) {
  const double z = ((static_cast<double>(y) - p.y_center) - h) / p.width;
  temp = p.tm - p.a * tanh(z);
  const double z0 = atanh(p.a / p.tm);
  const double integral = p.width * (p.tm * z + p.a * (log_cosh(z - z0) - log_cosh(-z0))) /
                          (p.tm * p.tm - p.a * p.a);
  rho = exp(R * p.gy * integral) / temp;
}

// Rayleigh-Taylor initial state: interface displaced by the Fourier modes
// h(x), populations at the zero-velocity equilibrium rho K_l(T).
template <class C>
__global__ void __launch_bounds__(256) init_rt_kernel(typename C::S* __restrict__ f, Geometry g,
                                                      RtParams p) {
  const C cd = C::of(g);
  const long long n = static_cast<long long>(g.lx) * g.ly;
  const long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const int x = static_cast<int>(i / g.ly);
  const int y = static_cast<int>(i - static_cast<long long>(x) * g.ly);
  const double two_pi = 6.283185307179586476925287;
  double h = 0.0;
  for (int k = 0; k < p.n_modes; ++k)
    h = h + p.amp[k] * cos(two_pi * static_cast<double>(k + 1) * static_cast<double>(x) /
                               static_cast<double>(g.lx) + p.phase[k]);
  double rho, temp;
  rt_fields(p, y, h, rho, temp);
  const double th = temp - 1.0;
#pragma unroll
  for (int l = 0; l < NPOP; ++l) {
    const double C2 = R2 * static_cast<double>(EX[l] * EX[l] + EY[l] * EY[l]);
    const double k = weight_of(l) * ((1.0 + th * (C2 - 2.0) / 2.0) + th * th * (C2 * C2 - 8.0 * C2 + 8.0) / 8.0);
    f[run_of(g, l, x + HALO) + y] = cd.enc(rho * k, l, y);
  }
}

// Reference state of the deviation storage, per row: density and
// temperature of the Rayleigh-Taylor state with a flat interface.
__global__ void __launch_bounds__(256) rt_reference_kernel(double* __restrict__ rho_out,
                                                           double* __restrict__ temp_out, int ly,
                                                           RtParams p) {
  const int y = blockIdx.x * 256 + threadIdx.x;
  if (y >= ly) return;
  double rho, temp;
  rt_fields(p, y, 0.0, rho, temp);
  rho_out[y] = rho;
  temp_out[y] = temp;
}

// Host-array transfers through the codec: one population at a time
// between binary64 values [x][y] and its stored runs.
template <class C>
__global__ void __launch_bounds__(256) encode_population_kernel(const double* __restrict__ in,
                                                           typename C::S* __restrict__ f,
                                                           Geometry g, int l) {
  const C cd = C::of(g);
  const long long n = static_cast<long long>(g.lx) * g.ly;
  const long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const int x = static_cast<int>(i / g.ly);
  const int y = static_cast<int>(i - static_cast<long long>(x) * g.ly);
  f[run_of(g, l, x + HALO) + y] = cd.enc(in[i], l, y);
}

template <class C>
__global__ void __launch_bounds__(256) decode_population_kernel(const typename C::S* __restrict__ f,
                                                           double* __restrict__ out, Geometry g, int l) {
  const C cd = C::of(g);
  const long long n = static_cast<long long>(g.lx) * g.ly;
  const long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const int x = static_cast<int>(i / g.ly);
  const int y = static_cast<int>(i - static_cast<long long>(x) * g.ly);
  out[i] = cd.dec(f[run_of(g, l, x + HALO) + y], l, y);
}

// ---------------------------------------------------------------------------
// Bandwidth probes
// ---------------------------------------------------------------------------

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_BLOCKS = 256 * 8;  // 8 work-groups per CU, grid-stride
constexpr int COPY_UNROLL = 4;         // 16-byte vectors per lane per pass
constexpr size_t COPY_MAX_BLOCKS = 65536;

// dst[i] = src[i] for i in [0, n) 16-byte vectors: the fastest plain copy
// found on this part.  Each lane loads COPY_UNROLL vectors one grid width
// apart, then stores them, all non-temporal; the last partial pass copies
// one vector per lane.
__global__ void __launch_bounds__(PROBE_THREADS) probe_copy_kernel(const double2* __restrict__ src,
                                                                   double2* __restrict__ dst,
                                                                   size_t n) {
  typedef double V __attribute__((ext_vector_type(2)));
  const V* s = reinterpret_cast<const V*>(src);
  V* d = reinterpret_cast<V*>(dst);
  const size_t stride = static_cast<size_t>(gridDim.x) * PROBE_THREADS;
  size_t i = static_cast<size_t>(blockIdx.x) * PROBE_THREADS + threadIdx.x;
  for (; i + (COPY_UNROLL - 1) * stride < n; i += COPY_UNROLL * stride) {
    V v[COPY_UNROLL];
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) v[u] = __builtin_nontemporal_load(&s[i + u * stride]);
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) __builtin_nontemporal_store(v[u], &d[i + u * stride]);
  }
  for (; i < n; i += stride) d[i] = s[i];
}

// dst[i + ws] = src[i + rs] for i in [0, n): one of rs, ws is the shift.
__global__ void __launch_bounds__(PROBE_THREADS) probe_shift_kernel(const double* __restrict__ src,
                                                                    double* __restrict__ dst,
                                                                    size_t n, long long rs,
                                                                    long long ws) {
  for (size_t i = static_cast<size_t>(blockIdx.x) * PROBE_THREADS + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * PROBE_THREADS)
    dst[static_cast<long long>(i) + ws] = src[static_cast<long long>(i) + rs];
}

}  // namespace

// Dispatch on the storage codec (C, element type S) and work-group size (BS).
#define D2Q37_DISPATCH(G, ...)                                                         \
  switch ((G).storage) {                                                               \
    case STORAGE_F64: { using C = CodecF64; using S = C::S; D2Q37_BLOCKS(G, __VA_ARGS__); break; }  \
    case STORAGE_F32: { using C = CodecF32; using S = C::S; D2Q37_BLOCKS(G, __VA_ARGS__); break; }  \
    case STORAGE_F16DEV: { using C = CodecF16Dev; using S = C::S; D2Q37_BLOCKS(G, __VA_ARGS__); break; } \
    default: return hipErrorInvalidValue;                                              \
  }
#define D2Q37_BLOCKS(G, ...)                                \
  switch ((G).block) {                                      \
    case 64: { constexpr int BS = 64; __VA_ARGS__; break; }        \
    case 128: { constexpr int BS = 128; __VA_ARGS__; break; }      \
    case 256: { constexpr int BS = 256; __VA_ARGS__; break; }      \
    case 512: { constexpr int BS = 512; __VA_ARGS__; break; }      \
    case 1024: { constexpr int BS = 1024; __VA_ARGS__; break; }    \
    default: return hipErrorInvalidValue;                   \
  }
#define D2Q37_STORAGE(G, ...)                                                          \
  switch ((G).storage) {                                                               \
    case STORAGE_F64: { using C = CodecF64; using S = C::S; __VA_ARGS__; break; }      \
    case STORAGE_F32: { using C = CodecF32; using S = C::S; __VA_ARGS__; break; }      \
    case STORAGE_F16DEV: { using C = CodecF16Dev; using S = C::S; __VA_ARGS__; break; } \
    default: return hipErrorInvalidValue;                                              \
  }

hipError_t launch_pbc(const Geometry& g, void* f, hipStream_t s) {
  (void)hipGetLastError();
  D2Q37_STORAGE(g, hipLaunchKernelGGL(pbc_kernel<S>, dim3((g.ly + 255) / 256, 52), dim3(256), 0, s,
                                      static_cast<S*>(f), g));
  return hipGetLastError();
}

hipError_t launch_propagate(const Geometry& g, const void* src, void* dst, hipStream_t s) {
  (void)hipGetLastError();
  D2Q37_DISPATCH(g, hipLaunchKernelGGL((propagate_kernel<C, BS>), dim3(g.lx * g.ny_blocks), dim3(BS),
                                       0, s, static_cast<const S*>(src), static_cast<S*>(dst), g));
  return hipGetLastError();
}

hipError_t launch_bc(const Geometry& g, void* f, const WallParams& w, hipStream_t s) {
  const int n = g.lx * 2 * WALL_ROWS;
  (void)hipGetLastError();
  D2Q37_STORAGE(g, hipLaunchKernelGGL(bc_kernel<C>, dim3((n + 255) / 256), dim3(256), 0, s,
                                      static_cast<S*>(f), g, w));
  return hipGetLastError();
}

hipError_t launch_collide(const Geometry& g, const void* src, void* dst, const CollideParams& c,
                          hipStream_t s) {
  (void)hipGetLastError();
  D2Q37_DISPATCH(g, hipLaunchKernelGGL((collide_kernel<C, BS>), dim3(g.lx * g.ny_blocks), dim3(BS),
                                       0, s, static_cast<const S*>(src), static_cast<S*>(dst), g, c));
  return hipGetLastError();
}

hipError_t launch_fused(const Geometry& g, const void* src, void* dst, const CollideParams& c,
                        const WallParams& w, hipStream_t s, const ColumnSet* cols, bool wrap) {
  const ColumnSet all{0, g.lx, 0};
  const ColumnSet cs = cols ? *cols : all;
  const int ncols = cs.na + (cols ? cs.nb : 0);
  if (ncols <= 0) return hipSuccess;
  hipError_t e = launch_fused_rows(g, src, dst, c, w, s, cs, ncols, g.ny_blocks, wrap);
  if (e != hipSuccess || g.storage != STORAGE_F16DEV || g.ysplit <= 0 || g.ysplit >= g.ly) return e;
  // the wavefronts that straddle the reference's temperature layers: first
  // rows y0 (multiples of 64) with y0 - 3 < ysplit <= y0 + 66
  const int first = std::max(0, (g.ysplit - WALL_ROWS) / WAVE * WAVE);
  const int last = std::min((g.ly - 1) / WAVE * WAVE, (g.ysplit + WALL_ROWS - 1) / WAVE * WAVE);
  ColumnSet band = cs;
  band.band = 1;
  band.y0 = first;
  band.nyb = (last + WAVE - first + g.block - 1) / g.block;
  return launch_fused_rows(g, src, dst, c, w, s, band, ncols, band.nyb, wrap);
}

hipError_t launch_fused2(const Geometry& g, const void* src, void* dst, const CollideParams& c,
                         const WallParams& w, const Fused2Strips& st, bool wall, hipStream_t s) {
  if (!(g.storage == STORAGE_F64 && g.ly >= F2_ROWS && st.seg_w >= 1 && st.count >= 0 &&
        st.nstrip == fused2_strips(g.ly)))
    return hipErrorInvalidValue;
  if (st.count == 0) return hipSuccess;
  const long long grid = static_cast<long long>(st.count) * ((g.lx + st.seg_w - 1) / st.seg_w);
  if (grid >= (1LL << 31)) return hipErrorInvalidValue;
  (void)hipGetLastError();
  if (wall)
    hipLaunchKernelGGL(fused2_kernel<true>, dim3(static_cast<unsigned>(grid)), dim3(WAVE), 0, s,
                       static_cast<const double*>(src), static_cast<double*>(dst), g, c, w, st);
  else
    hipLaunchKernelGGL(fused2_kernel<false>, dim3(static_cast<unsigned>(grid)), dim3(WAVE), 0, s,
                       static_cast<const double*>(src), static_cast<double*>(dst), g, c, w, st);
  return hipGetLastError();
}

hipError_t launch_fused_rows(const Geometry& g, const void* src, void* dst, const CollideParams& c,
                             const WallParams& w, hipStream_t s, const ColumnSet& cs, int ncols, int nyb,
                             bool wrap) {
  (void)hipGetLastError();
  if (cs.band) {
    if (g.storage != STORAGE_F16DEV) return hipErrorInvalidValue;
    using C = CodecF16Dev;
    using S = C::S;
    if (wrap) {
      D2Q37_BLOCKS(g, hipLaunchKernelGGL((fused_kernel<C, BS, true, true>), dim3(ncols * nyb), dim3(BS), 0, s,
                                         static_cast<const S*>(src), static_cast<S*>(dst), g, c, w, cs));
    } else {
      D2Q37_BLOCKS(g, hipLaunchKernelGGL((fused_kernel<C, BS, false, true>), dim3(ncols * nyb), dim3(BS), 0, s,
                                         static_cast<const S*>(src), static_cast<S*>(dst), g, c, w, cs));
    }
    return hipGetLastError();
  }
  if (wrap) {
    switch (g.storage) {
      case STORAGE_F64: {
        using C = CodecF64;
        using S = C::S;
        D2Q37_BLOCKS(g, hipLaunchKernelGGL((fused_kernel<C, BS, true>), dim3(ncols * nyb), dim3(BS),
                                           0, s, static_cast<const S*>(src), static_cast<S*>(dst), g, c, w, cs));
        break;
      }
      case STORAGE_F32: {
        using C = CodecF32;
        using S = C::S;
        D2Q37_BLOCKS(g, hipLaunchKernelGGL((fused_kernel<C, BS, true>), dim3(ncols * nyb), dim3(BS),
                                           0, s, static_cast<const S*>(src), static_cast<S*>(dst), g, c, w, cs));
        break;
      }
      case STORAGE_F16DEV: {
        using C = CodecF16Dev;
        using S = C::S;
        if (g.run_off) {
          D2Q37_BLOCKS(g, hipLaunchKernelGGL((fused_kernel<C, BS, true, false, true>), dim3(ncols * nyb),
                                             dim3(BS), 0, s, static_cast<const S*>(src), static_cast<S*>(dst), g,
                                             c, w, cs));
        } else {
          D2Q37_BLOCKS(g, hipLaunchKernelGGL((fused_kernel<C, BS, true>), dim3(ncols * nyb), dim3(BS),
                                             0, s, static_cast<const S*>(src), static_cast<S*>(dst), g, c, w, cs));
        }
        break;
      }
      default:
        return hipErrorInvalidValue;
    }
  } else if (g.storage == STORAGE_F16DEV && g.run_off) {
    using C = CodecF16Dev;
    using S = C::S;
    D2Q37_BLOCKS(g, hipLaunchKernelGGL((fused_kernel<C, BS, false, false, true>), dim3(ncols * nyb), dim3(BS),
                                       0, s, static_cast<const S*>(src), static_cast<S*>(dst), g, c, w, cs));
  } else {
    D2Q37_DISPATCH(g, hipLaunchKernelGGL((fused_kernel<C, BS, false>), dim3(ncols * nyb), dim3(BS),
                                         0, s, static_cast<const S*>(src), static_cast<S*>(dst), g, c, w, cs));
  }
  return hipGetLastError();
}

hipError_t launch_moments(const Geometry& g, const void* f, double* out, hipStream_t s) {
  const long long n = static_cast<long long>(g.lx) * g.ly;
  (void)hipGetLastError();
  D2Q37_STORAGE(g, hipLaunchKernelGGL(moments_kernel<C>, dim3(static_cast<unsigned>((n + 255) / 256)),
                                      dim3(256), 0, s, static_cast<const S*>(f), out, g));
  return hipGetLastError();
}

hipError_t launch_conservation(const Geometry& g, const void* f, double* partials, double* result,
                               hipStream_t s) {
  (void)hipGetLastError();
  D2Q37_STORAGE(g, hipLaunchKernelGGL(conservation_partial_kernel<C>, dim3(CONS_BLOCKS),
                                      dim3(CONS_THREADS), 0, s, static_cast<const S*>(f), g, partials));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(conservation_final_kernel, dim3(1), dim3(CONS_THREADS), 0, s, partials,
                     CONS_BLOCKS, result);
  return hipGetLastError();
}

hipError_t launch_get_sites(const Geometry& g, const void* f, const int* xs, const int* ys, int n,
                            double* out, hipStream_t s) {
  (void)hipGetLastError();
  D2Q37_STORAGE(g, hipLaunchKernelGGL(get_sites_kernel<C>, dim3((n + 255) / 256), dim3(256), 0, s,
                                      static_cast<const S*>(f), g, xs, ys, n, out));
  return hipGetLastError();
}

hipError_t launch_probe(int mode, const void* src, void* dst, size_t n16, int shift, hipStream_t s) {
  (void)hipGetLastError();
  if (mode == 0) {
    const size_t per_block = static_cast<size_t>(COPY_UNROLL) * PROBE_THREADS;
    const size_t blocks = std::min(COPY_MAX_BLOCKS, std::max<size_t>(1, (n16 + per_block - 1) / per_block));
    hipLaunchKernelGGL(probe_copy_kernel, dim3(static_cast<unsigned>(blocks)), dim3(PROBE_THREADS), 0, s,
                       static_cast<const double2*>(src), static_cast<double2*>(dst), n16);
  } else {
    // doubles: the aligned side is index i + 64 (a whole wavefront of
    // doubles in), the misaligned side i + 64 + shift, i in [0, n - 128),
    // so both stay inside [0, n) for |shift| <= 64.
    const long long n = 2 * static_cast<long long>(n16);
    const long long rs = mode == 1 ? 64 + shift : 64;
    const long long ws = mode == 1 ? 64 : 64 + shift;
    hipLaunchKernelGGL(probe_shift_kernel, dim3(PROBE_BLOCKS), dim3(PROBE_THREADS), 0, s,
                       static_cast<const double*>(src), static_cast<double*>(dst),
                       static_cast<size_t>(n - 128), rs, ws);
  }
  return hipGetLastError();
}

hipError_t launch_rt_reference(const Geometry& g, double* rho, double* temp, const RtParams& p,
                               hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(rt_reference_kernel, dim3((g.ly + 255) / 256), dim3(256), 0, s, rho, temp, g.ly, p);
  return hipGetLastError();
}

hipError_t launch_encode_population(const Geometry& g, const double* in, void* f, int l, hipStream_t s) {
  const long long n = static_cast<long long>(g.lx) * g.ly;
  (void)hipGetLastError();
  D2Q37_STORAGE(g, hipLaunchKernelGGL(encode_population_kernel<C>, dim3(static_cast<unsigned>((n + 255) / 256)),
                                      dim3(256), 0, s, in, static_cast<S*>(f), g, l));
  return hipGetLastError();
}

hipError_t launch_decode_population(const Geometry& g, const void* f, double* out, int l, hipStream_t s) {
  const long long n = static_cast<long long>(g.lx) * g.ly;
  (void)hipGetLastError();
  D2Q37_STORAGE(g, hipLaunchKernelGGL(decode_population_kernel<C>, dim3(static_cast<unsigned>((n + 255) / 256)),
                                      dim3(256), 0, s, static_cast<const S*>(f), out, g, l));
  return hipGetLastError();
}

hipError_t launch_init_rt(const Geometry& g, void* f, const RtParams& p, hipStream_t s) {
  const long long n = static_cast<long long>(g.lx) * g.ly;
  (void)hipGetLastError();
  D2Q37_STORAGE(g, hipLaunchKernelGGL(init_rt_kernel<C>, dim3(static_cast<unsigned>((n + 255) / 256)),
                                      dim3(256), 0, s, static_cast<S*>(f), g, p));
  return hipGetLastError();
}

}  // namespace d2q37
