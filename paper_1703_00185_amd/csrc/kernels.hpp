// Launch interface between the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "d2q37_model.hpp"

namespace d2q37 {

// Population storage types.
enum Storage : int { STORAGE_F64 = 0, STORAGE_F32 = 1, STORAGE_F16DEV = 2 };

// Population layouts.  X in [0, lx + 6) counts columns including 3 halo
// columns on each side (physical column x is X = x + 3), y in [0, ny) is
// the row, with rows >= ly being padding that is never read.  Element
// (l, X, y) sits at l * pstride + X * cstride + y:
//  * COLUMN f[X][l][y]: pstride = ny, cstride = 37 ny (+ pad).  Each column
//    holds its 37 population runs back to back, so a work-group's tile
//    streams through one contiguous column block;
//  * PLANAR f[l][X][y]: cstride = ny, pstride = (lx + 6) ny (+ pad), the
//    structure-of-arrays planes of Sec. 4 "Data Structure Analysis".
// In both, each population of a column is ny contiguous rows, so the 64
// lanes of a wavefront (consecutive rows) touch one contiguous segment.
enum PopLayout : int { LAYOUT_COLUMN = 0, LAYOUT_PLANAR = 1 };

struct Geometry {
  int lx, ly;
  int storage;       // Storage: element type of the populations
  int layout;        // PopLayout
  int ny;            // rows per column run (pitch), elements
  int block;         // work-group size of the lattice kernels
  int ny_blocks;     // ceil(ly / block)
  long long pstride; // elements between populations l and l + 1 of a site
  long long cstride; // elements between columns X and X + 1
  // deviation storage: the reference density per row and its reciprocal,
  // and the shell factors kf[KF_LEN] of the two temperature layers (rows
  // y < ysplit and y >= ysplit)
  const double* ref;
  const double* inv_ref;
  const double* kf;
  int ysplit;
  // 1 when the bytes from a column's start to 3 rows past its last run
  // stay below 2^31, so that one buffer descriptor per column with scalar
  // run offsets can address them (the binary16 fused kernel uses it)
  int run_off;
};

// Shell factors of the deviation-storage reference: K_s(T_lo), K_s(T_hi),
// 1 / K_s(T_lo), 1 / K_s(T_hi), W_s / K_s(T_lo), W_s / K_s(T_hi), NSHELL
// doubles each.
constexpr int KF_LO = 0, KF_HI = NSHELL, KF_INV_LO = 2 * NSHELL, KF_INV_HI = 3 * NSHELL;
constexpr int KF_WK_LO = 4 * NSHELL, KF_WK_HI = 5 * NSHELL;
constexpr int KF_LEN = 6 * NSHELL;

// Scalars of the collision (Eqs. 4-6): omega = 1/tau, the shift tau*g of
// the velocity and tau^2 |g|^2 / 2 of the temperature.
struct CollideParams {
  double omega;
  double one_minus_omega;
  double tgx, tgy;
  double dtemp;
};

// Wall factors K_l(T_wall) for the bottom and top walls.
struct WallParams {
  double kb[NPOP];
  double kt[NPOP];
};

// Columns covered by a lattice launch: na columns from xa, then nb
// columns from xb (nb is used by the host only, to size the grid).  band:
// a launch of the fused kernel over only the wavefronts that straddle the
// temperature layers of the binary16 deviation reference, rows from y0 in
// nyb work-group tiles (0: every other wavefront, rows from 0).
struct ColumnSet {
  int xa, na, xb;
  int nb = 0;
  int band = 0;
  int y0 = 0;
  int nyb = 0;  // 0: the geometry's ny_blocks
};

// Rayleigh-Taylor initial state parameters.
constexpr int MAX_MODES = 32;
struct RtParams {
  double tm, a;          // mean temperature, half contrast
  double width, y_center;
  double gy;
  int n_modes;
  double amp[MAX_MODES];
  double phase[MAX_MODES];
};

constexpr int CONS_BLOCKS = 1024;  // work-groups of the conservation pass
constexpr int CONS_THREADS = 256;
constexpr int CONS_FIELDS = 5;     // mass, jx, jy, energy, non-finite count

// Launchers: enqueue one kernel on stream s; the population pointers
// point to lattice copies in the geometry's layout and storage type.
hipError_t launch_pbc(const Geometry& g, void* f, hipStream_t s);
hipError_t launch_propagate(const Geometry& g, const void* src, void* dst, hipStream_t s);
hipError_t launch_bc(const Geometry& g, void* f, const WallParams& w, hipStream_t s);
hipError_t launch_collide(const Geometry& g, const void* src, void* dst, const CollideParams& c,
                          hipStream_t s);
// cols = nullptr: every column; else the two column ranges of *cols.
// wrap: periodic x by wrapping source columns (reads no halo column);
// else the halo columns written by pbc are read.
hipError_t launch_fused(const Geometry& g, const void* src, void* dst, const CollideParams& c,
                        const WallParams& w, hipStream_t s, const ColumnSet* cols = nullptr,
                        bool wrap = false);
// One launch of the fused kernel over ncols columns and nyb work-group
// tiles per column (launch_fused adds the band launch of binary16
// deviation lattices).
hipError_t launch_fused_rows(const Geometry& g, const void* src, void* dst, const CollideParams& c,
                             const WallParams& w, hipStream_t s, const ColumnSet& cs, int ncols, int nyb,
                             bool wrap);
// Two steps per launch (binary64 storage, ly >= 64, periodic x by
// wrapping): src -> dst equals two launch_fused steps through an
// intermediate lattice that is never stored.  The rows are cut into strips
// of 64 (58 output rows each, strip k from row 58 k); the interior strips
// and the strips holding wall rows take two kernels, which write disjoint
// rows and may run concurrently.  Strips of a launch: `count` strips from
// `first` (the wall launch: strip 0, then count - 1 strips from first),
// `nstrip` strips in all, `seg_w` output columns per wavefront.
struct Fused2Strips {
  int first, count, nstrip, seg_w;
};
struct Fused2Plan {
  int ok;  // 0: the lattice does not qualify (storage or ly < 64)
  Fused2Strips interior, wall;
};
// fused2_plan (fused2_plan.hpp) picks the strips and segments of a lattice.
hipError_t launch_fused2(const Geometry& g, const void* src, void* dst, const CollideParams& c,
                         const WallParams& w, const Fused2Strips& st, bool wall, hipStream_t s);
hipError_t launch_moments(const Geometry& g, const void* f, double* out, hipStream_t s);
hipError_t launch_conservation(const Geometry& g, const void* f, double* partials, double* result,
                               hipStream_t s);
// out[l * n + i] = f_l(xs[i], ys[i]) for n sites (device arrays).
hipError_t launch_get_sites(const Geometry& g, const void* f, const int* xs, const int* ys, int n,
                            double* out, hipStream_t s);
hipError_t launch_init_rt(const Geometry& g, void* f, const RtParams& p, hipStream_t s);
// Density and temperature of the flat-interface Rayleigh-Taylor state per
// row (the deviation-storage reference state), into rho[ly] and temp[ly].
hipError_t launch_rt_reference(const Geometry& g, double* rho, double* temp, const RtParams& p,
                               hipStream_t s);
hipError_t launch_encode_population(const Geometry& g, const double* in, void* f, int l, hipStream_t s);
hipError_t launch_decode_population(const Geometry& g, const void* f, double* out, int l, hipStream_t s);

// Copy probes (aligned copy, misaligned read / aligned write, aligned read /
// misaligned write); n16 = bytes / 16, shift in doubles.
hipError_t launch_probe(int mode, const void* src, void* dst, size_t n16, int shift, hipStream_t s);

}  // namespace d2q37
