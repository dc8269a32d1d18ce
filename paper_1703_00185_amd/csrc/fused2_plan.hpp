// Strips and segments of the two-step kernel (two steps per launch), for
// the host (the launch plan) and the device (each wavefront's rows).
//
// A strip is 64 consecutive rows, one wavefront, row base + lane.  Its
// second step pulls rows up to 3 beyond each output row, so an output row
// needs the first step of the 3 rows on either side inside the strip: a
// strip yields the 58 rows 3 .. 60 of its 64, and at a wall, where the
// rows beyond are replaced by bounce-back instead, the rows from or to the
// wall as well.  Strip k has base min(58 k, ly - 64) and outputs rows
// [k == 0 ? 0 : 58 k + 3, k == last ? ly : 58 k + 61); these ranges
// partition [0, ly) for every ly >= 64.
#pragma once

#include <algorithm>

#include "kernels.hpp"

namespace d2q37 {

constexpr int F2_ROWS = 64;                    // rows of a strip (one wavefront)
constexpr int F2_OUT = F2_ROWS - 2 * HALO;     // output rows of an interior strip
constexpr int F2_MIN_SEGMENT = 16;             // narrowest segment the plan picks

struct Fused2Rows {
  int base;            // first row of the strip
  int out_lo, out_hi;  // output rows [out_lo, out_hi)
};

D2Q37_HD inline int fused2_strips(int ly) { return (ly - F2_ROWS + F2_OUT - 1) / F2_OUT + 1; }

D2Q37_HD inline Fused2Rows fused2_rows(int strip, int nstrip, int ly) {
  Fused2Rows r;
  r.base = strip * F2_OUT < ly - F2_ROWS ? strip * F2_OUT : ly - F2_ROWS;
  r.out_lo = strip == 0 ? 0 : strip * F2_OUT + HALO;
  r.out_hi = strip == nstrip - 1 ? ly : strip * F2_OUT + F2_OUT + HALO;
  return r;
}

// Strips 1 .. n whose 64 rows hold no wall row (base + 64 <= ly - 3); the
// others (strip 0 and the last ones) take the wall kernel.
inline int fused2_interior_strips(int ly) {
  const int nstrip = fused2_strips(ly);
  int last = ly >= F2_ROWS + WALL_ROWS + F2_OUT ? (ly - WALL_ROWS - F2_ROWS) / F2_OUT : 0;
  last = std::min(last, nstrip - 2);
  return std::max(last, 0);
}

// Segments per strip: one wavefront per SIMD is resident (the kernel holds
// more than 256 registers and 36 KB of LDS), and a wavefront's time is the
// columns it steps, segment + 6.  Measured on 2048 x 8192: one round of
// wavefronts (7 segments of 293 columns) ran 9 % faster than any shape of
// several rounds, whatever their segment width, because the last round
// runs a fraction of the SIMDs for a whole segment.  The wall strips run
// beside the interior ones, each wall column costing about 1.7 interior
// ones (the wall gather and bounce-back), so their segments are a third as
// wide: they finish within the interior wavefronts' time and fill the
// SIMDs the interior round leaves.  So the plan minimises rounds x
// (segment + 6) over both launches, several rounds weighted by 1.1.
// simds: SIMDs of the device (4 per compute unit).
inline Fused2Plan fused2_plan(const Geometry& g, int simds) {
  Fused2Plan p{};
  if (g.storage != STORAGE_F64 || g.ly < F2_ROWS || g.lx < 1 || simds < 1) return p;
  const int nstrip = fused2_strips(g.ly);
  const int n_int = fused2_interior_strips(g.ly);
  const int n_wall = nstrip - n_int;
  auto wall_width = [&](int sw) { return std::min(g.lx, std::max(F2_MIN_SEGMENT / 2, (sw + 2) / 3)); };
  int best_n = 1;
  double best = -1.0;
  for (int nseg = 1; nseg <= g.lx; ++nseg) {
    const int sw = (g.lx + nseg - 1) / nseg;
    if (nseg > 1 && (g.lx + nseg - 2) / (nseg - 1) == sw) continue;  // same width as nseg - 1
    if (nseg > 1 && sw < F2_MIN_SEGMENT) break;  // 6 extra columns per few outputs
    const int ww = wall_width(sw);
    const long long waves =
        static_cast<long long>(n_int) * nseg + static_cast<long long>(n_wall) * ((g.lx + ww - 1) / ww);
    const long long rounds = (waves + simds - 1) / simds;
    const double cost = static_cast<double>(rounds) * (sw + 2 * HALO) * (rounds > 1 ? 1.1 : 1.0);
    if (best < 0.0 || cost < best) best = cost, best_n = nseg;
  }
  const int seg_w = (g.lx + best_n - 1) / best_n;
  p.interior = Fused2Strips{1, n_int, nstrip, seg_w};
  p.wall = Fused2Strips{1 + n_int, n_wall, nstrip, wall_width(seg_w)};
  p.ok = 1;
  return p;
}

// Strip of the i-th wavefront row of a launch: the interior launch takes
// strips first .. first + count - 1, the wall launch strip 0 and then
// strips first .. first + count - 2.
D2Q37_HD inline int fused2_strip_of(const Fused2Strips& st, bool wall, int i) {
  return wall ? (i == 0 ? 0 : st.first + i - 1) : st.first + i;
}

}  // namespace d2q37
