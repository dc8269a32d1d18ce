// Site-local device code of the D2Q37 step, shared by the single-lattice
// kernels and the ensemble engine: storage codecs, moment sums, the BGK
// collision and the thermal-wall reset.  Included by .hip files only; the
// including file must compile without floating-point contraction (every
// fused multiply-add below is an explicit fma()).
#pragma once

#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

#include "kernels.hpp"

namespace d2q37 {
namespace {

constexpr int WAVE = 64;
constexpr int NXCD = 8;  // accelerator complex dies of an MI355X

// Work-group ids are dealt round-robin over the 8 XCDs, each with its own
// L2.  Renumber them so that each XCD runs one contiguous range of logical
// tiles: neighbouring y-tiles of a column then share the 512-byte segments
// that straddle their boundary (the +-3-row misalignment of the pull) in
// the same L2.  Bijective for any number of groups.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
  const int xcd = bid % NXCD;
  const int idx = bid / NXCD;
  const int q = nblocks / NXCD;
  const int r = nblocks % NXCD;
  return xcd * q + (xcd < r ? xcd : r) + idx;
}

// Raw element access at a byte offset from a wavefront-uniform base,
// through a buffer descriptor built from that base (scalar instructions):
// the per-lane offset is the only vector operand, so no 64-bit vector
// address is formed per access (measured on the 2048 x 8192 fused step:
// binary16 +8 %, binary32 +2 %, binary64 +1 %).  The descriptor's range
// (2^31 - 1 bytes) is far above any offset used here (below one column
// run).  Cache-policy operand of the stores: nt | sc1 (non-temporal,
// system scope), measured on the fused step against nt alone: binary64
// +1.9 %, binary32 +1.3 %; default stores are 6 % slower and non-temporal
// loads slower too.  The bits set the write policy only, not what a later
// kernel reads.
constexpr int kBufferWord3 = 0x00020000;  // gfx9 raw buffer: 32-bit data format
constexpr int kNonTemporal = 2 | 16;      // nt | sc1

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_at(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, 0x7fffffff, kBufferWord3);
}

template <class S>
__device__ __forceinline__ S ld(const S* base, unsigned byte_off) {
  const __amdgpu_buffer_rsrc_t r = buffer_at(base);
  if constexpr (sizeof(S) == 2) {
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b16(r, byte_off, 0, 0));
  } else if constexpr (sizeof(S) == 4) {
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
  } else {
    static_assert(sizeof(S) == 8, "2-, 4- or 8-byte elements");
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
  }
}

// Element at voff + soff bytes from the base of descriptor r: voff per
// lane, soff wavefront-uniform (a scalar register operand of the buffer
// instruction), so one descriptor serves every run of a column and each
// access costs one scalar add instead of a 64-bit base and a descriptor.
// The caller keeps soff + voff below the descriptor's range.
template <class S>
__device__ __forceinline__ S ld_at(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (sizeof(S) == 2) {
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
  } else if constexpr (sizeof(S) == 4) {
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  } else {
    static_assert(sizeof(S) == 8, "2-, 4- or 8-byte elements");
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  }
}

// Non-temporal store at voff + soff bytes from the base of descriptor r.
template <class S>
__device__ __forceinline__ void st_nt_at(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, S v) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  if constexpr (sizeof(S) == 2) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, voff, soff, kNonTemporal);
  } else if constexpr (sizeof(S) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, kNonTemporal);
  } else {
    static_assert(sizeof(S) == 8, "2-, 4- or 8-byte elements");
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, kNonTemporal);
  }
}

// Non-temporal store (streaming: no reuse expected from the caches).
template <class S>
__device__ __forceinline__ void st_nt(S* base, unsigned byte_off, S v) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  const __amdgpu_buffer_rsrc_t r = buffer_at(base);
  if constexpr (sizeof(S) == 2) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, byte_off, 0, kNonTemporal);
  } else if constexpr (sizeof(S) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, byte_off, 0, kNonTemporal);
  } else {
    static_assert(sizeof(S) == 8, "2-, 4- or 8-byte elements");
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, byte_off, 0, kNonTemporal);
  }
}

// Population storage codecs.  Arithmetic is binary64 for every storage;
// a codec turns the stored element of population l at row y into the
// binary64 population and back.
//  * binary64: identity.
//  * binary32: exact widening; rounding to nearest on store.
//  * binary16 deviation: the element is d = (f - c) / c from the reference
//    c = K_l(T_L(y)) rho_ref(y), the zero-velocity equilibrium of a
//    reference state with a density per row and two temperature layers
//    (T_lo below row ysplit, T_hi from it up); stored as
//    d = f16(f32((f - c) * (K_l(T_L(y))^-1 * rho_ref(y)^-1))) and read
//    back as c (1 + d).  1 + d is exact in binary64, so decoding rounds
//    once.
// kMinWaves: wavefronts per SIMD the fused kernel's register budget must
// allow (1: no bound).  The binary16 kernel is VALU-bound; capped at 128
// VGPRs it keeps 4 wavefronts per SIMD.
// kLayered: the fused kernel gives a wavefront whose rows and pull sources
// all lie in one temperature layer the codec of that layer
// (CodecF16DevLayer), whose shell factors are wavefront-uniform.
// kWrapAlways: the wrapping fused kernel wraps every column's source
// columns (scalar arithmetic) instead of branching on the 3 + 3 edge
// columns.
using ConstD = const __attribute__((address_space(4))) double;
struct CodecF64 {
  static constexpr int kMinWaves = 1;
  static constexpr bool kLayered = false;
  static constexpr bool kWrapAlways = false;
  using S = double;
  static __device__ CodecF64 of(const Geometry&) { return {}; }
  __device__ double dec(S v, int, int) const { return v; }
  __device__ S enc(double f, int, int) const { return f; }
};
struct CodecF32 {
  static constexpr int kMinWaves = 1;
  static constexpr bool kLayered = false;
  static constexpr bool kWrapAlways = false;
  using S = float;
  static __device__ CodecF32 of(const Geometry&) { return {}; }
  __device__ double dec(S v, int, int) const { return static_cast<double>(v); }
  __device__ S enc(double f, int, int) const { return static_cast<float>(f); }
};
// Any rows: the layer is chosen per lane.
struct CodecF16Dev {
  static constexpr int kMinWaves = 4;
  static constexpr bool kLayered = true;
  static constexpr bool kWrapAlways = true;
  using S = _Float16;
  const double* ref;
  const double* inv_ref;
  ConstD* kf;
  int ysplit;
  static __device__ CodecF16Dev of(const Geometry& g) { return {g.ref, g.inv_ref, (ConstD*)(g.kf), g.ysplit}; }
  // the factors of both layers are scalar; the row picks one per lane
  __device__ double factor(int y, int k_lo, int k_hi) const { return y >= ysplit ? kf[k_hi] : kf[k_lo]; }
  __device__ double dec(S v, int l, int y) const {
    const int s = shell_of(l);
    const double c = factor(y, KF_LO + s, KF_HI + s) * ref[y];
    // c (1 + d) rounded once: 1 + d is exact, so the fused multiply-add
    // c d + c is the same correctly rounded value
    return fma(c, static_cast<double>(static_cast<float>(v)), c);
  }
  __device__ S enc(double f, int l, int y) const {
    const int s = shell_of(l);
    const double c = factor(y, KF_LO + s, KF_HI + s) * ref[y];
    const double q = (f - c) * (factor(y, KF_INV_LO + s, KF_INV_HI + s) * inv_ref[y]);
    return static_cast<_Float16>(static_cast<float>(q));
  }
};
// Rows of one temperature layer: k points at that layer's K_s, kinv at its
// 1 / K_s (wavefront-uniform).  Same arithmetic as CodecF16Dev.
struct CodecF16DevLayer {
  using S = _Float16;
  const double* ref;
  const double* inv_ref;
  ConstD* k;
  ConstD* kinv;
  __device__ double dec(S v, int l, int y) const {
    const double c = k[shell_of(l)] * ref[y];
    return fma(c, static_cast<double>(static_cast<float>(v)), c);
  }
  __device__ S enc(double f, int l, int y) const {
    const double c = k[shell_of(l)] * ref[y];
    const double q = (f - c) * (kinv[shell_of(l)] * inv_ref[y]);
    return static_cast<_Float16>(static_cast<float>(q));
  }
};

// Rows of one temperature layer, for the binary16 interior step at row y:
// decodes a population pulled from row y' of the same layer in units of
// the destination's reference, g = f_l / (K_s rho_ref(y)) =
// (rho_ref(y') / rho_ref(y)) (1 + d) (both rows have the layer's K_s, which
// cancels).  iy = 1 / rho_ref(y).
struct CodecF16DevRatio {
  using S = _Float16;
  const double* ref;
  double iy;
  __device__ double dec(S v, int, int ys) const {
    const double r = ref[ys] * iy;
    return fma(r, static_cast<double>(static_cast<float>(v)), r);
  }
};

// acc + k * v for a small integer k known after unrolling.
__device__ __forceinline__ double add_scaled(double acc, int k, double v) {
  if (k == 0) return acc;
  if (k == 1) return acc + v;
  if (k == -1) return acc - v;
  return fma(static_cast<double>(k), v, acc);
}
// k * v for a small integer k known after unrolling.
__device__ __forceinline__ double scaled(int k, double v) {
  if (k == 1) return v;
  if (k == -1) return -v;
  return static_cast<double>(k) * v;
}

// ---------------------------------------------------------------------------
// Site-local arithmetic
// ---------------------------------------------------------------------------

// Moment sums of one site: rho = sum f, jx = sum e_x f, jy = sum e_y f,
// eps = sum |e|^2 f (integer hops; velocities are r e).  Populations are
// summed pairwise (l, opp(l)) and shell by shell.
struct MomentSums {
  double rho, jx, jy, eps;
};

// moment_sums_of takes populations given as f_l = kf(s) g_l: it sums g
// shell by shell and applies each shell's factor once (UnitFactor: f = g,
// the same operations as summing f directly).
struct UnitFactor {
  static constexpr bool kUnit = true;
  __device__ double operator()(int) const { return 1.0; }
};
struct ShellFactor {
  static constexpr bool kUnit = false;
  const __attribute__((address_space(4))) double* k;
  __device__ double operator()(int s) const { return k[s]; }
};
template <class G, class K>
__device__ __forceinline__ MomentSums moment_sums_of(const G& g, const K& kf) {
  double shell[NSHELL];
  double jx = 0.0, jy = 0.0;
  shell[0] = K::kUnit ? g[0] : kf(0) * g[0];
#pragma unroll
  for (int s = 1; s < NSHELL; ++s) {
    const int lo = SHELL_START[s], hi = SHELL_START[s + 1], mid = (lo + hi) / 2;
    double acc = 0.0, jxs = 0.0, jys = 0.0;
#pragma unroll
    for (int l = lo; l < mid; ++l) {
      const int m = lo + hi - 1 - l;  // opposite population: e_m = -e_l
      const double sum = g[m] + g[l];
      const double dif = g[m] - g[l];
      acc = (l == lo) ? sum : acc + sum;
      if constexpr (K::kUnit) {
        jx = add_scaled(jx, EX[m], dif);
        jy = add_scaled(jy, EY[m], dif);
      } else {
        jxs = add_scaled(jxs, EX[m], dif);
        jys = add_scaled(jys, EY[m], dif);
      }
    }
    if constexpr (K::kUnit) {
      shell[s] = acc;
    } else {
      const double k = kf(s);
      shell[s] = k * acc;
      jx = fma(k, jxs, jx);
      jy = fma(k, jys, jy);
    }
  }
  double rho = shell[0];
  double eps = shell[1];
#pragma unroll
  for (int s = 1; s < NSHELL; ++s) rho = rho + shell[s];
#pragma unroll
  for (int s = 2; s < NSHELL; ++s) eps = fma(static_cast<double>(SHELL_N2[s]), shell[s], eps);
  return {rho, jx, jy, eps};
}
__device__ __forceinline__ MomentSums moment_sums(const double (&f)[NPOP]) {
  return moment_sums_of(f, UnitFactor{});
}

// BGK collision of one site (Eqs. 4-6): moments, shifted fields
// u + tau g and T - tau^2 |g|^2 / 2, the 4th-order Hermite equilibrium, and
// f <- (1 - omega) f + omega f^eq.  The equilibrium of population l is
// rho w_l P(s), s = u_shift . c_l, with per-shell coefficients
//   P(s) = p0 + p1 s + p2 s^2 + s^3/6 + s^4/24,
//   p0 = 1 - U/2 + U^2/8 + th (C-2)/2 + th U (4-C)/4 + th^2 (C^2-8C+8)/8,
//   p1 = 1 - U/2 + th (C-4)/2,   p2 = 1/2 - U/4 + th (C-6)/4,
// U = |u_shift|^2, th = T_shift - 1, C = |c_l|^2.  The even and odd parts
// of P serve both populations of a pair (s changes sign).
// collide_by hands omega f^eq of each population to the caller: rest(eq)
// for population 0 and pair(m, eq_m, l, eq_l) for the two populations of
// a pair.  With SHIFT, c(s) is subtracted from each shell's constant term
// e0, so the caller receives omega f^eq_l - c(s) without a subtraction per
// population.
// w(s): the weight of shell s (StdWeight: W_s); the binary16 interior step
// passes W_s / K_s, which puts f^eq in units of the reference.
struct StdWeight {
  __device__ double operator()(int s) const { return W_SHELL[s]; }
};
template <bool SHIFT, class Rest, class Pair, class Shift, class Weight = StdWeight>
__device__ __forceinline__ void collide_by(const MomentSums& m, const CollideParams& p, Rest&& rest, Pair&& pair,
                                           const Shift& c, const Weight& w = StdWeight{}) {
  const double inv_rho = 1.0 / m.rho;
  const double ux = R * m.jx * inv_rho;
  const double uy = R * m.jy * inv_rho;
  const double temp = 0.5 * (R2 * m.eps * inv_rho - (ux * ux + uy * uy));
  const double ubx = ux + p.tgx;
  const double uby = uy + p.tgy;
  const double th = (temp - p.dtemp) - 1.0;
  const double U = ubx * ubx + uby * uby;
  const double vx = R * ubx;
  const double vy = R * uby;
  const double th2 = th * th;
  // p0 = a0 + C (b0 + C d0), p1 = a1 + C b1, p2 = a2 + C b2
  const double a0 = (((1.0 - 0.5 * U) + 0.125 * U * U) - th) + (th * U + th2);
  const double b0 = (0.5 * th - 0.25 * th * U) - th2;
  const double d0 = 0.125 * th2;
  const double a1 = (1.0 - 0.5 * U) - 2.0 * th;
  const double b1 = 0.5 * th;
  const double a2 = (0.5 - 0.25 * U) - 1.5 * th;
  const double b2 = 0.25 * th;
  const double rw = m.rho * p.omega;

  if constexpr (SHIFT) rest((rw * w(0)) * a0 - c(0));
  else rest((rw * w(0)) * a0);
#pragma unroll
  for (int s = 1; s < NSHELL; ++s) {
    const double C = R2 * static_cast<double>(SHELL_N2[s]);
    const double cs = rw * w(s);
    double e0 = cs * fma(C, fma(C, d0, b0), a0);
    if constexpr (SHIFT) e0 = e0 - c(s);
    const double e2 = cs * fma(C, b2, a2);
    const double e4 = cs * (1.0 / 24.0);
    const double o1 = cs * fma(C, b1, a1);
    const double o3 = cs * (1.0 / 6.0);
    const int lo = SHELL_START[s], hi = SHELL_START[s + 1], mid = (lo + hi) / 2;
#pragma unroll
    for (int l = lo; l < mid; ++l) {
      const int mm = lo + hi - 1 - l;
      double sv;
      if (EX[mm] == 0)
        sv = scaled(EY[mm], vy);
      else if (EY[mm] == 0)
        sv = scaled(EX[mm], vx);
      else
        sv = add_scaled(scaled(EX[mm], vx), EY[mm], vy);
      const double ss = sv * sv;
      const double even = fma(ss, fma(ss, e4, e2), e0);
      const double odd = sv * fma(ss, o3, o1);
      pair(mm, even + odd, l, even - odd);
    }
  }
}

__device__ __forceinline__ void collide_site(double (&f)[NPOP], const CollideParams& p) {
  const MomentSums m = moment_sums(f);
  const double om1 = p.one_minus_omega;
  collide_by<false>(
      m, p, [&](double eq) { f[0] = fma(om1, f[0], eq); },
      [&](int a, double ea, int b, double eb) {
        f[a] = fma(om1, f[a], ea);
        f[b] = fma(om1, f[b], eb);
      },
      UnitFactor{});
}

// bc of one wall-row site: rho = f_0 + ... + f_36 (left fold), f_l = rho K_l.
// (WP: WallParams, possibly qualified with an address space.)
template <class WP>
__device__ __forceinline__ void thermalise(double (&f)[NPOP], bool bottom, const WP& w) {
  double rho = f[0];
#pragma unroll
  for (int l = 1; l < NPOP; ++l) rho = rho + f[l];
#pragma unroll
  for (int l = 0; l < NPOP; ++l) f[l] = rho * (bottom ? w.kb[l] : w.kt[l]);
}

}  // namespace
}  // namespace d2q37
