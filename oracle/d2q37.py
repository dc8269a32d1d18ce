"""Plain FP64 CPU oracle of the D2Q37 thermal lattice Boltzmann update.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
executes this module; only the tests, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code, tables or constants with the HIP
library: every constant below is derived here from its definition.

It follows Calore et al., "Massively parallel Lattice Boltzmann codes on
large GPU clusters" (arXiv:1703.00185):

* Sec. 2, Eqs. (4)-(5) and the sentence after them: BGK relaxation towards
  a Maxwellian evaluated at the shifted velocity u + tau*g and the shifted
  temperature T - tau^2 g^2 / D.
* Sec. 2, Eq. (6): the discrete master equation with time step 1,
  f_l(x + c_l, t + 1) = f_l(x, t) - (f_l(x, t) - f_l^eq) / tau.
* Sec. 2, the moment definitions under Eq. (6): rho = sum f,
  rho u = sum c f, D rho T = sum |c - u|^2 f.
* Sec. 2, Eq. (10) and the list of kernels after it: each step is a pull
  gather (propagate), then the top/bottom thermal walls on rows 0..2 and
  Ly-3..Ly-1 (bc), then the site-local collision (collide); x is periodic.

The paper does not print the velocity set, the weights, the discrete
equilibrium, the wall algorithm, the units or the initial state.  Each
function names the reading it takes; the readings are:

R1  velocity set: the 37 integer hops of the shells (0,0) (1,0) (1,1) (2,0)
    (2,1) (2,2) (3,0) (3,1) with all sign/axis images (reach 3 sites, and 26
    populations cross a vertical boundary, as Sec. 2 and Sec. 5 state).
R2  weights and the velocity scale r: the unique positive solution of the
    isotropy conditions (discrete moments of w equal the moments of a unit
    Gaussian through total order 8).
R3  equilibrium: the 4th-order Hermite projection of the Maxwellian of
    Eq. (5) at reference temperature 1.
R4  units: time step 1, a population hops e_l sites per step and carries the
    velocity c_l = r e_l; so one site is r length units.
R8  walls: in propagate, a population whose source lies beyond a wall is
    replaced by the opposite population of the same site (on-site bounce
    back); bc then sets the 37 populations of each wall-row site to
    rho_site * K_l(T_wall), the zero-velocity equilibrium at the wall
    temperature, with rho_site summed as a left fold in population order.
R9  gravity along -y; bottom wall hot.
R11 population order: by shell as in R1, then (e_x, e_y) ascending.
R12 Rayleigh-Taylor initial state in hydrostatic balance (closed form).
R15 binary16 deviation storage (the reduced-precision form beyond the
    paper's binary64 code): the deviation is taken from the zero-velocity
    equilibrium of a reference state with a density per row and two
    temperature layers (for the Rayleigh-Taylor workload: the density of
    the state with a flat interface, the wall temperatures below and above
    the interface), so that it holds little beyond each site's departure
    from the rest state of its row.
"""
from __future__ import annotations

import functools
import math
from types import SimpleNamespace

import numpy as np

D = 2  # space dimension (Sec. 2)
NPOP = 37
# Shell representatives of reading R1, in canonical order (R11).
SHELL_REPS = ((0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1))
# Isotropy conditions of reading R2: sum_l w_l Cx^(2a) Cy^(2b) equals the
# Gaussian moment (2a-1)!! (2b-1)!!, for these (a, b).  Together with the
# symmetry of the set they fix every moment through total order 8.
ISOTROPY_CONDITIONS = ((0, 0), (1, 0), (2, 0), (1, 1), (3, 0), (2, 1),
                       (4, 0), (3, 1), (2, 2))
WALL_ROWS = 3  # bc acts on y = 0, 1, 2 and Ly-3, Ly-2, Ly-1 (Sec. 4)


# ----------------------------------------------------------------------------
# Velocity set and weights (readings R1, R2, R11)
# ----------------------------------------------------------------------------

def _images(a: int, b: int) -> list[tuple[int, int]]:
    """All sign and axis images of the hop (a, b), sorted (R11)."""
    out = set()
    for p, q in ((a, b), (b, a)):
        for sx in (1, -1):
            for sy in (1, -1):
                out.add((sx * p, sy * q))
    return sorted(out)


def velocity_set():
    """Integer hops e_l (37 x 2), shell index per population, opposite index."""
    vecs, shell = [], []
    for s, (a, b) in enumerate(SHELL_REPS):
        for v in _images(a, b):
            vecs.append(v)
            shell.append(s)
    opp = [vecs.index((-x, -y)) for (x, y) in vecs]
    return (np.array(vecs, dtype=np.int64), np.array(shell, dtype=np.int64),
            np.array(opp, dtype=np.int64))


def _odd_double_factorial(n: int) -> int:
    """(n)!! for odd n >= -1, with (-1)!! = 1."""
    out = 1
    while n > 1:
        out *= n
        n -= 2
    return out


@functools.lru_cache(maxsize=None)
def solve_isotropy(dps: int = 60):
    """Solve the isotropy system of reading R2 in extended precision.

    For a trial q = r^2 the conditions are 9 linear equations in the 8 shell
    weights W_s:  sum_s W_s M_s(a,b) q^(a+b) = (2a-1)!!(2b-1)!!, with
    M_s(a,b) = sum over the hops of shell s of e_x^(2a) e_y^(2b).  They are
    consistent only where the determinant of the augmented 9x9 matrix
    vanishes; every such q with all W_s > 0 is a solution.  Returns
    (r, W) as strings of `dps` significant digits (converted to binary64
    by the caller, which rounds correctly).
    """
    import mpmath as mp

    shells = [_images(a, b) for (a, b) in SHELL_REPS]
    moments = [[sum(ex ** (2 * a) * ey ** (2 * b) for ex, ey in sh) for sh in shells]
               for (a, b) in ISOTROPY_CONDITIONS]
    gauss = [_odd_double_factorial(2 * a - 1) * _odd_double_factorial(2 * b - 1)
             for (a, b) in ISOTROPY_CONDITIONS]
    nk, ns = len(ISOTROPY_CONDITIONS), len(shells)

    with mp.workdps(dps):
        def matrix(q):
            A = mp.matrix(nk, ns)
            for k, (a, b) in enumerate(ISOTROPY_CONDITIONS):
                for s in range(ns):
                    A[k, s] = moments[k][s] * q ** (a + b)
            return A

        def consistency(q):
            A = matrix(q)
            aug = mp.matrix(nk, ns + 1)
            for k in range(nk):
                for s in range(ns):
                    aug[k, s] = A[k, s]
                aug[k, ns] = gauss[k]
            return mp.det(aug)

        grid = [mp.mpf(j) / 50 for j in range(10, 250)]  # q in [0.2, 5)
        solutions = []
        prev_q, prev_v = grid[0], consistency(grid[0])
        for q in grid[1:]:
            v = consistency(q)
            if prev_v == 0 or (prev_v < 0) != (v < 0):
                lo, hi, f_lo = prev_q, q, prev_v
                for _ in range(4 * dps):  # plain bisection, ~1 bit per pass
                    mid = (lo + hi) / 2
                    f_mid = consistency(mid)
                    if (f_mid < 0) == (f_lo < 0):
                        lo, f_lo = mid, f_mid
                    else:
                        hi = mid
                root = (lo + hi) / 2
                W, res = mp.qr_solve(matrix(root), mp.matrix(gauss))
                if res < mp.mpf(10) ** (-dps // 2) and all(W[s] > 0 for s in range(ns)):
                    solutions.append((root, [W[s] for s in range(ns)]))
            prev_q, prev_v = q, v
        if len(solutions) != 1:
            raise RuntimeError(f"isotropy system: expected one positive solution, got {len(solutions)}")
        q, W = solutions[0]
        return mp.nstr(mp.sqrt(q), dps - 5), tuple(mp.nstr(x, dps - 5) for x in W)


@functools.lru_cache(maxsize=None)
def constants() -> SimpleNamespace:
    """Model constants in binary64: e, shell, opp, r, w, c = r e (R1-R4)."""
    E, shell, opp = velocity_set()
    r_str, w_str = solve_isotropy()
    r = float(r_str)
    w_shell = np.array([float(x) for x in w_str])
    w = w_shell[shell]
    cx = r * E[:, 0].astype(np.float64)
    cy = r * E[:, 1].astype(np.float64)
    return SimpleNamespace(E=E, shell=shell, opp=opp, r=r, w_shell=w_shell, w=w,
                           cx=cx, cy=cy, r_str=r_str, w_shell_str=w_str)


def _col(v: np.ndarray, ndim: int) -> np.ndarray:
    """Reshape a per-population vector to broadcast over `ndim` site axes."""
    return v.reshape((NPOP,) + (1,) * ndim)


# ----------------------------------------------------------------------------
# Moments, equilibrium, collision (Sec. 2; readings R3, R4)
# ----------------------------------------------------------------------------

def moments(f: np.ndarray):
    """rho, u_x, u_y, T of populations f[37, ...] (Sec. 2, under Eq. 6).

    rho = sum_l f_l;  rho u = sum_l c_l f_l;  D rho T = sum_l |c_l - u|^2 f_l.
    """
    k = constants()
    nd = f.ndim - 1
    cx, cy = _col(k.cx, nd), _col(k.cy, nd)
    rho = f.sum(axis=0)
    ux = (cx * f).sum(axis=0) / rho
    uy = (cy * f).sum(axis=0) / rho
    T = (((cx - ux) ** 2 + (cy - uy) ** 2) * f).sum(axis=0) / (D * rho)
    return rho, ux, uy, T


def equilibrium(rho, ux, uy, T) -> np.ndarray:
    """Discrete equilibrium f_l^eq(rho, u, T), shape [37, ...] (reading R3).

    The Maxwellian of Eq. (5) expanded in tensor Hermite polynomials of the
    scaled velocity c_l around the reference temperature 1 and truncated
    after 4th order.  With s = u.c_l, U = |u|^2, C = |c_l|^2, th = T - 1 the
    fully contracted terms a^(n) : H^(n)(c_l) / rho are written out below.
    """
    k = constants()
    rho, ux, uy, T = (np.asarray(a, dtype=np.float64) for a in (rho, ux, uy, T))
    nd = np.broadcast(rho, ux, uy, T).ndim
    cx, cy, w = _col(k.cx, nd), _col(k.cy, nd), _col(k.w, nd)
    s = cx * ux + cy * uy
    U = ux * ux + uy * uy
    C = cx * cx + cy * cy
    th = T - 1.0
    h0 = 1.0
    h1 = s
    h2 = s * s - U + th * (C - D)
    h3 = s * s * s - 3.0 * s * U + 3.0 * th * s * (C - (D + 2))
    h4 = (s ** 4 - 6.0 * U * s * s + 3.0 * U * U
          + 6.0 * th * (s * s * (C - (D + 4)) + U * ((D + 2) - C))
          + 3.0 * th * th * (C * C - 2.0 * (D + 2) * C + D * (D + 2)))
    poly = h0 + h1 + h2 / 2.0 + h3 / 6.0 + h4 / 24.0
    return rho * w * poly


def collide(f: np.ndarray, tau: float, gx: float, gy: float) -> np.ndarray:
    """One BGK collision at every site of f[37, ...] (Eqs. 4-6, Sec. 2).

    The equilibrium is taken at the shifted fields u + tau g and
    T - tau^2 |g|^2 / D of the local moments, and each population relaxes
    towards it: f <- f - (f - f^eq) / tau.
    """
    rho, ux, uy, T = moments(f)
    ubx = ux + tau * gx
    uby = uy + tau * gy
    Tb = T - tau * tau * (gx * gx + gy * gy) / D
    feq = equilibrium(rho, ubx, uby, Tb)
    return f - (f - feq) / tau


# ----------------------------------------------------------------------------
# Propagate and walls (Sec. 2 kernel list, Sec. 4; reading R8)
# ----------------------------------------------------------------------------

def propagate(f: np.ndarray) -> np.ndarray:
    """Pull propagate over the physical lattice f[37, Lx, Ly] (Eq. 10).

    out_l(x, y) = f_l((x - e_lx) mod Lx, y - e_ly) when 0 <= y - e_ly < Ly
    (x periodic, Sec. 2); otherwise the source lies beyond a wall and
    out_l(x, y) = f_opp(l)(x, y) (reading R8).
    """
    k = constants()
    _, lx, ly = f.shape
    out = np.empty_like(f)
    y = np.arange(ly)
    for l in range(NPOP):
        ex, ey = int(k.E[l, 0]), int(k.E[l, 1])
        ysrc = y - ey
        inside = (ysrc >= 0) & (ysrc < ly)
        shifted = np.roll(f[l], ex, axis=0)  # shifted[x] = f_l[(x - ex) mod Lx]
        out[l][:, inside] = shifted[:, ysrc[inside]]
        out[l][:, ~inside] = f[k.opp[l]][:, ~inside]
    return out


def wall_factors(t_wall: float) -> list[float]:
    """K_l(T) = w_l [1 + th (C_l - 2)/2 + th^2 (C_l^2 - 8 C_l + 8)/8], th = T - 1.

    The zero-velocity equilibrium of reading R3 per unit density (D = 2),
    C_l = r^2 |e_l|^2.  Evaluated in binary64 in exactly this expression
    order, one Python float operation at a time, so that it is reproducible.
    """
    k = constants()
    r2 = k.r * k.r
    th = t_wall - 1.0
    out = []
    for l in range(NPOP):
        n2 = float(k.E[l, 0] * k.E[l, 0] + k.E[l, 1] * k.E[l, 1])
        C = r2 * n2
        out.append(float(k.w[l]) * (1.0 + th * (C - 2.0) / 2.0
                                    + th * th * (C * C - 8.0 * C + 8.0) / 8.0))
    return out


def thermalise(vals: np.ndarray, t_wall: float) -> np.ndarray:
    """Wall thermalisation of sites vals[37, ...] (Sec. 4 bc; reading R8).

    rho_site = f_0 + f_1 + ... + f_36 as a left fold in population order;
    every population becomes rho_site * K_l(T_wall).
    """
    K = wall_factors(t_wall)
    rho = vals[0].copy()
    for l in range(1, NPOP):
        rho = rho + vals[l]
    return np.stack([rho * K[l] for l in range(NPOP)])


def bc(f: np.ndarray, t_bottom: float, t_top: float) -> np.ndarray:
    """Thermal walls on rows 0..2 (t_bottom) and Ly-3..Ly-1 (t_top) (Sec. 4)."""
    _, lx, ly = f.shape
    out = f.copy()
    out[:, :, :WALL_ROWS] = thermalise(f[:, :, :WALL_ROWS], t_bottom)
    out[:, :, ly - WALL_ROWS:] = thermalise(f[:, :, ly - WALL_ROWS:], t_top)
    return out


# ----------------------------------------------------------------------------
# One time step, sampled sites, diagnostics
# ----------------------------------------------------------------------------

def step(f: np.ndarray, cfg) -> np.ndarray:
    """One time step: propagate, bc, collide (the kernel order of Sec. 2)."""
    g = propagate(f)
    g = bc(g, cfg.t_bottom, cfg.t_top)
    return collide(g, cfg.tau, cfg.gx, cfg.gy)


def fp16dev_reference(rho_ref, t_lo: float, t_hi: float, y_split: int):
    """Reference of the binary16 deviation storage (reading R15), [37, Ly]
    twice: c[l, y] = K_l(T(y)) * rho_ref(y) and the encoding factor
    inv[l, y] = (1 / K_l(T(y))) * (1 / rho_ref(y)), with T(y) = t_lo for
    y < y_split and t_hi for y >= y_split.  c is the zero-velocity
    equilibrium (reading R3 at u = 0, the factors of wall_factors) of a
    reference state with a density per row and two temperature layers.
    With t_lo = t_hi = 1 it reduces to w_l rho_ref(y)."""
    rho_ref = np.asarray(rho_ref, dtype=np.float64)
    ly = rho_ref.size
    K = {t: np.array(wall_factors(float(t))) for t in (t_lo, t_hi)}
    c = np.empty((NPOP, ly))
    inv = np.empty((NPOP, ly))
    for y in range(ly):
        k = K[t_lo] if y < y_split else K[t_hi]
        c[:, y] = k * rho_ref[y]
        inv[:, y] = (1.0 / k) * (1.0 / rho_ref[y])
    return c, inv


def encode_fp16dev(f: np.ndarray, ref) -> np.ndarray:
    """Binary16 scaled deviations d of f[37, Lx, Ly] from the reference
    ref = (c, inv) of fp16dev_reference: q = (f - c) * inv in binary64,
    rounded to binary32 and then to binary16 (nearest, ties to even, at
    each rounding)."""
    c, inv = ref
    q = (f - c[:, None, :]) * inv[:, None, :]
    return q.astype(np.float32).astype(np.float16)


def decode_fp16dev(d: np.ndarray, ref) -> np.ndarray:
    """Populations c (1 + d) from binary16 deviations (1 + d is exact)."""
    c, _ = ref
    return c[:, None, :] * (1.0 + d.astype(np.float64))


def stored(f: np.ndarray, storage: str, ref=None) -> np.ndarray:
    """Values as held in memory and read back: binary64 unchanged; binary32
    rounded to nearest (ties to even); binary16 deviations from the
    reference `ref` of fp16dev_reference (encode_fp16dev, then
    decode_fp16dev)."""
    if storage == "fp64":
        return f
    if storage == "fp32":
        return f.astype(np.float32).astype(np.float64)
    if storage == "fp16dev":
        return decode_fp16dev(encode_fp16dev(f, ref), ref)
    raise ValueError(storage)


def step_stored(f: np.ndarray, cfg, storage: str, fused: bool, ref=None) -> np.ndarray:
    """One step when populations are kept in `storage` between kernels.

    Arithmetic is binary64; each kernel that writes populations stores
    them in the storage type.  The separate sequence stores after
    propagate, after bc and after collide; the fused kernel stores once,
    after collide.  (Propagate only moves values, so its store changes
    nothing unless the encoding depends on the row, as the deviation
    storage's reference does.)
    """
    g = propagate(f)
    if not fused:
        g = stored(g, storage, ref)
    g = bc(g, cfg.t_bottom, cfg.t_top)
    if not fused:
        g = stored(g, storage, ref)
    return stored(collide(g, cfg.tau, cfg.gx, cfg.gy), storage, ref)


def run(f: np.ndarray, cfg, n: int) -> np.ndarray:
    for _ in range(n):
        f = step(f, cfg)
    return f


def gather_sites(f: np.ndarray, xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """Post-propagate populations [37, n] at the sites (xs, ys) only.

    Same rule as propagate(), evaluated per requested site, so that single
    sites of a large lattice can be checked without stepping all of it.
    """
    k = constants()
    _, lx, ly = f.shape
    xs = np.asarray(xs, dtype=np.int64)
    ys = np.asarray(ys, dtype=np.int64)
    out = np.empty((NPOP, xs.size), dtype=np.float64)
    for l in range(NPOP):
        ex, ey = int(k.E[l, 0]), int(k.E[l, 1])
        ysrc = ys - ey
        inside = (ysrc >= 0) & (ysrc < ly)
        pulled = f[l, (xs - ex) % lx, np.clip(ysrc, 0, ly - 1)]
        bounced = f[k.opp[l], xs, ys]
        out[l] = np.where(inside, pulled, bounced)
    return out


def step_sites(f: np.ndarray, cfg, xs, ys) -> np.ndarray:
    """Populations [37, n] after one step at the sites (xs, ys) of f."""
    _, lx, ly = f.shape
    ys = np.asarray(ys, dtype=np.int64)
    g = gather_sites(f, xs, ys)
    bottom = ys < WALL_ROWS
    top = ys >= ly - WALL_ROWS
    if bottom.any():
        g[:, bottom] = thermalise(g[:, bottom], cfg.t_bottom)
    if top.any():
        g[:, top] = thermalise(g[:, top], cfg.t_top)
    return collide(g, cfg.tau, cfg.gx, cfg.gy)


def totals(f: np.ndarray):
    """Global mass, momentum (x, y) and energy (1/2) sum |c|^2 f of f[37,...]."""
    k = constants()
    nd = f.ndim - 1
    cx, cy = _col(k.cx, nd), _col(k.cy, nd)
    return (float(f.sum()), float((cx * f).sum()), float((cy * f).sum()),
            float(0.5 * ((cx * cx + cy * cy) * f).sum()))


# ----------------------------------------------------------------------------
# Rayleigh-Taylor initial state (readings R9, R12)
# ----------------------------------------------------------------------------

def _log_cosh(z: np.ndarray) -> np.ndarray:
    """ln cosh z = |z| + log1p(exp(-2|z|)) - ln 2, without overflow."""
    a = np.abs(z)
    return a + np.log1p(np.exp(-2.0 * a)) - math.log(2.0)


def interface_height(lx: int, amps, phases) -> np.ndarray:
    """h(x) = sum_k a_k cos(2 pi k x / Lx + phi_k), k = 1..n (in sites)."""
    x = np.arange(lx, dtype=np.float64)
    h = np.zeros(lx)
    for k, (a, p) in enumerate(zip(amps, phases), start=1):
        h = h + a * np.cos(2.0 * math.pi * k * x / lx + p)
    return h


def rt_fields(lx: int, ly: int, cfg, rt):
    """Temperature and density of the Rayleigh-Taylor initial state [Lx, Ly].

    T(x, y) = T_m - a tanh(z), z = (y - y_c - h(x)) / width, with
    T_m = (T_bottom + T_top)/2 and a = (T_bottom - T_top)/2: a hot layer
    under a cold one.  Pressure p = rho T obeys hydrostatic balance in site
    units, d ln p / dy = r g_y / T (one site is r length units, R4); with
    T_m > |a| the integral is closed-form:
      int dy / T = width (T_m z' + a ln cosh z') / (T_m^2 - a^2),
      z' = z - atanh(a / T_m),
    taken from the interface (z = 0, where p = 1) to y.
    """
    k = constants()
    tm = 0.5 * (cfg.t_bottom + cfg.t_top)
    a = 0.5 * (cfg.t_bottom - cfg.t_top)
    h = interface_height(lx, rt.amps, rt.phases)
    y = np.arange(ly, dtype=np.float64)
    z = (y[None, :] - rt.y_center - h[:, None]) / rt.width
    T = tm - a * np.tanh(z)
    z0 = math.atanh(a / tm)
    zp = z - z0
    integral = rt.width * (tm * z + a * (_log_cosh(zp) - _log_cosh(-z0))) / (tm * tm - a * a)
    p = np.exp(k.r * cfg.gy * integral)
    rho = p / T
    return T, rho


def init_rt(lx: int, ly: int, cfg, rt) -> np.ndarray:
    """Populations [37, Lx, Ly] at rest, at equilibrium with the RT fields."""
    T, rho = rt_fields(lx, ly, cfg, rt)
    zero = np.zeros_like(T)
    return equilibrium(rho, zero, zero, T)
