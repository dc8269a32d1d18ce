"""Pins of the oracle's propagate and bc (Sec. 2 kernel list, Sec. 4; R8).

* propagate, against a brute-force push-view loop on tiny lattices: the
  value f_l(x, y) lands on (x + e_lx mod Lx, y + e_ly), or, if that row is
  beyond a wall, on population opp(l) of the same site.  It is a bijection.
* bc: wall-row sites keep their density, lose all momentum and take the
  wall temperature; the other rows are untouched.
"""
import numpy as np
import pytest

import oracle

TINY = [(3, 6), (4, 7), (5, 9), (7, 12), (3, 13)]


def _push_brute_force(f):
    E, _, opp = oracle.velocity_set()
    _, lx, ly = f.shape
    out = np.full_like(f, np.nan)
    for l in range(37):
        for x in range(lx):
            for y in range(ly):
                xd, yd = (x + E[l, 0]) % lx, y + E[l, 1]
                if 0 <= yd < ly:
                    out[l, xd, yd] = f[l, x, y]
                else:
                    out[opp[l], x, y] = f[l, x, y]
    return out


@pytest.mark.parametrize("lx,ly", TINY)
def test_propagate_matches_push_view(lx, ly):
    f = np.arange(37 * lx * ly, dtype=np.float64).reshape(37, lx, ly)
    got = oracle.propagate(f)
    want = _push_brute_force(f)
    assert not np.isnan(want).any()  # every destination written exactly once
    assert np.array_equal(got, want)
    assert np.array_equal(np.sort(got.ravel()), np.sort(f.ravel()))


def test_single_population_moves_by_its_hop():
    E, _, _ = oracle.velocity_set()
    lx, ly = 11, 20
    for l in range(37):
        f = np.zeros((37, lx, ly))
        f[l, 5, 9] = 1.0
        g = oracle.propagate(f)
        xs, ys = np.nonzero(g[l])
        assert (xs.tolist(), ys.tolist()) == ([5 + E[l, 0]], [9 + E[l, 1]])


def test_gather_sites_matches_propagate():
    lx, ly = 9, 14
    rng = np.random.default_rng(1)
    f = rng.random((37, lx, ly))
    full = oracle.propagate(f)
    xs, ys = np.meshgrid(np.arange(lx), np.arange(ly), indexing="ij")
    got = oracle.gather_sites(f, xs.ravel(), ys.ravel())
    assert np.array_equal(got, full.reshape(37, -1))


def _state(seed, lx, ly):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.8, 1.2, (lx, ly))
    ux = rng.uniform(-0.05, 0.05, (lx, ly))
    uy = rng.uniform(-0.05, 0.05, (lx, ly))
    T = rng.uniform(0.95, 1.05, (lx, ly))
    f = oracle.equilibrium(rho, ux, uy, T)
    return f * (1 + 0.02 * rng.standard_normal(f.shape))


@pytest.mark.parametrize("tb,tt", [(1.05, 0.95), (1.0, 1.0), (0.9, 1.2)])
def test_bc_wall_moments(tb, tt):
    lx, ly = 8, 16
    f = _state(2, lx, ly)
    g = oracle.bc(f, tb, tt)
    rho0 = f.sum(0)
    rho, ux, uy, T = oracle.moments(g)
    for rows, tw in ((slice(0, 3), tb), (slice(ly - 3, ly), tt)):
        assert np.max(np.abs(rho[:, rows] - rho0[:, rows]) / rho0[:, rows]) < 4e-15
        assert np.max(np.abs(ux[:, rows])) < 1e-15
        assert np.max(np.abs(uy[:, rows])) < 1e-15
        assert np.max(np.abs(T[:, rows] - tw)) < 1e-14
    assert np.array_equal(g[:, :, 3:ly - 3], f[:, :, 3:ly - 3])


def test_wall_factors_are_rest_equilibrium():
    for tw in (0.9, 1.0, 1.05, 1.2):
        K = np.array(oracle.wall_factors(tw))
        feq = oracle.equilibrium(np.array(1.0), np.array(0.0), np.array(0.0), np.array(tw))
        assert np.max(np.abs(K - feq)) < 1e-16
        assert (K > 0).all()


def test_thermalise_is_left_fold_times_factor():
    rng = np.random.default_rng(4)
    v = rng.random((37, 5))
    out = oracle.thermalise(v, 1.05)
    K = oracle.wall_factors(1.05)
    for i in range(5):
        s = 0.0
        for l in range(37):
            s = s + float(v[l, i]) if l else float(v[0, i])
        for l in range(37):
            assert out[l, i] == s * K[l]
