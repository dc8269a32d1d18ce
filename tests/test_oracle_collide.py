"""Pins of the oracle's equilibrium and collision (Sec. 2, Eqs. 4-6; R3, R4).

* Equilibrium moments through 4th order equal those of the continuous
  Maxwellian of Eq. (5), integrated by Gauss-Hermite quadrature.
* Collision conserves mass, adds rho g to the momentum and rho u.g to the
  energy (1/2) sum |c|^2 f (the macroscopic balance laws of Sec. 2).
* g = 0: the equilibrium is a fixed point, and a disturbance carrying no
  mass, momentum or energy decays by exactly (1 - 1/tau) per collision.
"""
import math

import numpy as np
import pytest
from numpy.polynomial.hermite_e import hermegauss

import oracle


def _maxwell_moment(rho, u, T, p):
    """E[(u + sqrt(T) X)^p] * rho-free, by 20-node Gauss-Hermite quadrature."""
    x, w = hermegauss(20)
    return float((w * (u + math.sqrt(T) * x) ** p).sum() / math.sqrt(2 * math.pi))


def _random_fields(seed, n):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 1.5, n)
    ux = rng.uniform(-0.1, 0.1, n)
    uy = rng.uniform(-0.1, 0.1, n)
    T = rng.uniform(0.9, 1.1, n)
    return rho, ux, uy, T


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_equilibrium_moments_match_maxwellian(seed):
    k = oracle.constants()
    rho, ux, uy, T = _random_fields(seed, 16)
    feq = oracle.equilibrium(rho, ux, uy, T)
    for i in range(rho.size):
        for p in range(5):
            for q in range(5 - p):
                disc = float((feq[:, i] * k.cx ** p * k.cy ** q).sum())
                cont = rho[i] * _maxwell_moment(rho[i], ux[i], T[i], p) * \
                    _maxwell_moment(rho[i], uy[i], T[i], q)
                assert abs(disc - cont) < 1e-13 * max(1.0, abs(cont)), (i, p, q, disc, cont)


def test_equilibrium_fifth_order_is_not_exact():
    """The projection stops at 4th order: a 5th moment differs at u != 0."""
    k = oracle.constants()
    rho, ux, uy, T = 1.0, 0.1, 0.05, 1.05
    feq = oracle.equilibrium(np.array(rho), np.array(ux), np.array(uy), np.array(T))
    disc = float((feq * k.cx ** 5).sum())
    cont = rho * _maxwell_moment(rho, ux, T, 5)
    assert abs(disc - cont) > 1e-8


def test_moments_recover_equilibrium_fields():
    rho, ux, uy, T = _random_fields(5, 64)
    m = oracle.moments(oracle.equilibrium(rho, ux, uy, T))
    for got, want in zip(m, (rho, ux, uy, T)):
        assert np.max(np.abs(got - want)) < 1e-14


def _noisy_state(seed, n):
    rho, ux, uy, T = _random_fields(seed, n)
    f = oracle.equilibrium(rho, ux, uy, T)
    rng = np.random.default_rng(seed + 100)
    return f * (1.0 + 0.05 * rng.standard_normal(f.shape))


@pytest.mark.parametrize("tau,gx,gy", [(0.8, 0.0, -1e-4), (0.6, 3e-4, 2e-4), (1.7, -1e-3, 5e-4)])
def test_collide_balance_laws(tau, gx, gy):
    k = oracle.constants()
    f = _noisy_state(7, 256)
    rho, ux, uy, _ = oracle.moments(f)
    g = oracle.collide(f, tau, gx, gy)
    C2 = (k.cx ** 2 + k.cy ** 2)[:, None]
    dm = g.sum(0) - f.sum(0)
    djx = (k.cx[:, None] * (g - f)).sum(0)
    djy = (k.cy[:, None] * (g - f)).sum(0)
    de = 0.5 * (C2 * (g - f)).sum(0)
    assert np.max(np.abs(dm)) < 1e-13
    assert np.max(np.abs(djx - rho * gx)) < 1e-13
    assert np.max(np.abs(djy - rho * gy)) < 1e-13
    assert np.max(np.abs(de - rho * (ux * gx + uy * gy))) < 1e-13


def test_equilibrium_is_fixed_point_without_gravity():
    rho, ux, uy, T = _random_fields(11, 128)
    feq = oracle.equilibrium(rho, ux, uy, T)
    out = oracle.collide(feq, 0.8, 0.0, 0.0)
    assert np.max(np.abs(out - feq)) < 4e-15


@pytest.mark.parametrize("tau", [0.55, 0.8, 2.0])
def test_invariant_free_disturbance_decays_by_one_minus_omega(tau):
    """f = feq + d, d with zero mass/momentum/energy: collide -> feq + (1-1/tau) d."""
    k = oracle.constants()
    rho, ux, uy, T = _random_fields(3, 32)
    feq = oracle.equilibrium(rho, ux, uy, T)
    rng = np.random.default_rng(9)
    d = 1e-3 * rng.standard_normal(feq.shape) * k.w[:, None]
    basis = np.stack([k.w, k.w * k.cx, k.w * k.cy, k.w * (k.cx ** 2 + k.cy ** 2)])  # 4 x 37
    probes = np.stack([np.ones(37), k.cx, k.cy, k.cx ** 2 + k.cy ** 2])
    A = probes @ basis.T
    coef = np.linalg.solve(A, probes @ d)
    d = d - basis.T @ coef
    assert np.max(np.abs(probes @ d)) < 1e-17
    out = oracle.collide(feq + d, tau, 0.0, 0.0)
    assert np.max(np.abs(out - (feq + (1 - 1 / tau) * d))) < 1e-15
