"""Seeded synthetic inputs for the Rayleigh-Taylor workloads.

This module holds no arithmetic of the method: it only draws the seeded
random numbers (perturbation amplitudes and phases, noise) and bundles the
run parameters, so that the HIP library and the CPU reference receive the
same inputs.  The random numbers are passed to both sides explicitly.
"""
from __future__ import annotations

import math
from types import SimpleNamespace

import numpy as np

# Parameters of the Rayleigh-Taylor workloads: relaxation time, gravity
# (lattice units, along -y), wall temperatures, interface width (sites) and
# number of Fourier modes of the interface perturbation.
TAU = 0.8
GRAVITY = 1e-4
T_BOTTOM = 1.05
T_TOP = 0.95
WIDTH = 2.0
N_MODES = 8


def rt_config(lx: int, ly: int, *, tau: float = TAU, gravity: float = GRAVITY,
              t_bottom: float = T_BOTTOM, t_top: float = T_TOP) -> SimpleNamespace:
    """Lattice size, relaxation time, gravity vector and wall temperatures."""
    return SimpleNamespace(lx=int(lx), ly=int(ly), tau=float(tau), gx=0.0,
                           gy=-float(gravity), t_bottom=float(t_bottom),
                           t_top=float(t_top))


def rt_perturbation(seed: int, ly: int, *, n_modes: int = N_MODES,
                    width: float = WIDTH, max_amp: float = 1.0) -> SimpleNamespace:
    """Interface shape: mode amplitudes a_k ~ U[0, max_amp] sites and phases
    phi_k ~ U[0, 2 pi), drawn from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    amps = rng.uniform(0.0, max_amp, n_modes)
    phases = rng.uniform(0.0, 2.0 * math.pi, n_modes)
    return SimpleNamespace(width=float(width), y_center=0.5 * (ly - 1),
                           amps=amps.astype(np.float64), phases=phases.astype(np.float64))


def flat_interface(ly: int, *, width: float = WIDTH) -> SimpleNamespace:
    """An unperturbed interface (every column identical)."""
    return SimpleNamespace(width=float(width), y_center=0.5 * (ly - 1),
                           amps=np.zeros(0), phases=np.zeros(0))


def noise(seed: int, shape, scale: float) -> np.ndarray:
    """scale * standard normal noise of the given shape."""
    return scale * np.random.default_rng(seed).standard_normal(shape)
