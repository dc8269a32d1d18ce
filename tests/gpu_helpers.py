"""Shared helpers of the GPU tests: lattice construction and the error metric.

The tolerance metric follows the FP64 bar of the hot path: the largest
population difference, scaled by the weight of its population and the
mean density, err = max |f_gpu - f_ref| / (w_l * mean rho).
"""
import sys

import numpy as np

import oracle
from paper_1703_00185_amd import inputs, lbm

FP64_TOL = 1e-12
LAYOUTS = [lbm.LBM_LAYOUT_COLUMN, lbm.LBM_LAYOUT_PLANAR]


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need an MI355X (gfx950); no GPU is visible")


def note(msg: str) -> None:
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def err_metric(got: np.ndarray, ref: np.ndarray) -> float:
    k = oracle.constants()
    shape = (37,) + (1,) * (ref.ndim - 1)
    rho_mean = float(ref.sum(axis=0).mean())
    return float(np.max(np.abs(got - ref) / (k.w.reshape(shape) * rho_mean)))


def lattice(ns, path=lbm.LBM_PATH_FUSED, block=0, **kw) -> lbm.Lattice:
    cfg = lbm.config_from(ns, path=path, block=block, **kw)
    note(f"lattice {ns.lx}x{ns.ly} path={path} block={block} layout={cfg.layout} "
         f"storage={cfg.storage}")
    return lbm.Lattice(cfg)


def noisy_state(seed: int, lx: int, ly: int, scale: float = 0.02) -> np.ndarray:
    """A seeded state near the Rayleigh-Taylor equilibrium (oracle-made)."""
    ns = inputs.rt_config(lx, ly)
    f = oracle.init_rt(lx, ly, ns, inputs.rt_perturbation(seed, ly))
    return f * (1.0 + inputs.noise(seed + 1000, f.shape, scale))
