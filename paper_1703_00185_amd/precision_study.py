"""Error of FP32 and FP16-deviation population storage against FP64.

Steps the 2048 x 8192 Rayleigh-Taylor lattice (seeded synthetic initial
state) with FP64, FP32 and FP16-deviation storage side by side on one GPU
and compares the density, temperature and velocity fields at the given
steps.  The FP64 path stands in for the FP64 CPU reference, which cannot
run thousands of steps at this size; the FP64 path itself is checked
against that reference per step at this size and for 100 steps at
64 x 128 by the test suite.

Usage: python -m paper_1703_00185_amd.precision_study [--steps 100 1000 5000]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def field_errors(ref, got) -> dict:
    rho0, ux0, uy0, T0 = ref
    rho, ux, uy, T = got
    return {
        "rho_max_rel": float(np.max(np.abs(rho - rho0) / rho0)),
        "rho_rms_rel": float(np.sqrt(np.mean(((rho - rho0) / rho0) ** 2))),
        "T_max_abs": float(np.max(np.abs(T - T0))),
        "T_rms_abs": float(np.sqrt(np.mean((T - T0) ** 2))),
        "u_max_abs": float(np.max(np.hypot(ux - ux0, uy - uy0))),
        "u_rms_abs": float(np.sqrt(np.mean((ux - ux0) ** 2 + (uy - uy0) ** 2))),
        "u_scale": float(np.max(np.hypot(ux0, uy0))),
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--lx", type=int, default=2048)
    ap.add_argument("--ly", type=int, default=8192)
    ap.add_argument("--steps", type=int, nargs="+", default=[100, 1000, 5000])
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    from paper_1703_00185_amd import inputs, lbm

    ns = inputs.rt_config(args.lx, args.ly)
    rt = inputs.rt_perturbation(args.seed, args.ly)
    kinds = (("fp64", lbm.LBM_FP64), ("fp32", lbm.LBM_FP32), ("fp16dev", lbm.LBM_FP16DEV))
    lats = {}
    for name, storage in kinds:
        lats[name] = lbm.Lattice(lbm.config_from(ns, storage=storage)).init_rt(rt)
    out = {"workload": f"rayleigh_taylor_{args.lx}x{args.ly}", "reference": "fp64 GPU path",
           "errors": {}}
    done = 0
    t0 = time.perf_counter()
    for target in sorted(args.steps):
        for lat in lats.values():
            lat.step(target - done)
        done = target
        ref = lats["fp64"].moments()
        for name in ("fp32", "fp16dev"):
            out["errors"].setdefault(name, {})[str(target)] = field_errors(ref, lats[name].moments())
        print(f"[precision] step {target}: "
              + ", ".join(f"{n} rho {out['errors'][n][str(target)]['rho_max_rel']:.2e}"
                          for n in ("fp32", "fp16dev")), file=sys.stderr, flush=True)
    out["wall_s"] = time.perf_counter() - t0
    for lat in lats.values():
        lat.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
