"""Batched ensemble of Rayleigh-Taylor lattices on one MI355X.

256 independent lattices (seeded): Lx uniform in {64, 128, ..., 1024}, Ly =
2 Lx or 4 Lx, temperature contrast uniform in [0.02, 0.2] around 1, 8
perturbation modes, FP32 storage, 500 steps each.  All of them advance
together through the ensemble engine (one persistent launch per step,
replayed from a HIP graph), with the tiling picked by the engine's
autotuner.  Beside it, the same lattices stepped one at a time with the
single-lattice fused path.  Prints one JSON line.

Usage: python -m paper_1703_00185_amd.ensemble_bench [--lattices 256] [--steps 500]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def draw_ensemble(seed: int, n: int):
    """(lx, ly, contrast, perturbation seed) for n lattices."""
    rng = np.random.default_rng(seed)
    lx = 64 * rng.integers(1, 17, n)
    ly = lx * rng.choice([2, 4], n)
    contrast = rng.uniform(0.02, 0.2, n)
    return [(int(a), int(b), float(c), int(seed * 100003 + i)) for i, (a, b, c) in
            enumerate(zip(lx, ly, contrast))]


def run_ensemble(lbm, inputs, lattices: int = 256, steps: int = 500, seed: int = 0,
                 storage_name: str = "fp32", tune_reps: int = 2, sequential_steps: int = 50,
                 log=None) -> dict:
    """Build the ensemble on the current GPU, autotune the engine, time
    `steps` engine steps (the first, which builds the step graph, is not
    timed) and `sequential_steps` steps of each lattice alone; returns the
    result record (the JSON object main() prints)."""
    import torch
    log = log or (lambda msg: print(msg, file=sys.stderr, flush=True))
    storage = lbm.LBM_FP32 if storage_name == "fp32" else lbm.LBM_FP64
    specs = draw_ensemble(seed, lattices)
    lats = []
    t0 = time.perf_counter()
    for lx, ly, contrast, pseed in specs:
        ns = inputs.rt_config(lx, ly, t_bottom=1 + contrast / 2, t_top=1 - contrast / 2)
        lat = lbm.Lattice(lbm.config_from(ns, storage=storage))
        lat.init_rt(inputs.rt_perturbation(pseed, ly))
        lats.append(lat)
    torch.cuda.synchronize()
    sites = sum(lx * ly for lx, ly, _, _ in specs)
    mem = sum(lat.nbytes for lat in lats)
    log(f"[ensemble] {len(lats)} lattices, {sites / 1e6:.1f} M sites, {mem / 2**30:.1f} GiB, "
        f"set up in {time.perf_counter() - t0:.1f} s")
    try:
        eng = lbm.Engine(max_slots=len(lats))
        for lat in lats:
            eng.add(lat, steps)
        (block, groups, sched), tuned_ms = eng.tune(reps=tune_reps)
        log(f"[ensemble] tuned: block {block}, groups {groups}, schedule {sched}, "
            f"{tuned_ms:.3f} ms per step")
        eng.step(1)  # graph build + warm-up (every lattice then runs steps - 1 more)
        eng.status()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eng.step(steps - 1)
        left = eng.status()
        wall = time.perf_counter() - t0
        assert int(left.max()) == 0
        mlups = sites * (steps - 1) / wall / 1e6
        log(f"[ensemble] engine: {mlups:.0f} MLUPS, {wall / (steps - 1) * 1e3:.3f} ms per step")
        eng.close()

        # one lattice at a time, same lattices, fused path, synchronised per lattice
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for lat in lats:
            lat.step(sequential_steps)
            torch.cuda.synchronize()
        seq_wall = time.perf_counter() - t0
        seq_mlups = sites * sequential_steps / seq_wall / 1e6
        log(f"[ensemble] one at a time: {seq_mlups:.0f} MLUPS")
    finally:
        for lat in lats:
            lat.close()
    return {
        "workload": f"{len(specs)} Rayleigh-Taylor lattices, Lx in 64..1024, Ly = 2 or 4 Lx, "
                    f"{storage_name}, {steps} engine steps",
        "lattices": len(specs), "sites": sites, "device_bytes": mem, "engine_mlups": mlups,
        "engine_steps_timed": steps - 1, "engine_ms_per_step": wall / (steps - 1) * 1e3,
        "tiling": {"block": block, "groups": groups, "schedule": ["chunked", "strided"][sched],
                   "tuned_ms_per_step": tuned_ms},
        "one_at_a_time_mlups": seq_mlups, "one_at_a_time_steps": sequential_steps,
        "speedup": mlups / seq_mlups,
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--lattices", type=int, default=256)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--storage", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--tune-reps", type=int, default=2)
    ap.add_argument("--sequential-steps", type=int, default=50,
                    help="steps per lattice for the one-at-a-time reference")
    args = ap.parse_args()

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    from paper_1703_00185_amd import inputs, lbm

    out = run_ensemble(lbm, inputs, args.lattices, args.steps, args.seed, args.storage,
                       args.tune_reps, args.sequential_steps)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
