"""Serving loop for Rayleigh-Taylor simulation requests (continuous batching).

Requests (seeded): lattice sizes log-uniform from 64 x 128 to 1024 x 4096,
step counts uniform in [100, 5000], FP64 or FP32 storage with equal odds,
arriving as a Poisson process whose rate is a fraction (default 0.8) of the
capacity measured on a calibration batch.  The loop keeps every admitted
lattice resident in HBM, admits queued requests first-come first-served
while they fit a device-memory budget, and advances all active lattices
together through the ensemble engine (one persistent launch per step,
replayed from a HIP graph).  It steps until the next lattice finishes
(at most `--chunk` steps, so that arrivals are admitted promptly), retires
finished lattices and frees their memory.

Reported: aggregate MLUPS over the run, p50/p99 completion latency
(completion minus arrival), and the same latencies for a one-request-at-a-
time plain FP64 server under the same arrivals.  That baseline is a FIFO
single server whose service times come from FP64 throughput measured on
the GPU for each lattice size.  A sample of served results is recomputed
alone and compared bit for bit.  Prints one JSON line.

Usage: python -m paper_1703_00185_amd.serve [--requests 5000] [--load 0.8]
"""
from __future__ import annotations

import argparse
import collections
import json
import math
import sys
import time

import numpy as np

Request = collections.namedtuple("Request", "rid arrival lx ly steps storage seed")


def draw_requests(seed: int, n: int):
    """Sizes, step counts and storage of n requests (arrival times later)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, n)
    lx = np.maximum(8, np.round(64 * 16.0 ** u)).astype(int)
    ly = np.maximum(16, np.round(128 * 32.0 ** u)).astype(int)
    steps = rng.integers(100, 5001, n)
    storage = rng.integers(0, 2, n)  # 0: FP64, 1: FP32
    return [(int(a), int(b), int(c), int(d), int(seed * 1000003 + i))
            for i, (a, b, c, d) in enumerate(zip(lx, ly, steps, storage))]


def poisson_arrivals(seed: int, n: int, rate: float) -> np.ndarray:
    rng = np.random.default_rng(seed + 1)
    return np.cumsum(rng.exponential(1.0 / rate, n))


def percentile(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else float("nan")


class Server:
    """Admission by memory budget, FIFO queue, continuous batching."""

    def __init__(self, lbm, inputs, budget_bytes: int, max_slots: int, chunk: int, keep=()):
        self.lbm, self.inputs = lbm, inputs
        self.budget = budget_bytes
        self.chunk = chunk
        self.engine = lbm.Engine(max_slots=max_slots)
        self.max_slots = max_slots
        self.keep = set(keep)       # request ids whose final populations are kept
        self.kept = {}
        self.used = 0
        self.events = []            # (time, "admit" | "retire", request id, slot)

    def config(self, r: Request):
        ns = self.inputs.rt_config(r.lx, r.ly)
        storage = self.lbm.LBM_FP32 if r.storage else self.lbm.LBM_FP64
        return self.lbm.config_from(ns, storage=storage)

    def run(self, requests):
        lbm = self.lbm
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue = collections.deque()
        active = {}                 # slot -> (request, lattice, bytes)
        left_of = {}                # slot -> steps still to run
        done = {}                   # rid -> completion time
        site_steps = 0
        t0 = time.perf_counter()
        next_report = 10.0
        while pending or queue or active:
            now = time.perf_counter() - t0
            if now >= next_report:
                print(f"[serve] t={now:.0f} s: {len(done)} done, {len(active)} active, "
                      f"{len(queue)} queued, {self.used / 2**30:.1f} GiB in use",
                      file=sys.stderr, flush=True)
                next_report = now + 10.0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            while queue and len(active) < self.max_slots:
                r = queue[0]
                cfg = self.config(r)
                need = lbm.lbm_required_bytes(cfg)
                if self.used + need > self.budget and active:
                    break           # wait for memory (first come, first served)
                queue.popleft()
                lat = lbm.Lattice(cfg)
                lat.init_rt(self.inputs.rt_perturbation(r.seed, r.ly))
                slot = self.engine.add(lat, r.steps)
                self.events.append((time.perf_counter() - t0, "admit", r.rid, slot))
                active[slot] = (r, lat, need)
                left_of[slot] = r.steps
                self.used += need
            if not active:
                if pending:
                    time.sleep(max(0.0, min(pending[0].arrival - (time.perf_counter() - t0), 0.05)))
                continue
            # step until the next lattice finishes (at most `chunk` steps)
            n = max(1, min(min(left_of.values()), self.chunk))
            self.engine.step(n)
            for s in left_of:
                left_of[s] = max(0, left_of[s] - n)
            self.engine.status()  # waits for the steps; finished lattices leave the tile table
            now = time.perf_counter() - t0
            for slot in [s for s in active if left_of[s] == 0]:
                r, lat, need = active.pop(slot)
                del left_of[slot]
                done[r.rid] = now
                site_steps += r.lx * r.ly * r.steps
                if r.rid in self.keep:
                    self.kept[r.rid] = lat.get()
                self.engine.remove(slot)
                self.events.append((now, "retire", r.rid, slot))
                lat.close()
                self.used -= need
        makespan = time.perf_counter() - t0
        self.engine.close()
        return done, makespan, site_steps


def measure_fp64_rates(lbm, inputs, sizes, steps: int = 30):
    """FP64 fused MLUPS of single lattices, per (lx, ly) (one at a time)."""
    import torch
    rates = {}
    for lx, ly in sizes:
        lat = lbm.Lattice(lbm.config_from(inputs.rt_config(lx, ly)))
        lat.init_rt(inputs.rt_perturbation(0, ly))
        lat.step(3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(steps)
        torch.cuda.synchronize()
        rates[(lx, ly)] = lx * ly * steps / (time.perf_counter() - t0) / 1e6
        lat.close()
    return rates


def fifo_latencies(arrivals, service):
    finish, out = 0.0, []
    for a, s in zip(arrivals, service):
        finish = max(finish, a) + s
        out.append(finish - a)
    return out


def serve_workload(lbm, inputs, requests: int = 5000, seed: int = 0, load: float = 0.8,
                   budget_gb: float = 200.0, max_slots: int = 1024, chunk: int = 25,
                   check: int = 12, log=None) -> dict:
    """Run the serving workload on the current GPU; returns the result
    record (the JSON object main() prints)."""
    log = log or (lambda msg: print(msg, file=sys.stderr, flush=True))
    drawn = draw_requests(seed, requests)
    work = np.array([lx * ly * st for lx, ly, st, _, _ in drawn], dtype=np.float64)

    # capacity: aggregate rate of the engine on a calibration batch of the mix
    cal = [d for d in drawn[:64]]
    cal_lats = []
    eng = lbm.Engine(max_slots=len(cal))
    for lx, ly, _, sto, s in cal:
        lat = lbm.Lattice(lbm.config_from(inputs.rt_config(lx, ly),
                                          storage=lbm.LBM_FP32 if sto else lbm.LBM_FP64))
        lat.init_rt(inputs.rt_perturbation(s, ly))
        eng.add(lat, 1000)
        cal_lats.append(lat)
    (block, groups, sched), _ = eng.tune(reps=2)
    eng.step(2)
    eng.status()
    t0 = time.perf_counter()
    eng.step(20)
    eng.status()
    cal_mlups = sum(lx * ly for lx, ly, _, _, _ in cal) * 20 / (time.perf_counter() - t0) / 1e6
    eng.close()
    for lat in cal_lats:
        lat.close()
    capacity = cal_mlups * 1e6 / float(work.mean())       # requests per second
    rate = load * capacity
    arrivals = poisson_arrivals(seed, requests, rate)
    reqs = [Request(i, float(arrivals[i]), lx, ly, st, sto, s)
            for i, (lx, ly, st, sto, s) in enumerate(drawn)]
    log(f"[serve] calibration {cal_mlups:.0f} MLUPS -> capacity {capacity:.2f} req/s, "
        f"arrival rate {rate:.2f} req/s, {requests} requests, "
        f"{work.sum() / 1e12:.2f} T site-updates")

    rng = np.random.default_rng(seed + 7)
    small = [r.rid for r in reqs if r.lx * r.ly <= 65536]
    keep = set(rng.choice(small, size=min(check, len(small)), replace=False).tolist()) if small else set()
    srv = Server(lbm, inputs, int(budget_gb * 2**30), max_slots, chunk, keep)
    srv.engine.set_tiling(block, groups, sched)
    done, makespan, site_steps = srv.run(reqs)
    lat_served = [done[r.rid] - r.arrival for r in reqs]
    mlups = site_steps / makespan / 1e6
    log(f"[serve] served {len(done)} requests in {makespan:.1f} s: {mlups:.0f} MLUPS, "
        f"p50 {percentile(lat_served, 50):.2f} s, p99 {percentile(lat_served, 99):.2f} s")

    # identical alone and in the mix
    mismatches = 0
    for rid in sorted(srv.kept):
        r = reqs[rid]
        lat = lbm.Lattice(srv.config(r))
        lat.init_rt(inputs.rt_perturbation(r.seed, r.ly))
        lat.step(r.steps)
        mismatches += int(not np.array_equal(lat.get(), srv.kept[rid]))
        lat.close()

    # one request at a time, plain FP64, same arrivals
    grid = sorted({(64 * 2 ** k, 128 * 2 ** k) for k in range(5)} |
                  {(64 * 2 ** k, 256 * 2 ** k) for k in range(5)})
    rates = measure_fp64_rates(lbm, inputs, [g for g in grid if g[0] <= 1024 and g[1] <= 4096])
    xs = np.log([lx * ly for lx, ly in rates])
    ys = np.array(list(rates.values()))
    order = np.argsort(xs)

    def fp64_rate(sites):
        return float(np.interp(math.log(sites), xs[order], ys[order]))

    service = [r.lx * r.ly * r.steps / (fp64_rate(r.lx * r.ly) * 1e6) for r in reqs]
    lat_base = fifo_latencies([r.arrival for r in reqs], service)
    base_mlups = float(work.sum()) / max(sum(service), 1e-9) / 1e6

    return {
        "workload": f"{requests} Rayleigh-Taylor requests, 64x128..1024x4096 log-uniform, "
                    f"100-5000 steps, FP64/FP32 50/50, Poisson arrivals at {load} of capacity",
        "arrival_rate_per_s": rate, "capacity_per_s": capacity, "calibration_mlups": cal_mlups,
        "tiling": {"block": block, "groups": groups, "schedule": sched},
        "served": {"mlups": mlups, "makespan_s": makespan,
                   "latency_p50_s": percentile(lat_served, 50),
                   "latency_p99_s": percentile(lat_served, 99),
                   "latency_mean_s": float(np.mean(lat_served))},
        "one_at_a_time_fp64": {"mlups": base_mlups,
                               "latency_p50_s": percentile(lat_base, 50),
                               "latency_p99_s": percentile(lat_base, 99),
                               "service_rates_measured": {f"{k[0]}x{k[1]}": v for k, v in rates.items()},
                               "note": "FIFO single server, service times from measured FP64 rates"},
        "identical_alone_and_in_mix": {"checked": len(srv.kept), "mismatches": mismatches},
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--requests", type=int, default=5000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--load", type=float, default=0.8)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--max-slots", type=int, default=1024)
    ap.add_argument("--chunk", type=int, default=25)
    ap.add_argument("--check", type=int, default=12, help="served results recomputed alone")
    args = ap.parse_args()

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    from paper_1703_00185_amd import inputs, lbm

    out = serve_workload(lbm, inputs, args.requests, args.seed, args.load, args.budget_gb,
                         args.max_slots, args.chunk, args.check)
    print(json.dumps(out), flush=True)
    return 0 if out["identical_alone_and_in_mix"]["mismatches"] == 0 else 1


if __name__ == "__main__":
    sys.exit(main())
