"""Serving loop for Rayleigh-Taylor simulation requests (continuous batching).

Requests (seeded): lattice sizes log-uniform from 64 x 128 to 1024 x 4096,
step counts uniform in [100, 5000], FP64 or FP32 storage with equal odds,
arriving as a Poisson process whose rate is a fraction (default 0.8) of the
capacity measured on a calibration batch.  The loop keeps every admitted
lattice resident in HBM, admits queued requests first-come first-served
while they fit a device-memory budget, and advances all active lattices
together through the ensemble engine (one persistent launch per step,
replayed from a HIP graph): by default the resident lattices with the
least remaining work, enough of them to fill the GPU (see Server).  It
steps until the next active lattice finishes (at most `--chunk` steps, so
that arrivals are admitted promptly), retires finished lattices and frees
their memory.

Reported: aggregate MLUPS over the run and over the time the engine was
busy, p50/p99 completion latency (completion minus arrival), and the same
latencies for a one-request-at-a-time plain FP64 server under the same
arrivals: run on the GPU (FIFO, each request a plain FP64 lattice stepped
alone) and, beside it, simulated from FP64 throughput measured per lattice
size.  A sample of served results (half of them small lattices, half of a
million sites or more, kept on the GPU until the run ends) is recomputed
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
    """Admission by memory budget (FIFO), continuous batching on the engine.

    Admitted requests stay resident in HBM until they finish.  Which of them
    the engine steps is the policy:
      * "srpt" (default): the resident lattices with the least remaining
        work (sites x steps left) first, as many as it takes to reach
        `fill_sites` active sites (enough to keep the GPU busy); the others
        wait, resident, and rejoin when they rank among the first.  Every
        engine step advances each active lattice by one step, so a lattice
        stepped beside others progresses at the pace of the whole batch:
        giving the batch to the requests nearest completion shortens most
        completion times, the longest ones included (on the serving
        workload at 0.8 load the model of this loop puts p99 at about half
        of "ps").
      * "ps": every resident lattice is stepped (processor sharing).
    Events (time, kind, request id, slot): "admit" (resident), "join" and
    "leave" (on and off the engine), "retire" (finished, memory freed).
    Requests in `keep` have their final populations kept: read back to the
    host at retirement, or with keep_lattices the finished lattices
    themselves, which then stay in device memory outside the budget until
    the caller closes them."""

    def __init__(self, lbm, inputs, budget_bytes: int, max_slots: int, chunk: int, keep=(),
                 policy: str = "srpt", fill_sites: int = 8_000_000, keep_lattices: bool = False):
        if policy not in ("srpt", "ps"):
            raise ValueError("policy must be 'srpt' or 'ps'")
        self.lbm, self.inputs = lbm, inputs
        self.budget = budget_bytes
        self.chunk = chunk
        self.policy = policy
        self.fill_sites = fill_sites
        self.engine = lbm.Engine(max_slots=max_slots)
        self.max_slots = max_slots
        self.keep = set(keep)       # request ids whose final populations are kept
        # keep_lattices: keep those lattices themselves (off the engine, not
        # closed; the caller reads and closes them), so that keeping a large
        # result costs the loop no copy to the host
        self.keep_lattices = keep_lattices
        self.kept = {}
        self.used = 0
        self.events = []
        self.busy = 0.0             # seconds with at least one lattice on the engine

    def config(self, r: Request):
        ns = self.inputs.rt_config(r.lx, r.ly)
        storage = self.lbm.LBM_FP32 if r.storage else self.lbm.LBM_FP64
        return self.lbm.config_from(ns, storage=storage)

    def _engine_set(self, resident):
        """Request ids the engine steps next."""
        if self.policy == "ps":
            return set(resident)
        order = sorted(resident, key=lambda rid: (resident[rid]["r"].lx * resident[rid]["r"].ly
                                                  * resident[rid]["left"], rid))
        out, sites = set(), 0
        for rid in order:
            out.add(rid)
            sites += resident[rid]["r"].lx * resident[rid]["r"].ly
            if sites >= self.fill_sites:
                break
        return out

    def run(self, requests):
        lbm = self.lbm
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue = collections.deque()
        resident = {}               # rid -> {"r", "lat", "bytes", "left", "slot"}
        done = {}                   # rid -> completion time
        site_steps = 0
        t0 = time.perf_counter()
        next_report = 10.0
        while pending or queue or resident:
            now = time.perf_counter() - t0
            if now >= next_report:
                on = sum(1 for e in resident.values() if e["slot"] is not None)
                print(f"[serve] t={now:.0f} s: {len(done)} done, {len(resident)} resident "
                      f"({on} on the engine), {len(queue)} queued, {self.used / 2**30:.1f} GiB in use",
                      file=sys.stderr, flush=True)
                next_report = now + 10.0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            while queue and len(resident) < self.max_slots:
                r = queue[0]
                cfg = self.config(r)
                need = lbm.lbm_required_bytes(cfg)
                if self.used + need > self.budget and resident:
                    break           # wait for memory (first come, first served)
                queue.popleft()
                lat = lbm.Lattice(cfg)
                lat.init_rt(self.inputs.rt_perturbation(r.seed, r.ly))
                resident[r.rid] = {"r": r, "lat": lat, "bytes": need, "left": r.steps, "slot": None}
                self.events.append((time.perf_counter() - t0, "admit", r.rid, None))
                self.used += need
            if not resident:
                if pending:
                    time.sleep(max(0.0, min(pending[0].arrival - (time.perf_counter() - t0), 0.05)))
                continue
            want = self._engine_set(resident)
            for rid, e in resident.items():
                if e["slot"] is not None and rid not in want:
                    self.engine.remove(e["slot"])
                    self.events.append((time.perf_counter() - t0, "leave", rid, e["slot"]))
                    e["slot"] = None
            for rid in sorted(want):
                e = resident[rid]
                if e["slot"] is None:
                    e["slot"] = self.engine.add(e["lat"], e["left"])
                    self.events.append((time.perf_counter() - t0, "join", rid, e["slot"]))
            # step until the next active lattice finishes (at most `chunk` steps)
            n = max(1, min(min(resident[rid]["left"] for rid in want), self.chunk))
            t_busy = time.perf_counter()
            self.engine.step(n)
            for rid in want:
                resident[rid]["left"] = max(0, resident[rid]["left"] - n)
            self.engine.status()  # waits for the steps; finished lattices leave the tile table
            self.busy += time.perf_counter() - t_busy
            now = time.perf_counter() - t0
            for rid in sorted(rid for rid in want if resident[rid]["left"] == 0):
                e = resident.pop(rid)
                r = e["r"]
                done[rid] = now
                site_steps += r.lx * r.ly * r.steps
                if rid in self.keep and not self.keep_lattices:
                    self.kept[rid] = e["lat"].get()
                self.engine.remove(e["slot"])
                self.events.append((now, "retire", rid, e["slot"]))
                if rid in self.keep and self.keep_lattices:
                    self.kept[rid] = e["lat"]
                else:
                    e["lat"].close()
                self.used -= e["bytes"]
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


def run_one_at_a_time(lbm, inputs, requests, log=None, sync=None):
    """The baseline server, run for real on the GPU: requests in arrival
    order, one at a time, each as a plain FP64 lattice stepped alone with
    the fused path (created, initialised, stepped, waited for, freed), each
    started no earlier than its arrival (the arrival times are seconds
    from the start of this call).  Returns the completion latencies and
    the busy time.  sync waits for the device (torch's by default)."""
    if sync is None:
        import torch
        sync = torch.cuda.synchronize
    out, busy = [], 0.0
    t0 = time.perf_counter()
    next_report = 10.0
    for r in sorted(requests, key=lambda q: q.arrival):
        now = time.perf_counter() - t0
        if now < r.arrival:
            time.sleep(r.arrival - now)
        start = time.perf_counter()
        lat = lbm.Lattice(lbm.config_from(inputs.rt_config(r.lx, r.ly)))
        lat.init_rt(inputs.rt_perturbation(r.seed, r.ly))
        lat.step(r.steps)
        sync()
        lat.close()
        end = time.perf_counter()
        busy += end - start
        out.append((r.rid, end - t0 - r.arrival))
        if log and end - t0 >= next_report:
            log(f"[serve] baseline t={end - t0:.0f} s: {len(out)} of {len(requests)} done")
            next_report = end - t0 + 10.0
    lat_by_rid = dict(out)
    return [lat_by_rid[r.rid] for r in requests], busy


def fifo_latencies(arrivals, service):
    finish, out = 0.0, []
    for a, s in zip(arrivals, service):
        finish = max(finish, a) + s
        out.append(finish - a)
    return out


def serve_workload(lbm, inputs, requests: int = 5000, seed: int = 0, load: float = 0.8,
                   budget_gb: float = 200.0, max_slots: int = 1024, chunk: int = 25,
                   check: int = 12, log=None, measure_baseline: bool = True,
                   policy: str = "srpt", rate: float | None = None, serve: bool = True) -> dict:
    """Run the serving workload on the current GPU; returns the result
    record (the JSON object main() prints).  With measure_baseline the
    one-request-at-a-time FP64 server is also run on the GPU under the same
    arrivals (as long again as the served run).  rate fixes the arrival
    rate (requests per second) instead of load x the measured capacity, so
    that two runs can share their arrivals; serve=False runs only the
    baselines."""
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
    if rate is None:
        rate = load * capacity
    arrivals = poisson_arrivals(seed, requests, rate)
    reqs = [Request(i, float(arrivals[i]), lx, ly, st, sto, s)
            for i, (lx, ly, st, sto, s) in enumerate(drawn)]
    log(f"[serve] calibration {cal_mlups:.0f} MLUPS -> capacity {capacity:.2f} req/s, "
        f"arrival rate {rate:.2f} req/s, {requests} requests, "
        f"{work.sum() / 1e12:.2f} T site-updates")

    served, identical, fill = None, None, None
    if serve:
        # half of the checked requests from the small lattices, half from
        # those of a million sites or more (the largest the workload draws)
        rng = np.random.default_rng(seed + 7)
        small = [r.rid for r in reqs if r.lx * r.ly <= 65536]
        large = [r.rid for r in reqs if r.lx * r.ly >= 1 << 20]
        n_large = min(check // 2, len(large))
        keep = set(rng.choice(large, size=n_large, replace=False).tolist()) if n_large else set()
        if small:
            keep |= set(rng.choice(small, size=min(check - n_large, len(small)), replace=False).tolist())
        srv = Server(lbm, inputs, int(budget_gb * 2**30), max_slots, chunk, keep, policy=policy,
                     keep_lattices=True)
        srv.engine.set_tiling(block, groups, sched)
        fill = srv.fill_sites
        done, makespan, site_steps = srv.run(reqs)
        lat_served = [done[r.rid] - r.arrival for r in reqs]
        mlups = site_steps / makespan / 1e6
        busy_mlups = site_steps / max(srv.busy, 1e-9) / 1e6
        log(f"[serve] served {len(done)} requests in {makespan:.1f} s: {mlups:.0f} MLUPS "
            f"({busy_mlups:.0f} over busy time), p50 {percentile(lat_served, 50):.2f} s, "
            f"p99 {percentile(lat_served, 99):.2f} s")
        served = {"mlups": mlups, "mlups_busy": busy_mlups, "busy_s": srv.busy,
                  "makespan_s": makespan,
                  "latency_p50_s": percentile(lat_served, 50),
                  "latency_p99_s": percentile(lat_served, 99),
                  "latency_mean_s": float(np.mean(lat_served))}

        # identical alone and in the mix (every population, bit for bit)
        mismatches = 0
        for rid in sorted(srv.kept):
            r = reqs[rid]
            mixed = srv.kept[rid]
            got = mixed.get()
            mixed.close()
            lat = lbm.Lattice(srv.config(r))
            lat.init_rt(inputs.rt_perturbation(r.seed, r.ly))
            lat.step(r.steps)
            mismatches += int(not np.array_equal(lat.get(), got))
            lat.close()
            del got
        identical = {"checked": len(srv.kept), "mismatches": mismatches,
                     "largest_sites": max((reqs[rid].lx * reqs[rid].ly for rid in srv.kept), default=0)}

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
    measured = None
    if measure_baseline:
        log(f"[serve] one-at-a-time FP64 server on the GPU, same {requests} arrivals")
        lat_m, busy_m = run_one_at_a_time(lbm, inputs, reqs, log)
        measured = {"mlups_busy": float(work.sum()) / max(busy_m, 1e-9) / 1e6,
                    "busy_s": busy_m,
                    "latency_p50_s": percentile(lat_m, 50),
                    "latency_p99_s": percentile(lat_m, 99),
                    "latency_mean_s": float(np.mean(lat_m)),
                    "note": "run on the GPU: FIFO, one FP64 lattice at a time (create, init, "
                            "step, wait, free), each started no earlier than its arrival"}
        log(f"[serve] one at a time (measured): p50 {measured['latency_p50_s']:.2f} s, "
            f"p99 {measured['latency_p99_s']:.2f} s, {measured['mlups_busy']:.0f} MLUPS busy")
    base = measured if measured else {"latency_p50_s": percentile(lat_base, 50),
                                      "latency_p99_s": percentile(lat_base, 99)}

    return {
        "workload": f"{requests} Rayleigh-Taylor requests, 64x128..1024x4096 log-uniform, "
                    f"100-5000 steps, FP64/FP32 50/50, Poisson arrivals at {load} of capacity",
        "policy": {"name": policy, "fill_sites": fill, "chunk_steps": chunk},
        "arrival_rate_per_s": rate, "capacity_per_s": capacity, "calibration_mlups": cal_mlups,
        "tiling": {"block": block, "groups": groups, "schedule": sched},
        "served": served,
        "one_at_a_time_fp64": {"latency_p50_s": base["latency_p50_s"],
                               "latency_p99_s": base["latency_p99_s"],
                               "measured": measured,
                               "simulated": {
                                   "mlups": base_mlups,
                                   "latency_p50_s": percentile(lat_base, 50),
                                   "latency_p99_s": percentile(lat_base, 99),
                                   "service_rates_measured": {f"{k[0]}x{k[1]}": v
                                                              for k, v in rates.items()},
                                   "note": "FIFO single server, service times from measured "
                                           "FP64 rates per lattice size"}},
        "identical_alone_and_in_mix": identical,
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
    ap.add_argument("--policy", choices=["srpt", "ps"], default="srpt",
                    help="which resident lattices the engine steps (see Server)")
    ap.add_argument("--no-measured-baseline", action="store_true",
                    help="only simulate the one-at-a-time FP64 server (it takes as long as serving)")
    ap.add_argument("--rate", type=float, default=None,
                    help="arrival rate in requests/s (default: --load x the measured capacity)")
    ap.add_argument("--baseline-only", action="store_true",
                    help="run only the one-at-a-time FP64 servers (with --rate, on another run's arrivals)")
    args = ap.parse_args()

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    from paper_1703_00185_amd import inputs, lbm

    out = serve_workload(lbm, inputs, args.requests, args.seed, args.load, args.budget_gb,
                         args.max_slots, args.chunk, args.check,
                         measure_baseline=not args.no_measured_baseline, policy=args.policy,
                         rate=args.rate, serve=not args.baseline_only)
    print(json.dumps(out), flush=True)
    ident = out["identical_alone_and_in_mix"]
    return 0 if ident is None or ident["mismatches"] == 0 else 1


if __name__ == "__main__":
    sys.exit(main())
