"""Throughput of the D2Q37 thermal LBM step on one MI355X.

Workload: the 2048 x 8192 Rayleigh-Taylor lattice in FP64 (16.8 M sites, 37
populations each), seeded synthetic initial state, column population
layout, stepped with the fused path (one propagate/bc/collide kernel per
step, periodic x by wrapping the source column).  A step is one update of
the whole lattice.  Inputs are resident in HBM before the timed region.
Beside it, for comparison: the same step in the planar layout, the
separate path (pbc, propagate, bc, collide), FP32 and FP16-deviation
storage with their field errors against the FP64 path after the same
steps, the region split, the two-step path (two steps per launch pair,
each site read and written once per two steps, bit-identical to the fused
path), the 64 x 128 workload (plain and graph-replayed launches), copy probes of the attainable bandwidth, the batched ensemble
(256 uneven FP32 lattices stepped by the autotuned engine, against the same
lattices one at a time), and a bounded sample of the serving workload
(Poisson arrivals of uneven FP64/FP32 requests stepped together by the
ensemble engine) for the p50/p99 completion latency against a
one-request-at-a-time FP64 server.

Prints one JSON line: MLUPS of the fused path as `value`, the roofline of
the dominant kernel (the fused kernel: 592 algorithmic bytes per site per
launch, HBM-bound) from two HIP events on the lattice's stream bracketing
the timed launches (one launch per step, so the span over the launch count
is the average launch duration, gaps between launches included), the measured HBM traffic of that kernel from the committed
rocprofv3 counter summary, the other paths' figures, and the FP64 CPU
oracle timed on a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "D2Q37 MLUPS, FP64 vs FP32-storage, 1 GPU; ensemble p50/p99 latency"
HBM_PEAK_GBS = 8000.0
BYTES_PER_SITE_FP64 = 2 * 37 * 8  # one read + one write of every population
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fused_2048x8192.json")
# the sources the fused kernel is compiled from
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1703_00185_amd", "csrc", f) for f in
                  ("kernels.hip", "d2q37_device.hpp", "kernels.hpp", "d2q37_model.hpp")]


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(lx: int, ly: int, layout: str):
    """HBM bytes per fused launch from the committed rocprofv3 counter
    summary, or None when it is missing, was taken on another workload or
    layout, or the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if (t.get("kernel_source_sha") != kernel_source_sha() or t.get("lx") != lx or t.get("ly") != ly
            or t.get("layout") != layout):
        return None
    return t.get("bytes_per_launch")


def time_path(lbm, ns, rt, path: int, steps: int, warmup: int, extra: dict,
              breakdown_steps: int = 0, graph_chunk: int = 0, fields: bool = False):
    """Time `steps` steps of one path.  The timed region holds only the
    step launches: no per-launch markers (they add a few microseconds per
    launch, and cross-stream ones more); two HIP events on the lattice's
    stream bracket it.  On a path with one launch per step the span over
    the launch count is that kernel's average launch duration (gaps between
    launches included).  With `breakdown_steps`, a separate run with a HIP
    event pair around every launch gives the per-kernel breakdown; with
    `graph_chunk`, the same steps are also replayed from a captured graph
    of that many steps.  With `fields`, the per-site moments (rho, ux, uy,
    T) after the warmup and timed steps are returned as well."""
    import torch
    cfg = lbm.config_from(ns, path=path, **extra)
    lat = lbm.Lattice(cfg)
    try:
        lat.init_rt(rt)
        lat.step(warmup)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(lat.stream)
        lat.step(steps)
        ev1.record(lat.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        span_ms = ev0.elapsed_time(ev1)
        moments = lat.moments() if fields else None
        kernels = {}
        if breakdown_steps:
            lbm.lbm_set_timing(lat.h, True)
            lat.step(breakdown_steps)
            ms, cnt = lbm.lbm_read_timing(lat.h)
            lbm.lbm_set_timing(lat.h, False)
            for p, name in enumerate(lbm.PHASE_NAMES):
                if cnt[p]:
                    kernels[name] = {"launches": int(cnt[p]), "avg_ms": float(ms[p] / cnt[p]),
                                     "timing": f"HIP events around every launch, separate run of "
                                               f"{breakdown_steps} steps"}
        graph_wall = None
        if graph_chunk:
            reps = max(1, steps // graph_chunk)
            lat.step_captured(graph_chunk)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                lat.step_captured(graph_chunk)
            torch.cuda.synchronize()
            graph_wall = (time.perf_counter() - t0) / (reps * graph_chunk)
        cons = lat.conservation()
        layout = lat.layout()
    finally:
        lat.close()
    return {"wall": wall, "span_ms": span_ms, "kernels": kernels, "cons": cons, "layout": layout,
            "graph_s_per_step": graph_wall, "moments": moments}


def field_errors(ref, got) -> dict:
    """Largest differences of the density (relative), temperature and
    velocity fields of `got` from `ref` (each a tuple rho, ux, uy, T)."""
    import numpy as np
    rho0, ux0, uy0, T0 = ref
    rho, ux, uy, T = got
    return {"rho_max_rel": float(np.max(np.abs(rho - rho0) / rho0)),
            "T_max_abs": float(np.max(np.abs(T - T0))),
            "u_max_abs": float(np.max(np.hypot(ux - ux0, uy - uy0))),
            "u_scale": float(np.max(np.hypot(ux0, uy0)))}


def cpu_model() -> str:
    """The host CPU as /proc/cpuinfo names it: model name, with the family,
    model and stepping numbers (some hosts report only a brand name)."""
    fields = {}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if ":" not in line:
                    if fields:
                        break       # end of the first processor's block
                    continue
                k, v = (t.strip() for t in line.split(":", 1))
                fields.setdefault(k, v)
    except OSError:
        pass
    if "model name" not in fields:
        import platform
        return platform.processor() or "unknown"
    ids = ", ".join(f"{k} {fields[k]}" for k in ("cpu family", "model", "stepping") if k in fields)
    return f"{fields['model name']} ({ids})" if ids else fields["model name"]


def single_kernel(name: str, run: dict, steps: int) -> dict:
    """Average launch duration of the one kernel a path launches per step,
    from the events bracketing the timed region."""
    return {name: {"launches": steps, "avg_ms": run["span_ms"] / steps,
                   "timing": "two HIP events bracketing the timed launches"}}


def probe_bandwidth(lbm, gib: float, reps: int = 10) -> dict:
    """Attainable-bandwidth reference: the library's copy probes on two
    buffers of `gib` GiB (the copy micro-benchmark of the paper's Sec. 4).
    COPY moves 2 x bytes per launch; MRAW/ARMW (doubles, shifted by
    -3..3 elements as the pull is) move 2 x (bytes - 1024).  The COPY
    launch is also the known-size kernel that calibrates the HBM byte
    counters."""
    import torch
    n = int(gib * (1 << 30)) // 16 * 16
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    stream = torch.cuda.current_stream().cuda_stream

    def timed(mode, shift):
        lbm.lbm_probe_bandwidth(mode, src.data_ptr(), dst.data_ptr(), n, shift, stream)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            lbm.lbm_probe_bandwidth(mode, src.data_ptr(), dst.data_ptr(), n, shift, stream)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        moved = 2 * n if mode == lbm.LBM_PROBE_COPY else 2 * (n - 1024)
        return {"bytes_per_launch": moved, "avg_ms": ms, "gbs": moved / (ms * 1e-3) / 1e9}

    out = {"copy": timed(lbm.LBM_PROBE_COPY, 0)}
    for name, mode in (("mraw", lbm.LBM_PROBE_MRAW), ("armw", lbm.LBM_PROBE_ARMW)):
        out[name] = {str(sh): timed(mode, sh)["gbs"] for sh in (-3, -1, 0, 1, 3)}
    del src, dst
    torch.cuda.empty_cache()
    return out


def small_lattice(lbm, inputs, reps: int = 5) -> dict:
    """The 64 x 128 Rayleigh-Taylor workload (100 steps): launch-latency
    bound (8,192 sites fill 128 wavefronts).  Median of `reps` runs of 100
    steps for the fused and separate paths, plain launches and replayed
    from a captured HIP graph."""
    import statistics
    import torch
    ns = inputs.rt_config(64, 128)
    rt = inputs.rt_perturbation(0, 128)
    out = {}
    for name, path in (("fused", lbm.LBM_PATH_FUSED), ("separate", lbm.LBM_PATH_SEPARATE)):
        for mode in ("plain", "graph"):
            lat = lbm.Lattice(lbm.config_from(ns, path=path)).init_rt(rt)
            step = lat.step if mode == "plain" else lat.step_captured
            step(100)
            torch.cuda.synchronize()
            times = []
            for _ in range(reps):
                t0 = time.perf_counter()
                step(100)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            lat.close()
            t = statistics.median(times)
            out[f"{name}_{mode}"] = {"us_per_step": t / 100 * 1e6, "mlups": 64 * 128 * 100 / t / 1e6}
    return out


def kernel_bandwidth(kernels: dict, sites: int, lx: int, ly: int, elem_bytes: int = 8) -> dict:
    """Algorithmic GB/s per kernel: fused/propagate/collide read and write
    every population once (592 B per site in FP64, 296 B in FP32); bc reads
    and writes 37 values at 6 Lx sites; pbc copies 52 rows of Ly values."""
    per_site = 2 * 37 * elem_bytes
    algo = {"fused": per_site * sites, "propagate": per_site * sites,
            "collide": per_site * sites, "bc": per_site * 6 * lx,
            "pbc": 2 * 52 * ly * elem_bytes, "fused_bulk": per_site * (lx - 6) * ly,
            "fused_border": per_site * 6 * ly}
    for name, k in kernels.items():
        k["algorithmic_bytes"] = algo[name]
        k["gbs"] = algo[name] / (k["avg_ms"] * 1e-3) / 1e9
        k["hbm_frac"] = k["gbs"] / HBM_PEAK_GBS
    return kernels


def cpu_baseline(seconds: float, small_steps: int = 100):
    """The FP64 oracle, as it stands, stepping a 2048 x 256 strip of the
    Rayleigh-Taylor workload (same Lx and initial-state recipe, 256 rows)
    for at least `seconds` of wall time; beside it, the oracle's run of the
    whole 64 x 128 workload (`small_steps` steps)."""
    import oracle
    from paper_1703_00185_amd import inputs
    lx, ly = 2048, 256
    ns = inputs.rt_config(lx, ly)
    f = oracle.init_rt(lx, ly, ns, inputs.rt_perturbation(0, ly))
    steps = 0
    t0 = time.perf_counter()
    while True:
        f = oracle.step(f, ns)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    small = None
    if small_steps > 0:
        ns1 = inputs.rt_config(64, 128)
        f1 = oracle.init_rt(64, 128, ns1, inputs.rt_perturbation(0, 128))
        t1 = time.perf_counter()
        f1 = oracle.run(f1, ns1, small_steps)
        el1 = time.perf_counter() - t1
        small = {"workload": "rayleigh_taylor_64x128_fp64", "steps": small_steps, "seconds": el1,
                 "us_per_step": el1 / small_steps * 1e6, "mlups": 64 * 128 * small_steps / el1 / 1e6}
    return {"value": lx * ly * steps / el / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{steps} FP64 oracle steps of a {lx}x{ly} Rayleigh-Taylor strip (NumPy, "
                      f"single-threaded elementwise ops; {len(os.sched_getaffinity(0))} host cores "
                      f"visible), {el:.1f} s",
            "small_lattice_64x128": small}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--lx", type=int, default=2048)
    ap.add_argument("--ly", type=int, default=8192)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--ny-pad", type=int, default=-1)
    ap.add_argument("--stride-pad", type=int, default=-1)
    ap.add_argument("--layout", choices=["column", "planar"], default="column",
                    help="population layout of the timed paths (planar is also timed for comparison)")
    ap.add_argument("--no-separate", action="store_true", help="time the fused path only")
    ap.add_argument("--no-layout-compare", action="store_true",
                    help="skip the fused run in the other population layout")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests of the bounded serving sample (p50/p99 latency); 0 skips it")
    ap.add_argument("--ensemble-lattices", type=int, default=256,
                    help="lattices of the batched-ensemble leg (FP32, autotuned engine); 0 skips it")
    ap.add_argument("--ensemble-steps", type=int, default=51,
                    help="engine steps of the ensemble leg (the first builds the graph, untimed)")
    ap.add_argument("--copy-gib", type=float, default=2.0,
                    help="size of the plain-copy reference (read GiB = write GiB)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the lattice is not sharded across GPUs)", file=sys.stderr)
        return 2
    if args.steps <= 0 or args.warmup < 0:
        print("--steps must be > 0 and --warmup >= 0", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible: bench.py needs an MI355X", file=sys.stderr)
        return 1
    from paper_1703_00185_amd import inputs, lbm

    lx, ly = args.lx, args.ly
    sites = lx * ly
    breakdown = min(args.steps, 200)  # steps of the per-launch timing runs
    ns = inputs.rt_config(lx, ly)
    rt = inputs.rt_perturbation(0, ly)
    layout_kind = lbm.LBM_LAYOUT_PLANAR if args.layout == "planar" else lbm.LBM_LAYOUT_COLUMN
    extra = {"block": args.block, "ny_pad": args.ny_pad, "stride_pad": args.stride_pad,
             "layout": layout_kind}

    copy = probe_bandwidth(lbm, args.copy_gib) if args.copy_gib > 0 else None
    if copy:
        log(f"copy probe of {args.copy_gib} GiB: {copy['copy']['gbs']:.0f} GB/s; "
            f"mraw(+1) {copy['mraw']['1']:.0f}, armw(+1) {copy['armw']['1']:.0f} GB/s")
    log(f"fused path {lx}x{ly}: {args.warmup} warmup + {args.steps} timed steps")
    run = time_path(lbm, ns, rt, lbm.LBM_PATH_FUSED, args.steps, args.warmup, extra, fields=True)
    wall, cons, layout = run["wall"], run["cons"], run["layout"]
    fp64_fields = run.pop("moments")
    kern = kernel_bandwidth(single_kernel("fused", run, args.steps), sites, lx, ly)
    mlups = sites * args.steps / wall / 1e6
    log(f"fused: {mlups:.1f} MLUPS, {wall / args.steps * 1e3:.3f} ms/step, "
        f"fused kernel {kern['fused']['avg_ms']:.3f} ms = {kern['fused']['gbs']:.0f} GB/s")
    if cons[4] != 0:
        log(f"non-finite populations after the run: {cons[4]}")
        return 1

    # the two-step path (two steps per launch pair, bit-identical to the
    # fused path): an even number of timed steps, so that every timed
    # launch is a two-step pair; its moments after the same number of
    # steps must equal the fused path's bit for bit
    steps2 = max(2, args.steps - args.steps % 2)
    log(f"two-step path {lx}x{ly}: {args.warmup} warmup + {steps2} timed steps")
    r6 = time_path(lbm, ns, rt, lbm.LBM_PATH_FUSED2, steps2, args.warmup, extra, fields=True)
    w6 = r6["wall"]
    pair_ms = r6["span_ms"] / (steps2 // 2)
    pair_bytes = 2 * 37 * 8 * sites  # each site read and written once per two steps
    two_step = {"mlups": sites * steps2 / w6 / 1e6, "ms_per_step": w6 / steps2 * 1e3,
                "steps": steps2, "speedup_vs_fused": (wall / args.steps) / (w6 / steps2),
                # null when the step counts differ (an odd --steps)
                "identical_to_fused": (all(np.array_equal(a, b) for a, b in zip(fp64_fields, r6["moments"]))
                                       if steps2 == args.steps else None),
                "launch_pair": {"launches": steps2 // 2, "avg_ms": pair_ms,
                                "timing": "two HIP events bracketing the timed launches",
                                "algorithmic_bytes": pair_bytes,
                                "gbs": pair_bytes / (pair_ms * 1e-3) / 1e9,
                                "hbm_frac": pair_bytes / (pair_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                "bytes_per_site_update": pair_bytes / (2 * sites)}}
    del r6
    log(f"two-step: {two_step['mlups']:.1f} MLUPS ({two_step['speedup_vs_fused']:.3f} x fused), "
        f"{pair_ms:.3f} ms per launch pair = {two_step['launch_pair']['gbs']:.0f} GB/s of "
        f"{two_step['launch_pair']['bytes_per_site_update']:.0f} B per site-update; identical to fused: "
        f"{two_step['identical_to_fused']}")

    other_layout = None
    if not args.no_layout_compare:
        other = "planar" if args.layout == "column" else "column"
        log(f"fused path, {other} layout {lx}x{ly}: {args.warmup} warmup + {args.steps} timed steps")
        r5 = time_path(lbm, ns, rt, lbm.LBM_PATH_FUSED, args.steps, args.warmup,
                       dict(extra, layout=lbm.LBM_LAYOUT_COLUMN + lbm.LBM_LAYOUT_PLANAR - layout_kind))
        w5 = r5["wall"]
        other_layout = {"layout": other, "mlups": sites * args.steps / w5 / 1e6,
                        "ms_per_step": w5 / args.steps * 1e3,
                        "kernels": kernel_bandwidth(single_kernel("fused", r5, args.steps), sites, lx, ly)}
        log(f"{other} layout: {other_layout['mlups']:.1f} MLUPS, "
            f"fused kernel {other_layout['kernels']['fused']['gbs']:.0f} GB/s")

    separate = None
    if not args.no_separate:
        log(f"separate path {lx}x{ly}: {args.warmup} warmup + {args.steps} timed steps")
        r2 = time_path(lbm, ns, rt, lbm.LBM_PATH_SEPARATE, args.steps, args.warmup, extra,
                       breakdown_steps=breakdown)
        w2 = r2["wall"]
        k2 = kernel_bandwidth(r2["kernels"], sites, lx, ly)
        separate = {"mlups": sites * args.steps / w2 / 1e6, "ms_per_step": w2 / args.steps * 1e3,
                    "kernels": k2}
        log(f"separate: {separate['mlups']:.1f} MLUPS")

    reduced = {}
    for name, storage, eb in (("fp32", lbm.LBM_FP32, 4), ("fp16dev", lbm.LBM_FP16DEV, 2)):
        log(f"fused path, {name} storage {lx}x{ly}: {args.warmup} warmup + {args.steps} timed steps")
        # one fused launch per step for every storage type
        r3 = time_path(lbm, ns, rt, lbm.LBM_PATH_FUSED, args.steps, args.warmup,
                       dict(extra, storage=storage), fields=True)
        errors = field_errors(fp64_fields, r3.pop("moments"))
        w3 = r3["wall"]
        k3 = single_kernel("fused", r3, args.steps)
        k3 = kernel_bandwidth(k3, sites, lx, ly, elem_bytes=eb)
        reduced[name] = {"mlups": sites * args.steps / w3 / 1e6, "ms_per_step": w3 / args.steps * 1e3,
                         "speedup_vs_fp64": wall / w3, "bytes_per_site": 2 * 37 * eb,
                         "kernels": k3,
                         "error_vs_fp64": dict(errors, steps=args.warmup + args.steps,
                                               reference="FP64 GPU path, same steps")}
        log(f"{name} storage: {reduced[name]['mlups']:.1f} MLUPS, "
            f"fused kernel {k3['fused']['gbs']:.0f} GB/s; after {args.warmup + args.steps} steps "
            f"max |drho|/rho {errors['rho_max_rel']:.1e}, |dT| {errors['T_max_abs']:.1e}, "
            f"|du| {errors['u_max_abs']:.1e} (max |u| {errors['u_scale']:.1e})")
    del fp64_fields

    log(f"region path {lx}x{ly}: {args.warmup} warmup + {args.steps} timed steps")
    r4 = time_path(lbm, ns, rt, lbm.LBM_PATH_REGIONS, args.steps, args.warmup, extra,
                   breakdown_steps=breakdown, graph_chunk=50)
    w4, g4 = r4["wall"], r4["graph_s_per_step"]
    regions = {"mlups": sites * args.steps / w4 / 1e6, "ms_per_step": w4 / args.steps * 1e3,
               "graph_replayed": {"mlups": sites / g4 / 1e6, "ms_per_step": g4 * 1e3,
                                  "graph_steps": 50},
               "kernels": kernel_bandwidth(r4["kernels"], sites, lx, ly)}
    log(f"regions: {regions['mlups']:.1f} MLUPS, graph-replayed "
        f"{regions['graph_replayed']['mlups']:.1f} MLUPS")

    log("64x128 workload, 100 steps: plain and graph-captured launches")
    small = small_lattice(lbm, inputs)
    log("64x128: " + ", ".join(f"{k} {v['us_per_step']:.1f} us/step" for k, v in small.items()))

    ensemble = None
    if args.ensemble_lattices > 0:
        from paper_1703_00185_amd.ensemble_bench import run_ensemble
        torch.cuda.empty_cache()
        log(f"batched ensemble: {args.ensemble_lattices} FP32 lattices, autotuned engine, "
            f"{args.ensemble_steps} steps")
        ensemble = run_ensemble(lbm, inputs, lattices=args.ensemble_lattices,
                                steps=args.ensemble_steps, sequential_steps=10, log=log)
        torch.cuda.empty_cache()

    serving = None
    if args.serve_requests > 0:
        from paper_1703_00185_amd.serve import serve_workload
        log(f"serving sample: {args.serve_requests} requests through the ensemble engine")
        serving = serve_workload(lbm, inputs, requests=args.serve_requests, log=log)
        log(f"serving: {serving['served']['mlups']:.0f} MLUPS, p50 {serving['served']['latency_p50_s']:.2f} s, "
            f"p99 {serving['served']['latency_p99_s']:.2f} s (one at a time FP64: p50 "
            f"{serving['one_at_a_time_fp64']['latency_p50_s']:.2f} s, "
            f"p99 {serving['one_at_a_time_fp64']['latency_p99_s']:.2f} s)")
        if serving["identical_alone_and_in_mix"]["mismatches"]:
            log("served results differ from the same requests run alone")
            return 1

    fk = kern["fused"]
    traffic = measured_traffic(lx, ly, args.layout)
    roofline = {"bound": "hbm", "achieved": fk["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": fk["gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "fused_kernel (propagate+bc+collide)",
                "algorithmic_bytes_per_launch": fk["algorithmic_bytes"],
                "avg_launch_ms": fk["avg_ms"]}

    cpu = None
    if not args.no_cpu_baseline:
        log(f"CPU oracle baseline, about {args.cpu_seconds:.0f} s")
        cpu = cpu_baseline(args.cpu_seconds)

    out = {
        "metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"rayleigh_taylor_{lx}x{ly}_fp64", "lx": lx, "ly": ly,
                   "path": "fused", "storage": "fp64", "layout": {
                       "kind": args.layout, "nx": layout[0], "ny_pitch": layout[1],
                       "pstride": layout[2], "cstride": layout[3], "block": layout[5]}},
        "roofline": roofline, "cpu_baseline": cpu, "kernels": kern, "separate": separate,
        "bandwidth_probe": copy, "reduced_storage": reduced, "regions": regions, "two_step": two_step,
        "other_layout": other_layout, "batched_ensemble": ensemble, "ensemble_serving": serving,
        "small_lattice_64x128": small,
        "paper_equivalent_gflops": 6472 * sites * args.steps / wall / 1e9,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
