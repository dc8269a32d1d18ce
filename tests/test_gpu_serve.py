"""Serving loop on the GPU: continuous batching through the ensemble engine.

A seeded stream of Rayleigh-Taylor requests of uneven sizes, step counts
and storage types (FP64 and FP32) arrives faster than the device-memory
budget admits them, so requests queue, lattices join the engine while
others are mid-run, finish at different steps, leave, and free slots and
memory for the queue.  Every request's final populations must be
bit-identical to the same request stepped alone with lbm_step (the engine
runs the fused kernel's arithmetic per lattice), under both policies (the
default one, which also takes unfinished lattices off the engine and puts
them back later, and processor sharing), and one FP64 request is checked
against the oracle.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import FP64_TOL, err_metric, need_gpu, note
from paper_1703_00185_amd import inputs, lbm
from paper_1703_00185_amd.serve import Request, Server

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _requests(n=20, seed=11):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        lx = int(rng.choice([8, 13, 24, 40, 64]))
        ly = int(rng.choice([16, 37, 64, 100, 256]))
        # a burst: every request is queued at once, so admission is bound by
        # the slots and the memory budget
        out.append(Request(rid=i, arrival=0.0, lx=lx, ly=ly, steps=int(rng.integers(3, 41)),
                           storage=i % 2, seed=1000 + i))
    return out


def _alone(srv, r):
    with lbm.Lattice(srv.config(r)) as lat:
        lat.init_rt(inputs.rt_perturbation(r.seed, r.ly))
        lat.step(r.steps)
        return lat.get()


@pytest.mark.parametrize("policy,fill", [("srpt", 6000), ("ps", 0)])
def test_served_results_equal_each_request_alone(policy, fill):
    reqs = _requests()
    # room for about three of these lattices at once: the rest queue
    sizes = sorted(lbm.lbm_required_bytes(lbm.config_from(
        inputs.rt_config(r.lx, r.ly), storage=lbm.LBM_FP32 if r.storage else lbm.LBM_FP64)) for r in reqs)
    budget = sum(sizes[-3:])
    note(f"serving {len(reqs)} requests ({policy}), budget {budget} bytes, 4 slots, chunk 3")
    srv = Server(lbm, inputs, budget, max_slots=4, chunk=3, keep=[r.rid for r in reqs],
                 policy=policy, fill_sites=fill)
    done, makespan, site_steps = srv.run(reqs)
    assert sorted(done) == [r.rid for r in reqs]
    assert site_steps == sum(r.lx * r.ly * r.steps for r in reqs)

    # continuous batching happened: several lattices on the engine at once,
    # a lattice joining while others were mid-run after one had left, and a
    # freed slot reused; under srpt, lattices also left the engine
    # unfinished and rejoined later
    on, peak, joined_after_leave, left_slots, reused = set(), 0, False, set(), False
    paused, resumed = set(), set()
    for _, kind, rid, slot in srv.events:
        if kind == "join":
            joined_after_leave |= bool(left_slots) and bool(on)
            reused |= slot in left_slots
            resumed |= {rid} & paused
            on.add(rid)
            peak = max(peak, len(on))
        elif kind in ("leave", "retire"):
            on.discard(rid)
            left_slots.add(slot)
            if kind == "leave":
                paused.add(rid)
    assert peak >= 2 and joined_after_leave and reused
    if policy == "srpt":
        assert resumed

    mismatches = [r.rid for r in reqs if not np.array_equal(srv.kept[r.rid], _alone(srv, r))]
    assert mismatches == []

    r = next(r for r in reqs if r.storage == 0)
    ns = inputs.rt_config(r.lx, r.ly)
    f = oracle.run(oracle.init_rt(r.lx, r.ly, ns, inputs.rt_perturbation(r.seed, r.ly)), ns, r.steps)
    assert err_metric(srv.kept[r.rid], f) < FP64_TOL
