"""Host logic of the serving loop, on the CPU with a stand-in engine.

The stand-in counts steps the way the engine does (each active lattice
advances one step per engine step until its count reaches zero), so the
scheduler's admission, FIFO order, memory accounting and completion
bookkeeping are exercised without a GPU.
"""
import types

import numpy as np
import pytest

from paper_1703_00185_amd import inputs, serve


class FakeLattice:
    def __init__(self, cfg):
        self.cfg = cfg
        self.closed = False

    def init_rt(self, rt):
        return self

    def get(self):
        return np.zeros(1)

    def close(self):
        self.closed = True


class FakeEngine:
    log = []

    def __init__(self, max_slots):
        self.left = {}
        self.next = 0

    def add(self, lat, steps):
        s = self.next
        self.next += 1
        self.left[s] = steps
        FakeEngine.log.append(("add", lat.cfg.rid))
        return s

    def step(self, n):
        for s in self.left:
            self.left[s] = max(0, self.left[s] - n)

    def status(self):
        return self.left

    def remove(self, slot):
        FakeEngine.log.append(("remove", slot, self.left[slot]))
        del self.left[slot]

    def set_tiling(self, *a):
        pass

    def close(self):
        pass


def fake_lbm(budget_log):
    m = types.SimpleNamespace()
    m.LBM_FP64, m.LBM_FP32 = 0, 1
    m.Lattice = FakeLattice
    m.Engine = FakeEngine

    def config_from(ns, storage=0):
        return types.SimpleNamespace(lx=ns.lx, ly=ns.ly, storage=storage, rid=None)

    m.config_from = config_from
    m.lbm_required_bytes = lambda cfg: cfg.lx * cfg.ly * 37 * (8 if cfg.storage == 0 else 4) * 2
    return m


@pytest.mark.parametrize("policy", ["srpt", "ps"])
def test_admission_budget_fifo_and_completion(policy):
    FakeEngine.log = []
    lbm = fake_lbm([])
    drawn = serve.draw_requests(3, 40)
    reqs = [serve.Request(i, 0.0, lx, ly, st // 50, sto, seed)
            for i, (lx, ly, st, sto, seed) in enumerate(drawn)]
    budget = 3 * max(lbm.lbm_required_bytes(lbm.config_from(inputs.rt_config(r.lx, r.ly), r.storage))
                     for r in reqs)
    srv = serve.Server(lbm, inputs, budget, max_slots=8, chunk=5, policy=policy)
    orig_config = srv.config

    def tagged(r):
        c = orig_config(r)
        c.rid = r.rid
        return c

    srv.config = tagged
    peak = [0]
    orig_add = FakeEngine.add

    def add(self, lat, steps):
        peak[0] = max(peak[0], srv.used + lbm.lbm_required_bytes(lat.cfg))
        return orig_add(self, lat, steps)

    FakeEngine.add = add
    try:
        done, makespan, site_steps = srv.run(reqs)
    finally:
        FakeEngine.add = orig_add
    assert sorted(done) == list(range(40))
    assert peak[0] <= budget
    admitted = [rid for _, kind, rid, _ in srv.events if kind == "admit"]
    assert admitted == sorted(admitted)          # first come, first served
    assert srv.used == 0
    assert site_steps == sum(r.lx * r.ly * r.steps for r in reqs)


def test_oversized_request_is_admitted_when_idle():
    FakeEngine.log = []
    lbm = fake_lbm([])
    reqs = [serve.Request(0, 0.0, 512, 2048, 3, 0, 1), serve.Request(1, 0.0, 64, 128, 2, 1, 2)]
    srv = serve.Server(lbm, inputs, budget_bytes=1000, max_slots=4, chunk=10)
    done, _, _ = srv.run(reqs)
    assert sorted(done) == [0, 1]


def test_fifo_latencies_closed_form():
    arr = [0.0, 1.0, 1.5, 10.0]
    svc = [2.0, 2.0, 1.0, 1.0]
    # finishes: 2, 4, 5, 11 -> latencies 2, 3, 3.5, 1
    assert serve.fifo_latencies(arr, svc) == [2.0, 3.0, 3.5, 1.0]


def test_request_distribution():
    d = serve.draw_requests(0, 4000)
    lx = np.array([x[0] for x in d])
    ly = np.array([x[1] for x in d])
    st = np.array([x[2] for x in d])
    assert lx.min() >= 64 and lx.max() <= 1024 and ly.min() >= 128 and ly.max() <= 4096
    assert st.min() >= 100 and st.max() <= 5000
    assert abs(np.mean([x[3] for x in d]) - 0.5) < 0.05
    # log-uniform sites: the median of log(sites) sits mid-range
    ls = np.log(lx * ly)
    assert abs(np.median(ls) - 0.5 * (np.log(64 * 128) + np.log(1024 * 4096))) < 0.3


def test_one_at_a_time_baseline_runs_in_arrival_order_after_arrival():
    """The measured baseline serves one request at a time, FIFO, each
    started no earlier than its arrival; FP64 storage for every request."""
    ran = []

    class TimedLattice(FakeLattice):
        def step(self, n):
            ran.append((n, self.cfg.storage))

    m = fake_lbm([])
    m.Lattice = TimedLattice
    reqs = [serve.Request(rid=i, arrival=a, lx=8, ly=16, steps=10 + i, storage=i % 2, seed=i)
            for i, a in enumerate([0.0, 0.05, 0.02, 0.3])]
    lat, busy = serve.run_one_at_a_time(m, inputs, reqs, sync=lambda: None)
    assert [n for n, _ in ran] == [10, 12, 11, 13]      # arrival order
    assert all(storage == 0 for _, storage in ran)      # plain FP64
    assert len(lat) == 4 and all(x >= 0.0 for x in lat)
    assert 0.0 <= busy < 0.3


def test_srpt_steps_least_remaining_work_first_up_to_fill():
    """The engine set is the resident lattices with the least remaining work
    (sites x steps left), taken until the fill size is reached; the others
    wait resident, and every lattice ends with its own step count."""
    FakeEngine.log = []
    lbm = fake_lbm([])
    reqs = [serve.Request(0, 0.0, 64, 128, 50, 0, 1),    # 409,600 site-steps
            serve.Request(1, 0.0, 64, 128, 10, 1, 2),    # 81,920
            serve.Request(2, 0.0, 128, 256, 4, 0, 3)]    # 131,072
    srv = serve.Server(lbm, inputs, 1 << 40, max_slots=4, chunk=100, fill_sites=2 * 64 * 128)
    steps_run = []
    orig_step = FakeEngine.step

    def step(self, n):
        steps_run.append((n, sorted(self.left)))
        orig_step(self, n)

    FakeEngine.step = step
    try:
        done, _, site_steps = srv.run(reqs)
    finally:
        FakeEngine.step = orig_step
    assert sorted(done) == [0, 1, 2]
    joins = [rid for _, kind, rid, _ in srv.events if kind == "join"]
    # 1 (least work) and 2 fill the engine first; 0 waits until one retires
    assert joins[:2] == [1, 2] and 0 in joins[2:]
    order = [rid for _, kind, rid, _ in srv.events if kind == "retire"]
    assert order == [2, 1, 0]
    assert site_steps == sum(r.lx * r.ly * r.steps for r in reqs)
