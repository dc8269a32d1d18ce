"""Region-split step (bulk columns on the caller's stream, pbc and the border
columns on a second stream, overlapped): bit-identical to the fused step,
and within the FP64 tolerance of the oracle."""
import numpy as np
import pytest

import oracle
from gpu_helpers import FP64_TOL, LAYOUTS, err_metric, lattice, need_gpu
from paper_1703_00185_amd import inputs, lbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("storage", [lbm.LBM_FP64, lbm.LBM_FP32, lbm.LBM_FP16DEV])
@pytest.mark.parametrize("lx,ly", [(3, 6), (6, 12), (7, 20), (37, 70), (64, 128), (130, 257)])
def test_regions_equal_fused(lx, ly, storage, layout):
    """Every storage type, including lattices too narrow for a bulk region
    (which take the fused step: pbc first for binary16 deviations)."""
    ns = inputs.rt_config(lx, ly)
    rt = inputs.rt_perturbation(2, ly)
    out = []
    for path in (lbm.LBM_PATH_FUSED, lbm.LBM_PATH_REGIONS):
        with lattice(ns, path=path, storage=storage, layout=layout) as lat:
            lat.init_rt(rt)
            lat.step(9)
            out.append(lat.get())
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("storage", [lbm.LBM_FP64, lbm.LBM_FP32, lbm.LBM_FP16DEV])
@pytest.mark.parametrize("lx,ly", [(1024, 1024), (515, 700)])
def test_regions_equal_fused_large(lx, ly, storage):
    """Lattices where one bulk launch takes long enough that a border launch
    on the other stream ordered wrongly against it would change the result;
    several step calls, so the ordering across calls is exercised too."""
    ns = inputs.rt_config(lx, ly)
    rt = inputs.rt_perturbation(4, ly)
    out = []
    for path in (lbm.LBM_PATH_FUSED, lbm.LBM_PATH_REGIONS):
        with lattice(ns, path=path, storage=storage) as lat:
            lat.init_rt(rt)
            lat.step(5)
            lat.conservation()
            lat.step(6)
            out.append(lat.get())
    assert np.array_equal(out[0], out[1])


def test_regions_match_oracle_and_time_both_parts():
    ns = inputs.rt_config(64, 128)
    f0 = oracle.init_rt(64, 128, ns, inputs.rt_perturbation(3, 128))
    with lattice(ns, path=lbm.LBM_PATH_REGIONS) as lat:
        lat.set(f0)
        lbm.lbm_set_timing(lat.h, True)
        lat.step(4)
        ms, cnt = lbm.lbm_read_timing(lat.h)
        got = lat.get()
    assert cnt.tolist() == [4, 0, 0, 0, 0, 4, 4, 0]
    assert err_metric(got, oracle.run(f0, ns, 4)) < FP64_TOL


@pytest.mark.parametrize("storage", [lbm.LBM_FP64, lbm.LBM_FP32, lbm.LBM_FP16DEV])
@pytest.mark.parametrize("path", [lbm.LBM_PATH_SEPARATE, lbm.LBM_PATH_FUSED, lbm.LBM_PATH_REGIONS])
def test_captured_steps_equal_plain_steps(path, storage):
    """Graph-replayed steps (odd and even counts, both buffer parities,
    replayed several times with eager work in between) equal plain steps,
    for every storage type (the deviation path adds a pbc launch)."""
    ns = inputs.rt_config(64, 128)
    rt = inputs.rt_perturbation(1, 128)
    with lattice(ns, path=path, storage=storage) as a, lattice(ns, path=path, storage=storage) as b:
        a.init_rt(rt)
        b.init_rt(rt)
        for n in (3, 4, 3, 3, 4, 1):
            a.step(n)
            b.step_captured(n)
            assert np.array_equal(a.get(), b.get()), n
            b.conservation()  # eager work between replays
