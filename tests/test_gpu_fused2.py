"""Two steps per launch (LBM_PATH_FUSED2): bit-identical to the fused step
on every shape class the strip and segment plan distinguishes, and within
the FP64 tolerance of the oracle.

Shapes: the lowest lattice the kernel takes (64 rows, one strip touching
both walls), 65 and 125 rows (two and three strips, the last strip's base
off the 58-row grid), a width of 3 (every column wraps, the segment of 9
columns steps each one three times), 7 columns, lattices of several
segments with a ragged last one, the full height of the benchmark on a
narrow lattice, and odd step counts (the last step takes the fused
kernel)."""
import numpy as np
import pytest

import oracle
from gpu_helpers import FP64_TOL, LAYOUTS, err_metric, lattice, need_gpu, noisy_state
from paper_1703_00185_amd import inputs, lbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _both(ns, rt, steps, **kw):
    out = []
    for path in (lbm.LBM_PATH_FUSED, lbm.LBM_PATH_FUSED2):
        with lattice(ns, path=path, **kw) as lat:
            lat.init_rt(rt)
            for n in steps:
                lat.step(n)
            out.append(lat.get())
    return out


@pytest.mark.parametrize("lx,ly,steps", [
    (64, 64, (2,)), (3, 64, (4,)), (7, 65, (2,)), (130, 125, (4,)), (67, 131, (3,)),
    (130, 257, (6,)), (515, 700, (4,)), (33, 1000, (2,)), (1100, 300, (2,)), (256, 8192, (2,)),
    (64, 128, (1, 2, 3, 2)),
])
def test_two_step_equals_fused(lx, ly, steps):
    ns = inputs.rt_config(lx, ly)
    a, b = _both(ns, inputs.rt_perturbation(5, ly), steps)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_two_step_equals_fused_layouts_and_padding(layout):
    """Strides come from the geometry: the planar layout and padded pitches."""
    ns = inputs.rt_config(131, 190)
    a, b = _both(ns, inputs.rt_perturbation(6, 190), (4,), layout=layout, ny_pad=64, stride_pad=96)
    assert np.array_equal(a, b)


def test_two_step_short_lattice_takes_fused_steps():
    """Below 64 rows the path steps with the fused kernel."""
    ns = inputs.rt_config(40, 50)
    a, b = _both(ns, inputs.rt_perturbation(7, 50), (4,))
    assert np.array_equal(a, b)


def test_two_step_matches_oracle_from_noisy_state():
    """100 steps of the 64 x 128 workload from a state off equilibrium
    (every population differs from its neighbours), against the oracle."""
    ns = inputs.rt_config(64, 128)
    f0 = noisy_state(11, 64, 128)
    with lattice(ns, path=lbm.LBM_PATH_FUSED2) as lat:
        lat.set(f0)
        lbm.lbm_set_timing(lat.h, True)
        lat.step(100)
        ms, cnt = lbm.lbm_read_timing(lat.h)
        got = lat.get()
    assert cnt[lbm.LBM_PHASE_FUSED2] == 50 and cnt[lbm.LBM_PHASE_FUSED] == 0
    assert err_metric(got, oracle.run(f0, ns, 100)) < FP64_TOL


def test_two_step_full_size_sampled():
    """The benchmark's 2048 x 8192 lattice, two steps, at sampled sites
    (walls, wrapped edge columns, strip and segment boundaries, random),
    equal to two fused steps."""
    lx, ly = 2048, 8192
    ns = inputs.rt_config(lx, ly)
    rng = np.random.default_rng(3)
    strip_rows = np.array([0, 1, 2, 3, 60, 61, 62, 63, 118, 119, 8120, 8128, 8180, 8181, ly - 4, ly - 3,
                           ly - 2, ly - 1])
    seg_cols = np.array([0, 1, 2, 292, 293, 294, 585, 586, 1757, 1758, lx - 3, lx - 2, lx - 1])
    xs = np.concatenate([rng.integers(0, lx, 6000), np.repeat(seg_cols, strip_rows.size)]).astype(np.int32)
    ys = np.concatenate([rng.integers(0, ly, 6000), np.tile(strip_rows, seg_cols.size)]).astype(np.int32)
    out = []
    for path in (lbm.LBM_PATH_FUSED, lbm.LBM_PATH_FUSED2):
        with lattice(ns, path=path) as lat:
            lat.init_rt(inputs.rt_perturbation(0, ly))
            lat.step(2)
            out.append(lbm.lbm_get_sites(lat.h, xs, ys))
    assert np.array_equal(out[0], out[1])


def test_two_step_captured_equals_plain():
    """Graph-replayed two-step launches (the side stream forked and joined
    inside the capture), odd and even counts, replayed with eager work in
    between, equal plain steps."""
    ns = inputs.rt_config(130, 200)
    rt = inputs.rt_perturbation(8, 200)
    p = lbm.LBM_PATH_FUSED2
    with lattice(ns, path=p) as a, lattice(ns, path=p) as b:
        a.init_rt(rt)
        b.init_rt(rt)
        for n in (4, 3, 4, 4, 1, 2):
            a.step(n)
            b.step_captured(n)
            assert np.array_equal(a.get(), b.get()), n
            b.conservation()


def test_two_step_on_a_user_stream():
    """Bound to a stream of the caller's (not the null stream): the wall
    launch on the library's second stream is still ordered inside each
    step call, so reading back right after equals the fused path."""
    import torch
    ns = inputs.rt_config(200, 190)
    rt = inputs.rt_perturbation(9, 190)
    with lattice(ns) as ref:
        ref.init_rt(rt)
        ref.step(6)
        want = ref.get()
    side = torch.cuda.Stream()
    lat = lbm.Lattice(lbm.config_from(ns, path=lbm.LBM_PATH_FUSED2), stream=side)
    try:
        lat.init_rt(rt)
        lat.step(2)
        lat.step(4)
        got = lat.get()
    finally:
        lat.close()
    assert np.array_equal(got, want)
