"""The 2048 x 8192 Rayleigh-Taylor lattice, in the launch configuration the
benchmark times (fused path, default work-group size).

The oracle cannot step 16.8 M sites in a test, so it checks sampled sites
one by one: its own initial state is built only on the columns the samples
pull from (the rest of its array stays untouched zero pages), and
oracle.step_sites computes the step at the samples.  Samples cover the
halo-crossing columns, the wall rows, the first rows beyond the walls and
random interior sites.  Properties that hold at any size back this up:
mass conservation and bit-identity of the fused and separate paths.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import FP64_TOL, err_metric, lattice, need_gpu, note
from paper_1703_00185_amd import inputs, lbm

pytestmark = pytest.mark.gpu

LX, LY = 2048, 8192


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _samples():
    """Edge columns and 32 random columns; on each, the edge rows and 20
    random rows (so the oracle needs only ~14% of the columns)."""
    rng = np.random.default_rng(2024)
    cols = [0, 1, 2, 3, 1023, LX - 4, LX - 3, LX - 2, LX - 1]
    cols += sorted(set(rng.integers(4, LX - 4, 32).tolist()))
    edge_y = [0, 1, 2, 3, 4, 63, 64, 4095, 4096, LY - 5, LY - 4, LY - 3, LY - 2, LY - 1]
    xs, ys = [], []
    for x in cols:
        rows = edge_y + rng.integers(0, LY, 20).tolist()
        xs += [x] * len(rows)
        ys += rows
    return np.array(xs, dtype=np.int64), np.array(ys, dtype=np.int64)


def _oracle_initial_state(ns, rt, xs):
    """Oracle initial populations on the columns within 3 of the samples."""
    T, rho = oracle.rt_fields(LX, LY, ns, rt)
    f0 = np.zeros((37, LX, LY))
    cols = np.unique(((xs[:, None] + np.arange(-3, 4)[None, :]) % LX).ravel())
    for c0 in range(0, cols.size, 64):
        c = cols[c0:c0 + 64]
        f0[:, c, :] = oracle.equilibrium(rho[c], np.zeros_like(T[c]), np.zeros_like(T[c]), T[c])
    return f0


@pytest.mark.timeout(600)
def test_full_size_step_at_sampled_sites():
    ns = inputs.rt_config(LX, LY)
    rt = inputs.rt_perturbation(0, LY)
    xs, ys = _samples()
    note("oracle initial state on sampled columns")
    f0 = _oracle_initial_state(ns, rt, xs)
    ref_init = f0[:, xs, ys]
    ref_step = oracle.step_sites(f0, ns, xs, ys)
    with lattice(ns, path=lbm.LBM_PATH_FUSED) as lat:
        lat.init_rt(rt)
        init = lat.sites(xs, ys)
        m0 = lat.conservation()
        lat.step(1)
        step1 = lat.sites(xs, ys)
        lat.step(1)
        m2 = lat.conservation()
        fused2 = lat.sites(xs, ys)
    e_init = err_metric(init, ref_init)
    e_step = err_metric(step1, ref_step)
    note(f"2048x8192: init err {e_init:.2e}, step err {e_step:.2e}, "
         f"mass drift {abs(m2[0] - m0[0]) / m0[0]:.2e}")
    assert e_init < 1e-14
    assert e_step < FP64_TOL
    assert abs(m2[0] - m0[0]) / m0[0] < 1e-13
    assert m2[4] == 0

    with lattice(ns, path=lbm.LBM_PATH_SEPARATE) as lat:
        lat.init_rt(rt)
        lat.step(2)
        sep2 = lat.sites(xs, ys)
    assert np.array_equal(sep2, fused2)


def _stored_at_sites(g, storage, ref_rows, ys):
    """oracle.stored() of populations g[37, n] at sites with rows ys
    (ref_rows: the deviation reference of oracle.fp16dev_reference)."""
    if storage == "fp32":
        return oracle.stored(g, "fp32")
    return oracle.stored(g[:, None, :], "fp16dev", (ref_rows[0][:, ys], ref_rows[1][:, ys]))[:, 0, :]


def _ulps_apart(got, want, storage, ref_rows, ys):
    """Largest distance in units in the last place of the stored type."""
    if storage == "fp32":
        a, b = got.astype(np.float32), want.astype(np.float32)
        return float(np.max(np.abs(a.view(np.int32).astype(np.int64) - b.view(np.int32).astype(np.int64))))
    r = (ref_rows[0][:, ys], ref_rows[1][:, ys])
    da = oracle.encode_fp16dev(got[:, None, :], r)[:, 0, :].astype(np.float64)
    db = oracle.encode_fp16dev(want[:, None, :], r)[:, 0, :]
    return float(np.max(np.abs(da - db.astype(np.float64)) / np.spacing(np.abs(db)).astype(np.float64)))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("storage", ["fp32", "fp16dev"])
def test_full_size_reduced_storage_step_at_sampled_sites(storage):
    """FP32 and FP16-deviation storage at 2048 x 8192 in the benchmark's
    launch configuration: the GPU's stored initial state is the oracle's
    initial state in the storage type, and one fused step equals the
    oracle's step of that stored state, stored once after collide, to 2
    units in the last place of the stored type (the GPU's own exp/tanh/log
    may put an initial value one unit to the other side of a rounding
    boundary)."""
    ns = inputs.rt_config(LX, LY)
    rt = inputs.rt_perturbation(0, LY)
    xs, ys = _samples()
    code = lbm.LBM_FP32 if storage == "fp32" else lbm.LBM_FP16DEV
    ref_rows = None
    if storage == "fp16dev":
        flat = inputs.flat_interface(LY)
        _, rho = oracle.rt_fields(1, LY, ns, flat)
        ref_rows = oracle.fp16dev_reference(rho[0], ns.t_bottom, ns.t_top, int(np.ceil(flat.y_center)))
    note(f"oracle initial state on sampled columns ({storage})")
    f0 = _oracle_initial_state(ns, rt, xs)
    cols = np.unique(((xs[:, None] + np.arange(-3, 4)[None, :]) % LX).ravel())
    for c0 in range(0, cols.size, 64):
        c = cols[c0:c0 + 64]
        f0[:, c, :] = oracle.stored(f0[:, c, :], storage, ref_rows)
    want_init = f0[:, xs, ys]
    want_step = _stored_at_sites(oracle.step_sites(f0, ns, xs, ys), storage, ref_rows, ys)
    with lattice(ns, path=lbm.LBM_PATH_FUSED, storage=code) as lat:
        lat.init_rt(rt)
        got_init = lat.sites(xs, ys)
        lat.step(1)
        got_step = lat.sites(xs, ys)
        cons = lat.conservation()
    u_init = _ulps_apart(got_init, want_init, storage, ref_rows, ys)
    u_step = _ulps_apart(got_step, want_step, storage, ref_rows, ys)
    note(f"2048x8192 {storage}: init {u_init:.0f} ulp, step {u_step:.0f} ulp, "
         f"{np.mean(got_step != want_step):.2e} of values differ")
    assert u_init <= 1
    assert u_step <= 2
    assert cons[4] == 0


@pytest.mark.timeout(600)
@pytest.mark.parametrize("storage", [lbm.LBM_FP64, lbm.LBM_FP16DEV])
def test_full_size_planar_equals_column_layout(storage):
    """At 2048 x 8192 the planar layout (population planes 37 x 16.8 M
    elements apart, element offsets past 2^32 bytes) and the benchmark's
    column layout give the same bits after three fused steps: at the
    sampled sites and in the conservation sums, which read every site in a
    fixed order."""
    ns = inputs.rt_config(LX, LY)
    rt = inputs.rt_perturbation(1, LY)
    xs, ys = _samples()
    out = {}
    for layout in (lbm.LBM_LAYOUT_COLUMN, lbm.LBM_LAYOUT_PLANAR):
        with lattice(ns, path=lbm.LBM_PATH_FUSED, layout=layout, storage=storage) as lat:
            lat.init_rt(rt)
            lat.step(3)
            out[layout] = (lat.sites(xs, ys), lat.conservation())
    col, pla = out[lbm.LBM_LAYOUT_COLUMN], out[lbm.LBM_LAYOUT_PLANAR]
    assert np.array_equal(col[0], pla[0])
    assert np.array_equal(col[1], pla[1])
    assert col[1][4] == 0


@pytest.mark.timeout(600)
def test_wide_planar_binary16_equals_column_layout():
    """Binary16 deviations on 4096 x 8192: in the planar layout the 37
    population planes of a column span 2.5 GB, past the 2^31-byte range
    of one buffer descriptor, so the fused kernel addresses each run with
    its own descriptor; in the column layout one descriptor per column with
    scalar run offsets covers them.  Both give the same bits after two
    fused steps, at sampled sites (edge columns, walls, the layer boundary
    of the reference, random rows) and in the conservation sums."""
    lx, ly = 4096, LY
    ns = inputs.rt_config(lx, ly)
    rt = inputs.rt_perturbation(2, ly)
    rng = np.random.default_rng(7)
    cols = [0, 1, 2, 3, lx // 2, lx - 4, lx - 3, lx - 2, lx - 1] + rng.integers(4, lx - 4, 24).tolist()
    rows = [0, 2, 3, 63, 64, 4093, 4095, 4096, 4098, 4160, ly - 4, ly - 1]
    xs = np.repeat(np.array(cols, dtype=np.int64), len(rows) + 12)
    ys = np.concatenate([rows + rng.integers(0, ly, 12).tolist() for _ in cols]).astype(np.int64)
    out = {}
    for layout in (lbm.LBM_LAYOUT_COLUMN, lbm.LBM_LAYOUT_PLANAR):
        with lattice(ns, path=lbm.LBM_PATH_FUSED, layout=layout, storage=lbm.LBM_FP16DEV) as lat:
            lat.init_rt(rt)
            lat.step(2)
            out[layout] = (lat.sites(xs, ys), lat.conservation())
    col, pla = out[lbm.LBM_LAYOUT_COLUMN], out[lbm.LBM_LAYOUT_PLANAR]
    assert np.array_equal(col[0], pla[0])
    assert np.array_equal(col[1], pla[1])
    assert col[1][4] == 0


@pytest.mark.timeout(600)
@pytest.mark.parametrize("storage", [lbm.LBM_FP64, lbm.LBM_FP16DEV])
def test_tall_narrow_lattice_step_at_sampled_sites(storage):
    """The narrowest lattice (Lx = 3: every column pulls across the periodic
    boundary on both sides) at 2^17 rows (2048 wavefronts per column, row
    offsets far past one work-group tile), weak gravity so the hydrostatic
    density stays within a factor of 1.2: one fused step at sampled rows of
    all three columns against the oracle (FP64 to the tolerance; binary16
    deviations to 2 units in the last place of the oracle's stored step),
    and two fused steps equal to two separate steps."""
    lx, ly = 3, 1 << 17
    ns = inputs.rt_config(lx, ly, gravity=1e-6)
    rt = inputs.rt_perturbation(3, ly)
    rng = np.random.default_rng(11)
    rows = np.concatenate([[0, 1, 2, 3, 63, 64, ly // 2 - 1, ly // 2, ly // 2 + 1, ly - 4, ly - 3, ly - 1],
                           rng.integers(0, ly, 40)])
    xs = np.repeat(np.arange(lx, dtype=np.int64), rows.size)
    ys = np.tile(rows.astype(np.int64), lx)
    f0 = oracle.init_rt(lx, ly, ns, rt)
    ref_rows = state = None
    if storage == lbm.LBM_FP16DEV:
        flat = inputs.flat_interface(ly)
        _, rho = oracle.rt_fields(1, ly, ns, flat)
        state = (rho[0].copy(), ns.t_bottom, ns.t_top, int(np.ceil(flat.y_center)))
        ref_rows = oracle.fp16dev_reference(*state)
        f0 = oracle.stored(f0, "fp16dev", ref_rows)
    want = oracle.step_sites(f0, ns, xs, ys)
    out = {}
    for path in (lbm.LBM_PATH_FUSED, lbm.LBM_PATH_SEPARATE):
        with lattice(ns, path=path, storage=storage) as lat:
            lat.init_rt(rt)
            if storage == lbm.LBM_FP16DEV:
                # the oracle's reference and stored initial state, so that
                # the step alone is compared
                lbm.lbm_set_reference(lat.h, *state)
                lat.set(f0)
            lat.step(1)
            out[path, 1] = lat.sites(xs, ys)
            lat.step(1)
            out[path, 2] = lat.sites(xs, ys)
            cons = lat.conservation()
        assert cons[4] == 0
    got = out[lbm.LBM_PATH_FUSED, 1]
    if storage == lbm.LBM_FP64:
        e = err_metric(got, want)
        note(f"{lx}x{ly} fp64: one fused step, err {e:.2e}")
        assert e < FP64_TOL
        assert np.array_equal(out[lbm.LBM_PATH_FUSED, 2], out[lbm.LBM_PATH_SEPARATE, 2])
    else:
        u = _ulps_apart(got, _stored_at_sites(want, "fp16dev", ref_rows, ys), "fp16dev", ref_rows, ys)
        note(f"{lx}x{ly} fp16dev: one fused step within {u:.0f} ulp of the oracle's stored step")
        assert u <= 2
