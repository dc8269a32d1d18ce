"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Bars: propagate and bc bit-exact; collide, the fused step and whole
trajectories within 1e-12 (gpu_helpers.err_metric); fused and separate
paths bit-identical to each other, and the column and planar population
layouts bit-identical to each other.  Sizes span several work-group tiles
with ragged tails, down to the smallest lattice the ABI accepts (3 x 6).
Every oracle input is made by the oracle or the seeded input module.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import FP64_TOL, LAYOUTS, err_metric, lattice, need_gpu, noisy_state, note
from paper_1703_00185_amd import inputs, lbm

pytestmark = pytest.mark.gpu

SIZES = [(3, 6), (4, 7), (5, 9), (3, 13), (37, 70), (64, 128), (130, 257), (9, 1100)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("lx,ly", [(3, 6), (37, 70), (64, 128), (130, 257)])
def test_init_rt_matches_oracle(lx, ly, layout):
    ns = inputs.rt_config(lx, ly)
    rt = inputs.rt_perturbation(lx + ly, ly)
    with lattice(ns, layout=layout) as lat:
        lat.init_rt(rt)
        got = lat.get()
    ref = oracle.init_rt(lx, ly, ns, rt)
    assert err_metric(got, ref) < 1e-14


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("block", [64, 128, 256, 512, 1024])
@pytest.mark.parametrize("lx,ly", SIZES)
def test_propagate_bit_exact(lx, ly, block, layout):
    f = 1.0 + inputs.noise(lx * 1000 + ly, (37, lx, ly), 0.3)
    with lattice(inputs.rt_config(lx, ly), path=lbm.LBM_PATH_SEPARATE, block=block, layout=layout) as lat:
        lat.set(f)
        lat.run_phase(lbm.LBM_PHASE_PBC)
        lat.run_phase(lbm.LBM_PHASE_PROPAGATE)
        got = lat.get()
    assert np.array_equal(got, oracle.propagate(f))


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("lx,ly", SIZES)
def test_bc_bit_exact(lx, ly, layout):
    ns = inputs.rt_config(lx, ly, t_bottom=1.1, t_top=0.93)
    f = noisy_state(7, lx, ly)
    with lattice(ns, path=lbm.LBM_PATH_SEPARATE, layout=layout) as lat:
        lat.set(f)
        lat.run_phase(lbm.LBM_PHASE_BC)
        got = lat.get()
    assert np.array_equal(got, oracle.bc(f, ns.t_bottom, ns.t_top))


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("tau,gy", [(0.8, -1e-4), (0.55, -3e-4), (1.9, 2e-4)])
@pytest.mark.parametrize("lx,ly", [(5, 9), (64, 128), (130, 257)])
def test_collide_matches_oracle(lx, ly, tau, gy, layout):
    ns = inputs.rt_config(lx, ly, tau=tau, gravity=-gy)
    f = noisy_state(3, lx, ly)
    with lattice(ns, path=lbm.LBM_PATH_SEPARATE, layout=layout) as lat:
        lat.set(f)
        lat.run_phase(lbm.LBM_PHASE_COLLIDE)
        got = lat.get()
    e = err_metric(got, oracle.collide(f, ns.tau, ns.gx, ns.gy))
    note(f"collide {lx}x{ly} tau={tau} err={e:.2e}")
    assert e < FP64_TOL


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("block", [64, 128, 256, 512, 1024])
@pytest.mark.parametrize("lx,ly", SIZES)
def test_fused_phase_matches_oracle_step(lx, ly, block, layout):
    ns = inputs.rt_config(lx, ly)
    f = noisy_state(11, lx, ly)
    with lattice(ns, block=block, layout=layout) as lat:
        lat.set(f)
        lat.run_phase(lbm.LBM_PHASE_PBC)
        lat.run_phase(lbm.LBM_PHASE_FUSED)
        got = lat.get()
    assert err_metric(got, oracle.step(f, ns)) < FP64_TOL


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("path", [lbm.LBM_PATH_SEPARATE, lbm.LBM_PATH_FUSED])
def test_trajectory_64x128_100_steps(path, layout):
    """The small Rayleigh-Taylor workload, every one of its 100 steps."""
    ns = inputs.rt_config(64, 128)
    f = oracle.init_rt(64, 128, ns, inputs.rt_perturbation(0, 128))
    worst = 0.0
    with lattice(ns, path=path, layout=layout) as lat:
        lat.set(f)
        for s in range(100):
            lat.step(1)
            f = oracle.step(f, ns)
            worst = max(worst, err_metric(lat.get(), f))
    note(f"trajectory path={path} layout={layout} worst err over 100 steps {worst:.2e}")
    assert worst < FP64_TOL


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("lx,ly", [(3, 6), (5, 13), (67, 131), (130, 257)])
def test_short_runs_on_ragged_lattices(lx, ly, layout):
    ns = inputs.rt_config(lx, ly)
    f0 = oracle.init_rt(lx, ly, ns, inputs.rt_perturbation(5, ly))
    ref = oracle.run(f0, ns, 5)
    for path in (lbm.LBM_PATH_SEPARATE, lbm.LBM_PATH_FUSED):
        with lattice(ns, path=path, layout=layout) as lat:
            lat.set(f0)
            lat.step(5)
            assert err_metric(lat.get(), ref) < FP64_TOL


@pytest.mark.parametrize("lx,ly", [(64, 128), (130, 257)])
def test_fused_and_separate_paths_bit_identical(lx, ly):
    ns = inputs.rt_config(lx, ly)
    out = []
    for path in (lbm.LBM_PATH_SEPARATE, lbm.LBM_PATH_FUSED):
        with lattice(ns, path=path) as lat:
            lat.init_rt(inputs.rt_perturbation(1, ly))
            lat.step(20)
            out.append(lat.get())
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("storage", [lbm.LBM_FP64, lbm.LBM_FP32, lbm.LBM_FP16DEV])
@pytest.mark.parametrize("path", [lbm.LBM_PATH_SEPARATE, lbm.LBM_PATH_FUSED, lbm.LBM_PATH_REGIONS])
def test_column_and_planar_layouts_bit_identical(path, storage):
    """Only addresses differ between the layouts: same bits after 15 steps,
    also with padded pitches and strides."""
    ns = inputs.rt_config(67, 131)
    out = []
    for layout, ny_pad, stride_pad in ((lbm.LBM_LAYOUT_COLUMN, -1, -1), (lbm.LBM_LAYOUT_PLANAR, -1, -1),
                                       (lbm.LBM_LAYOUT_COLUMN, 64, 8), (lbm.LBM_LAYOUT_PLANAR, 3, 100)):
        with lattice(ns, path=path, layout=layout, storage=storage, ny_pad=ny_pad, stride_pad=stride_pad) as lat:
            lat.init_rt(inputs.rt_perturbation(9, 131))
            lat.step(15)
            out.append(lat.get())
    for o in out[1:]:
        assert np.array_equal(out[0], o)


@pytest.mark.parametrize("lx,ly,ny_pad,stride_pad", [(64, 128, -1, -1), (37, 70, 5, 3), (3, 6, 64, 64)])
def test_layout_strides_reported(lx, ly, ny_pad, stride_pad):
    ns = inputs.rt_config(lx, ly)
    nx = lx + 6
    ny = -(-ly // 64) * 64 + max(ny_pad, 0)
    pad = max(stride_pad, 0)
    with lattice(ns, layout=lbm.LBM_LAYOUT_COLUMN, ny_pad=ny_pad, stride_pad=stride_pad) as lat:
        assert lat.layout()[:4] == (nx, ny, ny, 37 * ny + pad)
        assert lat.layout()[4] == -(-nx * (37 * ny + pad) * 8 // 256) * 256
        assert lat.layout()[5] == 64  # fewer wavefronts than SIMDs
    with lattice(ns, layout=lbm.LBM_LAYOUT_PLANAR, ny_pad=ny_pad, stride_pad=stride_pad) as lat:
        plane = -(-nx * ny // 64) * 64 + pad
        assert lat.layout()[:4] == (nx, ny, plane, ny)
        assert lat.layout()[4] == -(-37 * plane * 8 // 256) * 256


def test_moments_match_oracle():
    ns = inputs.rt_config(37, 70)
    f = noisy_state(2, 37, 70)
    with lattice(ns) as lat:
        lat.set(f)
        rho, ux, uy, T = lat.moments()
    r2, ux2, uy2, T2 = oracle.moments(f)
    assert np.max(np.abs(rho - r2) / r2) < 1e-14
    assert np.max(np.abs(ux - ux2)) < 1e-14
    assert np.max(np.abs(uy - uy2)) < 1e-14
    assert np.max(np.abs(T - T2)) < 1e-13


def test_conservation_matches_oracle_and_is_deterministic():
    ns = inputs.rt_config(130, 257)
    f = noisy_state(4, 130, 257)
    with lattice(ns) as lat:
        lat.set(f)
        a = lat.conservation()
        b = lat.conservation()
    assert np.array_equal(a, b)
    ref = oracle.totals(f)
    for got, want in zip(a[:4], ref):
        assert abs(got - want) <= 1e-12 * max(1.0, abs(ref[0]))
    assert a[4] == 0


def test_nonfinite_populations_are_counted():
    ns = inputs.rt_config(16, 32)
    f = noisy_state(8, 16, 32)
    f[5, 3, 7] = np.nan
    f[30, 15, 31] = np.inf
    f[0, 0, 0] = -np.inf
    with lattice(ns) as lat:
        lat.set(f)
        assert lat.conservation()[4] == 3


@pytest.mark.parametrize("path", [lbm.LBM_PATH_FUSED, lbm.LBM_PATH_REGIONS])
def test_failure_detected_and_recovered_from_checkpoint(path):
    """A corrupted population (forced from the host) is caught by the
    non-finite count of the conservation reduction after it has spread;
    restoring the last checkpoint and stepping again gives the bits of an
    undisturbed run."""
    ns = inputs.rt_config(64, 128)
    rt = inputs.rt_perturbation(5, 128)
    with lattice(ns, path=path) as lat:
        lat.init_rt(rt)
        lat.step(6)
        straight_ckpt = lat.get()
        lat.step(6)
        straight = lat.get()
    with lattice(ns, path=path) as lat:
        lat.init_rt(rt)
        lat.step(6)
        ckpt = lat.get()
        assert np.array_equal(ckpt, straight_ckpt)
        bad = ckpt.copy()
        bad[17, 40, 64] = np.nan
        lat.set(bad)
        lat.step(3)
        # the pull spreads a value up to 3 sites per step; collide mixes all
        # 37 populations of a site
        assert lat.conservation()[4] > 37
        lat.set(ckpt)
        assert lat.conservation()[4] == 0
        lat.step(6)
        assert np.array_equal(lat.get(), straight)


def test_mass_conserved_over_200_steps():
    ns = inputs.rt_config(64, 128)
    with lattice(ns) as lat:
        lat.init_rt(inputs.rt_perturbation(9, 128))
        m0 = lat.conservation()[0]
        lat.step(200)
        m1 = lat.conservation()[0]
    drift = abs(m1 - m0) / m0
    note(f"mass drift over 200 steps {drift:.2e}")
    assert drift < 1e-13 * np.sqrt(200)


def test_x_invariant_state_stays_x_invariant():
    ns = inputs.rt_config(24, 96)
    with lattice(ns) as lat:
        lat.init_rt(inputs.flat_interface(96))
        lat.step(30)
        f = lat.get()
    assert all(np.array_equal(f[:, 0, :], f[:, x, :]) for x in range(24))


def test_uniform_rest_state_stays_uniform():
    ns = inputs.rt_config(16, 40, gravity=0.0, t_bottom=1.0, t_top=1.0)
    f0 = oracle.equilibrium(np.full((16, 40), 1.2), np.zeros((16, 40)), np.zeros((16, 40)),
                            np.ones((16, 40)))
    with lattice(ns) as lat:
        lat.set(f0)
        lat.step(25)
        f = lat.get()
    # spatially uniform (every site equal to the lattice mean up to rounding
    # of the smallest-weight populations) and still the initial state
    mean = f.mean(axis=(1, 2), keepdims=True)
    assert err_metric(f, np.broadcast_to(mean, f.shape)) < 1e-13
    assert err_metric(f, f0) < 1e-13


def test_determinism_and_checkpoint_resume():
    ns = inputs.rt_config(64, 128)
    rt = inputs.rt_perturbation(6, 128)
    with lattice(ns) as lat:
        lat.init_rt(rt)
        lat.step(10)
        ckpt = lat.get()
        lat.step(10)
        straight = lat.get()
    with lattice(ns) as lat:
        lat.set(ckpt)
        lat.step(10)
        resumed = lat.get()
    with lattice(ns) as lat:
        lat.init_rt(rt)
        lat.step(20)
        again = lat.get()
    assert np.array_equal(straight, resumed)
    assert np.array_equal(straight, again)


def test_get_sites_matches_full_copy():
    ns = inputs.rt_config(37, 70)
    f = noisy_state(12, 37, 70)
    xs = np.array([0, 36, 5, 17, 36, 0])
    ys = np.array([0, 69, 33, 2, 0, 69])
    with lattice(ns) as lat:
        lat.set(f)
        got = lat.sites(xs, ys)
        with pytest.raises(lbm.LbmError):
            lat.sites(np.array([37]), np.array([0]))
        with pytest.raises(lbm.LbmError):
            lat.sites(np.array([0]), np.array([-1]))
    assert np.array_equal(got, f[:, xs, ys])


def test_timing_counters_and_state_errors():
    ns = inputs.rt_config(64, 128)
    with lattice(ns) as lat:
        with pytest.raises(lbm.LbmError) as ei:
            lat.step(1)
        assert ei.value.status == lbm.LBM_ESTATE
        lat.init_rt(inputs.rt_perturbation(0, 128))
        with pytest.raises(lbm.LbmError) as ei:
            lat.step(-1)
        assert ei.value.status == lbm.LBM_EINVAL
        lbm.lbm_set_timing(lat.h, True)
        lat.step(3)
        ms, cnt = lbm.lbm_read_timing(lat.h)
        lbm.lbm_set_timing(lat.h, False)
    # the fused path is one launch per step (periodic x by wrapping, no pbc)
    assert cnt.tolist() == [0, 0, 0, 0, 3, 0, 0, 0]
    assert ms[4] > 0
    with lattice(ns, path=lbm.LBM_PATH_SEPARATE) as lat:
        lat.init_rt(inputs.rt_perturbation(0, 128))
        lbm.lbm_set_timing(lat.h, True)
        lat.step(2)
        ms, cnt = lbm.lbm_read_timing(lat.h)
    assert cnt.tolist() == [2, 2, 2, 2, 0, 0, 0, 0]
    assert all(ms[p] > 0 for p in range(4))


def test_runs_on_a_side_stream():
    import torch
    ns = inputs.rt_config(64, 128)
    f0 = oracle.init_rt(64, 128, ns, inputs.rt_perturbation(2, 128))
    side = torch.cuda.Stream()
    cfg = lbm.config_from(ns)
    lat = lbm.Lattice(cfg, stream=side)
    try:
        lat.set(f0)
        lat.step(3)
        got = lat.get()
    finally:
        lat.close()
    assert err_metric(got, oracle.run(f0, ns, 3)) < FP64_TOL


def test_host_memory_pointer_rejected():
    cfg = lbm.lbm_config_default(16, 32)
    need = lbm.lbm_required_bytes(cfg)
    host = np.zeros(need // 8 + 64)
    addr = (host.ctypes.data + 255) // 256 * 256
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create(cfg, addr, need, 0)
    assert ei.value.status in (lbm.LBM_EINVAL, lbm.LBM_EDEVICE)


@pytest.mark.parametrize("mode,shift", [(0, 0), (1, 3), (1, -3), (1, 0), (2, 1), (2, -2), (2, 64),
                                        (1, -64)])
def test_bandwidth_probe_copies(mode, shift):
    import torch
    n = 4096
    src = torch.arange(n // 8, dtype=torch.float64, device="cuda")
    dst = torch.full((n // 8,), -1.0, dtype=torch.float64, device="cuda")
    lbm.lbm_probe_bandwidth(mode, src.data_ptr(), dst.data_ptr(), n, shift,
                            torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    s, d = src.cpu().numpy(), dst.cpu().numpy()
    if mode == 0:
        assert np.array_equal(d, s)
        return
    m = n // 8 - 128
    i = np.arange(m)
    rs, ws = (64 + shift, 64) if mode == 1 else (64, 64 + shift)
    assert np.array_equal(d[i + ws], s[i + rs])
    untouched = np.setdiff1d(np.arange(n // 8), i + ws)
    assert np.all(d[untouched] == -1.0)


@pytest.mark.parametrize("n16", [128, 3109, 1000003, 65536 * 1024 + 12345])
def test_bandwidth_probe_copy_sizes(n16):
    """The copy probe moves every 16-byte vector exactly once: sizes that
    leave a partial pass, and one above the grid cap (several passes)."""
    import torch
    src = torch.randint(-2**62, 2**62, (2 * n16,), dtype=torch.int64, device="cuda")
    dst = torch.zeros(2 * n16 + 2, dtype=torch.int64, device="cuda")
    lbm.lbm_probe_bandwidth(0, src.data_ptr(), dst.data_ptr(), 16 * n16, 0,
                            torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(dst[:2 * n16], src)
    assert int(dst[2 * n16:].abs().sum()) == 0
    del src, dst
    torch.cuda.empty_cache()


def test_bandwidth_probe_rejects_bad_arguments():
    import torch
    buf = torch.empty(4096, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    for args in [(3, 0), (0, 1), (1, 65)]:
        with pytest.raises(lbm.LbmError):
            lbm.lbm_probe_bandwidth(args[0], buf.data_ptr(), buf.data_ptr(), 4096, args[1], st)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_probe_bandwidth(0, buf.data_ptr() + 8, buf.data_ptr(), 2048, 0, st)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_probe_bandwidth(0, buf.data_ptr(), buf.data_ptr(), 1024, 0, st)


@pytest.mark.parametrize("storage,lx,ly,want", [
    (lbm.LBM_FP64, 8, 8192, 512), (lbm.LBM_FP32, 8, 8192, 256), (lbm.LBM_FP16DEV, 8, 8192, 64),
    (lbm.LBM_FP64, 256, 300, 512), (lbm.LBM_FP64, 256, 200, 256), (lbm.LBM_FP64, 512, 128, 128),
    (lbm.LBM_FP32, 1024, 100, 128), (lbm.LBM_FP64, 1024, 6, 64),
    # fewer wavefronts (lx * ceil(ly / 64)) than the 1024 SIMDs: one-wavefront groups
    (lbm.LBM_FP64, 64, 128, 64), (lbm.LBM_FP64, 8, 300, 64), (lbm.LBM_FP32, 127, 512, 64),
])
def test_default_work_group_size(storage, lx, ly, want):
    with lattice(inputs.rt_config(lx, ly), storage=storage) as lat:
        assert lat.layout()[5] == want
    with lattice(inputs.rt_config(lx, ly), storage=storage, block=1024) as lat:
        assert lat.layout()[5] == 1024


@pytest.mark.parametrize("path", [lbm.LBM_PATH_SEPARATE, lbm.LBM_PATH_FUSED, lbm.LBM_PATH_REGIONS])
def test_empty_requests_change_nothing(path):
    """Zero steps (plain and captured) and an empty site list are no-ops."""
    ns = inputs.rt_config(37, 70)
    with lattice(ns, path=path) as lat:
        lat.init_rt(inputs.rt_perturbation(4, 70))
        before = lat.get()
        lat.step(0)
        lat.step_captured(0)
        got = lat.sites(np.array([], dtype=np.int64), np.array([], dtype=np.int64))
        after = lat.get()
    assert got.shape == (37, 0)
    assert np.array_equal(before, after)
