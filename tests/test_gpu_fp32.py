"""FP32 population storage (binary64 arithmetic, binary32 in memory).

Bars:
* propagate moves stored values: bit-exact;
* bc: bit-exact against the oracle's bc rounded to binary32 (the fold and
  the product are binary64 on both sides, then one rounding);
* one fused or separate step: within one binary32 ulp per value of the
  oracle's step_stored (both round the same binary64 value, which the two
  sides compute equal to ~1e-16, so only values at a rounding boundary can
  land one ulp apart);
* 100 steps of the 64 x 128 workload: within 1e-6 (weight-scaled metric)
  of the oracle under the same storage rule, and the FP32-vs-FP64 error is
  reported and bounded by 100 steps x 2^-24 relative rounding per step.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import LAYOUTS, err_metric, lattice, need_gpu, noisy_state, note
from paper_1703_00185_amd import inputs, lbm

pytestmark = pytest.mark.gpu

SIZES = [(3, 6), (5, 9), (37, 70), (64, 128), (130, 257)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _fp32_state(seed, lx, ly):
    return oracle.stored(noisy_state(seed, lx, ly), "fp32")


def _within_one_ulp(got, ref):
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    return bool(np.all(np.abs(got - ref) <= ulp))


@pytest.mark.parametrize("lx,ly", SIZES)
def test_fp32_set_get_roundtrip_and_propagate(lx, ly):
    f = _fp32_state(1, lx, ly)
    with lattice(inputs.rt_config(lx, ly), path=lbm.LBM_PATH_SEPARATE, storage=lbm.LBM_FP32) as lat:
        lat.set(f)
        assert np.array_equal(lat.get(), f)
        lat.run_phase(lbm.LBM_PHASE_PBC)
        lat.run_phase(lbm.LBM_PHASE_PROPAGATE)
        got = lat.get()
    assert np.array_equal(got, oracle.propagate(f))


@pytest.mark.parametrize("lx,ly", SIZES)
def test_fp32_bc_bit_exact(lx, ly):
    ns = inputs.rt_config(lx, ly, t_bottom=1.08, t_top=0.97)
    f = _fp32_state(2, lx, ly)
    with lattice(ns, path=lbm.LBM_PATH_SEPARATE, storage=lbm.LBM_FP32) as lat:
        lat.set(f)
        lat.run_phase(lbm.LBM_PHASE_BC)
        got = lat.get()
    assert np.array_equal(got, oracle.stored(oracle.bc(f, ns.t_bottom, ns.t_top), "fp32"))


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("path", [lbm.LBM_PATH_SEPARATE, lbm.LBM_PATH_FUSED])
@pytest.mark.parametrize("lx,ly", SIZES)
def test_fp32_step_within_one_ulp(lx, ly, path, layout):
    ns = inputs.rt_config(lx, ly)
    f = _fp32_state(3, lx, ly)
    with lattice(ns, path=path, storage=lbm.LBM_FP32, layout=layout) as lat:
        lat.set(f)
        lat.step(1)
        got = lat.get()
    ref = oracle.step_stored(f, ns, "fp32", fused=path == lbm.LBM_PATH_FUSED)
    assert _within_one_ulp(got, ref)
    frac = float(np.mean(got != ref))
    note(f"fp32 {lx}x{ly} path={path}: {frac:.2e} of values one ulp apart")
    assert frac < 1e-3


def test_fp32_trajectory_64x128_100_steps():
    ns = inputs.rt_config(64, 128)
    f64 = oracle.init_rt(64, 128, ns, inputs.rt_perturbation(0, 128))
    f32 = oracle.stored(f64, "fp32")
    with lattice(ns, storage=lbm.LBM_FP32) as lat:
        lat.set(f32)
        lat.step(100)
        got = lat.get()
    for _ in range(100):
        f32 = oracle.step_stored(f32, ns, "fp32", fused=True)
        f64 = oracle.step(f64, ns)
    e_same = err_metric(got, f32)
    e_fp64 = err_metric(got, f64)
    note(f"fp32 64x128 after 100 steps: vs fp32 oracle {e_same:.2e}, vs fp64 oracle {e_fp64:.2e}")
    assert e_same < 1e-6
    assert e_fp64 < 100 * 2.0 ** -24 * 2


def test_fp32_fused_and_separate_agree_off_the_walls():
    ns = inputs.rt_config(64, 128)
    out = []
    for path in (lbm.LBM_PATH_SEPARATE, lbm.LBM_PATH_FUSED):
        with lattice(ns, path=path, storage=lbm.LBM_FP32) as lat:
            lat.set(_fp32_state(5, 64, 128))
            lat.step(1)
            out.append(lat.get())
    assert np.array_equal(out[0][:, :, 3:125], out[1][:, :, 3:125])


def test_fp32_init_and_diagnostics():
    ns = inputs.rt_config(37, 70)
    rt = inputs.rt_perturbation(4, 70)
    with lattice(ns, storage=lbm.LBM_FP32) as lat:
        lat.init_rt(rt)
        f = lat.get()
        rho, ux, uy, T = lat.moments()
        cons = lat.conservation()
    ref = oracle.init_rt(37, 70, ns, rt)
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(f - ref) <= ulp)
    r2, ux2, uy2, T2 = oracle.moments(f)
    assert np.max(np.abs(rho - r2) / r2) < 1e-14
    assert np.max(np.abs(T - T2)) < 1e-13
    tot = oracle.totals(f)
    assert abs(cons[0] - tot[0]) < 1e-12 * tot[0]
    assert cons[4] == 0


def test_fp32_layout_halves_memory():
    cfg64 = lbm.lbm_config_default(2048, 8192)
    cfg32 = lbm.lbm_config_default(2048, 8192, storage=lbm.LBM_FP32)
    assert lbm.lbm_required_bytes(cfg32) * 2 == lbm.lbm_required_bytes(cfg64)
