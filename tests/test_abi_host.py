"""Host-side checks of the C ABI (no GPU needed, no kernel launched).

* The library loads and exports every entry point include/lbm.h declares.
* Its model tables equal the oracle's independently solved constants bit
  for bit, and its wall factors K_l(T) equal the oracle's bit for bit (bc is
  checked bit-exact on the GPU, so both sides must start from equal factors).
* Config validation and lbm_create argument checks return the documented
  codes before any HIP call.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1703_00185_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_entry_points():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_entry_point():
    lib = lbm.load()
    names = _declared_entry_points()
    assert len(names) >= 19
    for name in names:
        assert hasattr(lib, name), name


def test_tables_equal_oracle_constants():
    e, opp, w, r = lbm.lbm_tables()
    k = oracle.constants()
    assert np.array_equal(e, k.E.astype(np.int32))
    assert np.array_equal(opp, k.opp.astype(np.int32))
    assert r == k.r
    assert np.array_equal(w, k.w)  # bit-equal binary64


@pytest.mark.parametrize("t", [0.9, 0.95, 1.0, 1.05, 1.1, 1.2345678901234567])
def test_wall_factors_bit_equal(t):
    assert lbm.lbm_wall_factors(t).tolist() == oracle.wall_factors(t)


def test_required_bytes_layout():
    cfg = lbm.lbm_config_default(64, 128)
    assert cfg.layout == lbm.LBM_LAYOUT_COLUMN
    nx, ny = 64 + 6, 128
    for layout, pad, elems in ((lbm.LBM_LAYOUT_COLUMN, -1, nx * 37 * ny),
                               (lbm.LBM_LAYOUT_PLANAR, -1, 37 * (-(-nx * ny // 64) * 64)),
                               (lbm.LBM_LAYOUT_COLUMN, 10, nx * (37 * ny + 10)),
                               (lbm.LBM_LAYOUT_PLANAR, 10, 37 * (-(-nx * ny // 64) * 64 + 10))):
        cfg.layout, cfg.stride_pad = layout, pad
        assert lbm.lbm_required_bytes(cfg) == 2 * (-(-elems * 8 // 256) * 256)


def test_config_from_rejects_unknown_fields():
    from paper_1703_00185_amd import inputs
    with pytest.raises(TypeError):
        lbm.config_from(inputs.rt_config(64, 128), plane_pad=3)


@pytest.mark.parametrize("field,value,needle", [
    ("lx", 2, "lx"), ("ly", 5, "ly"), ("tau", 0.5, "tau"), ("tau", float("nan"), "tau"),
    ("t_bottom", 0.0, "temperature"), ("t_top", -1.0, "temperature"),
    ("gy", float("inf"), "gravity"), ("storage", 7, "storage"), ("path", 4, "path"),
    ("block", 96, "block"), ("layout", 2, "layout"), ("layout", -1, "layout"),
])
def test_invalid_config_rejected(field, value, needle):
    cfg = lbm.lbm_config_default(64, 128)
    setattr(cfg, field, value)
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_required_bytes(cfg)
    assert ei.value.status == lbm.LBM_EINVAL
    assert needle in str(ei.value)
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create(cfg, 1 << 20, 1 << 40, 0)
    assert ei.value.status == lbm.LBM_EINVAL


@pytest.mark.parametrize("storage", [lbm.LBM_FP32, lbm.LBM_FP16DEV])
def test_two_step_path_takes_binary64_storage_only(storage):
    cfg = lbm.lbm_config_default(64, 128)
    cfg.path = lbm.LBM_PATH_FUSED2
    assert lbm.lbm_required_bytes(cfg) > 0
    cfg.storage = storage
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_required_bytes(cfg)
    assert ei.value.status == lbm.LBM_EINVAL and "LBM_PATH_FUSED2" in str(ei.value)


def test_lattice_too_large_rejected():
    cfg = lbm.lbm_config_default(40000, 40000)
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_required_bytes(cfg)
    assert "too large" in str(ei.value)


def test_create_argument_checks_before_device_calls():
    cfg = lbm.lbm_config_default(64, 128)
    need = lbm.lbm_required_bytes(cfg)
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create(cfg, 0, need, 0)
    assert ei.value.status == lbm.LBM_EINVAL
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create(cfg, 4096 + 8, need, 0)
    assert ei.value.status == lbm.LBM_ENOMEM and "aligned" in str(ei.value)
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create(cfg, 4096, need - 1, 0)
    assert ei.value.status == lbm.LBM_ENOMEM
    lib = lbm.load()
    assert lib.lbm_create(ctypes.byref(cfg), ctypes.c_void_p(4096), need, None, None) == lbm.LBM_EINVAL


def test_null_handle_calls_are_rejected():
    lib = lbm.load()
    assert lib.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert lib.lbm_run_phase(None, 0) == lbm.LBM_EINVAL
    assert lib.lbm_conservation(None, None) == lbm.LBM_EINVAL
    lbm.lbm_destroy(None)  # accepted
    assert isinstance(lbm.lbm_last_error(None), str)
