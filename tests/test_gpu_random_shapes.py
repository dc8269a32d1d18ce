"""Seeded random lattice shapes, paths, storages, layouts and work-group
sizes against the oracle.

Each case draws Lx in [3, 150] (every column is an edge column below 7)
and Ly in [6, 700] (mostly not a multiple of 64), a path, a storage, a
population layout and a work-group size, and checks one step from an
oracle-made state: binary64 within the FP64 bar, binary32 and binary16
deviations within one unit in the last place of the stored type of the
oracle's step under the same storage rule.  In binary64, three more steps
must give the same bits on the path drawn and on the separate path.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import FP64_TOL, err_metric, lattice, need_gpu, noisy_state, note
from paper_1703_00185_amd import inputs, lbm

pytestmark = pytest.mark.gpu

PATHS = [lbm.LBM_PATH_SEPARATE, lbm.LBM_PATH_FUSED, lbm.LBM_PATH_REGIONS]
STORAGES = [("fp64", lbm.LBM_FP64), ("fp32", lbm.LBM_FP32), ("fp16dev", lbm.LBM_FP16DEV)]
LAYOUTS = [lbm.LBM_LAYOUT_COLUMN, lbm.LBM_LAYOUT_PLANAR]
BLOCKS = [0, 64, 128, 256, 512, 1024]


def _cases(n=24, seed=20241202):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        lx = int(rng.integers(3, 151))
        ly = int(rng.integers(6, 701))
        out.append((i, lx, ly, PATHS[rng.integers(3)], STORAGES[rng.integers(3)],
                    LAYOUTS[rng.integers(2)], BLOCKS[rng.integers(len(BLOCKS))]))
    return out


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _ulps(got, want, name, ref):
    if name == "fp32":
        a = got.astype(np.float32).view(np.int32).astype(np.int64)
        b = want.astype(np.float32).view(np.int32).astype(np.int64)
        return int(np.max(np.abs(a - b)))
    da = oracle.encode_fp16dev(got, ref).astype(np.float64)
    db = oracle.encode_fp16dev(want, ref)
    return float(np.max(np.abs(da - db.astype(np.float64)) / np.spacing(np.abs(db)).astype(np.float64)))


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"{c[0]}-{c[1]}x{c[2]}")
def test_random_shape_step(case):
    i, lx, ly, path, (name, storage), layout, block = case
    ns = inputs.rt_config(lx, ly, tau=0.6 + 0.05 * (i % 8), gravity=1e-4 * (1 + i % 3),
                          t_bottom=1.0 + 0.01 * (i % 7), t_top=1.0 - 0.01 * (i % 5))
    ref = rows = None
    f = noisy_state(i, lx, ly)
    if name == "fp16dev":
        flat = inputs.flat_interface(ly)
        _, rho = oracle.rt_fields(1, ly, ns, flat)
        rows = (rho[0].copy(), ns.t_bottom, ns.t_top, int(np.ceil(flat.y_center)))
        ref = oracle.fp16dev_reference(*rows)
    f = oracle.stored(f, name, ref)
    with lattice(ns, path=path, storage=storage, layout=layout, block=block) as lat:
        if rows is not None:
            lbm.lbm_set_reference(lat.h, *rows)
        lat.set(f)
        lat.step(1)
        got = lat.get()
        lat.step(3)
        four = lat.get()
    if name == "fp64":
        e = err_metric(got, oracle.step(f, ns))
        note(f"case {case}: err {e:.2e}")
        assert e < FP64_TOL
    else:
        want = oracle.step_stored(f, ns, name, fused=path != lbm.LBM_PATH_SEPARATE, ref=ref)
        u = _ulps(got, want, name, ref)
        note(f"case {case}: {u} ulp")
        assert u <= 1
    with lattice(ns, path=lbm.LBM_PATH_SEPARATE, storage=storage, layout=layout, block=block) as lat:
        if rows is not None:
            lbm.lbm_set_reference(lat.h, *rows)
        lat.set(f)
        lat.step(4)
        sep = lat.get()
    if name == "fp64" or path == lbm.LBM_PATH_SEPARATE:
        assert np.array_equal(four, sep)
