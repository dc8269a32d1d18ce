"""Thin ctypes binding of libd2q37.so (the C ABI of include/lbm.h).

Each lbm_* function here has the name of the C entry point and only
marshals arguments: it converts Python/numpy values to C types, calls the
library, and raises LbmError with the library's message on a non-zero
status.  All computation happens in the HIP library.  PyTorch is used only
by `Lattice` to own the device memory and pick the stream.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

# The in-tree build of the library (paper_1703_00185_amd/build.py).
LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libd2q37.so")

NPOP = 37
MAX_MODES = 32
LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ESTATE = 0, -1, -2, -3, -4
LBM_FP64, LBM_FP32, LBM_FP16DEV = 0, 1, 2
LBM_PATH_SEPARATE, LBM_PATH_FUSED, LBM_PATH_REGIONS, LBM_PATH_FUSED2 = 0, 1, 2, 3
LBM_LAYOUT_COLUMN, LBM_LAYOUT_PLANAR = 0, 1
(LBM_PHASE_PBC, LBM_PHASE_PROPAGATE, LBM_PHASE_BC, LBM_PHASE_COLLIDE,
 LBM_PHASE_FUSED, LBM_PHASE_FUSED_BULK, LBM_PHASE_FUSED_BORDER, LBM_PHASE_FUSED2) = range(8)
LBM_NPHASES = 8
PHASE_NAMES = ("pbc", "propagate", "bc", "collide", "fused", "fused_bulk", "fused_border", "fused2")
STATUS_NAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE", -4: "LBM_ESTATE"}


class LbmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class lbm_config(ctypes.Structure):
    _fields_ = [("lx", c_int32), ("ly", c_int32), ("tau", c_double), ("gx", c_double),
                ("gy", c_double), ("t_bottom", c_double), ("t_top", c_double),
                ("storage", c_int32), ("path", c_int32), ("layout", c_int32), ("block", c_int32),
                ("ny_pad", c_int32), ("stride_pad", c_int64)]


class lbm_rt_params(ctypes.Structure):
    _fields_ = [("width", c_double), ("y_center", c_double), ("n_modes", c_int32),
                ("amp", POINTER(c_double)), ("phase", POINTER(c_double))]


_lib = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1703_00185_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    H = c_void_p
    sig = {
        "lbm_config_default": (c_int, [POINTER(lbm_config), c_int32, c_int32]),
        "lbm_required_bytes": (c_size_t, [POINTER(lbm_config)]),
        "lbm_create": (c_int, [POINTER(lbm_config), c_void_p, c_size_t, c_void_p, POINTER(H)]),
        "lbm_set_stream": (c_int, [H, c_void_p]),
        "lbm_init_rt": (c_int, [H, POINTER(lbm_rt_params)]),
        "lbm_step": (c_int, [H, c_int32]),
        "lbm_step_captured": (c_int, [H, c_int32]),
        "lbm_run_phase": (c_int, [H, c_int32]),
        "lbm_moments": (c_int, [H, c_void_p, c_void_p, c_void_p, c_void_p]),
        "lbm_conservation": (c_int, [H, c_void_p]),
        "lbm_get_populations": (c_int, [H, c_void_p]),
        "lbm_set_populations": (c_int, [H, c_void_p]),
        "lbm_get_sites": (c_int, [H, c_int32, c_void_p, c_void_p, c_void_p]),
        "lbm_get_sites_noalloc": (c_int, [H, c_int32, c_void_p, c_void_p, c_void_p]),
        "lbm_set_reference": (c_int, [H, c_void_p, c_double, c_double, c_int32]),
        "lbm_get_reference": (c_int, [H, c_void_p, c_void_p, c_void_p]),
        "lbm_set_timing": (c_int, [H, c_int32]),
        "lbm_read_timing": (c_int, [H, c_void_p, c_void_p]),
        "lbm_layout": (c_int, [H, c_void_p]),
        "lbm_tables": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
        "lbm_wall_factors": (c_int, [c_double, c_void_p]),
        "lbm_probe_bandwidth": (c_int, [c_int32, c_void_p, c_void_p, c_size_t, c_int32, c_void_p]),
        "lbm_engine_required_bytes": (c_size_t, [c_int32]),
        "lbm_engine_create": (c_int, [c_int32, c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]),
        "lbm_engine_add": (c_int, [c_void_p, H, c_int32, c_void_p]),
        "lbm_engine_remove": (c_int, [c_void_p, c_int32]),
        "lbm_engine_step": (c_int, [c_void_p, c_int32]),
        "lbm_engine_status": (c_int, [c_void_p, c_void_p]),
        "lbm_engine_set_tiling": (c_int, [c_void_p, c_int32, c_int32, c_int32]),
        "lbm_engine_get_tiling": (c_int, [c_void_p, c_void_p]),
        "lbm_engine_tune": (c_int, [c_void_p, c_int32, c_void_p, c_void_p]),
        "lbm_engine_last_error": (c_char_p, [c_void_p]),
        "lbm_engine_destroy": (None, [c_void_p]),
        "lbm_last_error": (c_char_p, [H]),
        "lbm_destroy": (None, [H]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _check(status: int, h=None) -> None:
    if status != LBM_OK:
        raise LbmError(status, lbm_last_error(h))


def lbm_last_error(h=None) -> str:
    msg = load().lbm_last_error(h)
    return msg.decode() if msg else ""


def lbm_config_default(lx: int, ly: int, **overrides) -> lbm_config:
    cfg = lbm_config()
    _check(load().lbm_config_default(byref(cfg), lx, ly))
    for k, v in overrides.items():
        if not hasattr(cfg, k):
            raise AttributeError(f"lbm_config has no field {k}")
        setattr(cfg, k, v)
    return cfg


def lbm_required_bytes(cfg: lbm_config) -> int:
    n = load().lbm_required_bytes(byref(cfg))
    if n == 0:
        raise LbmError(LBM_EINVAL, lbm_last_error(None))
    return int(n)


def lbm_create(cfg: lbm_config, dev_mem: int, dev_bytes: int, stream: int) -> c_void_p:
    h = c_void_p()
    _check(load().lbm_create(byref(cfg), c_void_p(dev_mem), dev_bytes, c_void_p(stream), byref(h)))
    return h


def lbm_set_stream(h, stream: int) -> None:
    _check(load().lbm_set_stream(h, c_void_p(stream)), h)


def lbm_init_rt(h, width: float, y_center: float, amps, phases) -> None:
    amps = np.ascontiguousarray(amps, dtype=np.float64)
    phases = np.ascontiguousarray(phases, dtype=np.float64)
    if amps.shape != phases.shape or amps.ndim != 1:
        raise ValueError("amps and phases must be 1-D arrays of equal length")
    p = lbm_rt_params(width, y_center, amps.size,
                      amps.ctypes.data_as(POINTER(c_double)), phases.ctypes.data_as(POINTER(c_double)))
    _check(load().lbm_init_rt(h, byref(p)), h)


def lbm_step(h, n: int) -> None:
    _check(load().lbm_step(h, n), h)


def lbm_step_captured(h, n: int) -> None:
    _check(load().lbm_step_captured(h, n), h)


def lbm_run_phase(h, phase: int) -> None:
    _check(load().lbm_run_phase(h, phase), h)


def lbm_moments(h, lx: int, ly: int):
    out = [np.empty((lx, ly), dtype=np.float64) for _ in range(4)]
    _check(load().lbm_moments(h, *[_ptr(a) for a in out]), h)
    return tuple(out)


def lbm_conservation(h) -> np.ndarray:
    out = np.empty(5, dtype=np.float64)
    _check(load().lbm_conservation(h, _ptr(out)), h)
    return out


def lbm_get_populations(h, lx: int, ly: int) -> np.ndarray:
    out = np.empty((NPOP, lx, ly), dtype=np.float64)
    _check(load().lbm_get_populations(h, _ptr(out)), h)
    return out


def lbm_set_populations(h, f: np.ndarray) -> None:
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.ndim != 3 or f.shape[0] != NPOP:
        raise ValueError("populations must have shape (37, lx, ly)")
    _check(load().lbm_set_populations(h, _ptr(f)), h)


def lbm_get_sites(h, xs, ys) -> np.ndarray:
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    if xs.shape != ys.shape or xs.ndim != 1:
        raise ValueError("xs and ys must be 1-D arrays of equal length")
    out = np.empty((NPOP, xs.size), dtype=np.float64)
    _check(load().lbm_get_sites(h, xs.size, _ptr(xs), _ptr(ys), _ptr(out)), h)
    return out


LBM_NOALLOC_MAX_SITES = 8192


def lbm_get_sites_noalloc(h, xs, ys) -> np.ndarray:
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    if xs.shape != ys.shape or xs.ndim != 1:
        raise ValueError("xs and ys must be 1-D arrays of equal length")
    out = np.empty((NPOP, xs.size), dtype=np.float64)
    _check(load().lbm_get_sites_noalloc(h, xs.size, _ptr(xs), _ptr(ys), _ptr(out)), h)
    return out


def lbm_set_reference(h, rho_ref, t_lo: float = 1.0, t_hi: float = 1.0, y_split: int = 0) -> None:
    rho_ref = np.ascontiguousarray(rho_ref, dtype=np.float64)
    _check(load().lbm_set_reference(h, _ptr(rho_ref), float(t_lo), float(t_hi), int(y_split)), h)


def lbm_get_reference(h, ly: int):
    """(rho_ref[ly], (t_lo, t_hi), y_split) of a deviation-storage lattice."""
    rho = np.empty(ly, dtype=np.float64)
    t = np.empty(2, dtype=np.float64)
    split = ctypes.c_int32(0)
    _check(load().lbm_get_reference(h, _ptr(rho), _ptr(t), ctypes.byref(split)), h)
    return rho, (float(t[0]), float(t[1])), int(split.value)


def lbm_set_timing(h, enable: bool) -> None:
    _check(load().lbm_set_timing(h, 1 if enable else 0), h)


def lbm_read_timing(h):
    ms = np.zeros(LBM_NPHASES, dtype=np.float64)
    cnt = np.zeros(LBM_NPHASES, dtype=np.int64)
    _check(load().lbm_read_timing(h, _ptr(ms), _ptr(cnt)), h)
    return ms, cnt


def lbm_layout(h):
    """(NX, NY, pstride, cstride, bytes of one lattice copy, work-group size)."""
    out = np.zeros(6, dtype=np.int64)
    _check(load().lbm_layout(h, _ptr(out)), h)
    return tuple(int(v) for v in out)


def lbm_tables():
    e = np.zeros((NPOP, 2), dtype=np.int32)
    opp = np.zeros(NPOP, dtype=np.int32)
    w = np.zeros(NPOP, dtype=np.float64)
    r = np.zeros(1, dtype=np.float64)
    _check(load().lbm_tables(_ptr(e), _ptr(opp), _ptr(w), _ptr(r)))
    return e, opp, w, float(r[0])


def lbm_wall_factors(t_wall: float) -> np.ndarray:
    out = np.zeros(NPOP, dtype=np.float64)
    _check(load().lbm_wall_factors(t_wall, _ptr(out)))
    return out


LBM_PROBE_COPY, LBM_PROBE_MRAW, LBM_PROBE_ARMW = 0, 1, 2


def lbm_probe_bandwidth(mode: int, src: int, dst: int, nbytes: int, shift: int, stream: int) -> None:
    _check(load().lbm_probe_bandwidth(mode, c_void_p(src), c_void_p(dst), nbytes, shift,
                                      c_void_p(stream)))


def lbm_destroy(h) -> None:
    load().lbm_destroy(h)


LBM_SCHED_CHUNKED, LBM_SCHED_STRIDED = 0, 1


def _echeck(status: int, e=None) -> None:
    if status != LBM_OK:
        msg = load().lbm_engine_last_error(e)
        raise LbmError(status, msg.decode() if msg else "")


def lbm_engine_required_bytes(max_slots: int) -> int:
    n = load().lbm_engine_required_bytes(max_slots)
    if n == 0:
        _echeck(LBM_EINVAL)
    return int(n)


def lbm_engine_create(max_slots: int, dev_mem: int, dev_bytes: int, stream: int) -> c_void_p:
    e = c_void_p()
    _echeck(load().lbm_engine_create(max_slots, c_void_p(dev_mem), dev_bytes, c_void_p(stream), byref(e)))
    return e


def lbm_engine_add(e, h, steps: int) -> int:
    slot = np.zeros(1, dtype=np.int32)
    _echeck(load().lbm_engine_add(e, h, steps, _ptr(slot)), e)
    return int(slot[0])


def lbm_engine_remove(e, slot: int) -> None:
    _echeck(load().lbm_engine_remove(e, slot), e)


def lbm_engine_step(e, n: int) -> None:
    _echeck(load().lbm_engine_step(e, n), e)


def lbm_engine_status(e, max_slots: int) -> np.ndarray:
    out = np.zeros(max_slots, dtype=np.int32)
    _echeck(load().lbm_engine_status(e, _ptr(out)), e)
    return out


def lbm_engine_set_tiling(e, block: int, groups: int, schedule: int) -> None:
    _echeck(load().lbm_engine_set_tiling(e, block, groups, schedule), e)


def lbm_engine_get_tiling(e):
    out = np.zeros(3, dtype=np.int32)
    _echeck(load().lbm_engine_get_tiling(e, _ptr(out)), e)
    return tuple(int(v) for v in out)


def lbm_engine_tune(e, reps: int):
    out = np.zeros(3, dtype=np.int32)
    ms = np.zeros(1, dtype=np.float64)
    _echeck(load().lbm_engine_tune(e, reps, _ptr(out), _ptr(ms)), e)
    return tuple(int(v) for v in out), float(ms[0])


def lbm_engine_destroy(e) -> None:
    load().lbm_engine_destroy(e)


class Lattice:
    """A lattice bound to device memory owned by a torch uint8 tensor.

    Convenience owner of the handle, the memory and the stream; every
    operation is one call of the C ABI above.
    """

    def __init__(self, cfg: lbm_config, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the D2Q37 library needs an MI355X (gfx950)")
        self.cfg = cfg
        self.lx, self.ly = int(cfg.lx), int(cfg.ly)
        self.device = torch.device(device if device is not None else "cuda")
        self.nbytes = lbm_required_bytes(cfg)
        self.mem = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = lbm_create(cfg, self.mem.data_ptr(), self.nbytes, self.stream.cuda_stream)

    def init_rt(self, rt) -> "Lattice":
        lbm_init_rt(self.h, rt.width, rt.y_center, rt.amps, rt.phases)
        return self

    def step(self, n: int = 1) -> None:
        lbm_step(self.h, n)

    def step_captured(self, n: int = 1) -> None:
        lbm_step_captured(self.h, n)

    def run_phase(self, phase: int) -> None:
        lbm_run_phase(self.h, phase)

    def moments(self):
        return lbm_moments(self.h, self.lx, self.ly)

    def conservation(self) -> np.ndarray:
        return lbm_conservation(self.h)

    def get(self) -> np.ndarray:
        return lbm_get_populations(self.h, self.lx, self.ly)

    def set(self, f: np.ndarray) -> None:
        lbm_set_populations(self.h, f)

    def sites(self, xs, ys) -> np.ndarray:
        return lbm_get_sites(self.h, xs, ys)

    def layout(self):
        return lbm_layout(self.h)

    def close(self) -> None:
        if getattr(self, "h", None) is not None:
            lbm_destroy(self.h)
            self.h = None
        self.mem = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Engine:
    """An ensemble engine on a torch-owned slot table (one C-ABI call per
    operation)."""

    def __init__(self, max_slots: int, device=None, stream=None):
        import torch
        self.max_slots = max_slots
        self.device = torch.device(device if device is not None else "cuda")
        n = lbm_engine_required_bytes(max_slots)
        self.mem = torch.empty(n, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.e = lbm_engine_create(max_slots, self.mem.data_ptr(), n, self.stream.cuda_stream)

    def add(self, lat: "Lattice", steps: int) -> int:
        return lbm_engine_add(self.e, lat.h, steps)

    def remove(self, slot: int) -> None:
        lbm_engine_remove(self.e, slot)

    def step(self, n: int = 1) -> None:
        lbm_engine_step(self.e, n)

    def status(self) -> np.ndarray:
        return lbm_engine_status(self.e, self.max_slots)

    def tune(self, reps: int = 3):
        return lbm_engine_tune(self.e, reps)

    def set_tiling(self, block: int, groups: int, schedule: int) -> None:
        lbm_engine_set_tiling(self.e, block, groups, schedule)

    def tiling(self):
        return lbm_engine_get_tiling(self.e)

    def close(self) -> None:
        if getattr(self, "e", None) is not None:
            lbm_engine_destroy(self.e)
            self.e = None
        self.mem = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def config_from(ns, **overrides) -> lbm_config:
    """lbm_config from a namespace with lx, ly, tau, gx, gy, t_bottom, t_top."""
    cfg = lbm_config_default(ns.lx, ns.ly)
    cfg.tau, cfg.gx, cfg.gy = ns.tau, ns.gx, ns.gy
    cfg.t_bottom, cfg.t_top = ns.t_bottom, ns.t_top
    fields = {name for name, _ in lbm_config._fields_}
    for k, v in overrides.items():
        if k not in fields:
            raise TypeError(f"lbm_config has no field {k!r}")
        setattr(cfg, k, v)
    return cfg
