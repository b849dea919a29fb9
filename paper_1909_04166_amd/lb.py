"""ctypes binding of the C-ABI in ``include/cmlb.h`` (``libcmlb.so``).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Function names equal the C names.  PyTorch supplies the device
workspace and the stream.  The library must have been built
(``python -m paper_1909_04166_amd.build``); if it is missing this module raises
on first use.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcmlb.so")

LB_OK, LB_E_INVALID_ARG, LB_E_WORKSPACE, LB_E_HIP, LB_E_UNSTABLE, LB_E_UNSUPPORTED, LB_E_STATE = (
    0, -1, -2, -3, -4, -5, -6)
LB_E_TOO_LARGE = -7
LB_PERIODIC, LB_HALFWAY_BB, LB_FREE_SLIP = 0, 1, 2
LB_BC = {"periodic": LB_PERIODIC, "wall": LB_HALFWAY_BB, "slip": LB_FREE_SLIP}
LB_COLLISION = {"cascaded": 0, "srt": 1, "printed": 2}
LB_FLOW = {"coupled": 0, "imposed": 1}
LB_SIGMA = {"linear": 0, "langmuir": 1}
LB_FREF = {"mean": 0, "light": 1, "heavy": 2, "none": 3}
LB_ST = {"geometric": 0, "chempot": 1}
PRECISION = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3}
LB_INIT = {"none": 0, "droplet": 1, "ellipse": 2, "interface": 3}
LB_ROUND = {"stochastic": 0, "nearest": 1}
STORE_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}


class lb_config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("force_ref", ctypes.c_int32), ("st_form", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("diag_every", ctypes.c_int32),
        ("rho_A", ctypes.c_double), ("rho_B", ctypes.c_double),
        ("nu_A", ctypes.c_double), ("nu_B", ctypes.c_double),
        ("sigma0", ctypes.c_double), ("sigma_T", ctypes.c_double),
        ("T0", ctypes.c_double), ("dTdy", ctypes.c_double), ("y_ref", ctypes.c_double),
        ("W", ctypes.c_double), ("M", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("shift_f", ctypes.c_double), ("shift_g", ctypes.c_double),
        ("u_max", ctypes.c_double),
        ("tile_x", ctypes.c_int32), ("tile_h", ctypes.c_int32),
        ("collision", ctypes.c_int32), ("flow", ctypes.c_int32),
        ("surf", ctypes.c_int32), ("tile_pf", ctypes.c_int32),
        ("beta", ctypes.c_double), ("psi_a", ctypes.c_double), ("psi_G", ctypes.c_double),
        ("init_kind", ctypes.c_int32), ("rounding", ctypes.c_int32), ("init_par", ctypes.c_double * 8),
    ]


class lb_diag(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("step", "sum_phi", "sum_rho", "max_u", "dp_laplace", "r_eff",
                 "spike_y", "bubble_y", "centroid_y", "nan_flag")]

    def as_dict(self) -> dict:
        return {n: float(getattr(self, n)) for n, _ in self._fields_}


class LBError(RuntimeError):
    def __init__(self, fn: str, code: int):
        self.code = code
        msg = lib().lb_status_string(code).decode() if _lib is not None else str(code)
        super().__init__(f"{fn} failed: {msg} ({code})")


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)

_SIGS = {
    "lb_status_string": ([ctypes.c_int32], ctypes.c_char_p),
    "lb_workspace_bytes": ([ctypes.POINTER(lb_config), _u64p], ctypes.c_int32),
    "lb_create": ([ctypes.POINTER(lb_config), _vp, ctypes.c_uint64, _vp, ctypes.POINTER(_vp)], ctypes.c_int32),
    "lb_init_fields": ([_vp, _dp], ctypes.c_int32),
    "lb_set_velocity": ([_vp, _dp, _dp], ctypes.c_int32),
    "lb_step": ([_vp, ctypes.c_int64], ctypes.c_int32),
    "lb_get_fields": ([_vp, _dp, _dp, _dp, _dp], ctypes.c_int32),
    "lb_get_coupling": ([_vp, _vp], ctypes.c_int32),
    "lb_diagnostics": ([_vp, ctypes.POINTER(lb_diag)], ctypes.c_int32),
    "lb_get_dist": ([_vp, _dp, _dp], ctypes.c_int32),
    "lb_set_dist": ([_vp, _dp, _dp, ctypes.c_int64], ctypes.c_int32),
    "lb_state_bytes": ([_vp, _u64p], ctypes.c_int32),
    "lb_save_state": ([_vp, _vp, ctypes.c_uint64], ctypes.c_int32),
    "lb_load_state": ([_vp, _vp, ctypes.c_uint64], ctypes.c_int32),
    "lb_get_step": ([_vp, _i64p], ctypes.c_int32),
    "lb_destroy": ([_vp], None),
    "lb_batch_workspace_bytes": ([ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _u64p], ctypes.c_int32),
    "lb_batch_create": ([ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                         _vp, ctypes.c_uint64, _vp, ctypes.POINTER(_vp)], ctypes.c_int32),
    "lb_batch_add": ([_vp, ctypes.POINTER(lb_config), _dp, _i32p], ctypes.c_int32),
    "lb_batch_remove": ([_vp, ctypes.c_int32], ctypes.c_int32),
    "lb_batch_step": ([_vp, ctypes.c_int64, ctypes.c_int32], ctypes.c_int32),
    "lb_batch_get_fields": ([_vp, ctypes.c_int32, _dp, _dp, _dp, _dp], ctypes.c_int32),
    "lb_batch_diagnostics": ([_vp, ctypes.c_int32, ctypes.POINTER(lb_diag)], ctypes.c_int32),
    "lb_batch_get_step": ([_vp, ctypes.c_int32, _i64p], ctypes.c_int32),
    "lb_batch_usage": ([_vp, _i32p, _i64p], ctypes.c_int32),
    "lb_batch_destroy": ([_vp], None),
    "lb_timing_enable": ([_vp, ctypes.c_int32], ctypes.c_int32),
    "lb_timing_read": ([_vp, _dp, _i64p], ctypes.c_int32),
    "lb_batch_timing_enable": ([_vp, ctypes.c_int32], ctypes.c_int32),
    "lb_batch_timing_read": ([_vp, _dp, _i64p], ctypes.c_int32),
    "lb_get_schedule": ([_vp, _i32p, _i32p, _i32p, _i32p], ctypes.c_int32),
    "lb_set_schedule": ([_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32], ctypes.c_int32),
    "lb_batch_get_schedule": ([_vp, _i32p, _i32p, _i32p, _i32p], ctypes.c_int32),
    "lb_batch_launch_counts": ([_vp, _i64p, _i64p], ctypes.c_int32),
    "lb_batch_set_schedule": ([_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
                              ctypes.c_int32),
    "lb_struct_sizes": ([_u64p, _u64p], ctypes.c_int32),
    "lb_copy_kernel": ([_vp, _vp, ctypes.c_uint64, _vp], ctypes.c_int32),
    "lb_bandwidth_probe": ([_vp, _vp, ctypes.c_uint64, ctypes.c_int32, _vp], ctypes.c_int32),
    "lb_step_noalloc": ([ctypes.POINTER(lb_config), _vp, _vp, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, _vp],
                        ctypes.c_int32),
}


def lib():
    """Load libcmlb.so (raises if it has not been built, or was built from other
    sources than the ones in the tree)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1909_04166_amd.build` (no CPU fallback exists)")
        from paper_1909_04166_amd import build as _build
        try:
            with open(LIB_PATH + _build.STAMP_SUFFIX) as fh:
                stamp = fh.read().strip()
        except OSError:
            stamp = None
        if stamp != _build.source_hash():
            raise RuntimeError(f"{LIB_PATH} does not match the sources in the tree (stale or foreign "
                               "build): rebuild it with `python -m paper_1909_04166_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        cb, db = ctypes.c_uint64(), ctypes.c_uint64()
        L.lb_struct_sizes(ctypes.byref(cb), ctypes.byref(db))
        if cb.value != ctypes.sizeof(lb_config) or db.value != ctypes.sizeof(lb_diag):
            raise RuntimeError("libcmlb.so struct layout does not match the binding")
        _lib = L
    return _lib


def _check(fn: str, rc: int) -> None:
    if rc != LB_OK:
        raise LBError(fn, rc)


def _dptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def default_shift_f(case: dict) -> float:
    """Storage shift of the phase-field values in 16-bit storage (f_a is stored as
    f_a - w_a shift_f): the light phase's phi, 0 when rho_A >= rho_B, else 1.  The
    light phase's values are then stored near zero, where the 16-bit formats
    resolve them finely, and rho(phi) = rho_B + phi (rho_A - rho_B) is most
    sensitive to phi there: a rounding error d phi moves rho by (ratio - 1) d phi
    relative to the light density, and only by about d phi relative to the heavy
    one.  With stochastic rounding (the default) the heavy phase then carries
    unbiased noise of about 1e-4 in phi and the light phase almost none; a shift
    of 9/16 (values of about w_a / 2 in both phases) put that noise into the light
    phase, and at density ratios near 1000 it drove lattices unstable."""
    return 0.0 if float(case["rho_A"]) >= float(case["rho_B"]) else 1.0


def config_from_case(case: dict, precision: str = "fp64", diag_every: int = 0,
                     tile: tuple = (0, 0), shift_f: float | None = None, shift_g: float = 0.0,
                     u_max: float = 0.0) -> lb_config:
    """Translate a case dictionary (paper_1909_04166_amd.workloads) into lb_config.
    tile: (tile_x, tile_h) or (tile_x, tile_h, tile_pf); zeros autotune.
    shift_f None: default_shift_f(case)."""
    c = lb_config()
    c.nx, c.ny = int(case["nx"]), int(case["ny"])
    c.bc_x = LB_BC[case.get("bc_x", "periodic")]
    c.bc_y = LB_BC[case.get("bc_y", "periodic")]
    c.force_ref = LB_FREF[case.get("force_ref", "mean")]
    c.st_form = LB_ST[case.get("st_form", "geometric")]
    c.precision = PRECISION[precision]
    c.diag_every = int(diag_every)
    c.rho_A, c.rho_B = float(case["rho_A"]), float(case["rho_B"])
    c.nu_A, c.nu_B = float(case["nu_A"]), float(case["nu_B"])
    c.sigma0, c.sigma_T = float(case.get("sigma0", 0.0)), float(case.get("sigma_T", 0.0))
    c.T0, c.dTdy, c.y_ref = float(case.get("T0", 0.0)), float(case.get("dTdy", 0.0)), float(case.get("y_ref", 0.0))
    c.W, c.M = float(case["W"]), float(case["M"])
    c.gx, c.gy = float(case.get("gx", 0.0)), float(case.get("gy", 0.0))
    if shift_f is None:
        shift_f = default_shift_f(case)
    c.shift_f, c.shift_g, c.u_max = float(shift_f), float(shift_g), float(u_max)
    c.tile_x, c.tile_h = int(tile[0]), int(tile[1])
    c.tile_pf = int(tile[2]) if len(tile) > 2 else 0
    c.collision = LB_COLLISION[case.get("collision", "cascaded")]
    c.flow = LB_FLOW[case.get("flow", "coupled")]
    c.surf = LB_SIGMA[case.get("surf", "linear")]
    c.beta = float(case.get("beta", 0.0))
    c.psi_a, c.psi_G = float(case.get("psi_a", 0.0)), float(case.get("psi_G", 0.0))
    c.rounding = LB_ROUND[case.get("rounding", "stochastic")]
    kind, par = case.get("init", ("none", ()))
    c.init_kind = LB_INIT[kind]
    for i, v in enumerate(par):
        c.init_par[i] = float(v)
    return c


# ------------------------------------------------------------ C-ABI mirrors

def lb_workspace_bytes(cfg: lb_config) -> int:
    b = ctypes.c_uint64()
    _check("lb_workspace_bytes", lib().lb_workspace_bytes(ctypes.byref(cfg), ctypes.byref(b)))
    return int(b.value)


def lb_create(cfg: lb_config, ws_ptr: int, ws_bytes: int, stream: int) -> int:
    h = _vp()
    _check("lb_create", lib().lb_create(ctypes.byref(cfg), _vp(ws_ptr), ws_bytes, _vp(stream), ctypes.byref(h)))
    return h.value


def lb_init_fields(h: int, phi0: np.ndarray | None) -> None:
    """phi0 None: the built-in initial field of the lattice's init_kind."""
    a = None if phi0 is None else np.ascontiguousarray(phi0, dtype=np.float64)
    _check("lb_init_fields", lib().lb_init_fields(_vp(h), _dptr(a)))


def lb_set_velocity(h: int, ux: np.ndarray, uy: np.ndarray) -> None:
    a = np.ascontiguousarray(ux, dtype=np.float64)
    b = np.ascontiguousarray(uy, dtype=np.float64)
    assert a.shape == b.shape
    _check("lb_set_velocity", lib().lb_set_velocity(_vp(h), _dptr(a), _dptr(b)))


def lb_step(h: int, n: int) -> int:
    """Returns the status (LB_E_UNSTABLE is reported, not raised)."""
    rc = lib().lb_step(_vp(h), int(n))
    if rc not in (LB_OK, LB_E_UNSTABLE):
        _check("lb_step", rc)
    return rc


def lb_get_fields(h: int, shape) -> tuple:
    out = [np.empty(shape) for _ in range(4)]
    _check("lb_get_fields", lib().lb_get_fields(_vp(h), *[_dptr(o) for o in out]))
    return tuple(out)


def lb_get_coupling(h: int, dev_ptr: int) -> None:
    _check("lb_get_coupling", lib().lb_get_coupling(_vp(h), _vp(dev_ptr)))


def lb_diagnostics(h: int) -> dict:
    d = lb_diag()
    _check("lb_diagnostics", lib().lb_diagnostics(_vp(h), ctypes.byref(d)))
    return d.as_dict()


def lb_get_dist(h: int, shape) -> tuple:
    f = np.empty((9,) + tuple(shape))
    g = np.empty((9,) + tuple(shape))
    _check("lb_get_dist", lib().lb_get_dist(_vp(h), _dptr(f), _dptr(g)))
    return f, g


def lb_set_dist(h: int, f: np.ndarray, g: np.ndarray | None, step: int = 0) -> None:
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = None if g is None else np.ascontiguousarray(g, dtype=np.float64)
    _check("lb_set_dist", lib().lb_set_dist(_vp(h), _dptr(f), _dptr(g), int(step)))


def lb_state_bytes(h: int) -> int:
    b = ctypes.c_uint64()
    _check("lb_state_bytes", lib().lb_state_bytes(_vp(h), ctypes.byref(b)))
    return int(b.value)


def lb_save_state(h: int) -> bytes:
    n = lb_state_bytes(h)
    buf = ctypes.create_string_buffer(n)
    _check("lb_save_state", lib().lb_save_state(_vp(h), ctypes.cast(buf, _vp), n))
    return buf.raw


def lb_load_state(h: int, state: bytes) -> None:
    buf = ctypes.create_string_buffer(state, len(state))
    _check("lb_load_state", lib().lb_load_state(_vp(h), ctypes.cast(buf, _vp), len(state)))


def lb_get_step(h: int) -> int:
    s = ctypes.c_int64()
    _check("lb_get_step", lib().lb_get_step(_vp(h), ctypes.byref(s)))
    return int(s.value)


def lb_destroy(h: int) -> None:
    lib().lb_destroy(_vp(h))


def lb_timing_enable(h: int, on: bool = True) -> None:
    _check("lb_timing_enable", lib().lb_timing_enable(_vp(h), int(bool(on))))


def lb_timing_read(h: int) -> tuple[float, int]:
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check("lb_timing_read", lib().lb_timing_read(_vp(h), ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


def lb_get_schedule(h: int) -> tuple[int, int, int, int]:
    """(workgroup width, rows per item or segment, persistent grid or 0, prefetch)."""
    a, b, c, d = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check("lb_get_schedule", lib().lb_get_schedule(_vp(h), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                                    ctypes.byref(d)))
    return int(a.value), int(b.value), int(c.value), int(d.value)


def lb_set_schedule(h: int, tile_x: int, mode: int, param: int, prefetch: int = 0) -> None:
    """Pin the schedule: mode 0 items of `param` rows; modes 1 and 2 persistent
    grids of `param` x resident workgroups per CU x CUs (balanced runs of strip
    rows; strip-aligned bands)."""
    _check("lb_set_schedule", lib().lb_set_schedule(_vp(h), int(tile_x), int(mode), int(param), int(prefetch)))


def lb_batch_get_schedule(b: int) -> tuple[int, int, int, int]:
    """(workgroup width, rows per segment, persistent grid or 0, prefetch) of a batch."""
    a, r, g, p = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check("lb_batch_get_schedule", lib().lb_batch_get_schedule(_vp(b), ctypes.byref(a), ctypes.byref(r),
                                                                ctypes.byref(g), ctypes.byref(p)))
    return int(a.value), int(r.value), int(g.value), int(p.value)


def lb_bandwidth_probe(dst: int, src: int, n: int, variant: int, stream: int) -> None:
    _check("lb_bandwidth_probe", lib().lb_bandwidth_probe(_vp(dst), _vp(src), int(n), int(variant), _vp(stream)))


def lb_batch_launch_counts(b: int) -> tuple[int, int]:
    """(steps replayed from graphs, steps launched one by one) since creation."""
    g, e = ctypes.c_int64(), ctypes.c_int64()
    _check("lb_batch_launch_counts", lib().lb_batch_launch_counts(_vp(b), ctypes.byref(g), ctypes.byref(e)))
    return int(g.value), int(e.value)


def lb_copy_kernel(dst: int, src: int, n: int, stream: int) -> None:
    _check("lb_copy_kernel", lib().lb_copy_kernel(_vp(dst), _vp(src), int(n), _vp(stream)))


def lb_step_noalloc(cfg: lb_config, state0: int, state1: int, state_bytes: int, step: int, n: int,
                    stream: int) -> None:
    """n steps of a lattice held in two caller-owned device buffers (the checkpoint
    payload layout) whose state is at step count `step`; the state ends in state0
    for even n, state1 for odd n."""
    _check("lb_step_noalloc", lib().lb_step_noalloc(ctypes.byref(cfg), _vp(state0), _vp(state1),
                                                     int(state_bytes), int(step), int(n), _vp(stream)))


def lb_batch_workspace_bytes(slots: int, node_capacity: int, precision: str) -> int:
    b = ctypes.c_uint64()
    _check("lb_batch_workspace_bytes",
           lib().lb_batch_workspace_bytes(slots, node_capacity, PRECISION[precision], ctypes.byref(b)))
    return int(b.value)


def lb_batch_create(slots: int, node_capacity: int, precision: str, tile: tuple[int, int],
                    ws_ptr: int, ws_bytes: int, stream: int) -> int:
    h = _vp()
    _check("lb_batch_create", lib().lb_batch_create(slots, node_capacity, PRECISION[precision],
                                                     int(tile[0]), int(tile[1]), _vp(ws_ptr), ws_bytes,
                                                     _vp(stream), ctypes.byref(h)))
    return h.value


def lb_batch_add(b: int, cfg: lb_config, phi0: np.ndarray | None) -> int:
    """Returns the slot index; raises LBError (code LB_E_WORKSPACE when full).
    phi0 None: the built-in initial field of cfg.init_kind."""
    a = None if phi0 is None else np.ascontiguousarray(phi0, dtype=np.float64)
    s = ctypes.c_int32()
    _check("lb_batch_add", lib().lb_batch_add(_vp(b), ctypes.byref(cfg), _dptr(a), ctypes.byref(s)))
    return int(s.value)


def lb_batch_remove(b: int, slot: int) -> None:
    _check("lb_batch_remove", lib().lb_batch_remove(_vp(b), int(slot)))


def lb_batch_step(b: int, n: int, use_graph: bool = True) -> None:
    _check("lb_batch_step", lib().lb_batch_step(_vp(b), int(n), int(bool(use_graph))))


def lb_batch_get_fields(b: int, slot: int, shape) -> tuple:
    out = [np.empty(shape) for _ in range(4)]
    _check("lb_batch_get_fields", lib().lb_batch_get_fields(_vp(b), int(slot), *[_dptr(o) for o in out]))
    return tuple(out)


def lb_batch_diagnostics(b: int, slot: int) -> dict:
    d = lb_diag()
    _check("lb_batch_diagnostics", lib().lb_batch_diagnostics(_vp(b), int(slot), ctypes.byref(d)))
    return d.as_dict()


def lb_batch_get_step(b: int, slot: int) -> int:
    s = ctypes.c_int64()
    _check("lb_batch_get_step", lib().lb_batch_get_step(_vp(b), int(slot), ctypes.byref(s)))
    return int(s.value)


def lb_batch_usage(b: int) -> tuple[int, int]:
    u, n = ctypes.c_int32(), ctypes.c_int64()
    _check("lb_batch_usage", lib().lb_batch_usage(_vp(b), ctypes.byref(u), ctypes.byref(n)))
    return int(u.value), int(n.value)


def lb_batch_destroy(b: int) -> None:
    lib().lb_batch_destroy(_vp(b))


def lb_batch_timing_enable(b: int, on: bool = True) -> None:
    _check("lb_batch_timing_enable", lib().lb_batch_timing_enable(_vp(b), int(bool(on))))


def lb_batch_timing_read(b: int) -> tuple[float, int]:
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check("lb_batch_timing_read", lib().lb_batch_timing_read(_vp(b), ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


# --------------------------------------------------------- torch plumbing

def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible: the lattice library runs on the GPU only")
    return torch


class Lattice:
    """One lattice in a torch-allocated device workspace on the current stream."""

    def __init__(self, case: dict, phi0: np.ndarray | None = None, precision: str = "fp64",
                 diag_every: int = 0, tile: tuple = (0, 0), shift_f: float | None = None,
                 shift_g: float = 0.0, u_max: float = 0.0, device: str = "cuda:0"):
        torch = _torch()
        self.case = dict(case)
        self.precision = precision
        self.shape = (int(case["ny"]), int(case["nx"]))
        self.cfg = config_from_case(case, precision, diag_every, tile, shift_f, shift_g, u_max)
        nbytes = lb_workspace_bytes(self.cfg)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream(self.ws.device).cuda_stream
        self.h = lb_create(self.cfg, self.ws.data_ptr(), nbytes, self.stream)
        if phi0 is not None:
            self.init(phi0)

    def close(self):
        if getattr(self, "h", None):
            lb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, phi0: np.ndarray | None) -> None:
        """phi0 None: the built-in initial field described by the case's "init" entry."""
        lb_init_fields(self.h, None if phi0 is None else np.asarray(phi0, dtype=np.float64).reshape(self.shape))

    def step(self, n: int = 1) -> int:
        return lb_step(self.h, n)

    def set_velocity(self, ux: np.ndarray, uy: np.ndarray) -> None:
        """Imposed velocity of a phase-field-only lattice (flow = "imposed")."""
        lb_set_velocity(self.h, np.asarray(ux, dtype=np.float64).reshape(self.shape),
                        np.asarray(uy, dtype=np.float64).reshape(self.shape))

    def fields(self):
        return lb_get_fields(self.h, self.shape)

    def coupling(self) -> dict:
        torch = _torch()
        buf = torch.empty((9,) + self.shape, dtype=torch.float64, device=self.ws.device)
        lb_get_coupling(self.h, buf.data_ptr())
        o = buf.cpu().numpy()
        names = ["dphix", "dphiy", "nx", "ny", "divn", "Ftx", "Fty", "Fpx", "Fpy"]
        return {k: o[i] for i, k in enumerate(names)}

    def diagnostics(self) -> dict:
        return lb_diagnostics(self.h)

    def get_dist(self):
        return lb_get_dist(self.h, self.shape)

    def set_dist(self, f, g, step: int = 0):
        lb_set_dist(self.h, f, g, step)

    def save(self) -> bytes:
        return lb_save_state(self.h)

    def load(self, state: bytes) -> None:
        lb_load_state(self.h, state)

    @property
    def t(self) -> int:
        return lb_get_step(self.h)

    @property
    def tile(self):
        return lb_get_schedule(self.h)

    def set_schedule(self, tile_x: int, mode: int, param: int, prefetch: int = 0) -> None:
        lb_set_schedule(self.h, tile_x, mode, param, prefetch)


class Batch:
    """Many lattices of uneven sizes in one workspace, advanced together by one
    persistent kernel launch per step (slots can be filled and freed between
    steps)."""

    def __init__(self, slots: int, node_capacity: int, precision: str = "fp32",
                 tile: tuple[int, int] = (0, 0), device: str = "cuda:0"):
        torch = _torch()
        self.precision = precision
        nbytes = lb_batch_workspace_bytes(slots, node_capacity, precision)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream(self.ws.device).cuda_stream
        self.b = lb_batch_create(slots, node_capacity, precision, tile, self.ws.data_ptr(), nbytes,
                                 self.stream)
        self.shapes = {}

    def close(self):
        if getattr(self, "b", None):
            lb_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, case: dict, phi0: np.ndarray, diag_every: int = 0, shift_f: float | None = None,
            shift_g: float = 0.0) -> int:
        cfg = config_from_case(case, self.precision, diag_every, (0, 0), shift_f, shift_g)
        shape = (int(case["ny"]), int(case["nx"]))
        slot = lb_batch_add(self.b, cfg, None if phi0 is None else np.asarray(phi0, dtype=np.float64).reshape(shape))
        self.shapes[slot] = shape
        return slot

    @property
    def tile(self):
        """Schedule of the persistent step (see lb_batch_get_schedule)."""
        return lb_batch_get_schedule(self.b)

    def remove(self, slot: int) -> None:
        lb_batch_remove(self.b, slot)
        self.shapes.pop(slot, None)

    def step(self, n: int = 1, use_graph: bool = True) -> None:
        lb_batch_step(self.b, n, use_graph)

    def fields(self, slot: int):
        return lb_batch_get_fields(self.b, slot, self.shapes[slot])

    def diagnostics(self, slot: int) -> dict:
        return lb_batch_diagnostics(self.b, slot)

    def t(self, slot: int) -> int:
        return lb_batch_get_step(self.b, slot)

    def usage(self) -> tuple[int, int]:
        return lb_batch_usage(self.b)

    def set_schedule(self, tile_x: int, mode: int, param: int, prefetch: int = 0) -> None:
        """Pin the persistent step's schedule (see Lattice.set_schedule)."""
        _check("lb_batch_set_schedule", lib().lb_batch_set_schedule(self.b, int(tile_x), int(mode), int(param),
                                                                    int(prefetch)))

    def launch_counts(self) -> tuple[int, int]:
        """(steps replayed from captured graphs, steps launched one by one)."""
        return lb_batch_launch_counts(self.b)
