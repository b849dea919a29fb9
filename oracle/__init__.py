"""FP64 CPU oracle for the coupled cascaded central-moment LB time step.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  The product library never imports
this package and this package never imports the product.

The arithmetic lives in ``lb_oracle.c`` (plain C, FP64, one function per step of
the method, in the paper's order: Secs. 2-5 of arXiv:1909.04166).  This module
only builds it with gcc and marshals arguments through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lb_oracle.c")
_LIB = os.path.join(_HERE, "liblboracle.so")

Q = 9


def build(force: bool = False) -> str:
    """Compile the oracle into ``oracle/liblboracle.so`` (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("bc_y", ctypes.c_int32), ("force_ref", ctypes.c_int32),
        ("st_form", ctypes.c_int32), ("collision", ctypes.c_int32),
        ("flow", ctypes.c_int32), ("surf", ctypes.c_int32),
        ("bc_x", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("rho_A", ctypes.c_double), ("rho_B", ctypes.c_double),
        ("nu_A", ctypes.c_double), ("nu_B", ctypes.c_double),
        ("sigma0", ctypes.c_double), ("sigma_T", ctypes.c_double),
        ("T0", ctypes.c_double), ("dTdy", ctypes.c_double), ("y_ref", ctypes.c_double),
        ("W", ctypes.c_double), ("M", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("beta", ctypes.c_double), ("psi_a", ctypes.c_double), ("psi_G", ctypes.c_double),
        ("q6_minus8", ctypes.c_int32), ("q8_printed", ctypes.c_int32), ("q11_lagged", ctypes.c_int32),
        ("pad3_", ctypes.c_int32),
    ]


_BC = {"periodic": 0, "wall": 1, "slip": 2}
# "printed": the cascaded pair with the printed closed forms of the hydrodynamic
# moment changes h_3..h_8 (the study switch q8_printed); "cascaded" solves the
# relaxation conditions they come from
_COLL = {"cascaded": 0, "srt": 1, "printed": 0}
_FLOW = {"coupled": 0, "imposed": 1}
_SURF = {"linear": 0, "langmuir": 1}
_FREF = {"mean": 0, "light": 1, "heavy": 2, "none": 3}
_ST = {"geometric": 0, "chempot": 1}

_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        lib.orc_create.argtypes = [ctypes.POINTER(OrcParams), ctypes.POINTER(vp)]
        lib.orc_create.restype = ctypes.c_int
        lib.orc_destroy.argtypes = [vp]
        lib.orc_init.argtypes = [vp, dp]
        lib.orc_step.argtypes = [vp, ctypes.c_int64]
        lib.orc_fields.argtypes = [vp, dp, dp, dp, dp]
        lib.orc_coupling.argtypes = [vp, dp]
        lib.orc_diagnostics.argtypes = [vp, dp]
        lib.orc_set_dist.argtypes = [vp, dp, dp, ctypes.c_int64]
        lib.orc_get_dist.argtypes = [vp, dp, dp]
        lib.orc_step_count.argtypes = [vp]
        lib.orc_step_count.restype = ctypes.c_int64
        lib.orc_hydro_collide.argtypes = [dp] + [ctypes.c_double] * 9 + [dp, dp]
        lib.orc_hydro_collide_study.argtypes = ([dp] + [ctypes.c_double] * 9 + [dp, ctypes.c_int, ctypes.c_int, dp])
        lib.orc_ace_collide.argtypes = [dp] + [ctypes.c_double] * 7 + [dp, dp]
        lib.orc_hydro_srt.argtypes = [dp] + [ctypes.c_double] * 9 + [dp]
        lib.orc_ace_srt.argtypes = [dp] + [ctypes.c_double] * 8 + [dp]
        lib.orc_set_velocity.argtypes = [vp, dp, dp]
        lib.orc_grad9.argtypes = [dp, dp, dp]
        lib.orc_lap9.argtypes = [dp]
        lib.orc_lap9.restype = ctypes.c_double
        lib.orc_sizeof_params.restype = ctypes.c_int
        assert lib.orc_sizeof_params() == ctypes.sizeof(OrcParams)
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def params_from_case(case: dict) -> OrcParams:
    """Translate a plain case dictionary (see the workload generators) into the
    oracle's own parameter struct."""
    P = OrcParams()
    P.nx, P.ny = int(case["nx"]), int(case["ny"])
    P.bc_y = _BC[case.get("bc_y", "periodic")]
    P.bc_x = _BC[case.get("bc_x", "periodic")]
    P.force_ref = _FREF[case.get("force_ref", "mean")]
    P.st_form = _ST[case.get("st_form", "geometric")]
    P.rho_A, P.rho_B = float(case["rho_A"]), float(case["rho_B"])
    P.nu_A, P.nu_B = float(case["nu_A"]), float(case["nu_B"])
    P.sigma0 = float(case.get("sigma0", 0.0))
    P.sigma_T = float(case.get("sigma_T", 0.0))
    P.T0 = float(case.get("T0", 0.0))
    P.dTdy = float(case.get("dTdy", 0.0))
    P.y_ref = float(case.get("y_ref", 0.0))
    P.W, P.M = float(case["W"]), float(case["M"])
    P.gx, P.gy = float(case.get("gx", 0.0)), float(case.get("gy", 0.0))
    P.collision = _COLL[case.get("collision", "cascaded")]
    P.flow = _FLOW[case.get("flow", "coupled")]
    P.surf = _SURF[case.get("surf", "linear")]
    P.beta = float(case.get("beta", 0.0))
    P.psi_a = float(case.get("psi_a", 0.0))
    P.psi_G = float(case.get("psi_G", 0.0))
    # study switches of the oracle only (other readings of Q6, Q8, Q11; off by default)
    P.q6_minus8 = int(bool(case.get("oracle_q6_minus8", False)))
    P.q8_printed = int(bool(case.get("oracle_q8_printed", False)) or case.get("collision") == "printed")
    P.q11_lagged = int(bool(case.get("oracle_q11_lagged", False)))
    return P


class Oracle:
    """One lattice advanced by the FP64 oracle."""

    def __init__(self, case: dict, phi0: np.ndarray | None = None):
        lib = _load()
        self.case = dict(case)
        self.nx, self.ny = int(case["nx"]), int(case["ny"])
        self._P = params_from_case(case)
        h = ctypes.c_void_p()
        rc = lib.orc_create(ctypes.byref(self._P), ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"oracle rejected the parameters (code {rc})")
        self._h = h
        if phi0 is not None:
            self.init(phi0)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    @property
    def shape(self):
        return (self.ny, self.nx)

    def init(self, phi0: np.ndarray) -> None:
        a = np.ascontiguousarray(phi0, dtype=np.float64).reshape(self.shape)
        _lib.orc_init(self._h, _dp(a))

    def step(self, n: int = 1) -> None:
        _lib.orc_step(self._h, int(n))

    @property
    def t(self) -> int:
        return int(_lib.orc_step_count(self._h))

    def fields(self):
        """(phi, p, ux, uy) at the current time, each (ny, nx) float64."""
        out = [np.empty(self.shape) for _ in range(4)]
        _lib.orc_fields(self._h, *[_dp(o) for o in out])
        return tuple(out)

    def coupling(self) -> dict:
        o = np.empty((9,) + self.shape)
        _lib.orc_coupling(self._h, _dp(o))
        names = ["dphix", "dphiy", "nx", "ny", "divn", "Ftx", "Fty", "Fpx", "Fpy"]
        return {k: o[i] for i, k in enumerate(names)}

    def diagnostics(self) -> dict:
        o = np.empty(10)
        _lib.orc_diagnostics(self._h, _dp(o))
        names = ["step", "sum_phi", "sum_rho", "max_u", "dp_laplace", "r_eff",
                 "spike_y", "bubble_y", "centroid_y", "nan_flag"]
        return {k: float(o[i]) for i, k in enumerate(names)}

    def set_velocity(self, ux: np.ndarray, uy: np.ndarray) -> None:
        """Imposed velocity of an ACE-only case (flow = "imposed")."""
        ux = np.ascontiguousarray(ux, dtype=np.float64).reshape(self.shape)
        uy = np.ascontiguousarray(uy, dtype=np.float64).reshape(self.shape)
        _lib.orc_set_velocity(self._h, _dp(ux), _dp(uy))

    def get_dist(self):
        f = np.empty((Q,) + self.shape)
        g = np.empty((Q,) + self.shape)
        _lib.orc_get_dist(self._h, _dp(f), _dp(g))
        return f, g

    def set_dist(self, f: np.ndarray, g: np.ndarray, step: int = 0) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        assert f.shape == (Q,) + self.shape and g.shape == f.shape
        _lib.orc_set_dist(self._h, _dp(f), _dp(g), int(step))


def hydro_collide(gbar, p, rho, psi, ux, uy, Ftx, Fty, Fpx, Fpy, omega):
    """Per-node hydrodynamic cascaded collision (post-collision gbar)."""
    lib = _load()
    g = np.ascontiguousarray(gbar, dtype=np.float64)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    out = np.empty(Q)
    lib.orc_hydro_collide(_dp(g), p, rho, psi, ux, uy, Ftx, Fty, Fpx, Fpy, _dp(om), _dp(out))
    return out


def hydro_collide_study(gbar, p, rho, psi, ux, uy, Ftx, Fty, Fpx, Fpy, omega, q6_minus8=False,
                        q8_printed=False):
    """The hydrodynamic collision under the study switches (other readings of
    m^s'_8's sigma'_00 coefficient and of h_3..h_8)."""
    lib = _load()
    g = np.ascontiguousarray(gbar, dtype=np.float64)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    out = np.empty(Q)
    lib.orc_hydro_collide_study(_dp(g), p, rho, psi, ux, uy, Ftx, Fty, Fpx, Fpy, _dp(om),
                                int(bool(q6_minus8)), int(bool(q8_printed)), _dp(out))
    return out


def ace_collide(f, phi, ux, uy, M, theta, nx, ny, omega):
    """Per-node phase-field cascaded collision (post-collision f)."""
    lib = _load()
    fi = np.ascontiguousarray(f, dtype=np.float64)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    out = np.empty(Q)
    lib.orc_ace_collide(_dp(fi), phi, ux, uy, M, theta, nx, ny, _dp(om), _dp(out))
    return out


def hydro_srt(gbar, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, omega):
    """Per-node hydrodynamic SRT collision (post-collision gbar)."""
    lib = _load()
    g = np.ascontiguousarray(gbar, dtype=np.float64)
    out = np.empty(Q)
    lib.orc_hydro_srt(_dp(g), p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, omega, _dp(out))
    return out


def ace_srt(f, phi, ux, uy, M, theta, nx, ny, omega):
    """Per-node phase-field SRT collision (post-collision f)."""
    lib = _load()
    fi = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty(Q)
    lib.orc_ace_srt(_dp(fi), phi, ux, uy, M, theta, nx, ny, omega, _dp(out))
    return out


def grad9(q9):
    lib = _load()
    q = np.ascontiguousarray(q9, dtype=np.float64)
    dx, dy = ctypes.c_double(), ctypes.c_double()
    lib.orc_grad9(_dp(q), ctypes.byref(dx), ctypes.byref(dy))
    return dx.value, dy.value


def lap9(q9):
    lib = _load()
    q = np.ascontiguousarray(q9, dtype=np.float64)
    return float(lib.orc_lap9(_dp(q)))
