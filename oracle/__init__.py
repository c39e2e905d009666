"""FP64 CPU oracle for the AIR reconstruction path (ctypes wrapper over oracle.c).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke entry point and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library ``paper_1310_1434_amd``; inputs reach both from ``synth``.

Operators follow the paper's Methods section: the filtered adjoint
A'^T = A^T C (text before Eq. (5)), the normal-equation operator of Eq. (5),
and the split Bregman L2 step; the framelet is the one-level piecewise-linear
tensor framelet of the Materials section.  See ``oracle.h`` for the exact
definitions, conventions and which parts are pinned.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile liboracle.so next to the source (gcc, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [("beam", ctypes.c_int32), ("n", ctypes.c_int32), ("pixel", ctypes.c_double),
                ("n_views", ctypes.c_int32), ("n_bins", ctypes.c_int32),
                ("cosv", ctypes.c_void_p), ("sinv", ctypes.c_void_p),
                ("bin", ctypes.c_double), ("sod", ctypes.c_double), ("sdd", ctypes.c_double),
                ("ramp", ctypes.c_int32)]


# filtration C (orc_geom.ramp): window in bits 0-3, symmetric cosine weighting in bit 4
RAMP_WINDOWS = {"ram-lak": 0, "shepp-logan": 1, "hann": 2}
RAMP_COSINE = 16


class _Params(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_double), ("mu", ctypes.c_double), ("n_outer", ctypes.c_int32),
                ("n_cg", ctypes.c_int32), ("reg", ctypes.c_int32), ("filter", ctypes.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        G = ctypes.POINTER(_Geom)
        sigs = {
            "orc_tables": [G, P, P, P],
            "orc_project": [G, P, P],
            "orc_backproject": [G, P, P],
            "orc_ramp": [G, P, P],
            "orc_filtered_backproject": [G, P, P, ctypes.c_int32],
            "orc_framelet": [ctypes.c_int32, P, P],
            "orc_framelet_adjoint": [ctypes.c_int32, P, P],
            "orc_apply_normal": [G, P, ctypes.c_double, ctypes.c_int32, P],
            "orc_cg": [G, P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, P],
            "orc_solve": [G, P, ctypes.POINTER(_Params), P, P, P],
            "orc_ramp_taps_kind": [ctypes.c_int32, ctypes.c_int32, P],
            "orc_ramp_weights": [G, P],
        }
        for name, args in sigs.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.orc_ramp_taps.argtypes = [ctypes.c_int32, P]
        lib.orc_ramp_taps.restype = None
        lib.orc_shrink.argtypes = [ctypes.c_int32, P, ctypes.c_double, P]
        lib.orc_shrink.restype = None
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = None
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Geom:
    """Oracle view of a scan geometry (any object with the ``synth.Geometry`` fields)."""

    def __init__(self, geom, ramp: int = 0):
        self.beam = 0 if geom.beam == "parallel" else 1
        self.ramp = int(ramp)
        self.n = int(geom.n)
        self.n_views = int(geom.n_views)
        self.n_bins = int(geom.n_bins)
        self._cos = _f64(geom.view_cos)
        self._sin = _f64(geom.view_sin)
        self._s = _Geom(self.beam, self.n, float(geom.pixel), self.n_views, self.n_bins,
                        self._cos.ctypes.data, self._sin.ctypes.data, float(geom.bin),
                        float(geom.sod), float(geom.sdd), self.ramp)

    @property
    def ref(self):
        return ctypes.byref(self._s)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def num_threads() -> int:
    return _load().orc_num_threads()


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def tables(g: Geom):
    nr = g.n_views * g.n_bins
    axis = np.empty(nr, np.int8)
    lo = np.empty(nr, np.int32)
    hi = np.empty(nr, np.int32)
    _check(_load().orc_tables(g.ref, _ptr(axis), _ptr(lo), _ptr(hi)), "tables")
    shape = (g.n_views, g.n_bins)
    return axis.reshape(shape), lo.reshape(shape), hi.reshape(shape)


def project(g: Geom, x) -> np.ndarray:
    x = _f64(x)
    y = np.empty((g.n_views, g.n_bins))
    _check(_load().orc_project(g.ref, _ptr(x), _ptr(y)), "project")
    return y


def backproject(g: Geom, y) -> np.ndarray:
    y = _f64(y)
    x = np.empty((g.n, g.n))
    _check(_load().orc_backproject(g.ref, _ptr(y), _ptr(x)), "backproject")
    return x


def ramp_taps(n_bins: int) -> np.ndarray:
    r = np.empty(n_bins)
    _load().orc_ramp_taps(int(n_bins), _ptr(r))
    return r


def ramp_taps_kind(kind: int, n_bins: int) -> np.ndarray:
    r = np.empty(n_bins)
    _check(_load().orc_ramp_taps_kind(int(kind), int(n_bins), _ptr(r)), "ramp_taps_kind")
    return r


def ramp_weights(g: Geom) -> np.ndarray:
    w = np.empty(g.n_bins)
    _check(_load().orc_ramp_weights(g.ref, _ptr(w)), "ramp_weights")
    return w


def ramp(g: Geom, y) -> np.ndarray:
    y = _f64(y)
    yf = np.empty_like(y)
    _check(_load().orc_ramp(g.ref, _ptr(y), _ptr(yf)), "ramp")
    return yf


def filtered_backproject(g: Geom, y, filter: int = 1) -> np.ndarray:
    y = _f64(y)
    x = np.empty((g.n, g.n))
    _check(_load().orc_filtered_backproject(g.ref, _ptr(y), _ptr(x), int(filter)), "filtered_backproject")
    return x


def framelet(x) -> np.ndarray:
    x = _f64(x)
    n = x.shape[-1]
    z = np.empty((9, n, n))
    _check(_load().orc_framelet(n, _ptr(x), _ptr(z)), "framelet")
    return z


def framelet_adjoint(z) -> np.ndarray:
    z = _f64(z)
    n = z.shape[-1]
    x = np.empty((n, n))
    _check(_load().orc_framelet_adjoint(n, _ptr(z), _ptr(x)), "framelet_adjoint")
    return x


def shrink(v, t: float) -> np.ndarray:
    v = _f64(v)
    d = np.empty_like(v)
    _load().orc_shrink(v.shape[-1], _ptr(v), float(t), _ptr(d))
    return d


def apply_normal(g: Geom, x, mu: float, filter: int = 1) -> np.ndarray:
    x = _f64(x)
    out = np.empty_like(x)
    _check(_load().orc_apply_normal(g.ref, _ptr(x), float(mu), int(filter), _ptr(out)), "apply_normal")
    return out


def cg(g: Geom, rhs, mu: float, n_iter: int, x0=None, filter: int = 1) -> np.ndarray:
    rhs = _f64(rhs)
    x = np.zeros_like(rhs) if x0 is None else _f64(x0).copy()
    _check(_load().orc_cg(g.ref, _ptr(rhs), float(mu), int(filter), int(n_iter), _ptr(x)), "cg")
    return x


def solve(g: Geom, y, lam: float, mu: float, n_outer: int, n_cg: int, reg: int = 0,
          filter: int = 1, x0=None, return_b: bool = False):
    """Split Bregman (reg=0), Eq. (5) L2 (reg=1) or forward-backward splitting (reg=2, mu = step of Eq. (6)).

    Returns (X, resid[n_outer]), plus the final Bregman variable b [9, n, n]
    when ``return_b`` is set."""
    y = _f64(y)
    x = np.zeros((g.n, g.n)) if x0 is None else _f64(x0).copy()
    resid = np.zeros(max(n_outer, 1))
    b = np.zeros((9, g.n, g.n)) if return_b else None
    p = _Params(float(lam), float(mu), int(n_outer), int(n_cg), int(reg), int(filter))
    _check(_load().orc_solve(g.ref, _ptr(y), ctypes.byref(p), _ptr(x), _ptr(resid),
                             _ptr(b) if return_b else None), "solve")
    return (x, resid[:n_outer], b) if return_b else (x, resid[:n_outer])
