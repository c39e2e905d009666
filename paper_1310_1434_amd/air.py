"""ctypes binding of libair.so, the MI355X AIR library (C ABI in include/air.h).

Argument marshalling only: every step of the reconstruction runs in the HIP
kernels of libair.so.  torch provides device memory and streams; tensors are
passed as raw device pointers on the current torch stream.  There is no CPU
fallback: if libair.so is missing this module raises at import time.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libair.so")

AIR_OK, AIR_E_INVALID, AIR_E_UNSUPPORTED, AIR_E_NOMEM, AIR_E_HIP, AIR_E_NONFINITE = 0, -1, -2, -3, -4, -5
PRECISIONS = {"fp32": 0, "mixed_f16": 1, "mixed_bf16": 2}
# plan flags: ramp window (bits 0-3) and symmetric cosine weighting of C
RAMP_WINDOWS = {"ram-lak": 0, "shepp-logan": 1, "hann": 2}
AIR_RAMP_COSINE_WEIGHTED = 16


class AirError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


class NonFiniteResult(AirError):
    """AIR_E_NONFINITE from air_state_retire: the slot was copied out and freed,
    but its residual history holds a non-finite value.  ``x`` and ``resid`` are
    the copied-out image and history."""

    def __init__(self, where: str, msg: str, x, resid):
        super().__init__(AIR_E_NONFINITE, where, msg)
        self.x, self.resid = x, resid


class _Geometry(ctypes.Structure):
    _fields_ = [("beam", ctypes.c_int), ("n", ctypes.c_int32), ("pixel_mm", ctypes.c_double),
                ("n_views", ctypes.c_int32), ("view_cos", ctypes.c_void_p), ("view_sin", ctypes.c_void_p),
                ("n_bins", ctypes.c_int32), ("bin_mm", ctypes.c_double), ("sod_mm", ctypes.c_double),
                ("sdd_mm", ctypes.c_double)]


class _SolveParams(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_double), ("mu", ctypes.c_double), ("n_outer", ctypes.c_int32),
                ("n_cg", ctypes.c_int32), ("reg", ctypes.c_int32), ("filter", ctypes.c_int32)]


KERNEL_KINDS = ("project", "backproject", "ramp", "cg", "framelet", "other")
# air_kernel_timing_enable modes
TIMING_MODES = {"off": 0, "on": 1, "one_stream": 2}


class _KernelStats(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * len(KERNEL_KINDS)), ("launches", ctypes.c_int64 * len(KERNEL_KINDS))]


# Every symbol include/air.h declares, with its ctypes signature.
_P = ctypes.c_void_p
_I = ctypes.c_int32
SIGNATURES = {
    "air_plan_create": ([ctypes.POINTER(_Geometry), _I, ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(_P)], ctypes.c_int),
    "air_plan_workspace_size": ([_P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "air_plan_bind_workspace": ([_P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "air_plan_tables": ([_P, _P, _P, _P], ctypes.c_int),
    "air_plan_destroy": ([_P], None),
    "air_project": ([_P, _P, _P, _I, _P], ctypes.c_int),
    "air_ramp": ([_P, _P, _P, _I, _P], ctypes.c_int),
    "air_filtered_backproject": ([_P, _P, _P, _I, _I, _P], ctypes.c_int),
    "air_normal_apply": ([_P, _P, _P, _I, ctypes.c_double, _I, _P], ctypes.c_int),
    "air_framelet": ([_P, _P, _P, _I, _I, _P], ctypes.c_int),
    "air_solve_workspace_size": ([_P, _I, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "air_solve": ([_P, _P, _P, _I, ctypes.POINTER(_SolveParams), _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "air_solve_noalloc": ([_P, _P, _P, _I, ctypes.POINTER(_SolveParams), _P, _P], ctypes.c_int),
    "air_state_workspace_size": ([_P, _I, ctypes.POINTER(_SolveParams), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "air_state_create": ([_P, _I, ctypes.POINTER(_SolveParams), _P, ctypes.c_size_t, ctypes.POINTER(_P)], ctypes.c_int),
    "air_state_destroy": ([_P], None),
    "air_state_admit": ([_P, _P, _P, _I, _P, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "air_state_step": ([_P, _I, _P, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "air_state_query": ([_P, _I, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "air_state_active": ([_P, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "air_state_poll": ([_P, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "air_state_retire": ([_P, _I, _P, _P, _P], ctypes.c_int),
    "air_state_snapshot_size": ([_P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "air_state_snapshot": ([_P, _I, _P, _P], ctypes.c_int),
    "air_state_restore": ([_P, _P, _P, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "air_kernel_timing_enable": ([_P, _I], ctypes.c_int),
    "air_kernel_timing_collect": ([_P, ctypes.POINTER(_KernelStats)], ctypes.c_int),
    "air_last_error": ([], ctypes.c_char_p),
}


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1310_1434_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def _check(status: int, where: str):
    if status != AIR_OK:
        raise AirError(status, where, lib.air_last_error().decode())


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_f32(t: torch.Tensor, device, shape, name):
    if not isinstance(t, torch.Tensor) or t.device != device or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 tensor on {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _geometry_struct(geom):
    cos = np.ascontiguousarray(geom.view_cos, dtype=np.float64)
    sin = np.ascontiguousarray(geom.view_sin, dtype=np.float64)
    g = _Geometry(0 if geom.beam == "parallel" else 1, int(geom.n), float(geom.pixel), int(geom.n_views),
                  cos.ctypes.data, sin.ctypes.data, int(geom.n_bins), float(geom.bin),
                  float(getattr(geom, "sod", 0.0)), float(getattr(geom, "sdd", 0.0)))
    return g, (cos, sin)


def host_tables(geom):
    """Index tables of a geometry, built on the host (no GPU needed):
    (axis int8, lo int32, hi int32), each [n_views, n_bins]."""
    g, keep = _geometry_struct(geom)
    h = ctypes.c_void_p()
    _check(lib.air_plan_create(ctypes.byref(g), 1, 0, 0, ctypes.byref(h)), "air_plan_create")
    try:
        nr = int(geom.n_views) * int(geom.n_bins)
        axis = np.empty(nr, np.int8)
        lo = np.empty(nr, np.int32)
        hi = np.empty(nr, np.int32)
        _check(lib.air_plan_tables(h, axis.ctypes.data, lo.ctypes.data, hi.ctypes.data), "air_plan_tables")
    finally:
        lib.air_plan_destroy(h)
    s = (int(geom.n_views), int(geom.n_bins))
    return axis.reshape(s), lo.reshape(s), hi.reshape(s)


def workspace_sizes(geom, capacity: int, lam: float, mu: float, n_cg: int, max_outer: int,
                    precision: str = "fp32", filter: int = 1) -> tuple[int, int]:
    """Device bytes of (the workspace of a max_batch = 1 plan of this geometry, a
    solve-slot state of `capacity` slots on it), from a host-only plan (no GPU)."""
    g, keep = _geometry_struct(geom)
    h = ctypes.c_void_p()
    _check(lib.air_plan_create(ctypes.byref(g), 1, PRECISIONS[precision], 0, ctypes.byref(h)), "air_plan_create")
    try:
        ps, ss = ctypes.c_size_t(), ctypes.c_size_t()
        prm = _SolveParams(float(lam), float(mu), int(max_outer), int(n_cg), 0, int(filter))
        _check(lib.air_plan_workspace_size(h, ctypes.byref(ps)), "air_plan_workspace_size")
        _check(lib.air_state_workspace_size(h, int(capacity), ctypes.byref(prm), ctypes.byref(ss)),
               "air_state_workspace_size")
    finally:
        lib.air_plan_destroy(h)
    return max(int(ps.value), 256), max(int(ss.value), 256)


class Plan:
    """A scan geometry with its device tables.

    ``geom`` is any object with the fields beam ("parallel"/"fan"), n, pixel,
    n_views, n_bins, bin, sod, sdd, view_cos, view_sin (float64 arrays).
    """

    def __init__(self, geom, max_batch: int = 1, precision: str = "fp32", device="cuda:0",
                 ramp: str = "ram-lak", cosine_weight: bool = False):
        """ramp / cosine_weight select the filtration C (the plan flags of air.h)."""
        if ramp not in RAMP_WINDOWS:
            raise ValueError(f"ramp must be one of {sorted(RAMP_WINDOWS)}")
        flags = RAMP_WINDOWS[ramp] | (AIR_RAMP_COSINE_WEIGHTED if cosine_weight else 0)
        self.ramp_window, self.cosine_weight = ramp, bool(cosine_weight)
        self.device = torch.device(device)
        self.n, self.n_views, self.n_bins = int(geom.n), int(geom.n_views), int(geom.n_bins)
        self.precision = precision
        self.max_batch = int(max_batch)
        g, self._keep = _geometry_struct(geom)
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        h = ctypes.c_void_p()
        _check(lib.air_plan_create(ctypes.byref(g), self.max_batch, PRECISIONS[precision], flags, ctypes.byref(h)),
               "air_plan_create")
        self._h = h
        size = ctypes.c_size_t()
        _check(lib.air_plan_workspace_size(h, ctypes.byref(size)), "air_plan_workspace_size")
        self._ws = torch.empty(max(int(size.value), 256), dtype=torch.uint8, device=self.device)
        _check(lib.air_plan_bind_workspace(h, ctypes.c_void_p(self._ws.data_ptr()), size.value,
                                           _stream(self.device)), "air_plan_bind_workspace")

    def __del__(self):
        h = getattr(self, "_h", None)
        # (at interpreter exit the module's globals may already be gone)
        if h is not None and h.value and lib is not None:
            lib.air_plan_destroy(h)
            self._h = None

    # ---- per-kernel event timing
    def kernel_timing(self, mode) -> None:
        """mode: "off", "on" (solves keep their two sub-batch streams) or
        "one_stream" (kernels run alone); True means "on", False "off"."""
        if isinstance(mode, bool):
            mode = "on" if mode else "off"
        _check(lib.air_kernel_timing_enable(self._h, TIMING_MODES[mode]), "air_kernel_timing_enable")

    def collect_kernel_timing(self) -> dict:
        """{kind: (total_ms, launches)} for the launches recorded since the last collect."""
        st = _KernelStats()
        _check(lib.air_kernel_timing_collect(self._h, ctypes.byref(st)), "air_kernel_timing_collect")
        return {k: (st.ms[i], int(st.launches[i])) for i, k in enumerate(KERNEL_KINDS)}

    # ---- host tables
    def tables(self):
        nr = self.n_views * self.n_bins
        axis = np.empty(nr, np.int8)
        lo = np.empty(nr, np.int32)
        hi = np.empty(nr, np.int32)
        _check(lib.air_plan_tables(self._h, axis.ctypes.data, lo.ctypes.data, hi.ctypes.data), "air_plan_tables")
        s = (self.n_views, self.n_bins)
        return axis.reshape(s), lo.reshape(s), hi.reshape(s)

    # ---- operators (batch = leading dimension)
    def _img(self, x, name="x"):
        return _dev_f32(x, self.device, (x.shape[0], self.n, self.n), name)

    def _sino(self, y, name="y"):
        return _dev_f32(y, self.device, (y.shape[0], self.n_views, self.n_bins), name)

    def project(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        b = x.shape[0]
        y = out if out is not None else torch.empty((b, self.n_views, self.n_bins), device=self.device)
        _check(lib.air_project(self._h, self._img(x), self._sino(y, "out"), b, _stream(self.device)), "air_project")
        return y

    def ramp(self, y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        b = y.shape[0]
        yf = out if out is not None else torch.empty_like(y)
        _check(lib.air_ramp(self._h, self._sino(y), self._sino(yf, "out"), b, _stream(self.device)), "air_ramp")
        return yf

    def filtered_backproject(self, y: torch.Tensor, filter: int = 1, out: torch.Tensor | None = None) -> torch.Tensor:
        b = y.shape[0]
        x = out if out is not None else torch.empty((b, self.n, self.n), device=self.device)
        _check(lib.air_filtered_backproject(self._h, self._sino(y), self._img(x, "out"), b, int(filter),
                                            _stream(self.device)), "air_filtered_backproject")
        return x

    def normal_apply(self, x: torch.Tensor, mu: float, filter: int = 1, out=None) -> torch.Tensor:
        b = x.shape[0]
        o = out if out is not None else torch.empty_like(x)
        _check(lib.air_normal_apply(self._h, self._img(x), self._img(o, "out"), b, float(mu), int(filter),
                                    _stream(self.device)), "air_normal_apply")
        return o

    def framelet(self, x: torch.Tensor) -> torch.Tensor:
        b = x.shape[0]
        z = torch.empty((b, 9, self.n, self.n), device=self.device)
        _check(lib.air_framelet(self._h, self._img(x), ctypes.c_void_p(z.data_ptr()), b, 0, _stream(self.device)),
               "air_framelet")
        return z

    def framelet_adjoint(self, z: torch.Tensor) -> torch.Tensor:
        b = z.shape[0]
        _dev_f32(z, self.device, (b, 9, self.n, self.n), "z")
        x = torch.empty((b, self.n, self.n), device=self.device)
        _check(lib.air_framelet(self._h, ctypes.c_void_p(z.data_ptr()), self._img(x, "out"), b, 1,
                                _stream(self.device)), "air_framelet")
        return x

    # ---- solver
    def solve_workspace_bytes(self, batch: int) -> int:
        size = ctypes.c_size_t()
        _check(lib.air_solve_workspace_size(self._h, int(batch), ctypes.byref(size)), "air_solve_workspace_size")
        return int(size.value)

    def solve(self, y: torch.Tensor, lam: float, mu: float, n_outer: int, n_cg: int, reg: int = 0,
              filter: int = 1, x0: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
              with_resid: bool = True):
        """Split Bregman AIR (reg=0), the L2 problem of Eq. (5) (reg=1), or forward-backward
        splitting of Eq. (6) (reg=2, mu = the step).

        Returns (X [B, n, n], resid [B, n_outer] float64 or None); asynchronous
        on the current stream (a batch of 8 or more runs as two halves on two
        library streams forked from and joined back to it; same results)."""
        b = y.shape[0]
        x = torch.zeros((b, self.n, self.n), device=self.device) if x0 is None else x0.clone()
        need = self.solve_workspace_bytes(b)
        ws = workspace if workspace is not None else torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        if ws.numel() < need:
            raise ValueError("workspace too small")
        resid = torch.zeros((b, max(n_outer, 1)), dtype=torch.float64, device=self.device) if with_resid else None
        p = _SolveParams(float(lam), float(mu), int(n_outer), int(n_cg), int(reg), int(filter))
        _check(lib.air_solve(self._h, self._sino(y), self._img(x), b, ctypes.byref(p),
                             ctypes.c_void_p(resid.data_ptr()) if resid is not None else None,
                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(self.device)), "air_solve")
        if resid is not None:
            resid = resid[:, :n_outer]
        return x, resid

    def solve_noalloc(self, y: torch.Tensor, x: torch.Tensor, lam: float, mu: float, n_outer: int, n_cg: int,
                      reg: int = 0, filter: int = 1, resid: torch.Tensor | None = None) -> None:
        """air_solve_noalloc: the solve with the library's static scratch, on the
        current stream; x [B, n, n] holds the start image and receives the
        result, resid (float64 [B, n_outer], optional) the residual history.
        Nothing is allocated here either: the caller passes every tensor."""
        b = y.shape[0]
        if resid is not None and (resid.dtype != torch.float64 or tuple(resid.shape) != (b, max(n_outer, 1))
                                  or resid.device != self.device or not resid.is_contiguous()):
            raise ValueError("resid must be a contiguous float64 tensor [batch, n_outer] on the plan's device")
        p = _SolveParams(float(lam), float(mu), int(n_outer), int(n_cg), int(reg), int(filter))
        _check(lib.air_solve_noalloc(self._h, self._sino(y), self._img(x), b, ctypes.byref(p),
                                     ctypes.c_void_p(resid.data_ptr()) if resid is not None else None,
                                     _stream(self.device)), "air_solve_noalloc")


class State:
    """Device-resident solve slots of one plan (continuous batching, see air_state_* in air.h).

    All calls are queued on ``stream`` (a torch.cuda.Stream; the current stream if
    None).  Steps on a non-default stream replay a captured HIP graph."""

    def __init__(self, plan: Plan, capacity: int, lam: float, mu: float, n_cg: int, max_outer: int,
                 filter: int = 1, stream=None):
        self.plan = plan
        self.stream = stream
        self.capacity = int(capacity)
        self.max_outer = int(max_outer)
        self._params = _SolveParams(float(lam), float(mu), int(max_outer), int(n_cg), 0, int(filter))
        size = ctypes.c_size_t()
        _check(lib.air_state_workspace_size(plan._h, self.capacity, ctypes.byref(self._params), ctypes.byref(size)),
               "air_state_workspace_size")
        self.workspace_bytes = int(size.value)
        with torch.cuda.stream(self._torch_stream()):
            self._ws = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device=plan.device)
        h = ctypes.c_void_p()
        _check(lib.air_state_create(plan._h, self.capacity, ctypes.byref(self._params),
                                    ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel(), ctypes.byref(h)),
               "air_state_create")
        self._h = h
        self._inputs = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.air_state_destroy(h)
            self._h = None

    def _torch_stream(self):
        return self.stream if self.stream is not None else torch.cuda.current_stream(self.plan.device)

    def _s(self):
        return ctypes.c_void_p(self._torch_stream().cuda_stream)

    @property
    def active(self) -> int:
        c = ctypes.c_int32()
        _check(lib.air_state_active(self._h, ctypes.byref(c)), "air_state_active")
        return int(c.value)

    def admit(self, y: torch.Tensor, x0: torch.Tensor | None = None, n_outer: int | None = None) -> int:
        """Start a reconstruction of sinogram y [V, D] (device); returns its slot id."""
        p = self.plan
        _dev_f32(y, p.device, (p.n_views, p.n_bins), "y")
        if x0 is not None:
            _dev_f32(x0, p.device, (p.n, p.n), "x0")
        slot = ctypes.c_int32()
        _check(lib.air_state_admit(self._h, ctypes.c_void_p(y.data_ptr()),
                                   ctypes.c_void_p(x0.data_ptr()) if x0 is not None else None,
                                   int(n_outer if n_outer is not None else self.max_outer), self._s(),
                                   ctypes.byref(slot)), "air_state_admit")
        st = self._torch_stream()
        y.record_stream(st)
        if x0 is not None:
            x0.record_stream(st)
        return int(slot.value)

    def step(self, max_iters: int = 1) -> int:
        done = ctypes.c_int32()
        _check(lib.air_state_step(self._h, int(max_iters), self._s(), ctypes.byref(done)), "air_state_step")
        return int(done.value)

    def finished(self) -> list[int]:
        """Slots through all their iterations (air_state_poll's bitmask)."""
        words = (self.capacity + 31) // 32
        mask = (ctypes.c_int32 * words)()
        _check(lib.air_state_poll(self._h, mask), "air_state_poll")
        return [s for s in range(self.capacity) if (mask[s // 32] & 0xFFFFFFFF) >> (s % 32) & 1]

    def query(self, slot: int):
        it, no = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.air_state_query(self._h, int(slot), ctypes.byref(it), ctypes.byref(no)), "air_state_query")
        return int(it.value), int(no.value)

    def retire(self, slot: int):
        """Copy out (X [n, n], resid [n_outer] float64) and free the slot (the
        library synchronises the state's stream once).  Raises NonFiniteResult,
        which carries both, if the residual history holds a non-finite value."""
        _, n_outer = self.query(slot)
        p = self.plan
        with torch.cuda.stream(self._torch_stream()):
            x = torch.empty((p.n, p.n), device=p.device)
            r = torch.empty((n_outer,), dtype=torch.float64, device=p.device)
        st = lib.air_state_retire(self._h, int(slot), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(r.data_ptr()),
                                  self._s())
        if st == AIR_E_NONFINITE:
            raise NonFiniteResult("air_state_retire", lib.air_last_error().decode(), x, r)
        _check(st, "air_state_retire")
        return x, r

    def snapshot(self, slot: int) -> np.ndarray:
        size = ctypes.c_size_t()
        _check(lib.air_state_snapshot_size(self._h, ctypes.byref(size)), "air_state_snapshot_size")
        buf = np.empty(int(size.value), np.uint8)
        _check(lib.air_state_snapshot(self._h, int(slot), ctypes.c_void_p(buf.ctypes.data), self._s()),
               "air_state_snapshot")
        self._torch_stream().synchronize()
        return buf

    def restore(self, buf: np.ndarray) -> int:
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        slot = ctypes.c_int32()
        _check(lib.air_state_restore(self._h, ctypes.c_void_p(buf.ctypes.data), self._s(), ctypes.byref(slot)),
               "air_state_restore")
        return int(slot.value)
