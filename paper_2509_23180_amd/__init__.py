"""Python binding of the MI355X FFT-preconditioned domain-decomposition solver.

Argument marshalling only: every step of the solve runs in the HIP library
`libfds.so` built from `csrc/` (see `build.py`).  PyTorch supplies device
memory and streams.  Importing this module does not load the library; the
first call does, and it raises if the library is missing or no GPU is present.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
# FDS_LIB selects another build of the library (e.g. a build variant)
LIB_PATH = os.environ.get("FDS_LIB") or os.path.join(HERE, "libfds.so")

FDS_OK = 0
FDS_PENDING = 1
STATUS = {0: "ok", 1: "pending", -1: "invalid argument", -2: "unsupported geometry",
          -3: "unsupported", -4: "singular", -5: "out of memory", -6: "not converged",
          -7: "non-finite input", -8: "device error", -9: "unsupported boundary condition"}
FLAG_INTERFACE_KRYLOV = 1   # fds_options.flags: Krylov basis on the centre's interface lines
BC_DIRICHLET = 0
BC_NEUMANN = 1
BC_PERIODIC = 2
FP64 = 0
FP32_PRECOND = 1
NO_PRECOND = 2       # P = I: the convergence baseline (flexible GMRES, z = v in FP32)
JACOBI = 3           # P = diag(L_c): the second baseline (flexible GMRES, z = P^-1 v in FP32)
STOP = {0: "none", 1: "tol", 2: "at_floor", 3: "max_cycles", 4: "stagnation"}

TIMING_CLASSES = {"dst": 0, "tridiag": 1, "operator": 2, "gram_dots": 3, "lines": 4, "other": 5,
                  "gram_update": 6, "cols": 7}


class FdsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Rect(ctypes.Structure):
    _fields_ = [("i0", ctypes.c_int32), ("j0", ctypes.c_int32), ("i1", ctypes.c_int32),
                ("j1", ctypes.c_int32)]


class _Bc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("edge_kinds", ctypes.POINTER(ctypes.c_int32))]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("admitted_mid_flight", ctypes.c_uint64),
                ("cycles", ctypes.c_uint64), ("queued", ctypes.c_int32), ("running", ctypes.c_int32),
                ("bytes_in_use", ctypes.c_uint64), ("peak_bytes_in_use", ctypes.c_uint64),
                ("host_admit_s", ctypes.c_double), ("host_retire_s", ctypes.c_double),
                ("host_tasks_s", ctypes.c_double), ("host_launch_s", ctypes.c_double),
                ("host_wait_s", ctypes.c_double)]


class _Options(ctypes.Structure):
    _fields_ = [("restart_m", ctypes.c_int32), ("max_cycles", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("cycles", ctypes.c_int32), ("stop_reason", ctypes.c_int32),
                ("relres_schur", ctypes.c_double), ("relres_global", ctypes.c_double),
                ("seconds", ctypes.c_double)]


@dataclass
class Result:
    status: int
    iterations: int
    cycles: int
    stop_reason: str
    relres_schur: float
    relres_global: float
    seconds: float

    @staticmethod
    def from_c(r: _Result) -> "Result":
        return Result(r.status, r.iterations, r.cycles, STOP.get(r.stop_reason, str(r.stop_reason)),
                      r.relres_schur, r.relres_global, r.seconds)


_lib = None

# exported symbols declared in include/fds.h
SYMBOLS = (
    "fds_plan_create", "fds_plan_destroy", "fds_plan_layout", "fds_plan_footprint", "fds_solve",
    "fds_solve_batch", "fds_server_create", "fds_server_destroy", "fds_batch_submit",
    "fds_batch_poll",
    "fds_batch_wait_any", "fds_server_stats_get", "fds_k_dst_rows", "fds_k_dst_rows_f32", "fds_k_tridiag_modes",
    "fds_k_tridiag_modes_f32", "fds_k_rect_solve", "fds_k_centre_operator", "fds_k_arnoldi_mgs",
    "fds_k_arnoldi_mgs_noalloc",
    "fds_status_str", "fds_last_error", "fds_timing_enable", "fds_timing_read", "fds_timing_bytes",
    "fds_timing_reset",
)


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libfds.so (no GPU needed to load).  Raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FdsError(-8, f"{path} is missing: run __graft_entry__.build() (or python "
                           f"paper_2509_23180_amd/build.py) first")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I32, I64, D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "fds_plan_create": ([ctypes.POINTER(_Rect), I32, D, D, ctypes.POINTER(_Bc),
                             ctypes.POINTER(_Options), ctypes.POINTER(P)], I32),
        "fds_plan_destroy": ([P], None),
        "fds_plan_layout": ([P, ctypes.POINTER(I64), ctypes.POINTER(I64)], I32),
        "fds_plan_footprint": ([P, ctypes.POINTER(ctypes.c_size_t)], I32),
        "fds_solve": ([P, P, P, P, D, P, ctypes.POINTER(_Result)], I32),
        "fds_solve_batch": ([ctypes.POINTER(P), I32, ctypes.POINTER(P), ctypes.POINTER(P),
                             ctypes.POINTER(P), ctypes.POINTER(D), P, ctypes.POINTER(_Result)], I32),
        "fds_server_create": ([ctypes.c_size_t, I32, ctypes.POINTER(P)], I32),
        "fds_server_destroy": ([P], None),
        "fds_batch_submit": ([P, P, P, P, P, D, P, ctypes.POINTER(ctypes.c_uint64)], I32),
        "fds_batch_poll": ([P, ctypes.c_uint64, ctypes.POINTER(_Result)], I32),
        "fds_batch_wait_any": ([P, I64, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_Result)], I32),
        "fds_server_stats_get": ([P, ctypes.POINTER(_ServerStats)], I32),
        "fds_k_dst_rows": ([P, P, I32, I32, D, P], I32),
        "fds_k_dst_rows_f32": ([P, P, I32, I32, ctypes.c_float, P], I32),
        "fds_k_tridiag_modes": ([P, I32, I32, D, D, D, P], I32),
        "fds_k_tridiag_modes_f32": ([P, I32, I32, D, D, D, P], I32),
        "fds_k_rect_solve": ([P, P, I32, I32, D, D, I32, P], I32),
        "fds_k_centre_operator": ([P, P, P, P], I32),
        "fds_k_arnoldi_mgs": ([P, I32, I64, P, P], I32),
        "fds_k_arnoldi_mgs_noalloc": ([P, I32, I64, P, P], I32),
        "fds_status_str": ([I32], ctypes.c_char_p),
        "fds_last_error": ([], ctypes.c_char_p),
        "fds_timing_enable": ([I32], I32),
        "fds_timing_read": ([I32, ctypes.POINTER(I64), ctypes.POINTER(D)], I32),
        "fds_timing_bytes": ([I32, ctypes.POINTER(D)], I32),
        "fds_timing_reset": ([], I32),
    }
    for name, (args, ret) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ret
    _lib = lib
    return lib


def _check(status: int, allow=(FDS_OK,)) -> int:
    if status not in allow:
        msg = load_library().fds_last_error().decode()
        raise FdsError(status, msg)
    return status


def _require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise FdsError(-8, "no HIP device available")
    load_library()


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


# --------------------------------------------------------------------------- plans

def _bc_struct(bc_kind: int, edge_kinds: Optional[Sequence[int]], nrect: int):
    if edge_kinds is None:
        return _Bc(int(bc_kind), None), None
    if len(edge_kinds) != 4 * nrect:
        raise ValueError("edge_kinds needs 4 entries per rectangle")
    arr = (ctypes.c_int32 * len(edge_kinds))(*map(int, edge_kinds))
    return _Bc(int(bc_kind), ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))), arr


class Plan:
    """fds_plan_create wrapper.  rects: closed node boxes (i0, j0, i1, j1).
    bc_kind / edge_kinds: boundary-condition kinds (BC_*; edge_kinds has four
    per rectangle, sides j=j0, i=i1, j=j1, i=i0)."""

    def __init__(self, rects: Sequence[Tuple[int, int, int, int]], h: float, kappa: float,
                 restart_m: int = 30, max_cycles: int = 200, precision: int = FP64,
                 bc_kind: int = BC_DIRICHLET, edge_kinds: Optional[Sequence[int]] = None,
                 flags: int = 0):
        _require_gpu()
        lib = load_library()
        arr = (_Rect * len(rects))(*[_Rect(*map(int, r)) for r in rects])
        opt = _Options(restart_m, max_cycles, precision, int(flags))
        bc, _keep = _bc_struct(bc_kind, edge_kinds, len(rects))
        out = ctypes.c_void_p()
        _check(lib.fds_plan_create(arr, len(rects), float(h), float(kappa), ctypes.byref(bc),
                                   ctypes.byref(opt), ctypes.byref(out)))
        self._h = out
        self.rects = [tuple(map(int, r)) for r in rects]
        self.h = float(h)
        self.kappa = float(kappa)
        self.restart_m = restart_m
        self.precision = precision
        self.flags = int(flags)
        n = len(rects)
        uo = (ctypes.c_int64 * (n + 1))()
        bo = (ctypes.c_int64 * (n + 1))()
        _check(lib.fds_plan_layout(self._h, uo, bo))
        self.unknown_offsets = list(uo)
        self.bc_offsets = list(bo)
        fp = ctypes.c_size_t()
        _check(lib.fds_plan_footprint(self._h, ctypes.byref(fp)))
        self.footprint = fp.value

    @property
    def n_unknowns(self) -> int:
        return self.unknown_offsets[-1]

    @property
    def n_bc(self) -> int:
        return self.bc_offsets[-1]

    def close(self):
        if getattr(self, "_h", None):
            load_library().fds_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(plan: Plan, rhs, x, tol: float, bc=None, stream=None) -> Result:
    """Blocking solve; returns the Result (raises on argument/device errors,
    not on FDS_E_NOT_CONVERGED / FDS_E_NONFINITE, which are in Result.status)."""
    lib = load_library()
    res = _Result()
    st = lib.fds_solve(plan._h, _ptr(rhs), _ptr(bc), _ptr(x), float(tol), _stream(stream),
                       ctypes.byref(res))
    _check(st, allow=(FDS_OK, -6, -7))
    return Result.from_c(res)


def solve_batch(plans: Sequence[Plan], rhs: Sequence, xs: Sequence, tols: Sequence[float],
                bcs: Optional[Sequence] = None, stream=None) -> List[Result]:
    lib = load_library()
    n = len(plans)
    P = ctypes.c_void_p
    ph = (P * n)(*[p._h for p in plans])
    rh = (P * n)(*[_ptr(r) for r in rhs])
    xh = (P * n)(*[_ptr(x) for x in xs])
    bh = (P * n)(*[_ptr(b) for b in bcs]) if bcs is not None else None
    th = (ctypes.c_double * n)(*map(float, tols))
    res = (_Result * n)()
    st = lib.fds_solve_batch(ph, n, rh, bh, xh, th, _stream(stream), res)
    _check(st, allow=(FDS_OK, -6, -7))
    return [Result.from_c(r) for r in res]


class Server:
    """Continuous-batching request server (fds_server_*)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int):
        _require_gpu()
        lib = load_library()
        out = ctypes.c_void_p()
        _check(lib.fds_server_create(int(hbm_budget_bytes), int(max_slots), ctypes.byref(out)))
        self._h = out
        self._held = {}   # ticket -> (plan, rhs, bc, x): alive until the result is collected
        import threading
        self._lock = threading.Lock()

    def submit(self, plan: Plan, rhs, x, tol: float, bc=None, stream=None) -> int:
        """Queue a solve.  The server reads rhs/bc after the work queued on
        `stream` (default: the current torch stream) up to this call."""
        t = ctypes.c_uint64()
        with self._lock:   # registered before a waiter can collect the ticket
            _check(load_library().fds_batch_submit(self._h, plan._h, _ptr(rhs), _ptr(bc), _ptr(x),
                                                   float(tol), _stream(stream), ctypes.byref(t)))
            self._held[t.value] = (plan, rhs, bc, x)
        return t.value

    def poll(self, ticket: int) -> Optional[Result]:
        res = _Result()
        st = load_library().fds_batch_poll(self._h, int(ticket), ctypes.byref(res))
        if st == FDS_PENDING:
            return None
        with self._lock:
            self._held.pop(int(ticket), None)
        _check(st, allow=(FDS_OK, -6, -7))
        return Result.from_c(res)

    def wait_any(self, timeout_s: Optional[float] = None) -> Optional[Tuple[int, Result]]:
        """The next finished request, (ticket, Result), waiting at most
        timeout_s seconds (None: no limit); None on time-out."""
        t = ctypes.c_uint64()
        res = _Result()
        us = -1 if timeout_s is None else int(timeout_s * 1e6)
        st = load_library().fds_batch_wait_any(self._h, us, ctypes.byref(t), ctypes.byref(res))
        if st == FDS_PENDING:
            return None
        with self._lock:
            self._held.pop(t.value, None)
        _check(st, allow=(FDS_OK, -6, -7))
        return t.value, Result.from_c(res)

    def stats(self) -> dict:
        s = _ServerStats()
        _check(load_library().fds_server_stats_get(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in _ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            load_library().fds_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------- kernel-level calls

def dst_rows(inp, out, scale: float = 1.0, stream=None):
    import torch
    rows, n = inp.shape
    lib = load_library()
    if inp.dtype == torch.float64:
        _check(lib.fds_k_dst_rows(_ptr(inp), _ptr(out), rows, n, float(scale), _stream(stream)))
    else:
        _check(lib.fds_k_dst_rows_f32(_ptr(inp), _ptr(out), rows, n, float(scale), _stream(stream)))


def tridiag_modes(data, h: float, kappa: float, scale: float = 1.0, stream=None):
    import torch
    rows, modes = data.shape
    lib = load_library()
    fn = lib.fds_k_tridiag_modes if data.dtype == torch.float64 else lib.fds_k_tridiag_modes_f32
    _check(fn(_ptr(data), rows, modes, float(h), float(kappa), float(scale), _stream(stream)))


def rect_solve(f, z, h: float, kappa: float, precision: int = FP64, stream=None):
    rows, cols = f.shape
    _check(load_library().fds_k_rect_solve(_ptr(f), _ptr(z), rows, cols, float(h), float(kappa),
                                           int(precision), _stream(stream)))


def centre_operator(plan: Plan, z, w, stream=None):
    _check(load_library().fds_k_centre_operator(plan._h, _ptr(z), _ptr(w), _stream(stream)))


def arnoldi_mgs(V, k: int, h, stream=None):
    _check(load_library().fds_k_arnoldi_mgs(_ptr(V), int(k), int(V.shape[1]), _ptr(h),
                                            _stream(stream)))


def arnoldi_mgs_noalloc(V, k: int, h, stream=None):
    """fds_k_arnoldi_mgs_noalloc: the same step with the library's fixed
    per-device working memory (no device allocation)."""
    _check(load_library().fds_k_arnoldi_mgs_noalloc(_ptr(V), int(k), int(V.shape[1]), _ptr(h),
                                                    _stream(stream)))


def timing_enable(classes=None):
    """Time the given kernel classes (names of TIMING_CLASSES; None = all,
    [] = off)."""
    if classes is None:
        mask = 0xFF
    else:
        mask = 0
        for c in classes:
            mask |= 1 << TIMING_CLASSES[c]
    _check(load_library().fds_timing_enable(mask))


def timing_reset():
    _check(load_library().fds_timing_reset())


def timing_read(cls: str) -> Tuple[int, float, float]:
    """(launches, total milliseconds, algorithmic bytes) of a kernel class."""
    c = ctypes.c_int64()
    ms = ctypes.c_double()
    b = ctypes.c_double()
    lib = load_library()
    _check(lib.fds_timing_read(TIMING_CLASSES[cls], ctypes.byref(c), ctypes.byref(ms)))
    _check(lib.fds_timing_bytes(TIMING_CLASSES[cls], ctypes.byref(b)))
    return c.value, ms.value, b.value
