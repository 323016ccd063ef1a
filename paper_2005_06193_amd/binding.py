"""ctypes binding of libegfem (include/egfem.h).

Argument marshalling only: torch tensors supply device memory and the current
HIP stream; every step of the computation runs in the library's HIP kernels.
There is no CPU fallback: without the built library (or without a HIP device)
every call raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import warnings
import weakref
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libegfem.so")

EGFEM_OK = 0
EGFEM_NOT_CONVERGED = 1
EGFEM_BREAKDOWN = 2
EGFEM_NONFINITE = 3
EGFEM_STAGNATED = 4
EGFEM_ERR_ARG = -1
EGFEM_ERR_SHAPE = -2
EGFEM_ERR_OOM = -3
EGFEM_ERR_HIP = -4
EGFEM_ERR_MESH = -5
STATUS_NAMES = {0: "ok", 1: "not_converged", 2: "breakdown", 3: "nonfinite", 4: "stagnated",
                -1: "err_arg", -2: "err_shape", -3: "err_oom", -4: "err_hip", -5: "err_mesh"}

FORM_STIFF = 0
FORM_MASS = 1
FORM_CONV = 2
W_P1 = 0
W_P2 = 1
W_IQ = 2
W_P0 = 3
HIST = 64


class EgfemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"egfem error {code} ({STATUS_NAMES.get(code, '?')}): {msg}")
        self.code = code


class _Info(C.Structure):
    _fields_ = [("dim", C.c_int), ("form", C.c_int), ("symmetric", C.c_int),
                ("n_nodes", C.c_int64), ("n_cells", C.c_int64), ("nnz", C.c_int64),
                ("nnz_b", C.c_int64), ("structural_nnz", C.c_int64), ("slots", C.c_int64),
                ("row_blocks", C.c_int64), ("device_bytes", C.c_int64),
                ("rowptr", C.c_void_p), ("col", C.c_void_p), ("kval", C.c_void_p),
                ("mval", C.c_void_p), ("wspace", C.c_int), ("n_w", C.c_int64), ("nnz_half", C.c_int64)]


class _Problem(C.Structure):
    _fields_ = [("a0", C.c_void_p), ("a0_const", C.c_double), ("load", C.c_void_p),
                ("dirichlet", C.c_void_p), ("add_stiffness", C.c_int)]


class _Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_newton", C.c_int), ("max_krylov", C.c_int),
                ("krylov_rtol", C.c_double), ("forcing", C.c_int), ("eta_max", C.c_double),
                ("max_backtracks", C.c_int), ("krylov_blocks", C.c_int),
                ("krylov_threads", C.c_int), ("timing", C.c_int)]


class _PicardOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_picard", C.c_int), ("max_krylov", C.c_int),
                ("krylov_rtol", C.c_double), ("krylov_blocks", C.c_int), ("krylov_threads", C.c_int),
                ("timing", C.c_int)]


class _PicardStats(C.Structure):
    _fields_ = [("status", C.c_int), ("picard_iters", C.c_int), ("krylov_iters", C.c_int),
                ("update", C.c_double), ("res0", C.c_double), ("res", C.c_double),
                ("update_hist", C.c_double * HIST), ("krylov_hist", C.c_int * HIST),
                ("t_matrix_ms", C.c_double), ("t_krylov_ms", C.c_double), ("krylov_kernels", C.c_int)]


class _BurgersOpts(C.Structure):
    _fields_ = [("dt", C.c_double), ("nu", C.c_double), ("steps", C.c_int), ("group", C.c_int),
                ("krylov_rtol", C.c_double), ("max_krylov", C.c_int), ("guess", C.c_int),
                ("krylov_blocks", C.c_int), ("krylov_threads", C.c_int), ("timing", C.c_int)]


class _BurgersStats(C.Structure):
    _fields_ = [("status", C.c_int), ("steps", C.c_int), ("krylov_iters", C.c_int64),
                ("max_step_krylov", C.c_int), ("max_relres", C.c_double), ("krylov_hist", C.c_int * HIST),
                ("t_rhs_ms", C.c_double), ("t_krylov_ms", C.c_double), ("krylov_kernels", C.c_int)]


class _GradCoef(C.Structure):
    _fields_ = [("c0", C.c_double), ("c1", C.c_double), ("q", C.c_double), ("start_linear", C.c_int)]


class _Shape(C.Structure):
    _fields_ = [("action_runs", C.c_int), ("action_pipe", C.c_int), ("krylov_blocks", C.c_int),
                ("krylov_threads", C.c_int), ("krylov_kernel", C.c_int), ("action_half", C.c_int),
                ("krylov_precond", C.c_int), ("krylov_cheb_ratio", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("status", C.c_int), ("newton_iters", C.c_int), ("krylov_iters", C.c_int),
                ("backtracks", C.c_int), ("res0", C.c_double), ("res", C.c_double),
                ("res_hist", C.c_double * HIST), ("krylov_hist", C.c_int * HIST),
                ("t_action_ms", C.c_double), ("t_jacobian_ms", C.c_double),
                ("t_krylov_ms", C.c_double), ("n_action", C.c_int), ("n_jacobian", C.c_int),
                ("n_krylov", C.c_int), ("krylov_status_hist", C.c_int * HIST),
                ("krylov_relres_hist", C.c_double * HIST), ("krylov_kernels", C.c_int)]


_lib = None

# Live handles and batch plans.  They own device memory, events, streams and
# graphs; an exit hook destroys them (batch plans first, they reference
# handles) while the HIP runtime is still up, instead of leaving it to object
# finalisers during interpreter shutdown.  The hook is registered after torch
# is imported, so it runs before torch's own exit hooks.
_live_tensors: "weakref.WeakSet" = weakref.WeakSet()
_live_batches: "weakref.WeakSet" = weakref.WeakSet()


def close_all() -> None:
    """Destroy every live batch plan, then every live tensor handle."""
    for b in list(_live_batches):
        b.close()
    for t in list(_live_tensors):
        t.close()


atexit.register(close_all)

EXPORTS = {
    "egfem_build_tensor": (C.c_int, [C.c_int, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                     C.c_int, C.c_double, C.POINTER(C.c_void_p)]),
    "egfem_build_tensor_w": (C.c_int, [C.c_int, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                       C.c_int, C.c_int, C.c_double, C.POINTER(C.c_void_p)]),
    "egfem_attach_elements": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]),
    "egfem_residual_elementwise": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "egfem_attach_unique": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                      C.POINTER(C.c_int64)]),
    "egfem_residual_unique": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "egfem_tensor_destroy": (None, [C.c_void_p]),
    "egfem_tensor_info": (C.c_int, [C.c_void_p, C.POINTER(_Info)]),
    "egfem_tensor_export": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "egfem_tensor_pattern": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "egfem_residual": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "egfem_jacobian": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "egfem_mode3": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "egfem_matvec": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                               C.c_void_p]),
    "egfem_problem_residual": (C.c_int, [C.c_void_p, C.POINTER(_Problem), C.c_void_p, C.c_void_p,
                                         C.POINTER(C.c_double), C.c_void_p]),
    "egfem_problem_residual_noalloc": (C.c_int, [C.c_void_p, C.POINTER(_Problem), C.c_void_p, C.c_void_p,
                                                 C.POINTER(C.c_double), C.c_void_p]),
    "egfem_problem_jacobian": (C.c_int, [C.c_void_p, C.POINTER(_Problem), C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_void_p]),
    "egfem_newton_opts_default": (None, [C.POINTER(_Opts)]),
    "egfem_newton": (C.c_int, [C.c_void_p, C.POINTER(_Problem), C.c_void_p, C.POINTER(_Opts),
                               C.POINTER(_Stats), C.c_void_p]),
    "egfem_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_double,
                              C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double), C.c_void_p]),
    "egfem_newton_batched": (C.c_int, [C.c_int, C.POINTER(C.c_void_p), C.POINTER(_Problem),
                                       C.POINTER(C.c_void_p), C.POINTER(_Opts), C.POINTER(_Stats),
                                       C.c_void_p]),
    "egfem_adjoint": (C.c_int, [C.c_void_p, C.POINTER(_Problem), C.c_void_p, C.c_void_p,
                                C.POINTER(_Opts), C.c_void_p, C.c_void_p, C.POINTER(C.c_int),
                                C.POINTER(C.c_double), C.c_void_p]),
    "egfem_batch_create": (C.c_int, [C.c_int, C.POINTER(C.c_void_p), C.POINTER(_Problem),
                                     C.POINTER(C.c_void_p), C.POINTER(_Opts), C.c_int, C.c_double,
                                     C.POINTER(C.c_void_p)]),
    "egfem_batch_create_sched": (C.c_int, [C.c_int, C.POINTER(C.c_void_p), C.POINTER(_Problem),
                                           C.POINTER(C.c_void_p), C.POINTER(_Opts), C.c_int, C.c_double,
                                           C.POINTER(C.c_void_p)]),
    "egfem_batch_run": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "egfem_batch_graph_run": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "egfem_batch_stats": (C.c_int, [C.c_void_p, C.POINTER(_Stats), C.c_void_p]),
    "egfem_batch_teams": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "egfem_batch_destroy": (None, [C.c_void_p]),
    "egfem_batch_autotune": (C.c_int, [C.c_int, C.POINTER(C.c_void_p), C.POINTER(_Problem),
                                       C.POINTER(C.c_void_p), C.POINTER(_Opts), C.POINTER(C.c_int),
                                       C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.c_void_p]),
    "egfem_get_shape": (C.c_int, [C.c_void_p, C.POINTER(_Shape)]),
    "egfem_set_shape": (C.c_int, [C.c_void_p, C.POINTER(_Shape)]),
    "egfem_autotune": (C.c_int, [C.c_void_p, C.POINTER(_Problem), C.c_int, C.POINTER(_Shape),
                                 C.POINTER(C.c_double), C.c_void_p]),
    "egfem_picard_opts_default": (None, [C.POINTER(_PicardOpts)]),
    "egfem_picard": (C.c_int, [C.c_void_p, C.POINTER(_Problem), C.c_void_p, C.POINTER(_PicardOpts),
                               C.POINTER(_PicardStats), C.c_void_p]),
    "egfem_burgers_opts_default": (None, [C.POINTER(_BurgersOpts)]),
    "egfem_burgers": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                C.POINTER(_BurgersOpts), C.POINTER(_BurgersStats), C.c_void_p]),
    "egfem_picard_grad": (C.c_int, [C.c_void_p, C.POINTER(_Problem), C.POINTER(_GradCoef), C.c_void_p,
                                    C.POINTER(_PicardOpts), C.POINTER(_PicardStats), C.c_void_p]),
    "egfem_newton_grad": (C.c_int, [C.c_void_p, C.POINTER(_Problem), C.POINTER(_GradCoef), C.c_void_p,
                                    C.POINTER(_Opts), C.POINTER(_Stats), C.c_void_p]),
    "egfem_solve_cg": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int,
                                 C.POINTER(C.c_int), C.POINTER(C.c_double), C.c_void_p]),
    "egfem_stream_read_chunks": (C.c_int64, [C.c_int64]),
    "egfem_stream_read": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]),
    "egfem_last_error": (C.c_char_p, []),
    "egfem_version": (C.c_char_p, []),
}


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load libegfem.so (torch is imported first so that its HIP runtime is the
    one the library binds to)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise EgfemError(EGFEM_ERR_HIP, f"{path} is not built; run __graft_entry__.build()")
    lib = C.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, allow_positive: bool = False) -> int:
    if rc < 0 or (rc > 0 and not allow_positive):
        msg = load_library().egfem_last_error().decode(errors="replace")
        raise EgfemError(rc, msg)
    return rc


def _require_device():
    if not torch.cuda.is_available():
        raise EgfemError(EGFEM_ERR_HIP, "no HIP device visible to torch")


def _dptr(t: Optional[torch.Tensor], dtype=torch.float64, n: Optional[int] = None) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise EgfemError(EGFEM_ERR_ARG, "tensor must live on the HIP device")
    if t.dtype != dtype:
        raise EgfemError(EGFEM_ERR_ARG, f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise EgfemError(EGFEM_ERR_ARG, "tensor must be contiguous")
    if n is not None and t.numel() != n:
        raise EgfemError(EGFEM_ERR_SHAPE, f"expected {n} entries, got {t.numel()}")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


@dataclass
class Info:
    dim: int
    form: int
    symmetric: int
    n_nodes: int
    n_cells: int
    nnz: int
    nnz_b: int
    structural_nnz: int
    slots: int
    row_blocks: int
    device_bytes: int
    wspace: int = 0
    n_w: int = 0
    nnz_half: int = 0


@dataclass
class NewtonOptions:
    tol: float = 1e-10
    max_newton: int = 50
    max_krylov: int = 20000
    krylov_rtol: float = 1e-12
    forcing: int = 0
    eta_max: float = 0.1
    max_backtracks: int = 10
    krylov_blocks: int = 0
    krylov_threads: int = 0
    timing: int = 0

    def c(self) -> _Opts:
        return _Opts(self.tol, self.max_newton, self.max_krylov, self.krylov_rtol, self.forcing,
                     self.eta_max, self.max_backtracks, self.krylov_blocks, self.krylov_threads,
                     self.timing)


@dataclass
class PicardOptions:
    """Mirror of egfem_picard_opts (defaults equal egfem_picard_opts_default)."""
    tol: float = 1e-12
    max_picard: int = 200
    max_krylov: int = 20000
    krylov_rtol: float = 0.1
    krylov_blocks: int = 0
    krylov_threads: int = 0
    timing: int = 0

    def c(self) -> _PicardOpts:
        return _PicardOpts(self.tol, self.max_picard, self.max_krylov, self.krylov_rtol, self.krylov_blocks,
                           self.krylov_threads, self.timing)


@dataclass
class PicardStats:
    status: int
    picard_iters: int
    krylov_iters: int
    update: float
    res0: float
    res: float
    update_hist: List[float]
    krylov_hist: List[int]
    t_matrix_ms: float
    t_krylov_ms: float
    krylov_kernels: int

    @property
    def status_name(self) -> str:
        return STATUS_NAMES.get(self.status, str(self.status))

    @classmethod
    def from_c(cls, s: _PicardStats) -> "PicardStats":
        k = min(s.picard_iters, HIST)
        return cls(s.status, s.picard_iters, s.krylov_iters, s.update, s.res0, s.res,
                   list(s.update_hist[:k]), list(s.krylov_hist[:k]), s.t_matrix_ms, s.t_krylov_ms,
                   s.krylov_kernels)


@dataclass
class BurgersOptions:
    """Mirror of egfem_burgers_opts (defaults equal egfem_burgers_opts_default)."""
    dt: float = 1e-2
    nu: float = 1.0
    steps: int = 100
    group: int = 0
    krylov_rtol: float = 1e-12
    max_krylov: int = 20000
    guess: int = 2
    krylov_blocks: int = 0
    krylov_threads: int = 0
    timing: int = 0

    def c(self) -> _BurgersOpts:
        return _BurgersOpts(self.dt, self.nu, self.steps, self.group, self.krylov_rtol, self.max_krylov,
                            self.guess, self.krylov_blocks, self.krylov_threads, self.timing)


@dataclass
class BurgersStats:
    status: int
    steps: int
    krylov_iters: int
    max_step_krylov: int
    max_relres: float
    krylov_hist: List[int]
    t_rhs_ms: float
    t_krylov_ms: float
    krylov_kernels: int

    @property
    def status_name(self) -> str:
        return STATUS_NAMES.get(self.status, str(self.status))

    @classmethod
    def from_c(cls, s: _BurgersStats) -> "BurgersStats":
        k = min(s.steps, HIST)
        return cls(s.status, s.steps, s.krylov_iters, s.max_step_krylov, s.max_relres, list(s.krylov_hist[:k]),
                   s.t_rhs_ms, s.t_krylov_ms, s.krylov_kernels)


@dataclass
class NewtonStats:
    status: int
    newton_iters: int
    krylov_iters: int
    backtracks: int
    res0: float
    res: float
    res_hist: List[float]
    krylov_hist: List[int]
    t_action_ms: float = 0.0
    t_jacobian_ms: float = 0.0
    t_krylov_ms: float = 0.0
    n_action: int = 0
    n_jacobian: int = 0
    n_krylov: int = 0
    krylov_status_hist: List[int] = None
    krylov_relres_hist: List[float] = None
    krylov_kernels: int = 0

    @property
    def status_name(self) -> str:
        return STATUS_NAMES.get(self.status, "?")

    @classmethod
    def from_c(cls, s: _Stats) -> "NewtonStats":
        k = min(s.newton_iters, HIST)
        return cls(s.status, s.newton_iters, s.krylov_iters, s.backtracks, s.res0, s.res,
                   list(s.res_hist[:k]), list(s.krylov_hist[:k]), s.t_action_ms, s.t_jacobian_ms,
                   s.t_krylov_ms, s.n_action, s.n_jacobian, s.n_krylov,
                   list(s.krylov_status_hist[:k + 1]), list(s.krylov_relres_hist[:k + 1]),
                   s.krylov_kernels)


class Problem:
    """Device-resident data of F(u) = [K u] + T:(u (x) (a0 + u^2)) - load = 0."""

    def __init__(self, n: int, load: torch.Tensor, dirichlet: Optional[torch.Tensor] = None,
                 a0: Optional[torch.Tensor] = None, a0_const: float = 1.0,
                 add_stiffness: bool = False):
        self.n = n
        self.load = load
        self.dirichlet = dirichlet
        self.a0 = a0
        self.a0_const = float(a0_const)
        self.add_stiffness = bool(add_stiffness)

    def c(self) -> _Problem:
        return _Problem(_dptr(self.a0, n=self.n), self.a0_const,
                        _dptr(self.load, n=self.n) if self.load is not None else None,
                        _dptr(self.dirichlet, torch.uint8, self.n), int(self.add_stiffness))


class Tensor:
    """Handle of a built EGFEM tensor with its CSR pattern and matrices."""

    def __init__(self, handle: int):
        self._h = C.c_void_p(handle)
        _live_tensors.add(self)
        inf = _Info()
        _check(load_library().egfem_tensor_info(self._h, C.byref(inf)))
        self.info = Info(inf.dim, inf.form, inf.symmetric, inf.n_nodes, inf.n_cells, inf.nnz,
                         inf.nnz_b, inf.structural_nnz, inf.slots, inf.row_blocks, inf.device_bytes,
                         inf.wspace, inf.n_w, inf.nnz_half)

    # -- construction ----------------------------------------------------
    @classmethod
    def build(cls, coords: np.ndarray, cells: np.ndarray, form: int = FORM_STIFF,
              drop_rel: float = 1e-13, wspace: int = W_P1) -> "Tensor":
        _require_device()
        lib = load_library()
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int32)
        if coords.ndim != 2 or cells.ndim != 2 or cells.shape[1] != coords.shape[1] + 1:
            raise EgfemError(EGFEM_ERR_SHAPE, "coords [N, d] and cells [E, d+1] expected")
        out = C.c_void_p()
        _check(lib.egfem_build_tensor_w(coords.shape[1], coords.shape[0], coords.ctypes.data,
                                        cells.shape[0], cells.ctypes.data, int(form), int(wspace),
                                        float(drop_rel), C.byref(out)))
        return cls(out.value)

    @classmethod
    def from_mesh(cls, mesh, form: int = FORM_STIFF, drop_rel: float = 1e-13, wspace: int = W_P1) -> "Tensor":
        return cls.build(mesh.coords, mesh.cells, form, drop_rel, wspace)

    def close(self):
        if self._h is not None and self._h.value:
            load_library().egfem_tensor_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self) -> C.c_void_p:
        if self._h is None:
            raise EgfemError(EGFEM_ERR_ARG, "tensor handle already closed")
        return self._h

    @property
    def n(self) -> int:
        return self.info.n_nodes

    # -- pattern ------------------------------------------------------------
    def pattern(self):
        """(rowptr, col) of the CSR pattern as host int32 arrays."""
        rp = np.empty(self.n + 1, np.int32)
        cl = np.empty(self.info.slots, np.int32)
        _check(load_library().egfem_tensor_pattern(self.handle, rp.ctypes.data, cl.ctypes.data))
        return rp, cl

    def export(self):
        """Host COO (i, j, k, v) of the stored tensor."""
        nnz = self.info.nnz
        i = np.empty(nnz, np.int32)
        j = np.empty(nnz, np.int32)
        k = np.empty(nnz, np.int32)
        v = np.empty(nnz, np.float64)
        _check(load_library().egfem_tensor_export(self.handle, i.ctypes.data, j.ctypes.data,
                                                  k.ctypes.data, v.ctypes.data))
        return i, j, k, v

    # -- online actions -----------------------------------------------------
    def residual(self, u: torch.Tensor, a: torch.Tensor, out: Optional[torch.Tensor] = None):
        """r_i = sum_jk T_ijk u_j a_k (a over the dofs of W_h)."""
        out = torch.empty_like(u) if out is None else out
        _check(load_library().egfem_residual(self.handle, _dptr(u, n=self.n), _dptr(a, n=self.info.n_w),
                                             _dptr(out, n=self.n), _stream()))
        return out

    def attach_elements(self, coords: np.ndarray, cells: np.ndarray):
        """Store the element-factored form (K^e per cell) of this stiffness tensor."""
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int32)
        _check(load_library().egfem_attach_elements(self.handle, coords.shape[1], coords.shape[0],
                                                    coords.ctypes.data, cells.shape[0], cells.ctypes.data))

    def residual_elementwise(self, u: torch.Tensor, a: torch.Tensor, out: Optional[torch.Tensor] = None):
        """r_i = sum_jk T_ijk u_j a_k through the element-factored form."""
        out = torch.empty_like(u) if out is None else out
        _check(load_library().egfem_residual_elementwise(self.handle, _dptr(u, n=self.n), _dptr(a, n=self.n),
                                                         _dptr(out, n=self.n), _stream()))
        return out

    def attach_unique(self, coords: np.ndarray, cells: np.ndarray) -> int:
        """Store the fully symmetric mass tensor once per index multiset;
        returns the number of stored values (N + 2E + F)."""
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int32)
        nu = C.c_int64(0)
        _check(load_library().egfem_attach_unique(self.handle, coords.shape[1], coords.shape[0],
                                                  coords.ctypes.data, cells.shape[0], cells.ctypes.data,
                                                  C.byref(nu)))
        return int(nu.value)

    def residual_unique(self, u: torch.Tensor, a: torch.Tensor, out: Optional[torch.Tensor] = None):
        """r_i = sum_jk T_ijk u_j a_k through the unique storage."""
        out = torch.empty_like(u) if out is None else out
        _check(load_library().egfem_residual_unique(self.handle, _dptr(u, n=self.n), _dptr(a, n=self.n),
                                                    _dptr(out, n=self.n), _stream()))
        return out

    def jacobian(self, u, a, dadu=None, add_stiffness=False, dirichlet=None, out=None,
                 dinv=None):
        out = torch.empty(self.info.slots, dtype=torch.float64, device="cuda") if out is None else out
        _check(load_library().egfem_jacobian(self.handle, _dptr(u, n=self.n), _dptr(a, n=self.info.n_w),
                                             _dptr(dadu, n=self.info.n_w), int(add_stiffness),
                                             _dptr(dirichlet, torch.uint8, self.n),
                                             _dptr(out, n=self.info.slots), _dptr(dinv, n=self.n),
                                             _stream()))
        return out

    def mode3(self, w, u, out=None):
        """out_k = sum_ij w_i T_ijk u_j."""
        out = torch.empty_like(u) if out is None else out
        _check(load_library().egfem_mode3(self.handle, _dptr(w, n=self.n), _dptr(u, n=self.n),
                                          _dptr(out, n=self.n), _stream()))
        return out

    def matvec(self, x, which: str = "J", jval=None, transpose=False, out=None):
        sel = {"J": 0, "K": 1, "M": 2}[which]
        out = torch.empty_like(x) if out is None else out
        _check(load_library().egfem_matvec(self.handle, sel, _dptr(jval, n=self.info.slots),
                                           int(transpose), _dptr(x, n=self.n),
                                           _dptr(out, n=self.n), _stream()))
        return out

    def problem_residual(self, p: Problem, u, out=None, with_norm=False):
        out = torch.empty_like(u) if out is None else out
        pc = p.c()
        nrm = C.c_double(0.0)
        _check(load_library().egfem_problem_residual(self.handle, C.byref(pc), _dptr(u, n=self.n),
                                                     _dptr(out, n=self.n),
                                                     C.byref(nrm) if with_norm else None,
                                                     _stream()))
        return (out, nrm.value) if with_norm else out

    def problem_residual_noalloc(self, p: Problem, u, out, with_norm=False):
        """egfem_problem_residual_noalloc: the caller passes the output; the
        library allocates nothing (its fixed per-device array holds the
        partial sums)."""
        pc = p.c()
        nrm = C.c_double(0.0)
        _check(load_library().egfem_problem_residual_noalloc(self.handle, C.byref(pc), _dptr(u, n=self.n),
                                                             _dptr(out, n=self.n),
                                                             C.byref(nrm) if with_norm else None,
                                                             _stream()))
        return (out, nrm.value) if with_norm else out

    def problem_jacobian(self, p: Problem, u, out=None, dinv=None):
        out = torch.empty(self.info.slots, dtype=torch.float64, device="cuda") if out is None else out
        pc = p.c()
        _check(load_library().egfem_problem_jacobian(self.handle, C.byref(pc), _dptr(u, n=self.n),
                                                     _dptr(out, n=self.info.slots),
                                                     _dptr(dinv, n=self.n), _stream()))
        return out

    def newton(self, p: Problem, u: torch.Tensor, opts: Optional[NewtonOptions] = None,
               warn: bool = True) -> NewtonStats:
        """Damped Newton in place on u; returns the statistics."""
        o = (opts or NewtonOptions()).c()
        pc = p.c()
        st = _Stats()
        rc = load_library().egfem_newton(self.handle, C.byref(pc), _dptr(u, n=self.n), C.byref(o),
                                         C.byref(st), _stream())
        _check(rc, allow_positive=True)
        stats = NewtonStats.from_c(st)
        if rc not in (EGFEM_OK, EGFEM_STAGNATED) and warn:
            warnings.warn(f"egfem_newton ended with status {stats.status_name}")
        return stats

    def adjoint(self, p: Problem, u, ubar, opts: Optional[NewtonOptions] = None,
                grad_a0: bool = True):
        """lambda = DF(u)^-T ubar (free nodes) and dJ/da0 = -(T ._2 u)^T lambda.
        Returns (lambda, grad_a0 or None, status, krylov_iters, relres)."""
        lam = torch.empty_like(u)
        ga = torch.empty_like(u) if grad_a0 else None
        o = (opts or NewtonOptions()).c()
        pc = p.c()
        it = C.c_int(0)
        rr = C.c_double(0.0)
        rc = load_library().egfem_adjoint(self.handle, C.byref(pc), _dptr(u, n=self.n),
                                          _dptr(ubar, n=self.n), C.byref(o), _dptr(lam, n=self.n),
                                          _dptr(ga, n=self.n), C.byref(it), C.byref(rr), _stream())
        _check(rc, allow_positive=True)
        return lam, ga, rc, it.value, rr.value

    # -- launch shapes / autotuner ------------------------------------------
    def get_shape(self) -> dict:
        s = _Shape()
        _check(load_library().egfem_get_shape(self.handle, C.byref(s)))
        return {f: getattr(s, f) for f, _ in _Shape._fields_}

    def set_shape(self, **kw):
        cur = self.get_shape()
        cur.update(kw)
        s = _Shape(**cur)
        _check(load_library().egfem_set_shape(self.handle, C.byref(s)))

    def autotune(self, problem: Optional[Problem] = None, action: bool = True,
                 krylov: bool = True, cache: Optional[str] = None) -> dict:
        """Pick the tensor-action run shape and the Krylov grid by timing
        candidates on this tensor; with `cache` (a JSON path) reuse/store the
        choice keyed by the tensor's sizes."""
        import json
        key = (f"d{self.info.dim}-f{self.info.form}-w{self.info.wspace}-n{self.n}-z{self.info.nnz}"
               f"-s{self.info.slots}")
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                db = json.load(fh)
            if key in db:
                self.set_shape(**db[key]["shape"])
                return db[key]
        what = (1 if action else 0) | (2 if (krylov and problem is not None) else 0)
        pc = problem.c() if problem is not None else None
        s = _Shape()
        us = (C.c_double * 2)()
        _check(load_library().egfem_autotune(self.handle, C.byref(pc) if pc is not None else None,
                                             what, C.byref(s), us, _stream()))
        res = {"shape": {f: getattr(s, f) for f, _ in _Shape._fields_},
               "action_us": us[0], "krylov_iter_us": us[1]}
        if cache:
            db = {}
            if os.path.exists(cache):
                with open(cache) as fh:
                    db = json.load(fh)
            db[key] = res
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            with open(cache, "w") as fh:
                json.dump(db, fh, indent=1)
        return res

    def picard(self, p: Problem, u: torch.Tensor, opts: Optional[PicardOptions] = None,
               warn: bool = True) -> PicardStats:
        """Picard iteration in place on u (Sec. 4, Example picard_iteration);
        returns the statistics."""
        o = (opts or PicardOptions()).c()
        pc = p.c()
        st = _PicardStats()
        rc = load_library().egfem_picard(self.handle, C.byref(pc), _dptr(u, n=self.n), C.byref(o),
                                         C.byref(st), _stream())
        _check(rc, allow_positive=True)
        stats = PicardStats.from_c(st)
        if rc != EGFEM_OK and warn:
            warnings.warn(f"egfem_picard ended with status {stats.status_name}")
        return stats

    def picard_grad(self, p: Problem, u: torch.Tensor, c0: float, c1: float, q: float,
                    start_linear: bool = True, opts: Optional[PicardOptions] = None,
                    warn: bool = True) -> PicardStats:
        """Picard iteration for a(grad u) = (c0 + c1 |grad u|^2)^q on a W_h = P0
        handle (p-Laplace: c0 = eps^2, c1 = 1, q = (p-2)/2), in place on u."""
        o = (opts or PicardOptions()).c()
        pc = p.c()
        g = _GradCoef(float(c0), float(c1), float(q), int(bool(start_linear)))
        st = _PicardStats()
        rc = load_library().egfem_picard_grad(self.handle, C.byref(pc), C.byref(g), _dptr(u, n=self.n),
                                              C.byref(o), C.byref(st), _stream())
        _check(rc, allow_positive=True)
        stats = PicardStats.from_c(st)
        if rc != EGFEM_OK and warn:
            warnings.warn(f"egfem_picard_grad ended with status {stats.status_name}")
        return stats

    def newton_grad(self, p: Problem, u: torch.Tensor, c0: float, c1: float, q: float,
                    start_linear: bool = True, opts: Optional[NewtonOptions] = None,
                    warn: bool = True) -> NewtonStats:
        """Damped Newton for a(grad u) = (c0 + c1 |grad u|^2)^q on a W_h = P0 handle."""
        o = (opts or NewtonOptions()).c()
        pc = p.c()
        g = _GradCoef(float(c0), float(c1), float(q), int(bool(start_linear)))
        st = _Stats()
        rc = load_library().egfem_newton_grad(self.handle, C.byref(pc), C.byref(g), _dptr(u, n=self.n),
                                              C.byref(o), C.byref(st), _stream())
        _check(rc, allow_positive=True)
        stats = NewtonStats.from_c(st)
        if rc != EGFEM_OK and warn:
            warnings.warn(f"egfem_newton_grad ended with status {stats.status_name}")
        return stats

    def burgers(self, u: torch.Tensor, dirichlet: Optional[torch.Tensor] = None,
                source: Optional[torch.Tensor] = None, opts: Optional[BurgersOptions] = None,
                warn: bool = True) -> BurgersStats:
        """Semi-implicit Burgers steps in place on u (Sec. 5.2) with this
        convection tensor.  source: None, one nodal vector [n] used at every
        step, or [steps, n] (row m = nodal source values at t_{m+1})."""
        o = opts or BurgersOptions()
        stride = 0
        sp_ = None
        if source is not None:
            if source.dim() == 1:
                sp_ = _dptr(source, n=self.n)
            else:
                if source.dim() != 2 or source.shape[1] != self.n or source.shape[0] < o.steps:
                    raise EgfemError(EGFEM_ERR_SHAPE, "source must be [n] or [>= steps, n]")
                sp_ = _dptr(source)
                stride = self.n
        st = _BurgersStats()
        oc = o.c()
        rc = load_library().egfem_burgers(self.handle, _dptr(dirichlet, dtype=torch.uint8, n=self.n), sp_,
                                          stride, _dptr(u, n=self.n), C.byref(oc), C.byref(st), _stream())
        _check(rc, allow_positive=True)
        stats = BurgersStats.from_c(st)
        if rc != EGFEM_OK and warn:
            warnings.warn(f"egfem_burgers ended with status {stats.status_name}")
        return stats

    def solve_cg(self, jval, rhs, x=None, rtol=1e-12, max_iter=20000):
        """Preconditioned conjugate gradients (the handle's preconditioner:
        block-Jacobi or Jacobi) for an SPD matrix in the tensor's pattern;
        returns (x, status, iterations, relres)."""
        x = torch.zeros_like(rhs) if x is None else x
        it = C.c_int(0)
        rr = C.c_double(0.0)
        rc = load_library().egfem_solve_cg(self.handle, _dptr(jval, n=self.info.slots), _dptr(rhs, n=self.n),
                                           _dptr(x, n=self.n), float(rtol), int(max_iter), C.byref(it),
                                           C.byref(rr), _stream())
        _check(rc, allow_positive=True)
        return x, rc, it.value, rr.value

    def solve(self, jval, rhs, x=None, transpose=False, rtol=1e-12, max_iter=20000):
        x = torch.zeros_like(rhs) if x is None else x
        it = C.c_int(0)
        rr = C.c_double(0.0)
        rc = load_library().egfem_solve(self.handle, _dptr(jval, n=self.info.slots), int(transpose),
                                        _dptr(rhs, n=self.n), _dptr(x, n=self.n), float(rtol),
                                        int(max_iter), C.byref(it), C.byref(rr), _stream())
        _check(rc, allow_positive=True)
        return x, rc, it.value, rr.value


class Batch:
    """Reusable batch plan: all instances solved by one persistent launch,
    optionally replayed from a captured hipGraph.  kind 0: streaming teams
    (egfem_batch_create; threads 512/1024, weight_exp the team weight
    exponent); kind 1: scheduled resident teams (egfem_batch_create_sched;
    threads 256/512, weight_exp the duration exponent)."""

    def __init__(self, tensors: Sequence[Tensor], problems: Sequence[Problem],
                 us: Sequence[torch.Tensor], opts: Optional[NewtonOptions] = None,
                 threads: int = 0, weight_exp: float = 0.0, kind: int = 0):
        m = len(tensors)
        if not (m == len(problems) == len(us)) or m == 0:
            raise EgfemError(EGFEM_ERR_SHAPE, "tensors/problems/us must have equal nonzero length")
        self.count = m
        self._keep = (list(tensors), list(problems), list(us))   # buffers must outlive the plan
        hs = (C.c_void_p * m)(*[t.handle.value for t in tensors])
        self._ps = (_Problem * m)(*[p.c() for p in problems])
        up = (C.c_void_p * m)(*[_dptr(u, n=t.n) for u, t in zip(us, tensors)])
        o = (opts or NewtonOptions()).c()
        out = C.c_void_p()
        if kind not in (0, 1):
            raise EgfemError(EGFEM_ERR_ARG, "kind must be 0 (streaming teams) or 1 (scheduled teams)")
        create = load_library().egfem_batch_create_sched if kind == 1 else load_library().egfem_batch_create
        _check(create(m, hs, self._ps, up, C.byref(o), int(threads), float(weight_exp), C.byref(out)))
        self.kind = kind
        self._h = out
        _live_batches.add(self)

    def run(self, zero_init: bool = True, graph: bool = False):
        fn = load_library().egfem_batch_graph_run if graph else load_library().egfem_batch_run
        _check(fn(self._h, int(zero_init), _stream()))

    def stats(self):
        st = (_Stats * self.count)()
        rc = load_library().egfem_batch_stats(self._h, st, _stream())
        _check(rc, allow_positive=True)
        return [NewtonStats.from_c(st[i]) for i in range(self.count)], rc

    def teams(self):
        t = (C.c_int * self.count)()
        tot = C.c_int(0)
        _check(load_library().egfem_batch_teams(self._h, t, C.byref(tot)))
        return list(t), tot.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().egfem_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def newton_batched(tensors: Sequence[Tensor], problems: Sequence[Problem],
                   us: Sequence[torch.Tensor], opts: Optional[NewtonOptions] = None):
    """All instances in one persistent launch; returns a list of NewtonStats."""
    m = len(tensors)
    if not (m == len(problems) == len(us)) or m == 0:
        raise EgfemError(EGFEM_ERR_SHAPE, "tensors/problems/us must have equal nonzero length")
    hs = (C.c_void_p * m)(*[t.handle.value for t in tensors])
    ps = (_Problem * m)(*[p.c() for p in problems])
    up = (C.c_void_p * m)(*[_dptr(u, n=t.n) for u, t in zip(us, tensors)])
    st = (_Stats * m)()
    o = (opts or NewtonOptions()).c()
    rc = load_library().egfem_newton_batched(m, hs, ps, up, C.byref(o), st, _stream())
    _check(rc, allow_positive=True)
    return [NewtonStats.from_c(st[i]) for i in range(m)], rc


def batch_autotune(tensors: Sequence[Tensor], problems: Sequence[Problem], us: Sequence[torch.Tensor],
                   opts: Optional[NewtonOptions] = None, cache: Optional[str] = None) -> dict:
    """egfem_batch_autotune: the batch plan's kind, workgroup size and team
    weight (or duration) exponent by timing; with `cache` (a JSON path)
    reuse/store the choice keyed by the instances' sizes.  Returns {"kind",
    "threads", "weight_exp", "ms"}, the arguments of Batch."""
    import json
    m = len(tensors)
    if not (m == len(problems) == len(us)) or m == 0:
        raise EgfemError(EGFEM_ERR_SHAPE, "tensors/problems/us must have equal nonzero length")
    key = "batch2-" + "-".join(f"{t.n}x{t.info.nnz}" for t in tensors)
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            db = json.load(fh)
        if key in db:
            return db[key]
    hs = (C.c_void_p * m)(*[t.handle.value for t in tensors])
    ps = (_Problem * m)(*[p.c() for p in problems])
    up = (C.c_void_p * m)(*[_dptr(u, n=t.n) for u, t in zip(us, tensors)])
    o = (opts or NewtonOptions()).c()
    kind = C.c_int(0)
    thr = C.c_int(0)
    wexp = C.c_double(0.0)
    ms = C.c_double(0.0)
    _check(load_library().egfem_batch_autotune(m, hs, ps, up, C.byref(o), C.byref(kind), C.byref(thr),
                                               C.byref(wexp), C.byref(ms), _stream()))
    res = {"kind": kind.value, "threads": thr.value, "weight_exp": wexp.value, "ms": ms.value}
    if cache:
        db = {}
        if os.path.exists(cache):
            with open(cache) as fh:
                db = json.load(fh)
        db[key] = res
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as fh:
            json.dump(db, fh, indent=1)
    return res


def stream_read(x: torch.Tensor, partial: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Streaming-read ceiling probe: per-chunk sums of x (float64, contiguous)
    written into `partial` (allocated when None); see egfem_stream_read."""
    n = x.numel()
    nc = int(load_library().egfem_stream_read_chunks(n))
    if partial is None:
        partial = torch.empty(max(nc, 1), dtype=torch.float64, device=x.device)
    _check(load_library().egfem_stream_read(_dptr(x), n, _dptr(partial), partial.numel(), _stream()))
    return partial


def version() -> str:
    return load_library().egfem_version().decode()
