"""Thin ctypes binding of libtpsurf (include/tpsurf.h).

Argument marshalling only: every step runs in the HIP library.  Tensors must live on a
HIP device (torch "cuda" device), be contiguous and have the documented dtype; results
are returned as new device tensors.  There is no CPU fallback: if the library is not
built, loading fails with an error.
"""
from __future__ import annotations

import atexit
import ctypes
import math
import os
import weakref
from dataclasses import dataclass
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtpsurf.so")

TP_OK = 0
TP_E_INVALID_ARGUMENT, TP_E_NOT_CONVERGED, TP_E_DEVICE = 1, 5, 8
STATUS_NAMES = {
    0: "TP_OK", 1: "TP_E_INVALID_ARGUMENT", 2: "TP_E_DEGENERATE_FACE", 3: "TP_E_BAD_INDEX",
    4: "TP_E_NONFINITE", 5: "TP_E_NOT_CONVERGED", 6: "TP_E_OUT_OF_MEMORY",
    7: "TP_E_SINGULAR_CONSTRAINTS", 8: "TP_E_DEVICE",
}
PREC_FP32_HILO, PREC_FP32, PREC_FP64, PREC_FP32_NEAR64, PREC_FP32_ACC32, PREC_FP32_KAHAN = 0, 1, 2, 3, 4, 5
KIND_ENERGY, KIND_GRAD, KIND_FRAC, KIND_SOBOLEV = 0, 1, 2, 3

# Every symbol the C-ABI exports (the header declares exactly these).
EXPORTED = [
    "tp_params_default", "tp_energy", "tp_gradient", "tp_energy_faces", "tp_energy_faces_noalloc",
    "tp_fractional_apply",
    "tp_precond_apply", "tp_problem_create", "tp_problem_destroy", "tp_problem_set_vertices",
    "tp_problem_get_vertices", "tp_problem_energy", "tp_problem_gradient",
    "tp_problem_fractional_apply", "tp_sobolev_apply", "tp_problem_sobolev_apply",
    "tp_problem_sobolev_solve", "tp_problem_set_obstacle", "tp_problem_obstacle_energy",
    "tp_problem_add_implicit", "tp_problem_implicit_energy",
    "tp_problem_precond_apply", "tp_step_opts_default",
    "tp_precond_step", "tp_last_error", "tp_profile_enable", "tp_profile_reset", "tp_profile_get",
    "tp_problem_poisson_solve", "tp_batch_step", "tp_problem_device_bytes",
    "tp_estimate_device_bytes", "tp_problem_bh_stats", "tp_set_allocator", "tp_problem_set_pins",
    "tp_problem_bct_stats", "tp_remesh", "tp_problem_obstacle_stats",
]


class TpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("sigma", ctypes.c_double),
                ("precision", ctypes.c_int), ("cg_rtol", ctypes.c_double), ("cg_maxiter", ctypes.c_int),
                ("cg_precond", ctypes.c_int), ("theta", ctypes.c_double), ("leaf_size", ctypes.c_int),
                ("chi", ctypes.c_double), ("sym_pairs", ctypes.c_int), ("sym_band", ctypes.c_int)]


class SolveReport(ctypes.Structure):
    _fields_ = [("cg_iters", ctypes.c_int * 2), ("cg_relres", ctypes.c_double * 2),
                ("t_ms", ctypes.c_double * 4)]


class GmresReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("cycles", ctypes.c_int), ("relres", ctypes.c_double),
                ("precond_cg_iters", ctypes.c_int), ("t_ms", ctypes.c_double), ("omega", ctypes.c_double)]


class StepOpts(ctypes.Structure):
    _fields_ = [("tau0", ctypes.c_double), ("line_search", ctypes.c_int), ("armijo_c", ctypes.c_double),
                ("shrink", ctypes.c_double), ("max_backtracks", ctypes.c_int),
                ("constrain_area", ctypes.c_int), ("constrain_volume", ctypes.c_int),
                ("area_target", ctypes.c_double), ("volume_target", ctypes.c_double),
                ("solver", ctypes.c_int), ("solver_rtol", ctypes.c_double), ("solver_maxiter", ctypes.c_int),
                ("area_penalty", ctypes.c_double), ("volume_penalty", ctypes.c_double),
                ("barycenter_motion", ctypes.c_int), ("warm_start", ctypes.c_int)]


class StepReport(ctypes.Structure):
    _fields_ = [("E", ctypes.c_double), ("E_new", ctypes.c_double), ("grad_norm", ctypes.c_double),
                ("slope", ctypes.c_double), ("tau", ctypes.c_double), ("backtracks", ctypes.c_int),
                ("n_constraints", ctypes.c_int), ("cg_iters", ctypes.c_int * 2),
                ("cg_relres", ctypes.c_double * 2), ("phi_before", ctypes.c_double * 2),
                ("phi_trial", ctypes.c_double * 2), ("phi_after", ctypes.c_double * 2),
                ("t_ms", ctypes.c_double * 8), ("warm_started", ctypes.c_int)]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


class KernelStats(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double), ("pairs_total", ctypes.c_double),
                ("cols_total", ctypes.c_double), ("launches", ctypes.c_int64)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libtpsurf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2107_01664_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, d, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "tp_params_default": [P(Params)],
        "tp_energy": [vp, i64, vp, i64, P(Params), P(d), vp],
        "tp_gradient": [vp, i64, vp, i64, P(Params), P(d), vp, vp],
        "tp_energy_faces": [vp, vp, vp, i64, P(Params), P(d), vp],
        "tp_energy_faces_noalloc": [vp, vp, vp, i64, P(Params), P(d), vp],
        "tp_fractional_apply": [vp, i64, vp, i64, P(Params), vp, i32, vp, vp],
        "tp_precond_apply": [vp, i64, vp, i64, P(Params), vp, i32, vp, P(SolveReport), vp],
        "tp_problem_create": [vp, i64, vp, i64, P(Params), vp, P(vp)],
        "tp_problem_set_vertices": [vp, vp],
        "tp_problem_get_vertices": [vp, vp],
        "tp_problem_energy": [vp, P(d)],
        "tp_problem_gradient": [vp, P(d), vp],
        "tp_problem_fractional_apply": [vp, vp, i32, vp],
        "tp_sobolev_apply": [vp, i64, vp, i64, P(Params), vp, i32, vp, vp],
        "tp_problem_sobolev_apply": [vp, vp, i32, vp],
        "tp_problem_set_obstacle": [vp, vp, i64, vp, i64, ctypes.c_double, ctypes.c_double],
        "tp_problem_obstacle_energy": [vp, P(d), vp],
        "tp_problem_add_implicit": [vp, i32, P(d), d, d, d, i32],
        "tp_problem_implicit_energy": [vp, P(d), vp],
        "tp_problem_sobolev_solve": [vp, vp, i32, ctypes.c_double, i32, i32, i32, vp, P(GmresReport)],
        "tp_problem_precond_apply": [vp, vp, i32, vp, P(SolveReport)],
        "tp_problem_poisson_solve": [vp, vp, i32, vp, P(SolveReport)],
        "tp_step_opts_default": [P(StepOpts)],
        "tp_precond_step": [vp, P(StepOpts), P(StepReport), vp],
        "tp_batch_step": [P(vp), i32, P(StepOpts), P(StepReport), P(i32)],
        "tp_problem_device_bytes": [vp, P(ctypes.c_uint64)],
        "tp_problem_bh_stats": [vp, P(i64), P(i64)],
        "tp_problem_bct_stats": [vp, P(i64), P(i64)],
        "tp_problem_obstacle_stats": [vp, P(i64), P(i64)],
        "tp_estimate_device_bytes": [i64, i64, i32, i32, P(Params), i32, P(ctypes.c_uint64)],
        "tp_profile_enable": [i32],
        "tp_profile_reset": [],
        "tp_profile_get": [i32, P(KernelStats)],
        "tp_set_allocator": [ctypes.c_void_p, ctypes.c_void_p, vp],
        "tp_problem_set_pins": [vp, P(i32), i64],
        "tp_remesh": [vp, i64, vp, i64, d, i32, d, vp, i64, vp, i64, P(i64), P(i64)],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.tp_problem_destroy.argtypes = [vp]
    L.tp_problem_destroy.restype = None
    L.tp_last_error.argtypes = []
    L.tp_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


# tp_set_allocator callbacks: alloc(bytes, stream, user) -> pointer, free(ptr, bytes, stream, user)
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_torch_allocator = None     # the registered callbacks (kept alive while registered)
allocator_calls = {"alloc": 0, "free": 0}


def use_torch_allocator(on: bool = True) -> None:
    """Route every device buffer of the library through PyTorch's caching allocator
    (tp_set_allocator), or back to hipMalloc.  Switch only while no problem exists."""
    global _torch_allocator
    if not on:
        _check(lib().tp_set_allocator(None, None, None))
        _torch_allocator = None
        return

    def _alloc(nbytes, stream, user):
        try:
            allocator_calls["alloc"] += 1
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), int(stream or 0))
        except Exception:       # reported to the library as NULL -> TP_E_OUT_OF_MEMORY
            return None

    def _free(ptr, nbytes, stream, user):
        allocator_calls["free"] += 1
        torch.cuda.caching_allocator_delete(ptr)

    cbs = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    _check(lib().tp_set_allocator(ctypes.cast(cbs[0], ctypes.c_void_p), ctypes.cast(cbs[1], ctypes.c_void_p), None))
    _torch_allocator = cbs


def _check(status: int, allow=()):
    if status != TP_OK and status not in allow:
        raise TpError(status, (lib().tp_last_error() or b"").decode())
    return status


def default_params(**kw) -> Params:
    p = Params()
    _check(lib().tp_params_default(ctypes.byref(p)))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev(t: torch.Tensor, dtype, name: str, cols: Optional[int] = None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
        raise ValueError(f"{name} must have shape (n, {cols})")
    return t.contiguous()


def _mesh(V, F):
    return _dev(V, torch.float64, "V", 3), _dev(F, torch.int32, "F", 3)


def tp_energy(V, F, params: Optional[Params] = None) -> float:
    V, F = _mesh(V, F)
    E = ctypes.c_double()
    _check(lib().tp_energy(V.data_ptr(), V.shape[0], F.data_ptr(), F.shape[0],
                           ctypes.byref(params or default_params()), ctypes.byref(E), _stream()))
    return E.value


def tp_gradient(V, F, params: Optional[Params] = None):
    V, F = _mesh(V, F)
    dE = torch.empty_like(V)
    E = ctypes.c_double()
    _check(lib().tp_gradient(V.data_ptr(), V.shape[0], F.data_ptr(), F.shape[0],
                             ctypes.byref(params or default_params()), ctypes.byref(E),
                             dE.data_ptr(), _stream()))
    return E.value, dE


def tp_energy_faces(X, N, a, params: Optional[Params] = None) -> float:
    X = _dev(X, torch.float64, "X", 3)
    N = _dev(N, torch.float64, "N", 3)
    a = _dev(a, torch.float64, "a")
    E = ctypes.c_double()
    _check(lib().tp_energy_faces(X.data_ptr(), N.data_ptr(), a.data_ptr(), a.shape[0],
                                 ctypes.byref(params or default_params()), ctypes.byref(E), _stream()))
    return E.value


def tp_energy_faces_noalloc(X, N, a, params: Optional[Params] = None) -> float:
    """tp_energy_faces through the entry point that allocates nothing (nF <= 65536)."""
    X = _dev(X, torch.float64, "X", 3)
    N = _dev(N, torch.float64, "N", 3)
    a = _dev(a, torch.float64, "a")
    E = ctypes.c_double()
    _check(lib().tp_energy_faces_noalloc(X.data_ptr(), N.data_ptr(), a.data_ptr(), a.shape[0],
                                         ctypes.byref(params or default_params()), ctypes.byref(E), _stream()))
    return E.value


def tp_remesh(V, F, L0: float, iterations: int = 5, rho: float = 0.5):
    """Remesh on the host (splits, collapses, Delaunay flips, tangential smoothing).
    V (nV, 3) and F (nF, 3) as numpy arrays or CPU tensors; returns new (V, F) numpy
    arrays (float64, int32)."""
    import numpy as np
    V = np.ascontiguousarray(np.asarray(V.cpu() if isinstance(V, torch.Tensor) else V, dtype=np.float64))
    F = np.ascontiguousarray(np.asarray(F.cpu() if isinstance(F, torch.Tensor) else F, dtype=np.int32))
    if V.ndim != 2 or V.shape[1] != 3 or F.ndim != 2 or F.shape[1] != 3:
        raise ValueError("V must be (nV, 3) and F (nF, 3)")
    nv, nf = ctypes.c_int64(), ctypes.c_int64()
    capV, capF = V.shape[0] + 3 * F.shape[0] // 2 + 16, 4 * F.shape[0] + 16
    for _ in range(2):
        Vo = np.empty((capV, 3), np.float64)
        Fo = np.empty((capF, 3), np.int32)
        st = lib().tp_remesh(V.ctypes.data, V.shape[0], F.ctypes.data, F.shape[0], float(L0), int(iterations),
                             float(rho), Vo.ctypes.data, capV, Fo.ctypes.data, capF,
                             ctypes.byref(nv), ctypes.byref(nf))
        if st == 0:
            return Vo[:nv.value].copy(), Fo[:nf.value].copy()
        if nv.value <= capV and nf.value <= capF:
            break
        capV, capF = nv.value, nf.value
    _check(st)


def _cols(u, nV, name):
    u = _dev(u, torch.float64, name)
    if u.dim() == 1:
        u = u.reshape(-1, 1)
    if u.shape[0] != nV:
        raise ValueError(f"{name} must have {nV} rows")
    return u.contiguous()


def tp_fractional_apply(V, F, u, params: Optional[Params] = None):
    V, F = _mesh(V, F)
    squeeze = u.dim() == 1
    u = _cols(u, V.shape[0], "u")
    Lu = torch.empty_like(u)
    _check(lib().tp_fractional_apply(V.data_ptr(), V.shape[0], F.data_ptr(), F.shape[0],
                                     ctypes.byref(params or default_params()), u.data_ptr(),
                                     u.shape[1], Lu.data_ptr(), _stream()))
    return Lu[:, 0] if squeeze else Lu


def tp_sobolev_apply(V, F, u, params: Optional[Params] = None):
    """A u = (B + B0) u, the operator of the inner product, for u of shape (nV,) or (nV, k)."""
    V, F = _mesh(V, F)
    squeeze = u.dim() == 1
    u = _cols(u, V.shape[0], "u")
    Au = torch.empty_like(u)
    _check(lib().tp_sobolev_apply(V.data_ptr(), V.shape[0], F.data_ptr(), F.shape[0],
                                  ctypes.byref(params or default_params()), u.data_ptr(),
                                  u.shape[1], Au.data_ptr(), _stream()))
    return Au[:, 0] if squeeze else Au


def tp_precond_apply(V, F, b, params: Optional[Params] = None):
    V, F = _mesh(V, F)
    squeeze = b.dim() == 1
    b = _cols(b, V.shape[0], "b")
    x = torch.empty_like(b)
    rep = SolveReport()
    _check(lib().tp_precond_apply(V.data_ptr(), V.shape[0], F.data_ptr(), F.shape[0],
                                  ctypes.byref(params or default_params()), b.data_ptr(), b.shape[1],
                                  x.data_ptr(), ctypes.byref(rep), _stream()))
    return (x[:, 0] if squeeze else x), rep


def step_opts(**kw) -> StepOpts:
    o = StepOpts()
    _check(lib().tp_step_opts_default(ctypes.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


_live_problems: "weakref.WeakSet[Problem]" = weakref.WeakSet()


@atexit.register
def _close_live_problems():
    """Destroy problems still open when the interpreter exits, while the HIP runtime and
    (with a registered allocator) the Python free callback are both still usable."""
    for P in list(_live_problems):
        P.close()


class Problem:
    """Resident problem (tp_problem_*): topology, vertices and work buffers stay on the device."""

    def __init__(self, V, F, params: Optional[Params] = None):
        V, F = _mesh(V, F)
        self.nV, self.nF = V.shape[0], F.shape[0]
        self.device = V.device
        h = ctypes.c_void_p()
        _check(lib().tp_problem_create(V.data_ptr(), self.nV, F.data_ptr(), self.nF,
                                       ctypes.byref(params or default_params()), _stream(),
                                       ctypes.byref(h)))
        self._h = h
        _live_problems.add(self)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().tp_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_vertices(self, V):
        V = _dev(V, torch.float64, "V", 3)
        _check(lib().tp_problem_set_vertices(self._h, V.data_ptr()))

    def vertices(self):
        out = torch.empty((self.nV, 3), dtype=torch.float64, device=self.device)
        _check(lib().tp_problem_get_vertices(self._h, out.data_ptr()))
        return out

    def energy(self) -> float:
        E = ctypes.c_double()
        _check(lib().tp_problem_energy(self._h, ctypes.byref(E)))
        return E.value

    def gradient(self, out=None):
        dE = out if out is not None else torch.empty((self.nV, 3), dtype=torch.float64, device=self.device)
        E = ctypes.c_double()
        _check(lib().tp_problem_gradient(self._h, ctypes.byref(E), dE.data_ptr()))
        return E.value, dE

    def fractional_apply(self, u, out=None):
        squeeze = u.dim() == 1
        u = _cols(u, self.nV, "u")
        Lu = out if out is not None else torch.empty_like(u)
        _check(lib().tp_problem_fractional_apply(self._h, u.data_ptr(), u.shape[1], Lu.data_ptr()))
        return Lu[:, 0] if squeeze else Lu

    def sobolev_solve(self, b, rtol: float = 1e-6, restart: int = 30, maxiter: int = 300, precond: int = 1,
                      out=None, check: bool = True):
        """x = A^+ P b by preconditioned GMRES; returns (x, report dict).  precond = 0 uses the
        paper's preconditioner alone, 1 adds the weighted diagonal of A."""
        squeeze = b.dim() == 1
        b = _cols(b, self.nV, "b")
        x = out if out is not None else torch.empty_like(b)
        r = GmresReport()
        st = lib().tp_problem_sobolev_solve(self._h, b.data_ptr(), b.shape[1], rtol, restart, maxiter,
                                            precond, x.data_ptr(), ctypes.byref(r))
        if check:
            _check(st)
        rep = {"iters": r.iters, "cycles": r.cycles, "relres": r.relres,
               "precond_cg_iters": r.precond_cg_iters, "t_ms": r.t_ms, "omega": r.omega, "status": st}
        return (x[:, 0] if squeeze else x), rep

    def set_obstacle(self, Vo, Fo, p: float = 6.0, weight: float = 1.0):
        """Static obstacle mesh (device tensors) with potential exponent p and weight."""
        Vo, Fo = _mesh(Vo, Fo)
        _check(lib().tp_problem_set_obstacle(self._h, Vo.data_ptr(), Vo.shape[0], Fo.data_ptr(), Fo.shape[0],
                                             p, weight))

    def add_implicit(self, kind: int, q, c: float, p: float = 6.0, weight: float = 1.0, attract: bool = False):
        """kind 0: plane q . x = c; kind 1: sphere |x - q| = c; obstacle or attractor."""
        qa = (ctypes.c_double * 3)(*[float(v) for v in q])
        _check(lib().tp_problem_add_implicit(self._h, kind, qa, c, p, weight, 1 if attract else 0))

    def clear_implicit(self):
        _check(lib().tp_problem_add_implicit(self._h, -1, None, 0.0, 0.0, 0.0, 0))

    def implicit_energy(self, out=None):
        dE = out if out is not None else torch.empty((self.nV, 3), dtype=torch.float64, device=self.device)
        E = ctypes.c_double()
        _check(lib().tp_problem_implicit_energy(self._h, ctypes.byref(E), dE.data_ptr()))
        return E.value, dE

    def obstacle_energy(self, out=None):
        dE = out if out is not None else torch.empty((self.nV, 3), dtype=torch.float64, device=self.device)
        E = ctypes.c_double()
        _check(lib().tp_problem_obstacle_energy(self._h, ctypes.byref(E), dE.data_ptr()))
        return E.value, dE

    def sobolev_apply(self, u, out=None):
        squeeze = u.dim() == 1
        u = _cols(u, self.nV, "u")
        Au = out if out is not None else torch.empty_like(u)
        _check(lib().tp_problem_sobolev_apply(self._h, u.data_ptr(), u.shape[1], Au.data_ptr()))
        return Au[:, 0] if squeeze else Au

    def precond_apply(self, b, out=None, allow_not_converged=False):
        squeeze = b.dim() == 1
        b = _cols(b, self.nV, "b")
        x = out if out is not None else torch.empty_like(b)
        rep = SolveReport()
        allow = (5,) if allow_not_converged else ()
        _check(lib().tp_problem_precond_apply(self._h, b.data_ptr(), b.shape[1], x.data_ptr(),
                                              ctypes.byref(rep)), allow)
        return (x[:, 0] if squeeze else x), rep

    def poisson_solve(self, b, out=None, allow_not_converged=False):
        """Per-component mean-zero solution of C x = P b (FP64 CG)."""
        squeeze = b.dim() == 1
        b = _cols(b, self.nV, "b")
        x = out if out is not None else torch.empty_like(b)
        rep = SolveReport()
        allow = (5,) if allow_not_converged else ()
        _check(lib().tp_problem_poisson_solve(self._h, b.data_ptr(), b.shape[1], x.data_ptr(),
                                              ctypes.byref(rep)), allow)
        return (x[:, 0] if squeeze else x), rep

    def step(self, opts: Optional[StepOpts] = None, direction=None):
        rep = StepReport()
        ptr = direction.data_ptr() if direction is not None else None
        _check(lib().tp_precond_step(self._h, ctypes.byref(opts or step_opts()), ctypes.byref(rep), ptr))
        return rep

    def bh_stats(self):
        """(far, near) term counts of the last Barnes-Hut evaluation."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().tp_problem_bh_stats(self._h, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def bct_stats(self):
        """(admissible, inadmissible) blocks of the last block cluster tree."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().tp_problem_bct_stats(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def obstacle_stats(self):
        """(far, near) terms of the last obstacle evaluation (tp_problem_obstacle_stats)."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().tp_problem_obstacle_stats(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_pins(self, idx) -> None:
        """Pin the listed vertices at their current positions (tp_problem_set_pins)."""
        import numpy as np
        a = np.ascontiguousarray(np.asarray(idx, dtype=np.int32).reshape(-1))
        _check(lib().tp_problem_set_pins(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), a.size))

    def device_bytes(self) -> int:
        b = ctypes.c_uint64()
        _check(lib().tp_problem_device_bytes(self._h, ctypes.byref(b)))
        return int(b.value)


def batch_step(problems, opts=None):
    """tp_batch_step: one descent step of every problem, same-phase work in shared launches.

    opts: None (defaults), one StepOpts for all, or a list of len(problems).
    Returns (statuses, reports); a failed problem's status is nonzero, the others are valid.
    """
    n = len(problems)
    if n == 0:
        return [], []
    hs = (ctypes.c_void_p * n)(*[p._h.value for p in problems])
    if opts is None or isinstance(opts, StepOpts):
        one = opts or step_opts()
        arr = (StepOpts * n)(*([one] * n))
    else:
        if len(opts) != n:
            raise ValueError("opts must have one entry per problem")
        arr = (StepOpts * n)(*opts)
    reps = (StepReport * n)()
    sts = (ctypes.c_int * n)()
    rc = lib().tp_batch_step(hs, n, arr, reps, sts)
    if rc == TP_E_DEVICE or (rc != TP_OK and all(int(x) == TP_OK for x in sts)):
        _check(rc)      # a failure of the whole call, not of one problem
    return [int(x) for x in sts], [reps[i] for i in range(n)]


def estimate_device_bytes(nV: int, nF: int, max_degree: int, ncomp: int = 1,
                          params: Optional[Params] = None, n_constraints: int = 2) -> int:
    b = ctypes.c_uint64()
    _check(lib().tp_estimate_device_bytes(nV, nF, max_degree, ncomp, ctypes.byref(params or default_params()),
                                          n_constraints, ctypes.byref(b)))
    return int(b.value)


def profile_enable(on: bool = True):
    _check(lib().tp_profile_enable(1 if on else 0))


def profile_reset():
    _check(lib().tp_profile_reset())


def profile_get(kind: int) -> dict:
    st = KernelStats()
    _check(lib().tp_profile_get(kind, ctypes.byref(st)))
    return {"ms_total": st.ms_total, "pairs_total": st.pairs_total, "cols_total": st.cols_total,
            "launches": int(st.launches)}
