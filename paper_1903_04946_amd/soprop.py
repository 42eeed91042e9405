"""Thin ctypes binding of libsoprop (include/soprop.h).

Argument marshalling only: every step of the propagation runs in the HIP
library.  PyTorch supplies device memory (the caller's psi tensors) and the
stream.  If the library is missing or cannot be loaded, every entry point
raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsoprop.so")

SPLITS = {"VTV": 0, "TVT": 1, "VT": 2, "TV": 3}
COMPS = {"strang": 0, "triple_jump": 1, "tj": 1, "suzuki": 2, "sf": 2, "custom": 3}
ABI_VERSION = 3
C128, C64 = 0, 1


class SopError(RuntimeError):
    pass


class _Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]


class _Desc(ctypes.Structure):
    _fields_ = [("grid", _Grid), ("nsurf", ctypes.c_int),
                ("inv_mass", ctypes.POINTER(ctypes.c_double)),
                ("vtable", ctypes.POINTER(ctypes.c_double)),
                ("split", ctypes.c_int), ("comp", ctypes.c_int), ("order", ctypes.c_int),
                ("dt", ctypes.c_double), ("hbar", ctypes.c_double), ("dtype", ctypes.c_int),
                ("nparams", ctypes.c_int), ("dvtables", ctypes.POINTER(ctypes.c_double)),
                ("ngamma", ctypes.c_int), ("gamma", ctypes.POINTER(ctypes.c_double))]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("alloc", _ALLOC_FN), ("free", _FREE_FN)]


def _torch_allocator():
    """sop_allocator hooks onto PyTorch's caching allocator (current device):
    the plan's tables then live in torch's memory pool."""
    import torch
    dev = torch.cuda.current_device()

    def alloc(ctx, nbytes, stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0))
        except Exception:  # out of memory: the library reports SOP_ERR_NOMEM
            return None

    def free(ctx, ptr, stream):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:  # interpreter shutdown: the process releases the pool
            pass

    fa, ff = _ALLOC_FN(alloc), _FREE_FN(free)
    return _Allocator(None, fa, ff), (fa, ff)


class _Info(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("n_a", ctypes.c_int), ("n_b", ctypes.c_int),
                ("n_a_unq", ctypes.c_int), ("n_b_unq", ctypes.c_int),
                ("n_v_tables", ctypes.c_int), ("n_t_tables", ctypes.c_int),
                ("npts", ctypes.c_int64), ("table_bytes", ctypes.c_size_t),
                ("scratch_bytes", ctypes.c_size_t)]


EXPORTS = ["sop_abi_version", "sop_status_string", "sop_last_error", "sop_supported_length",
           "sop_scheme_sequence", "sop_custom_sequence", "sop_plan_create", "sop_plan_create_with_allocator",
           "sop_plan_destroy", "sop_plan_info_get",
           "sop_plan_set_stream", "sop_propagate", "sop_observables", "sop_overlap",
           "sop_distance", "sop_interpolate", "sop_propagate_trapezoid",
           "sop_propagate_trapezoid_noalloc", "sop_apply_action", "sop_plan_set_timing", "sop_timing_read",
           "sop_plan_set_params",
           "sop_plan_update_v", "sop_action_times", "sop_propagate_driven",
           "sop_adjoint_workspace_bytes", "sop_adjoint_forward", "sop_adjoint_backward",
           "sop_adjoint",
           "sop_propagate_many", "sop_plan_set_option", "sop_batch_create",
           "sop_batch_destroy", "sop_batch_propagate", "sop_batch_set_option",
           "sop_batch_check", "sop_batch_describe"]
KINDS = ["zpass", "ypass", "xpass", "k1d", "other", "plane", "interp"]

_lib = None


def lib():
    """Loads libsoprop.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SopError(f"{LIB_PATH} is not built; run python -m paper_1903_04946_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    dp, ip, vp = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), ctypes.c_void_p
    L.sop_abi_version.restype = ctypes.c_int
    if L.sop_abi_version() != ABI_VERSION:
        raise SopError(f"{LIB_PATH} has ABI version {L.sop_abi_version()}, the binding "
                       f"expects {ABI_VERSION}; rebuild it")
    L.sop_status_string.restype = ctypes.c_char_p
    L.sop_status_string.argtypes = [ctypes.c_int]
    L.sop_last_error.restype = ctypes.c_char_p
    L.sop_supported_length.argtypes = [ctypes.c_int, ctypes.c_int]
    L.sop_scheme_sequence.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      dp, dp, dp, dp, ip, ip, ip]
    L.sop_custom_sequence.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int,
                                      dp, dp, dp, dp, ip, ip, ip]
    L.sop_plan_create.argtypes = [ctypes.POINTER(_Desc), vp, ctypes.POINTER(vp)]
    L.sop_plan_create_with_allocator.argtypes = [ctypes.POINTER(_Desc), vp,
                                                 ctypes.POINTER(_Allocator), ctypes.POINTER(vp)]
    L.sop_plan_destroy.argtypes = [vp]
    L.sop_plan_info_get.argtypes = [vp, ctypes.POINTER(_Info)]
    L.sop_plan_set_stream.argtypes = [vp, vp]
    L.sop_propagate.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int]
    L.sop_observables.argtypes = [vp, vp, dp]
    L.sop_overlap.argtypes = [vp, vp, vp, dp]
    L.sop_distance.argtypes = [vp, vp, vp, dp]
    L.sop_interpolate.argtypes = [vp, vp, vp, vp]
    L.sop_propagate_trapezoid.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                                          ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
    L.sop_propagate_trapezoid_noalloc.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int64,
                                                  ctypes.c_double, ctypes.c_int,
                                                  ctypes.POINTER(ctypes.c_int64)]
    L.sop_apply_action.argtypes = [vp, vp, ctypes.c_int, ctypes.c_double]
    L.sop_plan_set_timing.argtypes = [vp, ctypes.c_int]
    L.sop_plan_set_params.argtypes = [vp, dp]
    L.sop_plan_update_v.argtypes = [vp, dp]
    L.sop_action_times.argtypes = [vp, dp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.sop_propagate_driven.argtypes = [vp, vp, ctypes.c_int64, dp]
    L.sop_propagate_many.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int64, ctypes.c_int]
    L.sop_plan_set_option.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.sop_adjoint_workspace_bytes.argtypes = [vp, ctypes.c_int64, ctypes.c_int,
                                              ctypes.POINTER(ctypes.c_size_t)]
    L.sop_adjoint_forward.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int, vp, dp]
    L.sop_adjoint_backward.argtypes = [vp, ctypes.c_int64, ctypes.c_int, dp, vp, dp]
    L.sop_adjoint.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int, dp, vp, dp, dp]
    L.sop_timing_read.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64), dp]
    L.sop_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.POINTER(vp)]
    L.sop_batch_destroy.argtypes = [vp]
    L.sop_batch_propagate.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.c_int]
    L.sop_batch_set_option.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.sop_batch_check.argtypes = [vp]
    L.sop_batch_describe.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t,
                                     ctypes.POINTER(ctypes.c_size_t)]
    for f in ("sop_scheme_sequence", "sop_plan_create", "sop_plan_create_with_allocator",
              "sop_plan_destroy", "sop_plan_info_get",
              "sop_plan_set_stream", "sop_propagate", "sop_observables", "sop_overlap",
              "sop_distance", "sop_interpolate", "sop_propagate_trapezoid",
           "sop_propagate_trapezoid_noalloc", "sop_apply_action", "sop_plan_set_timing", "sop_timing_read",
              "sop_plan_set_params",
              "sop_plan_update_v", "sop_action_times", "sop_propagate_driven",
              "sop_adjoint_workspace_bytes", "sop_adjoint_forward", "sop_adjoint_backward",
              "sop_propagate_many", "sop_plan_set_option", "sop_batch_create",
              "sop_batch_destroy", "sop_batch_propagate", "sop_batch_set_option",
              "sop_batch_check", "sop_batch_describe"):
        getattr(L, f).restype = ctypes.c_int
    L.sop_supported_length.restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc != 0:
        L = lib()
        raise SopError(f"{what}: {L.sop_status_string(rc).decode()} "
                       f"({L.sop_last_error().decode()})")


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def interpolate(src: "Plan", psi_src, dst: "Plan", psi_dst) -> None:
    """psi_dst <- the trigonometric interpolant of psi_src (src's grid)
    evaluated on dst's grid, zero outside src's box (sop_interpolate)."""
    for plan, psi in ((src, psi_src), (dst, psi_dst)):
        plan._check_psi(psi)
    _check(lib().sop_interpolate(src._h, ctypes.c_void_p(psi_src.data_ptr()), dst._h,
                                 ctypes.c_void_p(psi_dst.data_ptr())), "sop_interpolate")


def scheme_sequence(split: str, comp: str, order: int = 2, gamma=None):
    """Pruned sequence and unique coefficients from the library's planner
    (comp = 'custom' takes the symmetric coefficients gamma)."""
    cap = 4096
    a, b, au, bu = (np.zeros(cap) for _ in range(4))
    ia = np.zeros(cap, np.int32)
    ib = np.zeros(cap, np.int32)
    counts = np.zeros(4, np.int32)
    if comp == "custom":
        g = np.ascontiguousarray(gamma, dtype=np.float64)
        _check(lib().sop_custom_sequence(SPLITS[split], g.size, _dp(g), cap, _dp(a), _dp(b),
                                         _dp(au), _dp(bu), _ip(ia), _ip(ib), _ip(counts)),
               "sop_custom_sequence")
    else:
        _check(lib().sop_scheme_sequence(SPLITS[split], COMPS[comp], order, cap, _dp(a),
                                         _dp(b), _dp(au), _dp(bu), _ip(ia), _ip(ib),
                                         _ip(counts)),
               "sop_scheme_sequence")
    N, na, nb, M = (int(c) for c in counts)
    return {"a": a[:N].copy(), "b": b[:N].copy(), "a_unq": au[:na].copy(),
            "b_unq": bu[:nb].copy(), "ia": ia[:N].copy(), "ib": ib[:N].copy(), "M": M}


@dataclass
class PlanInfo:
    M: int
    n_a: int
    n_b: int
    n_a_unq: int
    n_b_unq: int
    n_v_tables: int
    n_t_tables: int
    npts: int
    table_bytes: int
    scratch_bytes: int


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A propagation plan (sop_plan_create).

    n, lo, hi: per-axis grid (1D or cubic 3D); nsurf; inv_mass per axis;
    vtable: float64 [S(S+1)/2][npts] packed upper triangle of V(q);
    split: 'VTV' | 'TVT' | 'VT' | 'TV'; comp: 'strang' | 'triple_jump' |
    'suzuki' | 'custom' (gamma: the symmetric composition coefficients);
    order; dt; dtype: torch.complex128 or torch.complex64;
    allocator: None (the library's hipMalloc) or 'torch' (the plan's device
    buffers come from PyTorch's caching allocator,
    sop_plan_create_with_allocator).
    """

    def __init__(self, n, lo, hi, nsurf, inv_mass, vtable, split="VTV", comp="strang",
                 order=2, dt=0.01, hbar=1.0, dtype=None, stream=None, dvtables=None,
                 allocator=None, gamma=None):
        import torch
        if dtype is None:
            dtype = torch.complex128
        if dtype not in (torch.complex128, torch.complex64):
            raise ValueError("dtype must be complex128 or complex64")
        L = lib()
        self.dtype = dtype
        self.n = list(n)
        self.nsurf = int(nsurf)
        self.shape = (self.nsurf, *self.n)
        g = _Grid()
        g.ndim = len(self.n)
        for d in range(3):
            g.n[d] = self.n[d] if d < g.ndim else 1
            g.lo[d] = lo[d] if d < g.ndim else 0.0
            g.hi[d] = hi[d] if d < g.ndim else 1.0
        self._inv_mass = np.ascontiguousarray(inv_mass, dtype=np.float64)
        ne = self.nsurf * (self.nsurf + 1) // 2
        self._vt = np.ascontiguousarray(vtable, dtype=np.float64).reshape(ne, -1)
        if self._vt.shape[1] != int(np.prod(self.n)):
            raise ValueError("vtable size does not match the grid")
        d = _Desc()
        d.grid = g
        d.nsurf = self.nsurf
        d.inv_mass = _dp(self._inv_mass)
        d.vtable = _dp(self._vt)
        d.split = SPLITS[split]
        d.comp = COMPS[comp]
        d.order = int(order)
        if gamma is not None:
            self._gamma = np.ascontiguousarray(gamma, dtype=np.float64).ravel()
            d.ngamma = self._gamma.size
            d.gamma = _dp(self._gamma)
        d.dt = float(dt)
        self.dt = float(dt)
        d.hbar = float(hbar)
        d.dtype = C128 if dtype == torch.complex128 else C64
        self.nparams = 0
        if dvtables is not None:
            self._dv = np.ascontiguousarray(dvtables, dtype=np.float64).reshape(-1, ne,
                                                                               self._vt.shape[1])
            self.nparams = self._dv.shape[0]
            d.nparams = self.nparams
            d.dvtables = _dp(self._dv)
        self._stream = stream
        h = ctypes.c_void_p()
        if allocator is None:
            _check(L.sop_plan_create(ctypes.byref(d), _stream_handle(stream), ctypes.byref(h)),
                   "sop_plan_create")
        elif allocator == "torch":
            self._hooks = _torch_allocator()  # kept alive until the plan is destroyed
            _check(L.sop_plan_create_with_allocator(ctypes.byref(d), _stream_handle(stream),
                                                    ctypes.byref(self._hooks[0]),
                                                    ctypes.byref(h)),
                   "sop_plan_create_with_allocator")
        else:
            raise ValueError("allocator must be None or 'torch'")
        self._h = h

    @classmethod
    def from_model(cls, model, **kw):
        return cls(model.n, model.lo, model.hi, model.nsurf, model.inv_mass, model.vtable,
                   hbar=model.hbar, **kw)

    def set_params(self, theta):
        """V <- vtable + sum_k theta_k dvtables[k]; tables formed again."""
        th = np.ascontiguousarray(theta, dtype=np.float64).reshape(self.nparams)
        _check(lib().sop_plan_set_params(self._h, _dp(th)), "sop_plan_set_params")

    def action_times(self) -> np.ndarray:
        """Times of one step's potential actions, in units of dt from its start."""
        cnt = ctypes.c_int()
        _check(lib().sop_action_times(self._h, None, 0, ctypes.byref(cnt)), "sop_action_times")
        c = np.zeros(cnt.value)
        _check(lib().sop_action_times(self._h, _dp(c), cnt.value, ctypes.byref(cnt)),
               "sop_action_times")
        return c

    def propagate_driven(self, psi, nsteps: int, drive=None, f=None, t0: float = 0.0):
        """psi <- the composed steps with V + s D, s sampled per potential
        action: `drive` [nsteps][count], or a callable f(t) evaluated at
        t0 + (n + c_v) dt (c from action_times).  Synchronises."""
        self._check_psi(psi)
        c = self.action_times()
        if drive is None:
            if f is None:
                raise ValueError("give drive samples or f")
            t = t0 + (np.arange(int(nsteps))[:, None] + c[None, :]) * self.dt
            drive = np.vectorize(f, otypes=[float])(t) if t.size else np.zeros((0, len(c)))
        s = np.ascontiguousarray(drive, dtype=np.float64).reshape(-1)
        if s.size != int(nsteps) * len(c):
            raise ValueError("drive must hold nsteps x count samples")
        _check(lib().sop_propagate_driven(self._h, ctypes.c_void_p(psi.data_ptr()),
                                          int(nsteps), _dp(s)), "sop_propagate_driven")
        return psi

    def update_v(self, vtable):
        """Replaces the V-table ([S(S+1)/2][npts] FP64) and forms the tables again."""
        vt = np.ascontiguousarray(vtable, dtype=np.float64)
        if vt.size != self._vt.size:
            raise ValueError("vtable must hold S(S+1)/2 x npts values")
        vt = vt.reshape(self._vt.shape)
        _check(lib().sop_plan_update_v(self._h, _dp(vt)), "sop_plan_update_v")
        self._vt = vt

    def adjoint_workspace_bytes(self, nsteps: int, K: int) -> int:
        b = ctypes.c_size_t()
        _check(lib().sop_adjoint_workspace_bytes(self._h, int(nsteps), int(K), ctypes.byref(b)),
               "sop_adjoint_workspace_bytes")
        return int(b.value)

    def adjoint_workspace(self, nsteps: int, K: int):
        import torch
        return torch.empty(self.adjoint_workspace_bytes(nsteps, K), dtype=torch.uint8,
                           device="cuda")

    def adjoint_forward(self, psi0, nsteps: int, K: int, workspace) -> np.ndarray:
        """Populations P_s(T) after nsteps from psi0, checkpoints every K steps."""
        self._check_psi(psi0)
        pops = np.zeros(self.nsurf)
        _check(lib().sop_adjoint_forward(self._h, ctypes.c_void_p(psi0.data_ptr()), int(nsteps),
                                         int(K), ctypes.c_void_p(workspace.data_ptr()), _dp(pops)),
               "sop_adjoint_forward")
        return pops

    def adjoint_backward(self, nsteps: int, K: int, weights, workspace) -> np.ndarray:
        """sum_s weights[s] dP_s/dtheta_k after adjoint_forward."""
        w = np.ascontiguousarray(weights, dtype=np.float64).reshape(self.nsurf)
        g = np.zeros(self.nparams)
        _check(lib().sop_adjoint_backward(self._h, int(nsteps), int(K), _dp(w),
                                          ctypes.c_void_p(workspace.data_ptr()), _dp(g)),
               "sop_adjoint_backward")
        return g

    def adjoint(self, psi0, nsteps: int, K: int, weights, workspace):
        """(P_s(T), sum_s weights[s] dP_s/dtheta_k) in one call (sop_adjoint)."""
        self._check_psi(psi0)
        w = np.ascontiguousarray(weights, dtype=np.float64).reshape(self.nsurf)
        pops = np.zeros(self.nsurf)
        g = np.zeros(self.nparams)
        _check(lib().sop_adjoint(self._h, ctypes.c_void_p(psi0.data_ptr()), int(nsteps), int(K),
                                 _dp(w), ctypes.c_void_p(workspace.data_ptr()), _dp(pops),
                                 _dp(g)), "sop_adjoint")
        return pops, g

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().sop_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def info(self) -> PlanInfo:
        i = _Info()
        _check(lib().sop_plan_info_get(self._h, ctypes.byref(i)), "sop_plan_info_get")
        return PlanInfo(i.M, i.n_a, i.n_b, i.n_a_unq, i.n_b_unq, i.n_v_tables, i.n_t_tables,
                        i.npts, i.table_bytes, i.scratch_bytes)

    def _check_psi(self, psi):
        import torch
        if not isinstance(psi, torch.Tensor) or not psi.is_cuda:
            raise TypeError("psi must be a CUDA (HIP) tensor")
        if psi.dtype != self.dtype:
            raise TypeError(f"psi dtype {psi.dtype} != plan dtype {self.dtype}")
        if tuple(psi.shape) != self.shape or not psi.is_contiguous():
            raise ValueError(f"psi must be a contiguous tensor of shape {self.shape}")

    def propagate_trapezoid(self, psi, nsteps: int, tol: float = 1e-13,
                            max_iter: int = 10000, noalloc: bool = False) -> int:
        """psi ([S, N], or [count, S, N] independent states) advanced in place
        by nsteps steps of the plan's composition of the trapezoidal rule
        (sop_propagate_trapezoid, or with noalloc=True
        sop_propagate_trapezoid_noalloc, whose workspace is the library's
        static device scratch); returns the number of linear-solver
        iterations."""
        import torch
        if psi.dim() == len(self.shape) + 1:
            count = psi.shape[0]
            if (not isinstance(psi, torch.Tensor) or not psi.is_cuda or psi.dtype != self.dtype
                    or tuple(psi.shape[1:]) != self.shape or not psi.is_contiguous()):
                raise ValueError(f"psi must be a contiguous CUDA tensor [count, {self.shape}]")
        else:
            self._check_psi(psi)
            count = 1
        it = ctypes.c_int64()
        name = "sop_propagate_trapezoid_noalloc" if noalloc else "sop_propagate_trapezoid"
        _check(getattr(lib(), name)(self._h, ctypes.c_void_p(psi.data_ptr()), int(count),
                                    int(nsteps), float(tol), int(max_iter), ctypes.byref(it)),
               name)
        return int(it.value)

    def set_stream(self, stream=None):
        self._stream = stream
        _check(lib().sop_plan_set_stream(self._h, _stream_handle(stream)), "sop_plan_set_stream")

    def propagate(self, psi, nsteps: int, direction: int = 1):
        """psi <- U(direction dt)^nsteps psi in place (asynchronous)."""
        self._check_psi(psi)
        _check(lib().sop_propagate(self._h, ctypes.c_void_p(psi.data_ptr()), int(nsteps),
                                   int(direction)), "sop_propagate")
        return psi

    def propagate_many(self, psis, nsteps: int, direction: int = 1):
        """Propagates a contiguous [count, S, n...] tensor of states in place."""
        import torch
        if not isinstance(psis, torch.Tensor) or not psis.is_cuda or psis.dtype != self.dtype:
            raise TypeError("psis must be a CUDA tensor of the plan's dtype")
        if tuple(psis.shape[1:]) != self.shape or not psis.is_contiguous() or psis.dim() < 2:
            raise ValueError(f"psis must be contiguous of shape [count, {self.shape}]")
        _check(lib().sop_propagate_many(self._h, ctypes.c_void_p(psis.data_ptr()),
                                        int(psis.shape[0]), int(nsteps), int(direction)),
               "sop_propagate_many")
        return psis

    def apply_action(self, psi, op: str, coef: float):
        self._check_psi(psi)
        _check(lib().sop_apply_action(self._h, ctypes.c_void_p(psi.data_ptr()),
                                      0 if op == "V" else 1, float(coef)), "sop_apply_action")
        return psi

    def set_graphs(self, enable: bool):
        """3D runs of >= 4 steps as captured HIP graphs (default on)."""
        _check(lib().sop_plan_set_option(self._h, 1, int(bool(enable))), "sop_plan_set_option")

    def set_plane_pass(self, enable: bool):
        """Fused xy plane pass on 3D grids whose plane fits in LDS (default on
        for n <= 64)."""
        _check(lib().sop_plan_set_option(self._h, 2, int(bool(enable))), "sop_plan_set_option")

    def set_timing(self, enable: bool):
        """Brackets every kernel launch with HIP events (measurement aid)."""
        _check(lib().sop_plan_set_timing(self._h, int(bool(enable))), "sop_plan_set_timing")

    def timing_read(self) -> dict:
        """Per kernel kind: summed event ms, launch count, algorithmic bytes."""
        ms = np.zeros(len(KINDS))
        counts = np.zeros(len(KINDS), np.int64)
        by = np.zeros(len(KINDS))
        _check(lib().sop_timing_read(self._h, _dp(ms),
                                     counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     _dp(by)), "sop_timing_read")
        return {k: {"ms": float(ms[i]), "count": int(counts[i]), "bytes": float(by[i])}
                for i, k in enumerate(KINDS) if counts[i] > 0}

    def observables(self, psi) -> dict:
        self._check_psi(psi)
        out = np.zeros(4 + self.nsurf)
        _check(lib().sop_observables(self._h, ctypes.c_void_p(psi.data_ptr()), _dp(out)),
               "sop_observables")
        S = self.nsurf
        return {"norm": out[0], "energy": out[1], "pops": out[2:2 + S].copy(),
                "kinetic": out[2 + S], "potential": out[3 + S]}

    def overlap(self, psi, phi) -> complex:
        self._check_psi(psi)
        self._check_psi(phi)
        out = np.zeros(2)
        _check(lib().sop_overlap(self._h, ctypes.c_void_p(psi.data_ptr()),
                                 ctypes.c_void_p(phi.data_ptr()), _dp(out)), "sop_overlap")
        return complex(out[0], out[1])

    def distance(self, psi, phi) -> tuple:
        """(||psi - phi||, ||psi - phi|| / ||phi||) with the volume element."""
        self._check_psi(psi)
        self._check_psi(phi)
        out = np.zeros(2)
        _check(lib().sop_distance(self._h, ctypes.c_void_p(psi.data_ptr()),
                                  ctypes.c_void_p(phi.data_ptr()), _dp(out)), "sop_distance")
        return float(out[0]), float(out[1])


class Batch:
    """Many independent plans propagated by one graph launch (sop_batch_create).

    plans: Plan objects (kept alive by the batch); stream: the torch stream
    the propagate calls run on (default: the current stream).
    """

    def __init__(self, plans, stream=None):
        L = lib()
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(L.sop_batch_create(arr, len(self.plans), _stream_handle(stream), ctypes.byref(h)),
               "sop_batch_create")
        self._h = h

    def propagate(self, psis, nsteps, direction: int = 1):
        """psis[i] <- U_i(direction dt_i)^nsteps[i] psis[i] in place (asynchronous)."""
        if len(psis) != len(self.plans):
            raise ValueError("one state per member")
        ns = np.ascontiguousarray(np.broadcast_to(np.asarray(nsteps, dtype=np.int64),
                                                  (len(self.plans),)))
        for p, x in zip(self.plans, psis):
            p._check_psi(x)
        ptrs = (ctypes.c_void_p * len(psis))(*[x.data_ptr() for x in psis])
        _check(lib().sop_batch_propagate(self._h, ptrs,
                                         ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                         int(direction)), "sop_batch_propagate")
        return psis

    def set_graphs(self, enable: bool):
        _check(lib().sop_batch_set_option(self._h, 1, int(bool(enable))), "sop_batch_set_option")

    def set_plane_pass(self, enable: bool):
        _check(lib().sop_batch_set_option(self._h, 2, int(bool(enable))), "sop_batch_set_option")

    def set_queue(self, enable: bool):
        """3D groups as one work-queue launch each, or (default) as lockstep pass launches."""
        _check(lib().sop_batch_set_option(self._h, 3, int(bool(enable))), "sop_batch_set_option")

    def set_queue_spin(self, polls: int):
        """Bound on the polls of one wait in a work-queue launch."""
        _check(lib().sop_batch_set_option(self._h, 4, int(polls)), "sop_batch_set_option")

    def check(self):
        """Synchronises; raises if a work-queue wait ran out of polls since the last check."""
        _check(lib().sop_batch_check(self._h), "sop_batch_check")

    def describe(self) -> dict:
        import json
        need = ctypes.c_size_t()
        _check(lib().sop_batch_describe(self._h, None, 0, ctypes.byref(need)),
               "sop_batch_describe")
        buf = ctypes.create_string_buffer(need.value)
        _check(lib().sop_batch_describe(self._h, buf, need.value, None), "sop_batch_describe")
        return json.loads(buf.value.decode())

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().sop_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _populations_fn():
    import torch

    class PopulationsFn(torch.autograd.Function):
        """P(theta): final surface populations as a function of the plan's
        parameters; the backward pass runs the library's adjoint sweep.

        apply(theta, plan, psi0, nsteps, K) -> tensor [S] (float64, CPU)
        theta: float64 CPU tensor [nparams]; plan: Plan with dvtables;
        psi0: device tensor of the plan's shape and dtype (complex128).
        """

        @staticmethod
        def forward(ctx, theta, plan, psi0, nsteps, K):
            plan.set_params(theta.detach().cpu().numpy())
            ws = plan.adjoint_workspace(nsteps, K)
            pops = plan.adjoint_forward(psi0, nsteps, K, ws)
            ctx.plan, ctx.ws, ctx.nsteps, ctx.K = plan, ws, nsteps, K
            return torch.from_numpy(pops)

        @staticmethod
        def backward(ctx, grad_pops):
            g = ctx.plan.adjoint_backward(ctx.nsteps, ctx.K, grad_pops.detach().cpu().numpy(),
                                          ctx.ws)
            ctx.ws = None
            return torch.from_numpy(g), None, None, None, None

    return PopulationsFn


_PFN = None


def __getattr__(name):
    global _PFN
    if name == "PopulationsFn":
        if _PFN is None:
            _PFN = _populations_fn()
        return _PFN
    raise AttributeError(name)
