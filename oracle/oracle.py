"""ctypes wrapper of the plain FP64 CPU oracle (``oracle/soref.cpp``).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The product
library (``paper_1903_04946_amd``) never imports this module.

The oracle follows arXiv:1903.04946 (Roulet, Choi, Vanicek): composition
coefficients (Sec. "Symmetric composition schemes"), splitting, pruning and
unique coefficients (Sec. "Pruning splitting coefficients", Table II), the
dynamic Fourier method (Sec. "Dynamic Fourier method"), the Jacobi-based
potential exponential (Sec. "Molecular Hamiltonian in the diabatic basis")
and the exact evolution operator (Eq. exact_evol_op) by dense
diagonalisation on tiny grids.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "soref.cpp")

STRANG, TRIPLE_JUMP, SUZUKI = 0, 1, 2
VTV, TVT, VT, TV = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (plain -O2, OpenMP over independent loops)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["g++", "-O2", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp",
               "-std=c++17", "-shared", "-fPIC", _SRC, "-o", _LIB_PATH + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Problem(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("nsurf", ctypes.c_int),
        ("inv_mass", ctypes.c_double * 3),
        ("hbar", ctypes.c_double),
        ("vtable", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        pp = ctypes.POINTER(_Problem)
        L.orc_gammas.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int]
        L.orc_splitting.argtypes = [ctypes.c_int] * 4 + [dp, dp, ctypes.c_int]
        L.orc_unique.argtypes = [ctypes.c_int] * 3 + [dp, dp, ip, ip, ctypes.c_int, ip]
        L.orc_fft.argtypes = [ctypes.c_int, ctypes.c_int, dp]
        L.orc_expm_potential.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_eigh.argtypes = [ctypes.c_int, dp, dp, dp]
        L.orc_propagate.argtypes = [pp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_int64, ctypes.c_int, dp]
        L.orc_action.argtypes = [pp, ctypes.c_int, ctypes.c_double, dp]
        L.orc_propagate_timed.argtypes = [pp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_int64, dp, dp]
        L.orc_threads.argtypes = []
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_expm_frechet.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_double,
                                       dp, dp]
        L.orc_gradient.argtypes = [pp, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_double, ctypes.c_int64, dp, dp, dp, dp]
        L.orc_observables.argtypes = [pp, dp, dp]
        L.orc_overlap.argtypes = [pp, dp, dp, dp]
        L.orc_distance.argtypes = [pp, dp, dp, dp]
        L.orc_propagate_driven.argtypes = [pp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_double, ctypes.c_int64, dp, dp]
        L.orc_exact.argtypes = [pp, ctypes.c_double, dp]
        ip_ = ctypes.POINTER(ctypes.c_int)
        L.orc_interpolate.argtypes = [ctypes.c_int, ctypes.c_int, ip_, dp, dp, dp, ip_, dp, dp, dp]
        L.orc_propagate_gamma.argtypes = [pp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_double,
                                          ctypes.c_int64, dp]
        for f in ("orc_gammas", "orc_splitting", "orc_unique", "orc_fft", "orc_expm_potential",
                  "orc_eigh", "orc_propagate", "orc_action", "orc_observables", "orc_overlap",
                  "orc_distance", "orc_propagate_driven", "orc_propagate_gamma",
                  "orc_interpolate",
                  "orc_exact", "orc_propagate_timed", "orc_threads", "orc_set_threads",
                  "orc_expm_frechet",
                  "orc_gradient"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


class Problem:
    """Grid, surfaces, masses and V-table of a diabatic model (Eq. diab_mol_ham)."""

    def __init__(self, n, lo, hi, nsurf, inv_mass, vtable, hbar=1.0):
        n = list(n)
        self.ndim = len(n)
        self.n = n
        self.lo = list(lo)
        self.hi = list(hi)
        self.nsurf = int(nsurf)
        self.inv_mass = list(inv_mass)
        self.hbar = float(hbar)
        npts = int(np.prod(n))
        ne = self.nsurf * (self.nsurf + 1) // 2
        self.vtable = np.ascontiguousarray(vtable, dtype=np.float64).reshape(ne, npts)
        self._s = _Problem()
        self._s.ndim = self.ndim
        for d in range(3):
            self._s.n[d] = n[d] if d < self.ndim else 1
            self._s.lo[d] = self.lo[d] if d < self.ndim else 0.0
            self._s.hi[d] = self.hi[d] if d < self.ndim else 1.0
            self._s.inv_mass[d] = self.inv_mass[d] if d < self.ndim else 0.0
        self._s.nsurf = self.nsurf
        self._s.hbar = self.hbar
        self._s.vtable = _dp(self.vtable)

    @property
    def npts(self) -> int:
        return int(np.prod(self.n))

    @property
    def shape(self):
        return (self.nsurf, *self.n)

    def ptr(self):
        return ctypes.byref(self._s)


def gammas(scheme: int, order: int) -> np.ndarray:
    out = np.zeros(4096)
    m = lib().orc_gammas(scheme, order, _dp(out), out.size)
    if m < 0:
        raise ValueError("invalid scheme/order")
    return out[:m].copy()


def splitting(split: int, scheme: int, order: int, pruned: bool):
    a = np.zeros(8192)
    b = np.zeros(8192)
    n = lib().orc_splitting(split, scheme, order, int(pruned), _dp(a), _dp(b), a.size)
    if n < 0:
        raise ValueError("invalid split/scheme/order")
    return a[:n].copy(), b[:n].copy()


def unique(split: int, scheme: int, order: int):
    cap = 4096
    au = np.zeros(cap)
    bu = np.zeros(cap)
    ia = np.zeros(cap, dtype=np.int32)
    ib = np.zeros(cap, dtype=np.int32)
    counts = np.zeros(4, dtype=np.int32)
    if lib().orc_unique(split, scheme, order, _dp(au), _dp(bu), _ip(ia), _ip(ib), cap,
                        _ip(counts)) != 0:
        raise ValueError("invalid split/scheme/order")
    n, na, nb, _ = (int(c) for c in counts)
    return au[:na].copy(), bu[:nb].copy(), ia[:n].copy(), ib[:n].copy()


def fft(x: np.ndarray, inverse: bool = False) -> np.ndarray:
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    lib().orc_fft(a.size, int(inverse), _dp(a.view(np.float64)))
    return a


def expm_potential(V: np.ndarray, tau: float, hbar: float = 1.0) -> np.ndarray:
    V = np.ascontiguousarray(V, dtype=np.float64)
    S = V.shape[0]
    U = np.zeros((S, S), dtype=np.complex128)
    lib().orc_expm_potential(S, _dp(V), tau, hbar, _dp(U.view(np.float64)))
    return U


def eigh(A: np.ndarray):
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    lam = np.zeros(n)
    R = np.zeros((n, n))
    lib().orc_eigh(n, _dp(A), _dp(lam), _dp(R))
    return lam, R


def propagate(prob: Problem, psi: np.ndarray, split: int, scheme: int, order: int,
              dt: float, nsteps: int, pruned: bool = True) -> np.ndarray:
    a = np.ascontiguousarray(psi, dtype=np.complex128).reshape(prob.shape).copy()
    rc = lib().orc_propagate(prob.ptr(), split, scheme, order, float(dt), int(nsteps),
                             int(pruned), _dp(a.view(np.float64)))
    if rc != 0:
        raise ValueError("oracle propagate rejected its arguments")
    return a


def propagate_gamma(prob: Problem, psi: np.ndarray, split: int, gamma, dt: float,
                    nsteps: int) -> np.ndarray:
    """nsteps steps of the composition S(gamma_M dt) ... S(gamma_1 dt) of Strang
    stages (Sec. "Symmetric composition schemes"), each applied unmerged."""
    a = np.ascontiguousarray(psi, dtype=np.complex128).reshape(prob.shape).copy()
    g = np.ascontiguousarray(gamma, dtype=np.float64).ravel()
    rc = lib().orc_propagate_gamma(prob.ptr(), split, g.size, _dp(g), float(dt), int(nsteps),
                                   _dp(a.view(np.float64)))
    if rc != 0:
        raise ValueError("oracle propagate_gamma rejected its arguments")
    return a


def interpolate(psi: np.ndarray, n_src, lo_src, hi_src, n_dst, lo_dst, hi_dst) -> np.ndarray:
    """Trigonometric interpolant of psi [S][grid] (grid n_src on [lo, hi) per
    axis) evaluated on the grid n_dst on [lo_dst, hi_dst); zero outside."""
    nd = len(n_src)
    a = np.ascontiguousarray(psi, dtype=np.complex128)
    S = a.shape[0]
    assert tuple(a.shape[1:]) == tuple(n_src)
    out = np.zeros((S, *n_dst), np.complex128)
    ns = np.ascontiguousarray(n_src, dtype=np.int32)
    nn = np.ascontiguousarray(n_dst, dtype=np.int32)
    f = [np.ascontiguousarray(v, dtype=np.float64) for v in (lo_src, hi_src, lo_dst, hi_dst)]
    rc = lib().orc_interpolate(nd, S, _ip(ns), _dp(f[0]), _dp(f[1]), _dp(a.view(np.float64)),
                               _ip(nn), _dp(f[2]), _dp(f[3]), _dp(out.view(np.float64)))
    if rc != 0:
        raise ValueError("oracle interpolate rejected its arguments")
    return out


def dense_hamiltonian_1d(n, lo, hi, nsurf, inv_mass, vtable, hbar=1.0) -> np.ndarray:
    """H = T (x) 1_S + V on an n-point 1D grid (Eq. diab_mol_ham with the
    Fourier grid of Sec. "Dynamic Fourier method"): T = F^-1 diag(T_k) F with
    F the DFT matrix, T_k = (hbar kappa_k)^2 inv_mass / 2, kappa_k = 2 pi k / L
    over the signed frequencies; V = the S x S blocks of point-wise diagonals.
    Rows and columns ordered [surface][point]."""
    n = int(n)
    L = float(hi) - float(lo)
    m = np.arange(n)
    F = np.exp(-2j * np.pi * np.outer(m, m) / n)
    ks = np.where(m <= n // 2, m, m - n).astype(float)
    Tk = (hbar * 2 * np.pi * ks / L) ** 2 * float(np.ravel(inv_mass)[0]) / 2
    T = (F.conj().T * Tk) @ F / n
    S = int(nsurf)
    vt = np.asarray(vtable, dtype=float).reshape(-1, n)
    H = np.kron(np.eye(S), T)
    pk = 0
    for i in range(S):
        for j in range(i, S):
            blk = np.diag(vt[pk])
            H[i * n:(i + 1) * n, j * n:(j + 1) * n] += blk
            if j != i:
                H[j * n:(j + 1) * n, i * n:(i + 1) * n] += blk
            pk += 1
    return H


def trapezoid_stage_maps(H: np.ndarray, gammas, dt: float, hbar: float = 1.0) -> dict:
    """The stage maps (1 + i tau H)^-1 (1 - i tau H) of the trapezoidal rule,
    tau = g dt / (2 hbar), one per distinct coefficient g, by dense direct
    solves."""
    eye = np.eye(H.shape[0])
    maps = {}
    for g in np.ravel(gammas):
        tau = float(g) * dt / (2 * hbar)
        if tau not in maps:
            maps[tau] = np.linalg.solve(eye + 1j * tau * H, eye - 1j * tau * H)
    return maps


def propagate_trapezoid(H: np.ndarray, psi: np.ndarray, gammas, dt: float, nsteps: int,
                        hbar: float = 1.0, per_stage: bool = False,
                        maps: dict | None = None) -> np.ndarray:
    """nsteps steps of the composition of the trapezoidal rule with the
    coefficients gammas: each stage solves (1 + i tau H) x = (1 - i tau H) psi,
    tau = g dt / (2 hbar), by a dense direct solve.  By default the stage
    maps are formed once per distinct tau (trapezoid_stage_maps, or `maps`
    when given); per_stage=True solves for the one right-hand side at every
    stage instead (the cheaper choice on large grids with few stages)."""
    shape = np.shape(psi)
    x = np.ascontiguousarray(psi, dtype=np.complex128).ravel().copy()
    if per_stage:
        eye = np.eye(H.shape[0])
        for _ in range(int(nsteps)):
            for g in np.ravel(gammas):
                tau = float(g) * dt / (2 * hbar)
                x = np.linalg.solve(eye + 1j * tau * H, x - 1j * tau * (H @ x))
        return x.reshape(shape)
    if maps is None:
        maps = trapezoid_stage_maps(H, gammas, dt, hbar)
    for _ in range(int(nsteps)):
        for g in np.ravel(gammas):
            x = maps[float(g) * dt / (2 * hbar)] @ x
    return x.reshape(shape)


def apply_hamiltonian(n, lo, hi, nsurf, inv_mass, vtable, u, hbar: float = 1.0) -> np.ndarray:
    """H u on a periodic grid of any dimension (Eq. diab_mol_ham with the
    Fourier grid of Sec. "Dynamic Fourier method"): the kinetic energy as
    sum_d F_d^-1 diag(T_d) F_d along each axis d (numpy's FFT), T_d(k) =
    (hbar kappa_k)^2 inv_mass_d / 2, kappa_k = 2 pi k / L_d over the signed
    frequencies (Nyquist as +n/2), plus the S x S matvec with the real
    symmetric V(x).  u: [S][n_0]..[n_{D-1}]."""
    n = [int(v) for v in n]
    S = int(nsurf)
    u = np.asarray(u, dtype=np.complex128).reshape(S, *n)
    out = np.zeros_like(u)
    for d in range(len(n)):
        L = float(hi[d]) - float(lo[d])
        m = np.arange(n[d])
        ks = np.where(m <= n[d] // 2, m, m - n[d]).astype(float)
        Tk = (hbar * 2 * np.pi * ks / L) ** 2 * float(inv_mass[d]) / 2
        shape = [1] * (len(n) + 1)
        shape[d + 1] = n[d]
        out += np.fft.ifft(Tk.reshape(shape) * np.fft.fft(u, axis=d + 1), axis=d + 1)
    vt = np.asarray(vtable, dtype=float).reshape(-1, *n)
    pk = 0
    for i in range(S):
        for j in range(i, S):
            out[i] += vt[pk] * u[j]
            if j != i:
                out[j] += vt[pk] * u[i]
            pk += 1
    return out


def propagate_trapezoid_krylov(n, lo, hi, nsurf, inv_mass, vtable, psi, gammas, dt: float,
                               nsteps: int, hbar: float = 1.0, tol: float = 1e-15) -> np.ndarray:
    """The trapezoidal-rule composition of propagate_trapezoid on grids too
    large for dense matrices: every stage solves (1 + i tau H) x =
    (1 - i tau H) psi, tau = g dt / (2 hbar), with H applied matrix-free
    (apply_hamiltonian) by restarted GMRES (scipy) to a relative residual
    tol, started from psi.  Since |1 + i tau lambda| >= 1 for real lambda,
    the error of x is at most the residual."""
    import scipy.sparse.linalg as sla
    shape = np.shape(psi)
    x = np.ascontiguousarray(psi, dtype=np.complex128).ravel().copy()
    N = x.size

    def H(u):
        return apply_hamiltonian(n, lo, hi, nsurf, inv_mass, vtable, u, hbar).ravel()

    for _ in range(int(nsteps)):
        for g in np.ravel(gammas):
            tau = float(g) * dt / (2 * hbar)
            A = sla.LinearOperator((N, N), matvec=lambda u, t=tau: u + 1j * t * H(u),
                                   dtype=np.complex128)
            b = x - 1j * tau * H(x)
            y, info = sla.gmres(A, b, x0=x, rtol=tol, atol=0.0, restart=60, maxiter=400)
            if info != 0:
                raise RuntimeError(f"oracle GMRES did not reach {tol} (info {info})")
            x = y
    return x.reshape(shape)


def set_threads(n: int) -> int:
    """Threads of the oracle's OpenMP loops; returns the count now in use."""
    if lib().orc_set_threads(int(n)) != 0:
        raise ValueError("thread count must be >= 1")
    return int(lib().orc_threads())


def propagate_timed(prob: Problem, psi: np.ndarray, split: int, scheme: int, order: int,
                    dt: float, nsteps: int):
    """Pruned propagation; returns (psi, seconds of the step loop, threads)."""
    a = np.ascontiguousarray(psi, dtype=np.complex128).reshape(prob.shape).copy()
    sec = np.zeros(1)
    rc = lib().orc_propagate_timed(prob.ptr(), split, scheme, order, float(dt), int(nsteps),
                                   _dp(a.view(np.float64)), _dp(sec))
    if rc != 0:
        raise ValueError("oracle propagate rejected its arguments")
    return a, float(sec[0]), int(lib().orc_threads())


def expm_frechet(V: np.ndarray, D: np.ndarray, tau: float, hbar: float = 1.0):
    """(exp(-i tau V/hbar), its Frechet derivative in direction D)."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    D = np.ascontiguousarray(D, dtype=np.float64)
    S = V.shape[0]
    U = np.zeros((S, S), np.complex128)
    L = np.zeros((S, S), np.complex128)
    lib().orc_expm_frechet(S, _dp(V), _dp(D), tau, hbar, _dp(U.view(np.float64)),
                           _dp(L.view(np.float64)))
    return U, L


def gradient(prob: Problem, dvtables: np.ndarray, psi0: np.ndarray, split: int, scheme: int,
             order: int, dt: float, nsteps: int, weights):
    """(populations at the end, sum_s w_s dP_s/dtheta_k) by tangent propagation."""
    dv = np.ascontiguousarray(dvtables, dtype=np.float64)
    npar = dv.shape[0]
    a = np.ascontiguousarray(psi0, dtype=np.complex128).reshape(prob.shape)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    pops = np.zeros(prob.nsurf)
    grad = np.zeros(max(npar, 1))
    rc = lib().orc_gradient(prob.ptr(), npar, _dp(dv), split, scheme, order, float(dt),
                            int(nsteps), _dp(a.view(np.float64)), _dp(w), _dp(pops), _dp(grad))
    if rc != 0:
        raise ValueError("oracle gradient rejected its arguments")
    return pops, grad[:npar]


def action(prob: Problem, psi: np.ndarray, op: str, tau: float) -> np.ndarray:
    a = np.ascontiguousarray(psi, dtype=np.complex128).reshape(prob.shape).copy()
    rc = lib().orc_action(prob.ptr(), 0 if op == "V" else 1, float(tau), _dp(a.view(np.float64)))
    if rc != 0:
        raise ValueError("oracle action rejected its arguments")
    return a


def observables(prob: Problem, psi: np.ndarray) -> dict:
    a = np.ascontiguousarray(psi, dtype=np.complex128).reshape(prob.shape)
    out = np.zeros(4 + prob.nsurf)
    if lib().orc_observables(prob.ptr(), _dp(a.view(np.float64)), _dp(out)) != 0:
        raise ValueError("oracle observables rejected its arguments")
    S = prob.nsurf
    return {"norm": out[0], "energy": out[1], "pops": out[2:2 + S].copy(),
            "kinetic": out[2 + S], "potential": out[3 + S]}


def overlap(prob: Problem, psi: np.ndarray, phi: np.ndarray) -> complex:
    a = np.ascontiguousarray(psi, dtype=np.complex128).reshape(prob.shape)
    b = np.ascontiguousarray(phi, dtype=np.complex128).reshape(prob.shape)
    out = np.zeros(2)
    lib().orc_overlap(prob.ptr(), _dp(a.view(np.float64)), _dp(b.view(np.float64)), _dp(out))
    return complex(out[0], out[1])


def propagate_driven(prob: Problem, dtable: np.ndarray, psi: np.ndarray, split: int,
                     scheme: int, order: int, dt: float, nsteps: int,
                     drive: np.ndarray) -> np.ndarray:
    """Pruned propagation with V(x, t) = V0 + s D: drive[n, v] is the value
    s for the v-th potential action of step n (shape [nsteps, nv])."""
    a = np.ascontiguousarray(psi, dtype=np.complex128).reshape(prob.shape).copy()
    d = np.ascontiguousarray(dtable, dtype=np.float64).reshape(-1)
    s = np.ascontiguousarray(drive, dtype=np.float64).reshape(-1)
    rc = lib().orc_propagate_driven(prob.ptr(), _dp(d), split, scheme, order, float(dt),
                                    int(nsteps), _dp(s), _dp(a.view(np.float64)))
    if rc != 0:
        raise ValueError("oracle driven propagation rejected its arguments")
    return a


def distance(prob: Problem, psi: np.ndarray, phi: np.ndarray) -> float:
    """||psi - phi|| with the volume element (the error norm of the paper's
    convergence studies)."""
    a = np.ascontiguousarray(psi, dtype=np.complex128).reshape(prob.shape)
    b = np.ascontiguousarray(phi, dtype=np.complex128).reshape(prob.shape)
    out = np.zeros(1)
    if lib().orc_distance(prob.ptr(), _dp(a.view(np.float64)), _dp(b.view(np.float64)),
                          _dp(out)) != 0:
        raise ValueError("oracle distance rejected its arguments")
    return float(out[0])


def exact(prob: Problem, psi: np.ndarray, t: float) -> np.ndarray:
    a = np.ascontiguousarray(psi, dtype=np.complex128).reshape(prob.shape).copy()
    if lib().orc_exact(prob.ptr(), float(t), _dp(a.view(np.float64))) != 0:
        raise ValueError("grid too large for the dense exact propagator")
    return a


def l2(prob: Problem, psi: np.ndarray) -> float:
    """L2 norm with the volume element."""
    dV = float(np.prod([(h - l) / n for n, l, h in zip(prob.n, prob.lo, prob.hi)]))
    return float(np.sqrt(np.sum(np.abs(psi) ** 2) * dV))
