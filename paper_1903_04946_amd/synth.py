"""Seeded synthetic inputs: grids, diabatic potential tables and initial states.

This module holds input recipes only (model potentials evaluated on a grid,
Gaussian wavepackets, seeded parameter draws).  It contains none of the
propagation method's arithmetic, imports nothing else from this package and
is the one module both the HIP path's tests and the oracle's tests draw
inputs from.

The models stand in for the paper's NaI (1D, two surfaces) and pyrazine
(3 modes, three surfaces, box [-7, 7], Sec. "Three-dimensional model of
pyrazine") whose parameters are not reproduced here.  Atomic units, hbar = 1.

V-tables are real symmetric S x S matrices per grid point, stored as the
packed upper triangle (V00, V01, .., V0,S-1, V11, ..) in an array
[S(S+1)/2][npts] with the grid flattened C-order (last axis fastest).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

EV_PER_HARTREE = 27.211386245988


def packed_index(S: int, i: int, j: int) -> int:
    if i > j:
        i, j = j, i
    return i * S - (i * (i - 1)) // 2 + (j - i)


@dataclass
class Model:
    n: list            # points per axis
    lo: list
    hi: list
    nsurf: int
    inv_mass: list     # 1/m_d per axis
    vtable: np.ndarray  # [S(S+1)/2][npts] float64
    psi0: np.ndarray    # [S, *n] complex128
    hbar: float = 1.0
    dvtables: np.ndarray | None = None  # [nparams][S(S+1)/2][npts] (optional)
    meta: dict = field(default_factory=dict)

    @property
    def npts(self) -> int:
        return int(np.prod(self.n))

    @property
    def dx(self):
        return [(h - l) / n for n, l, h in zip(self.n, self.lo, self.hi)]

    @property
    def dV(self) -> float:
        return float(np.prod(self.dx))

    def axes(self):
        return [l + np.arange(n) * d for n, l, d in zip(self.n, self.lo, self.dx)]


def gaussian_1d(x: np.ndarray, x0: float, p0: float, sigma: float, hbar: float = 1.0):
    """(pi sigma^2)^(-1/4) exp(-(x-x0)^2/(2 sigma^2) + i p0 (x-x0)/hbar)."""
    return (np.pi * sigma**2) ** (-0.25) * np.exp(
        -((x - x0) ** 2) / (2 * sigma**2) + 1j * p0 * (x - x0) / hbar)


def normalise(psi: np.ndarray, dV: float) -> np.ndarray:
    return psi / np.sqrt(np.sum(np.abs(psi) ** 2) * dV)


# ----------------------------------------------------------------- 1D model
def two_surface_1d(n: int = 1024, lo: float = -10.0, hi: float = 10.0,
                   x0: float = -2.0, p0: float = 0.0,
                   sigma: float = 1.0 / np.sqrt(2.0), v22_cap: float | None = None) -> Model:
    """1D two-surface diabatic model with a Gaussian on surface 1.

    V11 = 0.5 (x+1)^2, V22 = 0.1 (1 - exp(-0.8 (x-1.5)))^2 + 0.3,
    V12 = 0.05 exp(-x^2/2); mass 1.  V22 reaches about 1e7 Ha at x = -10;
    v22_cap, if given, clips it there (min(V22, v22_cap)).
    """
    x = lo + np.arange(n) * ((hi - lo) / n)
    v11 = 0.5 * (x + 1.0) ** 2
    v22 = 0.1 * (1.0 - np.exp(-0.8 * (x - 1.5))) ** 2 + 0.3
    if v22_cap is not None:
        v22 = np.minimum(v22, v22_cap)
    v12 = 0.05 * np.exp(-x**2 / 2.0)
    vt = np.stack([v11, v12, v22]).astype(np.float64)
    psi = np.zeros((2, n), dtype=np.complex128)
    psi[0] = gaussian_1d(x, x0, p0, sigma)
    psi = normalise(psi, (hi - lo) / n)
    return Model([n], [lo], [hi], 2, [1.0], vt, psi,
                 meta={"name": "two_surface_1d", "x0": x0, "p0": p0, "sigma": sigma,
                       "v22_cap": v22_cap})


# ----------------------------------------------------------------- 3D LVC
def lvc_parameters(seed: int = 1903):
    """Linear vibronic coupling parameters (eV), drawn in the order omega[3],
    E[3], kappa[3][3] from numpy's PCG64 with the given seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    omega = rng.uniform(0.05, 0.15, size=3)
    energy = rng.uniform(0.0, 1.0, size=3)
    kappa = rng.uniform(-0.3, 0.3, size=(3, 3))  # kappa[s][mode]
    return omega, energy, kappa


def lvc_3d(n: int = 64, seed: int = 1903, lo: float = -7.0, hi: float = 7.0,
           couplings=None, dv_params=False, q0=(0.0, 0.0, 0.0), p0=(0.0, 0.0, 0.0)) -> Model:
    """Three-mode, three-surface linear vibronic coupling model.

    V_ss(q) = E_s + sum_k (omega_k q_k^2 / 2 + kappa_k^(s) q_k),
    V_st(q) = sum over couplings (s, t, mode, lambda) of lambda q_mode;
    T = sum_k omega_k p_k^2 / 2 (mass 1/omega_k).  Default couplings: one
    interstate coupling of 0.2 eV between surfaces 2 and 3 on mode 3.
    psi0 = the ground-state Gaussian (sigma = 1 per mode), on surface 3.
    With dv_params, the model carries dV/dtheta tables for the couplings
    theta = (lambda12 on mode 1, lambda13 on mode 2, lambda23 on mode 3)
    at (0.05, 0.05, 0.2) eV (derivatives per eV).
    """
    omega, energy, kappa = lvc_parameters(seed)
    if couplings is None:
        couplings = [(1, 2, 2, 0.2)]
        if dv_params:
            couplings = [(0, 1, 0, 0.05), (0, 2, 1, 0.05), (1, 2, 2, 0.2)]
    h = EV_PER_HARTREE
    ax = lo + np.arange(n) * ((hi - lo) / n)
    q = np.meshgrid(ax, ax, ax, indexing="ij")
    S = 3
    npts = n**3
    vt = np.zeros((6, npts))
    for s in range(S):
        v = np.full(q[0].shape, energy[s])
        for k in range(3):
            v = v + omega[k] * q[k] ** 2 / 2 + kappa[s, k] * q[k]
        vt[packed_index(S, s, s)] = (v / h).ravel()
    for (s, t, mode, lam) in couplings:
        vt[packed_index(S, s, t)] += (lam * q[mode] / h).ravel()
    psi = np.zeros((S, n, n, n), dtype=np.complex128)
    g = [gaussian_1d(ax, q0[k], p0[k], 1.0) for k in range(3)]
    psi[2] = g[0][:, None, None] * g[1][None, :, None] * g[2][None, None, :]
    dxv = ((hi - lo) / n) ** 3
    psi = normalise(psi, dxv)
    dv = None
    if dv_params:
        dv = np.zeros((len(couplings), 6, npts))
        for i, (s, t, mode, lam) in enumerate(couplings):
            dv[i, packed_index(S, s, t)] = (q[mode] / h).ravel()
    return Model([n, n, n], [lo] * 3, [hi] * 3, S, list(omega / h), vt, psi,
                 dvtables=dv,
                 meta={"name": "lvc_3d", "seed": seed, "omega_eV": omega.tolist(),
                       "E_eV": energy.tolist(), "kappa_eV": kappa.tolist(),
                       "couplings": couplings})


def lvc_vtable_theta(model: Model, theta) -> np.ndarray:
    """V-table at coupling parameters theta (eV): V0 with the couplings of
    ``dvtables`` replaced by theta (the model is linear in them)."""
    base = model.vtable.copy()
    cs = model.meta["couplings"]
    for i, (s, t, mode, lam) in enumerate(cs):
        base += (theta[i] - lam) * model.dvtables[i]
    return base


# ----------------------------------------------------------------- tiny cases
def random_small(n, nsurf, seed, lo=-4.0, hi=4.0, coupling=0.3):
    """Small random smooth model for brute-force comparisons (any ndim)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ndim = len(n)
    axes = [lo + np.arange(m) * ((hi - lo) / m) for m in n]
    q = np.meshgrid(*axes, indexing="ij")
    ne = nsurf * (nsurf + 1) // 2
    vt = np.zeros((ne, int(np.prod(n))))
    for s in range(nsurf):
        v = np.full(q[0].shape, rng.uniform(-0.5, 0.5))
        for k in range(ndim):
            c = rng.uniform(-0.5, 0.5)
            v = v + 0.5 * rng.uniform(0.2, 1.0) * (q[k] - c) ** 2
        vt[packed_index(nsurf, s, s)] = v.ravel()
    for s in range(nsurf):
        for t in range(s + 1, nsurf):
            c = rng.uniform(-1, 1, size=ndim)
            r2 = sum((q[k] - c[k]) ** 2 for k in range(ndim))
            vt[packed_index(nsurf, s, t)] = (coupling * rng.uniform(0.5, 1.0) *
                                             np.exp(-r2 / 2)).ravel()
    psi = np.zeros((nsurf, *n), dtype=np.complex128)
    g = np.ones(n, dtype=np.complex128)
    for k in range(ndim):
        shape = [1] * ndim
        shape[k] = n[k]
        g = g * gaussian_1d(axes[k], rng.uniform(-1, 1), rng.uniform(-1, 1), 1.0).reshape(shape)
    psi[0] = g
    dV = float(np.prod([(hi - lo) / m for m in n]))
    psi = normalise(psi, dV)
    return Model(list(n), [lo] * ndim, [hi] * ndim, nsurf,
                 list(rng.uniform(0.5, 1.5, size=ndim)), vt, psi,
                 meta={"name": "random_small", "seed": seed})


def random_state(shape, seed, dV=1.0) -> np.ndarray:
    """Random normalised complex state (for parity tests of single actions)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    psi = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return normalise(psi, dV)


# ----------------------------------------------------------------- compositions
# Coefficients handed to a custom symmetric composition, as inputs.
# Yoshida (1990), the sixth-order symmetric composition of seven Strang stages
# (his "solution A", 15 digits as published): (w3, w2, w1, w0, w1, w2, w3)
# with w0 = 1 - 2 (w1 + w2 + w3).
_YOSHIDA6_W = (-1.17767998417887, 0.235573213359357, 0.784513610477560)


def yoshida6_gammas() -> np.ndarray:
    w1, w2, w3 = _YOSHIDA6_W
    w0 = 1.0 - 2.0 * (w1 + w2 + w3)
    return np.array([w3, w2, w1, w0, w1, w2, w3])


def random_symmetric_gammas(M: int, seed: int, spread: float = 0.4) -> np.ndarray:
    """M coefficients, symmetric (g_j = g_{M+1-j}), summing to one, whose first
    (M+1)/2 values are distinct: uniform draws around 1/M, the middle one then
    set so that the sum is one."""
    rng = np.random.Generator(np.random.PCG64(seed))
    half = (M + 1) // 2
    g = np.empty(M)
    h = (1.0 + spread * rng.uniform(-1.0, 1.0, size=half)) / M
    g[:half] = h
    g[M - half:] = h[::-1]
    if M % 2:
        g[half - 1] = 1.0 - 2.0 * h[:half - 1].sum()
    else:
        g *= 1.0 / g.sum()
    return g


# ----------------------------------------------------------------- batches
def batch_manifest(count: int = 256, seed: int = 4946, t_final: float = 0.5):
    """Members of a batched ensemble: grid type, x0, p0, dt, order, scheme.

    Grid type uniform over {512, 1024, 2048, 4096, 8192 (1D, two surfaces),
    32^3, 48^3 (3D, three surfaces)}; x0 ~ U[-3, 3], p0 ~ U[-2, 2] (per mode
    in 3D); dt ~ U[0.005, 0.05], snapped so that every member reaches the
    same final time (nsteps * dt = t_final, so the step counts are uneven);
    order in {2, 4, 6, 8}; triple jump or Suzuki fractal for order >= 4.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    grids = [("1d", 512), ("1d", 1024), ("1d", 2048), ("1d", 4096), ("1d", 8192),
             ("3d", 32), ("3d", 48)]
    out = []
    for i in range(count):
        kind, n = grids[int(rng.integers(0, len(grids)))]
        ndim = 1 if kind == "1d" else 3
        x0 = rng.uniform(-3, 3, size=ndim)
        p0 = rng.uniform(-2, 2, size=ndim)
        dt = rng.uniform(0.005, 0.05)
        nsteps = int(np.ceil(t_final / dt))
        dt = t_final / nsteps
        order = int(rng.choice([2, 4, 6, 8]))
        scheme = "strang" if order == 2 else ("triple_jump" if rng.integers(0, 2) == 0 else "suzuki")
        out.append({"kind": kind, "n": n, "x0": x0.tolist(), "p0": p0.tolist(), "dt": dt,
                    "nsteps": nsteps, "order": order, "scheme": scheme})
    return out


def ensemble_model(entry) -> Model:
    """The model of one manifest entry: the 1D two-surface model with its
    packet at (x0, p0), or the 32^3 / 48^3 three-surface LVC model with the
    packet on surface 3 at (q0, p0)."""
    if entry["kind"] == "1d":
        return two_surface_1d(n=entry["n"], x0=entry["x0"][0], p0=entry["p0"][0])
    return lvc_3d(n=entry["n"], q0=tuple(entry["x0"]), p0=tuple(entry["p0"]))
