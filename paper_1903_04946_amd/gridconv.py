"""Convergence with grid density (Appendix B), on the three-surface LVC model.

A family of cubic grids whose number of points per axis doubles from one
member to the next while the range and the density of the position grid --
and so of the momentum grid -- each grow by sqrt(2) per axis.  Every member
propagates the same initial state (the ground-state Gaussian on surface 3,
sampled on its own grid) with the same composition and step; states are
compared on the densest grid, reached from the sparser ones by trigonometric
interpolation (sop_interpolate).  Per member n, at the final time t_f:

  total error        ||I_{n->N} psi_n(t_f) - psi_N(t_f)||
  integration error  ||I_{n->N} I_{N->n} psi_N(t_f) - psi_N(t_f)||,
                     psi_N(t_f) represented on n's grid only after the
                     propagation (so the part of the error that the reduced
                     grid costs the representation and its overlap integrals)
  ratio              integration error / total error

and the initial error ||I_{n->N} psi_n(0) - psi_N(0)||; N is the densest
member, taken as converged.  Norms carry the volume element of the densest
grid.  Every step (propagation, interpolation, distance) runs in the HIP
library; this module only sequences the calls.
"""
from __future__ import annotations

import math

from . import soprop, synth


def box_half_width(n: int, n0: int = 64, half0: float = 7.0) -> float:
    """Half-width of the box [-L, L) of the n-point member: [-7, 7) (the
    paper's pyrazine box) at 64 points per axis, scaled by sqrt(2) per
    doubling of the points (so 32 points span [-4.95, 4.95), narrower than
    the packet's excursion, and 256 points [-14, 14))."""
    return half0 * math.sqrt(n / n0)


def grid_convergence(torch, ns=(32, 64, 128, 256), comp: str = "suzuki", order: int = 6,
                     t_final: float = 500.0, nsteps: int = 128, seed: int = 1903) -> dict:
    """Runs the study on the members ns (ascending; the last is the
    converged reference) with nsteps steps of size t_final / nsteps.
    Returns the per-member errors and the grids."""
    ns = sorted(ns)
    dt = t_final / nsteps
    members = {}
    for n in ns:
        L = box_half_width(n)
        m = synth.lvc_3d(n=n, seed=seed, lo=-L, hi=L)
        plan = soprop.Plan.from_model(m, comp=comp, order=order, dt=dt)
        psi0 = torch.from_numpy(m.psi0).cuda()
        psi = psi0.clone()
        plan.propagate(psi, nsteps)
        members[n] = (m, plan, psi0, psi)
    torch.cuda.synchronize()
    N = ns[-1]
    mN, pN, psi0N, psiN = members[N]
    up = torch.empty_like(psiN)
    back = torch.empty_like(psiN)
    rows = []
    for n in ns[:-1]:
        m, plan, psi0, psi = members[n]
        soprop.interpolate(plan, psi0, pN, up)
        e0 = pN.distance(up, psi0N)[0]
        soprop.interpolate(plan, psi, pN, up)
        tot = pN.distance(up, psiN)[0]
        down = torch.empty_like(psi)
        soprop.interpolate(pN, psiN, plan, down)
        soprop.interpolate(plan, down, pN, back)
        integ = pN.distance(back, psiN)[0]
        rows.append({"n": n, "npts": n**3, "box": [m.lo[0], m.hi[0]], "dx": m.dx[0],
                     "initial_error": e0, "total_error": tot, "integration_error": integ,
                     "ratio": integ / tot if tot > 0 else None,
                     "norm_final": plan.observables(psi)["norm"]})
    out = {"model": "LVC 3 modes x 3 surfaces (seed %d), psi0 = ground-state Gaussian on "
                    "surface 3" % seed,
           "scheme": f"{comp}-{order} VTV", "t_final": t_final, "nsteps": nsteps, "dt": dt,
           "reference": {"n": N, "box": [mN.lo[0], mN.hi[0]], "dx": mN.dx[0]},
           "members": rows}
    for _, plan, _, _ in members.values():
        plan.close()
    return out
