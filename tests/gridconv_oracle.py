"""The grid-convergence study of Appendix B computed with the oracle alone
(its propagation and its trigonometric interpolation, distances in numpy),
for the parity test of the GPU study and for the oracle's own pins.  The
definitions are those of paper_1903_04946_amd.gridconv: states compared on
the densest grid, reached from the sparser ones by interpolation; total
error, integration error (the converged final state represented on the
sparser grid only after propagation, and back) and their ratio."""
import numpy as np


def dist(a, b, dV):
    return float(np.sqrt(np.sum(np.abs(a - b) ** 2) * dV))


def study(orc, models, split, scheme, order, dt, nsteps):
    """models: the members, ascending in grid size; the last is the
    reference.  Returns rows of (n, initial, total, integration, ratio)."""
    def prob(m):
        return orc.Problem(m.n, m.lo, m.hi, m.nsurf, m.inv_mass, m.vtable, m.hbar)

    finals = [orc.propagate(prob(m), m.psi0, split, scheme, order, dt, nsteps) for m in models]
    R, psiR = models[-1], finals[-1]

    def to_ref(m, psi):
        return orc.interpolate(psi, m.n, m.lo, m.hi, R.n, R.lo, R.hi)

    rows = []
    for m, psi in zip(models[:-1], finals[:-1]):
        e0 = dist(to_ref(m, m.psi0), R.psi0, R.dV)
        tot = dist(to_ref(m, psi), psiR, R.dV)
        down = orc.interpolate(psiR, R.n, R.lo, R.hi, m.n, m.lo, m.hi)
        integ = dist(to_ref(m, down), psiR, R.dV)
        rows.append({"n": m.n[0], "initial_error": e0, "total_error": tot,
                     "integration_error": integ, "ratio": integ / tot})
    return rows
