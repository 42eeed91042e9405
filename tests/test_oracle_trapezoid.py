"""Pins of the oracle's compositions of the trapezoidal rule (the implicit,
energy-conserving comparison integrator; for a linear equation it is the
implicit midpoint rule too).

Independent references: the exact evolution by scipy.linalg.expm of the
dense Hamiltonian built with numpy's FFT (a second construction of H), the
free particle's closed form per momentum, (1 - i tau T_k)/(1 + i tau T_k),
and the properties the mathematics fixes: unitarity, conservation of <H>,
time reversibility, and global errors O(dt^2) for the rule and O(dt^4) for
its triple-jump composition.
"""
import numpy as np
import pytest

from paper_1903_04946_amd import synth
from test_oracle_propagator import dense_h, exact_scipy, fitted_slope, l2


def H_of(orc, m):
    return orc.dense_hamiltonian_1d(m.n[0], m.lo[0], m.hi[0], m.nsurf, m.inv_mass, m.vtable,
                                    m.hbar)


def test_dense_h_agrees_with_fft_construction(orc):
    m = synth.random_small([24], 2, seed=3, lo=-5, hi=5, coupling=0.5)
    np.testing.assert_allclose(H_of(orc, m), dense_h(m), rtol=0, atol=1e-10)


def test_free_particle_closed_form(orc):
    m = synth.random_small([32], 1, seed=2, lo=-6, hi=6)
    m.vtable[:] = 0
    H = H_of(orc, m)
    dt = 0.37
    got = orc.propagate_trapezoid(H, m.psi0, [1.0], dt, 3, m.hbar)
    k = 2 * np.pi * np.fft.fftfreq(32, d=m.dx[0]) * m.hbar
    Tk = 0.5 * m.inv_mass[0] * k**2
    tau = dt / (2 * m.hbar)
    ref = np.fft.ifft(((1 - 1j * tau * Tk) / (1 + 1j * tau * Tk)) ** 3 * np.fft.fft(m.psi0[0]))
    np.testing.assert_allclose(got[0], ref, rtol=0, atol=1e-13)


def test_unitary_energy_conserving_reversible(orc):
    m = synth.random_small([32], 2, seed=3, lo=-5, hi=5, coupling=0.5)
    H = H_of(orc, m)
    g = orc.gammas(1, 4)
    psi = orc.propagate_trapezoid(H, m.psi0, g, 0.3, 7, m.hbar)
    n0 = np.vdot(m.psi0.ravel(), m.psi0.ravel()).real
    assert abs(np.vdot(psi.ravel(), psi.ravel()).real / n0 - 1) < 1e-13
    e0 = np.vdot(m.psi0.ravel(), H @ m.psi0.ravel()).real
    e1 = np.vdot(psi.ravel(), H @ psi.ravel()).real
    assert abs(e1 - e0) < 1e-12 * abs(e0)
    back = orc.propagate_trapezoid(H, psi, g, -0.3, 7, m.hbar)
    assert l2(m, back - m.psi0) < 1e-12


@pytest.mark.parametrize("scheme,order,ks", [(0, 2, range(5, 10)), (1, 4, range(7, 11))])
def test_orders_against_exact(orc, scheme, order, ks):
    m = synth.random_small([16], 2, seed=3, lo=-5, hi=5, coupling=0.5)
    H = H_of(orc, m)
    tf = 4.0
    ref = exact_scipy(m, m.psi0, tf)
    g = orc.gammas(scheme, order)
    dts, errs = [], []
    for k in ks:
        ns = 2**k
        dts.append(tf / ns)
        errs.append(l2(m, orc.propagate_trapezoid(H, m.psi0, g, tf / ns, ns, m.hbar) - ref))
    slope = fitted_slope(dts, errs)
    print(f"[trapezoid order {order}] errors {['%.1e' % e for e in errs]}, slope {slope:.2f}")
    assert abs(slope - order) < 0.35, errs
