"""Pins of the oracle's tangent-mode population gradient.

* the Frechet derivative of exp(-i tau V) against scipy.linalg.expm_frechet
  (a library routine), for 2 x 2 and 3 x 3 real symmetric V;
* d P_s / d theta against central finite differences of the oracle's own
  propagator (a different computation: no derivative code involved);
* an x-independent two-level potential [[E1, theta], [theta, E2]]: kinetic
  and potential parts commute, every splitting is exact, and
  P_2(t) = theta^2 sin^2(Omega t) / Omega^2, Omega^2 = theta^2 + ((E1-E2)/2)^2
  (Rabi formula), whose derivative in theta is written out below;
* the norm is conserved, so sum_s dP_s/dtheta_k = 0.
"""
import numpy as np
import pytest
import scipy.linalg

from paper_1903_04946_amd import synth


def problem(orc, m, vt=None):
    return orc.Problem(m.n, m.lo, m.hi, m.nsurf, m.inv_mass, m.vtable if vt is None else vt, m.hbar)


@pytest.mark.parametrize("S", [2, 3])
@pytest.mark.parametrize("seed", range(3))
def test_frechet_vs_scipy(orc, S, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((S, S))
    V = (A + A.T) / 2
    B = rng.standard_normal((S, S))
    D = (B + B.T) / 2
    for tau in (0.3, -1.1, 7.0):
        U, L = orc.expm_frechet(V, D, tau)
        Us, Ls = scipy.linalg.expm_frechet(-1j * tau * V, -1j * tau * D)
        assert np.max(np.abs(U - Us)) < 1e-13
        assert np.max(np.abs(L - Ls)) < 1e-13 * max(1, abs(tau))


def small_lvc_params(n=8):
    m = synth.lvc_3d(n=n, dv_params=True, lo=-5, hi=5)
    return m


def test_gradient_vs_finite_differences_3d(orc):
    m = small_lvc_params(8)
    theta0 = np.array([c[3] for c in m.meta["couplings"]])
    w = np.array([0.0, 0.0, 1.0])
    P = problem(orc, m)
    pops, grad = orc.gradient(P, m.dvtables, m.psi0, orc.VTV, orc.TRIPLE_JUMP, 4, 40.0, 6, w)
    h = 1e-4
    for k in range(3):
        vals = {}
        for j in (-2, -1, 1, 2):
            th = theta0.copy()
            th[k] += j * h
            Pk = problem(orc, m, synth.lvc_vtable_theta(m, th))
            psi = orc.propagate(Pk, m.psi0, orc.VTV, orc.TRIPLE_JUMP, 4, 40.0, 6)
            vals[j] = orc.observables(Pk, psi)["pops"] @ w
        # fourth-order central difference
        fd = (-vals[2] + 8 * vals[1] - 8 * vals[-1] + vals[-2]) / (12 * h)
        assert abs(grad[k] - fd) < 1e-9 + 1e-8 * abs(fd), (k, grad[k], fd)
    # populations from the tangent run equal the plain propagation
    psi = orc.propagate(P, m.psi0, orc.VTV, orc.TRIPLE_JUMP, 4, 40.0, 6)
    np.testing.assert_allclose(pops, orc.observables(P, psi)["pops"], atol=1e-13)


def test_gradient_vs_finite_differences_1d(orc):
    m = synth.two_surface_1d(n=128)
    x = m.axes()[0]
    dv = np.zeros((1, 3, 128))
    dv[0, 1] = np.exp(-x**2 / 2)  # V12 = theta exp(-x^2/2)
    w = np.array([0.0, 1.0])
    P = problem(orc, m)
    _, grad = orc.gradient(P, dv, m.psi0, orc.VTV, orc.SUZUKI, 4, 0.05, 30, w)
    h = 1e-3
    vals = {}
    for j in (-2, -1, 1, 2):
        Pk = problem(orc, m, m.vtable + j * h * dv[0])
        psi = orc.propagate(Pk, m.psi0, orc.VTV, orc.SUZUKI, 4, 0.05, 30)
        vals[j] = orc.observables(Pk, psi)["pops"][1]
    fd = (-vals[2] + 8 * vals[1] - 8 * vals[-1] + vals[-2]) / (12 * h)
    assert abs(grad[0] - fd) < 1e-11 + 1e-8 * abs(fd), (grad[0], fd)


def test_rabi_closed_form(orc):
    n, lo, hi = 32, -6.0, 6.0
    E1, E2, th, t = 0.1, -0.25, 0.07, 9.0
    vt = np.zeros((3, n))
    vt[0], vt[1], vt[2] = E1, th, E2
    dv = np.zeros((1, 3, n))
    dv[0, 1] = 1.0
    x = lo + np.arange(n) * (hi - lo) / n
    psi0 = np.zeros((2, n), complex)
    psi0[0] = synth.gaussian_1d(x, 0.3, 0.5, 1.0)
    psi0 = synth.normalise(psi0, (hi - lo) / n)
    P = orc.Problem([n], [lo], [hi], 2, [1.0], vt)
    for split, scheme, order, nsteps in [(orc.VTV, 0, 2, 3), (orc.TVT, 1, 4, 2), (orc.VT, 0, 1, 5)]:
        pops, grad = orc.gradient(P, dv, psi0, split, scheme, order, t / nsteps, nsteps, [0.0, 1.0])
        d = (E1 - E2) / 2
        Om = np.sqrt(th**2 + d**2)
        s, c = np.sin(Om * t), np.cos(Om * t)
        p2 = th**2 * s**2 / Om**2
        dp2 = (2 * th * s**2 + th**2 * 2 * s * c * t * th / Om) / Om**2 - th**2 * s**2 * 2 * th / Om**4
        assert abs(pops[1] - p2) < 1e-13
        assert abs(grad[0] - dp2) < 1e-12


def test_norm_gradient_vanishes(orc):
    m = small_lvc_params(8)
    P = problem(orc, m)
    _, grad = orc.gradient(P, m.dvtables, m.psi0, orc.VTV, orc.SUZUKI, 4, 30.0, 4, [1.0, 1.0, 1.0])
    assert np.max(np.abs(grad)) < 1e-12
