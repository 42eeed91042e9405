"""Pins of the oracle's propagation by a composition with given coefficients
(Sec. "Symmetric composition schemes"; the paper's "optimal" schemes are
compositions of this kind whose coefficients it does not print).

Independent references: the exact evolution by scipy.linalg.expm of the
dense discrete Hamiltonian, Yoshida's published sixth-order coefficients
(their order is what the mathematics fixes: global error O(dt^6)), and
special cases that reduce to the built-in schemes.
"""
import numpy as np
import pytest

from paper_1903_04946_amd import synth
from test_oracle_propagator import exact_scipy, fitted_slope, l2, problem


def _model():
    return synth.random_small([16], 2, seed=3, lo=-5, hi=5, coupling=0.5)


def test_yoshida6_coefficients_satisfy_moment_conditions():
    g = synth.yoshida6_gammas()
    assert np.allclose(g, g[::-1], rtol=0, atol=0)
    assert abs(g.sum() - 1) < 1e-15
    # sums of odd powers vanish for a symmetric order-6 composition of a
    # symmetric second-order method (orders 3 and 5 of the error expansion)
    assert abs(np.sum(g**3)) < 1e-13
    assert abs(np.sum(g**5)) < 1e-12


@pytest.mark.parametrize("split", ["VTV", "TVT"])
def test_yoshida6_converges_at_order_6(orc, split):
    m = _model()
    P = problem(orc, m)
    tf = 4.0
    ref = exact_scipy(m, m.psi0, tf)
    g = synth.yoshida6_gammas()
    dts, errs = [], []
    for k in range(2, 7):
        ns = int(round(tf / (2.0 / 2**k)))
        dts.append(tf / ns)
        errs.append(l2(m, orc.propagate_gamma(P, m.psi0, getattr(orc, split), g, tf / ns, ns)
                       - ref))
    slope = fitted_slope(dts, errs)
    print(f"[yoshida6 {split}] errors {['%.1e' % e for e in errs]}, slope {slope:.2f}")
    assert abs(slope - 6) < 0.5, errs


def test_generic_symmetric_gammas_are_second_order(orc):
    m = _model()
    P = problem(orc, m)
    tf = 4.0
    ref = exact_scipy(m, m.psi0, tf)
    g = synth.random_symmetric_gammas(5, seed=2)
    assert abs(np.sum(g**3)) > 1e-3  # no fourth-order cancellation
    dts, errs = [], []
    for k in range(3, 8):
        ns = 2**k
        dts.append(tf / ns)
        errs.append(l2(m, orc.propagate_gamma(P, m.psi0, orc.VTV, g, tf / ns, ns) - ref))
    assert abs(fitted_slope(dts, errs) - 2) < 0.35, errs


def test_half_stages_equal_strang_at_half_step(orc):
    m = _model()
    P = problem(orc, m)
    a = orc.propagate_gamma(P, m.psi0, orc.VTV, [0.5, 0.5], 0.3, 7)
    b = orc.propagate(P, m.psi0, orc.VTV, 0, 2, 0.15, 14, pruned=False)
    assert l2(m, a - b) < 1e-14


@pytest.mark.parametrize("scheme,order", [(1, 4), (2, 4), (1, 6)])
def test_builtin_gammas_given_as_custom(orc, scheme, order):
    """The recursive schemes' coefficients given as a custom list reproduce
    the built-in schemes (here against their pruned, merged sequence)."""
    m = _model()
    P = problem(orc, m)
    g = orc.gammas(scheme, order)
    a = orc.propagate_gamma(P, m.psi0, orc.TVT, g, 0.2, 5)
    b = orc.propagate(P, m.psi0, orc.TVT, scheme, order, 0.2, 5, pruned=True)
    assert l2(m, a - b) < 1e-13
