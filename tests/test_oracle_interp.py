"""Pins of the oracle's trigonometric interpolation (Appendix B: states on
grids of different range and density are compared through the trigonometric
interpolant of the one on the sparser grid).

Independent references: closed forms of band-limited trigonometric
polynomials (interpolated exactly at any point), the Nyquist mode, the
identity on equal grids, and an analytic Gaussian wavepacket, which the
interpolant approaches exponentially fast with the number of samples (the
convergence Appendix B reports).
"""
import numpy as np
import pytest


def grid(n, lo, hi):
    return lo + np.arange(n) * ((hi - lo) / n)


def trig_poly(x, lo, hi, modes):
    L = hi - lo
    return sum(a * np.exp(2j * np.pi * k * (x - lo) / L) for k, a in modes)


@pytest.mark.parametrize("n", [16, 15])
def test_band_limited_polynomial_is_reproduced_anywhere(orc, n):
    lo, hi = -3.0, 5.0
    modes = [(-3, 0.7 - 0.2j), (0, 0.3), (2, -0.5j), (n // 2 - 1, 0.25 + 0.1j)]
    u = trig_poly(grid(n, lo, hi), lo, hi, modes)[None]
    lod, hid, nd = -4.0, 6.5, 37  # partly outside the source box
    got = orc.interpolate(u, [n], [lo], [hi], [nd], [lod], [hid])[0]
    x = grid(nd, lod, hid)
    inside = (x >= lo) & (x < hi)
    assert inside.sum() > 10 and (~inside).sum() > 3
    np.testing.assert_allclose(got[inside], trig_poly(x[inside], lo, hi, modes), rtol=0,
                               atol=1e-13)
    assert np.all(got[~inside] == 0)


def test_nyquist_mode_is_the_cosine(orc):
    n, lo, hi = 16, 0.0, 2.0
    u = ((-1.0) ** np.arange(n)).astype(complex)[None]
    nd, lod, hid = 50, 0.0, 2.0
    got = orc.interpolate(u, [n], [lo], [hi], [nd], [lod], [hid])[0]
    x = grid(nd, lod, hid)
    np.testing.assert_allclose(got, np.cos(np.pi * n * (x - lo) / (hi - lo)), rtol=0, atol=1e-14)


def test_equal_grids_are_the_identity(orc):
    rng = np.random.default_rng(5)
    for n in ([32], [8, 8, 8], [6, 5, 7]):
        u = rng.standard_normal((2, *n)) + 1j * rng.standard_normal((2, *n))
        lo, hi = [-1.0] * len(n), [2.0] * len(n)
        got = orc.interpolate(u, n, lo, hi, n, lo, hi)
        np.testing.assert_allclose(got, u, rtol=0, atol=1e-13)


def gaussian(x, x0=0.3, p0=1.5, sigma=1.0):
    return np.exp(-((x - x0) ** 2) / (4 * sigma**2) + 1j * p0 * x)


def test_gaussian_converges_exponentially(orc):
    """Range and density grow by sqrt(2) per doubling of the points, as in
    Appendix B; the interpolant on the finest grid approaches the analytic
    packet exponentially fast in the number of source points."""
    L0 = 8.0
    nd, Ld = 256, 8.0 * 2.0
    xd = grid(nd, -Ld, Ld)
    errs = []
    for n, L in [(16, L0 / 2**0.5), (32, L0), (64, L0 * 2**0.5)]:
        u = gaussian(grid(n, -L, L))[None]
        got = orc.interpolate(u, [n], [-L], [L], [nd], [-Ld], [Ld])[0]
        ref = np.where((xd >= -L) & (xd < L), gaussian(xd), 0)
        errs.append(np.max(np.abs(got - ref)))
    print("[interp gaussian] max errors", ["%.1e" % e for e in errs])
    assert errs[0] > 1e-4 and errs[1] < 1e-5 and errs[2] < 1e-12
    assert errs[1] < 1e-2 * errs[0] and errs[2] < 1e-4 * errs[1]


def test_axes_separate_in_3d(orc):
    n, lo, hi = [8, 8, 8], [-1.0, 0.0, 2.0], [1.0, 3.0, 4.0]
    modes = [[(1, 1.0), (-2, 0.3j)], [(0, 0.5), (3, -0.2)], [(-1, 0.4 + 0.1j), (2, 0.6)]]
    axes = [grid(n[a], lo[a], hi[a]) for a in range(3)]
    f = [trig_poly(axes[a], lo[a], hi[a], modes[a]) for a in range(3)]
    u = np.einsum("i,j,k->ijk", *f)[None]
    nd, lod, hid = [5, 11, 9], [-0.9, -0.5, 2.1], [1.3, 3.2, 3.9]
    got = orc.interpolate(u, n, lo, hi, nd, lod, hid)[0]
    ref = []
    for a in range(3):
        x = grid(nd[a], lod[a], hid[a])
        ref.append(np.where((x >= lo[a]) & (x < hi[a]), trig_poly(x, lo[a], hi[a], modes[a]), 0))
    np.testing.assert_allclose(got, np.einsum("i,j,k->ijk", *ref), rtol=0, atol=1e-13)
