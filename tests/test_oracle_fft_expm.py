"""Pins of the oracle's FFT and per-point potential exponential.

FFT: brute-force DFT sums in extended precision, numpy's FFT (a library
routine), round trip, Parseval, delta and plane-wave transforms.
Exponential (Sec. "Molecular Hamiltonian in the diabatic basis"): the 2 x 2
closed form (the case where one Jacobi rotation is exact), unitarity, the
group property U(t1) U(t2) = U(t1 + t2), U(t) U(-t) = 1, and scipy's expm
for 3 x 3 and 4 x 4.
"""
import numpy as np
import pytest
import scipy.linalg


def dft_brute(x, inverse=False):
    n = len(x)
    j = np.arange(n)
    out = np.zeros(n, dtype=np.clongdouble)
    sign = 1 if inverse else -1
    xl = np.asarray(x, dtype=np.clongdouble)
    for k in range(n):
        ang = sign * 2 * np.pi * np.longdouble(1) * ((j * k) % n) / n
        out[k] = np.sum(xl * (np.cos(ang.astype(np.longdouble)) + 1j * np.sin(ang.astype(np.longdouble))))
    if inverse:
        out /= n
    return out.astype(np.complex128)


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 48, 64, 12, 3])
def test_fft_vs_brute_force(orc, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for inv in (False, True):
        ref = dft_brute(x, inv)
        got = orc.fft(x, inv)
        assert np.max(np.abs(got - ref)) <= 1e-15 * max(1, n) * np.max(np.abs(ref)) * 4


@pytest.mark.parametrize("n", [128, 1024, 4096])
def test_fft_vs_numpy(orc, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    np.testing.assert_allclose(orc.fft(x), np.fft.fft(x), rtol=0, atol=1e-12 * np.sqrt(n))
    np.testing.assert_allclose(orc.fft(x, True), np.fft.ifft(x), rtol=0, atol=1e-14)
    y = orc.fft(orc.fft(x), True)
    assert np.max(np.abs(y - x)) < 1e-14 * np.log2(n)
    # Parseval
    X = orc.fft(x)
    assert abs(np.sum(np.abs(X) ** 2) / n - np.sum(np.abs(x) ** 2)) < 1e-12 * np.sum(np.abs(x) ** 2)


def test_fft_delta_and_plane_wave(orc):
    n = 64
    d = np.zeros(n, dtype=complex)
    d[0] = 1
    np.testing.assert_array_equal(orc.fft(d), np.ones(n))
    k0 = 5
    w = np.exp(2j * np.pi * k0 * np.arange(n) / n)
    W = orc.fft(w)
    ref = np.zeros(n)
    ref[k0] = n
    assert np.max(np.abs(W - ref)) < 1e-12


def closed_form_2x2(a, b, c, tau):
    # exp(-i tau V) for V = [[a, c], [c, b]]
    m = (a + b) / 2
    om = np.sqrt(((a - b) / 2) ** 2 + c**2)
    Vm = np.array([[a - m, c], [c, b - m]])
    s = np.sin(om * tau) / om if om > 0 else tau
    return np.exp(-1j * tau * m) * (np.cos(om * tau) * np.eye(2) - 1j * s * Vm)


@pytest.mark.parametrize("seed", range(6))
def test_expm_2x2_closed_form(orc, seed):
    rng = np.random.default_rng(seed)
    a, b, c = rng.uniform(-3, 3, 3)
    tau = rng.uniform(-2, 2)
    V = np.array([[a, c], [c, b]])
    U = orc.expm_potential(V, tau)
    np.testing.assert_allclose(U, closed_form_2x2(a, b, c, tau), rtol=0, atol=1e-14)
    np.testing.assert_allclose(U @ U.conj().T, np.eye(2), rtol=0, atol=1e-15 * 4)
    # complex symmetric: U = U^T for real symmetric V
    np.testing.assert_allclose(U, U.T, rtol=0, atol=1e-15)


def test_expm_2x2_large_phase(orc):
    # the steep wall of the 1D model: V ~ 1e7 with tau = 5e-3
    V = np.array([[40.5, 1e-20], [1e-20, 9.8e6]])
    U = orc.expm_potential(V, 5e-3)
    np.testing.assert_allclose(U, closed_form_2x2(40.5, 9.8e6, 1e-20, 5e-3), rtol=0, atol=1e-10)


@pytest.mark.parametrize("S", [3, 4])
@pytest.mark.parametrize("seed", range(4))
def test_expm_vs_scipy(orc, S, seed):
    rng = np.random.default_rng(100 + seed)
    A = rng.standard_normal((S, S))
    V = (A + A.T) / 2
    tau = rng.uniform(-1.5, 1.5)
    U = orc.expm_potential(V, tau)
    np.testing.assert_allclose(U, scipy.linalg.expm(-1j * tau * V), rtol=0, atol=1e-14)
    np.testing.assert_allclose(U @ U.conj().T, np.eye(S), rtol=0, atol=1e-14)
    U2 = orc.expm_potential(V, 0.7)
    U3 = orc.expm_potential(V, tau + 0.7)
    np.testing.assert_allclose(U @ U2, U3, rtol=0, atol=1e-14)
    np.testing.assert_allclose(U @ orc.expm_potential(V, -tau), np.eye(S), rtol=0, atol=1e-14)


def test_expm_hbar(orc):
    V = np.array([[1.0, 0.3], [0.3, -0.5]])
    np.testing.assert_allclose(orc.expm_potential(V, 0.8, hbar=2.0),
                               scipy.linalg.expm(-1j * 0.4 * V), atol=1e-14)


@pytest.mark.parametrize("n", [2, 3, 7, 20])
def test_jacobi_eigh_vs_numpy(orc, n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    A = A + A.T
    lam, R = orc.eigh(A)
    np.testing.assert_allclose(np.sort(lam), np.linalg.eigvalsh(A), atol=1e-13 * n)
    np.testing.assert_allclose(R @ np.diag(lam) @ R.T, A, atol=1e-13 * n)
    np.testing.assert_allclose(R.T @ R, np.eye(n), atol=1e-14 * n)


def test_jacobi_degenerate(orc):
    # constant diagonal (already diagonal, degenerate)
    lam, R = orc.eigh(np.eye(3) * 2.0)
    np.testing.assert_array_equal(lam, [2, 2, 2])
    np.testing.assert_array_equal(R, np.eye(3))
