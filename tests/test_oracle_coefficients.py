"""Pins of the oracle's composition, splitting, pruning and dedupe.

Each expectation comes from the paper's printed formulas or table, or from a
mathematical identity, not from the oracle itself:
  * Eq. triple_jump_fourth_order_so / Eq. suzukis_fractals_fourth_order_so
    (the fourth-order coefficients, closed form);
  * Eq. symmetric_splitting_coefficients (a_{N-j+1} = a_j, b_{N-j} = b_j);
  * the sum rules sum a = sum b = 1 (Sec. "Compositions of split-operator
    algorithms") and sum gamma = 1 (Sec. "Symmetric composition schemes");
  * Table II counts (tests/golden/table2_counts.txt);
  * the order conditions of the recursive construction: every level that
    raises p -> p+2 has sum c^(p+1) = 0, so the flattened coefficient list
    has sum gamma^q = 0 for q = 3, 5, ..., order-1.
"""
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_counts.txt")
SCHEME = {"strang": 0, "tj": 1, "sf": 2}


def table2_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        s, o, before, after, na, nb = line.split()
        rows.append((s, int(o), int(before), int(after), int(na), int(nb)))
    return rows


def test_triple_jump_fourth_order_closed_form(orc):
    c = 2.0 ** (1.0 / 3.0)
    g1 = 1.0 / (2.0 - c)
    a, b = orc.splitting(orc.VTV, orc.TRIPLE_JUMP, 4, pruned=False)
    assert len(a) == 6
    # a1 = a2 = 1/(2(2-2^{1/3})), a3 = -2^{1/3}/(2(2-2^{1/3}))
    np.testing.assert_allclose(a[0], 1.0 / (2 * (2 - c)), rtol=1e-15)
    np.testing.assert_allclose(a[1], 1.0 / (2 * (2 - c)), rtol=1e-15)
    np.testing.assert_allclose(a[2], -c / (2 * (2 - c)), rtol=1e-15)
    # b1 = 1/(2-2^{1/3}), b3 = -2^{1/3}/(2-2^{1/3}), b2 = b6 = 0
    np.testing.assert_allclose(b[0], g1, rtol=1e-15)
    np.testing.assert_allclose(b[2], -c / (2 - c), rtol=1e-15)
    assert b[1] == 0.0 and b[5] == 0.0
    # remaining by symmetry
    N = 6
    for j in range(1, N + 1):
        assert a[N - j] == pytest.approx(a[j - 1], rel=1e-15)
    for j in range(1, N):
        assert b[N - j - 1] == pytest.approx(b[j - 1], rel=1e-15, abs=0)


def test_suzuki_fourth_order_closed_form(orc):
    c = 4.0 ** (1.0 / 3.0)
    a, b = orc.splitting(orc.VTV, orc.SUZUKI, 4, pruned=False)
    assert len(a) == 10
    for j in range(4):
        np.testing.assert_allclose(a[j], 1.0 / (2 * (4 - c)), rtol=1e-15)
    np.testing.assert_allclose(a[4], -c / (2 * (4 - c)), rtol=1e-15)
    np.testing.assert_allclose(b[0], 1.0 / (4 - c), rtol=1e-15)
    np.testing.assert_allclose(b[2], 1.0 / (4 - c), rtol=1e-15)
    np.testing.assert_allclose(b[4], -c / (4 - c), rtol=1e-15)
    assert b[1] == 0.0 and b[3] == 0.0 and b[9] == 0.0
    N = 10
    for j in range(1, N + 1):
        assert a[N - j] == pytest.approx(a[j - 1], rel=1e-15)
    for j in range(1, N):
        assert b[N - j - 1] == pytest.approx(b[j - 1], rel=1e-15, abs=0)


@pytest.mark.parametrize("row", table2_rows(), ids=lambda r: f"{r[0]}{r[1]}")
def test_table2_counts(orc, row):
    scheme, order, before, after, na, nb = row
    a, b = orc.splitting(orc.VTV, SCHEME[scheme], order, pruned=False)
    assert len(a) + np.count_nonzero(b) == before
    ap, bp = orc.splitting(orc.VTV, SCHEME[scheme], order, pruned=True)
    assert len(ap) + np.count_nonzero(bp) == after
    # footnotes of Table II: N_A = 2 N_B before, N_A = N_B + 1 after the merge
    assert len(a) == 2 * np.count_nonzero(b)
    assert len(ap) == np.count_nonzero(bp) + 1
    au, bu, ia, ib = orc.unique(orc.VTV, SCHEME[scheme], order)
    assert (len(au), len(bu)) == (na, nb)
    # index arrays reproduce the pruned sequence (Eq. range_index_unq)
    np.testing.assert_array_equal(au[ia], ap)
    nz = bp != 0
    np.testing.assert_array_equal(bu[ib[nz]], bp[nz])
    assert np.all(ib[~nz] == -1)
    assert ia.min() >= 0 and ia.max() < na


def test_first_order_counts(orc):
    # Table II, elementary order 1: 2 actions, 1 + 1 unique
    for split in (orc.VT, orc.TV):
        a, b = orc.splitting(split, 0, 1, pruned=True)
        assert list(a) == [1.0] and list(b) == [1.0]


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("order", [2, 4, 6, 8, 10])
def test_sum_rules_and_symmetry(orc, scheme, order):
    g = orc.gammas(scheme, order)
    # each gamma is rounded once from extended precision: the exact sum of
    # the rounded values is within sum|gamma| * 2^-53 of 1
    bound = np.sum(np.abs(g)) * 2.0**-53 + 1e-16
    assert abs(math.fsum(g) - 1.0) <= bound
    np.testing.assert_array_equal(g, g[::-1])  # palindromic
    for pruned in (False, True):
        a, b = orc.splitting(orc.VTV, scheme, order, pruned)
        bound = np.sum(np.abs(g)) * 2.0**-52 + 1e-16
        assert abs(math.fsum(a) - 1.0) <= bound
        assert abs(math.fsum(b) - 1.0) <= bound
        N = len(a)
        # Eq. symmetric_splitting_coefficients
        for j in range(1, N + 1):
            assert a[N - j] == pytest.approx(a[j - 1], rel=1e-14, abs=1e-300)
        for j in range(1, N):
            assert b[N - j - 1] == pytest.approx(b[j - 1], rel=1e-14, abs=1e-300)


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("order", [4, 6, 8, 10])
def test_order_conditions(orc, scheme, order):
    g = np.array(orc.gammas(scheme, order), dtype=np.longdouble)
    for q in range(3, order, 2):
        s = np.sum(g**q)
        assert abs(float(s)) < 1e-12 * float(np.sum(np.abs(g) ** q)) + 1e-14, (q, s)
    # the next odd power does not vanish (the order is not higher)
    q = order + 1
    assert abs(float(np.sum(g**q))) > 1e-3 * float(np.sum(np.abs(g) ** q))


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("order", [4, 6, 8])
def test_pruned_is_merged_unpruned(orc, scheme, order):
    # Eq. merging_splitting_coeff_b_zero: each zero b_j (j != N) merges
    # a_j + a_{j+1}; the pruned a's are sums of consecutive unpruned pairs.
    a, b = orc.splitting(orc.VTV, scheme, order, False)
    ap, bp = orc.splitting(orc.VTV, scheme, order, True)
    M = len(a) // 2
    assert len(ap) == M + 1
    np.testing.assert_allclose(ap[0], a[0], rtol=1e-15)
    np.testing.assert_allclose(ap[-1], a[-1], rtol=1e-15)
    for j in range(1, M):
        np.testing.assert_allclose(ap[j], a[2 * j - 1] + a[2 * j], rtol=1e-14, atol=1e-15)
    np.testing.assert_array_equal(bp[:M], b[0::2])
    assert bp[M] == 0.0


def test_invalid_inputs(orc):
    with pytest.raises(ValueError):
        orc.gammas(1, 3)
    with pytest.raises(ValueError):
        orc.gammas(0, 4)
    with pytest.raises(ValueError):
        orc.splitting(orc.VT, 0, 2, True)
