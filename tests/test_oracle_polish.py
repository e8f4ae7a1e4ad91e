"""Pins of the oracle's whole-matrix polish (oracle_cur_select_polish): the
swap loop on every column from the root's cross.  Checked against the
definition of a dominant cross (Sec. 1.1: no single row or column exchange
raises |det A(I,J)|), by numpy solves and by brute-force determinants, not
by the oracle's own arithmetic."""
import numpy as np
import pytest

from paper_2502_11017_amd import workloads as W
from tests.helpers import col_interp, rand, row_interp, single_swap_gain


def _logvol(A, I, J):
    return np.linalg.slogdet(A[np.ix_(I, J)])[1]


@pytest.mark.parametrize("shape,r,w,seed", [((120, 300), 6, 16, 1), ((200, 512), 16, 64, 2), ((64, 90), 5, 8, 3)])
def test_polish_is_dominant_over_all_columns(orc, shape, r, w, seed):
    m, n = shape
    A = rand(m, r + 4, seed) @ np.diag(0.7 ** np.arange(r + 4)) @ rand(r + 4, n, seed + 10) + 1e-3 * rand(m, n, seed + 20)
    base = orc.select(A, r, w=w)
    pol = orc.select(A, r, w=w, polish=True)
    assert base["status"] == 0 and pol["status"] == 0
    I, J = pol["I"], pol["J"]
    # dominance on the whole matrix, both directions
    assert np.abs(row_interp(A, I, J)).max() <= 1 + 1e-12
    assert np.abs(col_interp(A, I, J, np.arange(n))).max() <= 1 + 1e-12
    # the tree's cross was dominant over its root's candidates only; the
    # polish made further swaps, never lowering the volume; one node more
    assert np.abs(col_interp(A, base["I"], base["J"], np.arange(n))).max() > 1 + 1e-12
    assert pol["swaps"] > base["swaps"]
    assert _logvol(A, I, J) > _logvol(A, base["I"], base["J"])
    assert pol["nodes"] == base["nodes"] + 1
    assert abs(pol["logvol"] - _logvol(A, I, J)) <= 1e-12 * abs(pol["logvol"]) + 1e-12


def test_polish_brute_force_single_swaps(orc):
    # tiny: no single row swap and no single column swap over all columns
    # raises |det| (brute-force determinants)
    for seed in range(4):
        A = rand(9, 12, 700 + seed)
        for r in (1, 2, 3):
            pol = orc.select(A, r, w=max(r, 3), polish=True)
            assert pol["status"] == 0
            assert single_swap_gain(A, pol["I"], pol["J"], np.arange(12)) <= 1 + 1e-10


def test_polish_of_a_dominant_root_makes_no_swap(orc):
    # one leaf covering every column: the root is already dominant over all
    # columns, so the polish only confirms it
    A = W.c1(1).numpy()
    r = 16
    base = orc.select(A, r, w=A.shape[1], trace=True)
    pol = orc.select(A, r, w=A.shape[1], polish=True, trace=True)
    np.testing.assert_array_equal(base["I"], pol["I"])
    np.testing.assert_array_equal(base["J"], pol["J"])
    meta = pol["trace"]["meta"]
    assert len(meta) == len(base["trace"]["meta"]) + 1
    last = meta[-1]
    assert last[0] == base["trace"]["meta"][-1][0] + 1 and last[1] == 0  # level after the root, index 0
    assert last[6] == 0  # no swap


def test_polish_leaves_a_rank_short_root(orc):
    A = rand(40, 3, 5) @ rand(3, 60, 6)  # rank 3
    base = orc.select(A, 5, w=8, trace=True)
    pol = orc.select(A, 5, w=8, polish=True, trace=True)
    assert base["status"] == pol["status"] == orc.ERR_RANK
    np.testing.assert_array_equal(base["I"], pol["I"])
    assert pol["nodes"] == base["nodes"]
    # no polish record either
    np.testing.assert_array_equal(pol["trace"]["meta"], base["trace"]["meta"])


@pytest.mark.parametrize("shape,r,w,seed", [((150, 260), 8, 32, 31), ((300, 200), 12, 24, 32), ((64, 90), 5, 8, 33)])
def test_rect_polish_is_dominant_over_the_whole_matrix(orc, shape, r, w, seed):
    # the symmetric form of Alg. 2: I from the row tree, J from the column
    # tree, chosen apart; the polish makes the square cross dominant on all
    # of A (numpy solves over every row and column) and never lowers |det|
    m, n = shape
    A = rand(m, r + 5, seed) @ np.diag(0.6 ** np.arange(r + 5)) @ rand(r + 5, n, seed + 10) + 1e-3 * rand(m, n, seed + 20)
    base = orc.select_rect(A, r, r, w=w)
    pol = orc.select_rect(A, r, r, w=w, polish=True)
    assert base["status"] == pol["status"] == 0
    I, J = pol["I"], pol["J"]
    assert np.abs(row_interp(A, I, J)).max() <= 1 + 1e-12
    assert np.abs(col_interp(A, I, J, np.arange(n))).max() <= 1 + 1e-12
    assert _logvol(A, I, J) >= _logvol(A, base["I"], base["J"]) - 1e-12
    assert abs(pol["logvol"] - _logvol(A, I, J)) <= 1e-12 * abs(pol["logvol"]) + 1e-12
    assert list(I) == sorted(I) and list(J) == sorted(J)


def test_rect_polish_brute_force_single_swaps(orc):
    for seed in range(3):
        A = rand(10, 11, 800 + seed)
        for r in (1, 2, 3):
            pol = orc.select_rect(A, r, r, w=max(r, 3), polish=True)
            assert pol["status"] == 0
            assert single_swap_gain(A, pol["I"], pol["J"], np.arange(11)) <= 1 + 1e-10


def test_rect_polish_applies_to_square_crosses_only(orc):
    A = rand(80, 90, 41)
    a = orc.select_rect(A, 4, 6, w=8)
    b = orc.select_rect(A, 4, 6, w=8, polish=True)
    assert "polish" not in b
    np.testing.assert_array_equal(a["I"], b["I"])
    np.testing.assert_array_equal(a["J"], b["J"])
