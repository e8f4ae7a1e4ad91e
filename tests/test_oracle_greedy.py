"""Pins of the oracle's norm-greedy selection (Alg. 2 with Alg. 3), CPU only.

The rule picks, r times, the vector of largest norm and projects it out of all
vectors (orthogonal projection): in exact arithmetic its choices are the
pivots of QR with column pivoting, which LAPACK computes independently (with
norm downdating rather than recomputation), so equal pivot sequences on
generic matrices pin the projection, the norm and the argmax.  Closed cases
pin the rest: r = 1, orthogonal vectors, exact low rank, and the invariances
of the rule.
"""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import oracle as orc


@pytest.mark.parametrize("seed", range(6))
def test_choice_order_is_the_qrcp_pivot_order(seed):
    rng = np.random.default_rng(100 + seed)
    A = rng.standard_normal((150 + 7 * seed, 110 + 5 * seed))
    r = 15
    g = orc.greedy(A, r)
    assert g["status"] == orc.OK
    np.testing.assert_array_equal(g["order_J"], sl.qr(A, pivoting=True, mode="r")[1][:r])
    np.testing.assert_array_equal(g["order_I"], sl.qr(A.T, pivoting=True, mode="r")[1][:r])
    np.testing.assert_array_equal(g["I"], np.sort(g["order_I"]))
    np.testing.assert_array_equal(g["J"], np.sort(g["order_J"]))


def test_r1_is_the_largest_row_and_column():
    A = np.random.default_rng(7).standard_normal((300, 200))
    g = orc.greedy(A, 1)
    assert g["order_J"][0] == np.argmax((A * A).sum(axis=0))
    assert g["order_I"][0] == np.argmax((A * A).sum(axis=1))


def test_orthogonal_columns_come_in_norm_order():
    # orthogonal vectors are unchanged by the projections: the order is by norm
    rng = np.random.default_rng(8)
    Q, _ = np.linalg.qr(rng.standard_normal((64, 40)))
    d = rng.permutation(np.arange(1, 41, dtype=np.float64))
    A = Q * d
    g = orc.greedy(A, 10)
    np.testing.assert_array_equal(g["order_J"], np.argsort(-d)[:10])


def test_exact_low_rank_stops_short():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((120, 5)) @ rng.standard_normal((5, 90))
    g = orc.greedy(A, 8)
    assert g["status"] == orc.ERR_RANK
    assert g["rank_rows"] == 5 and g["rank_cols"] == 5
    assert (g["I"][5:] == -1).all() and (g["J"][5:] == -1).all()
    # the five chosen columns span the column space
    C = A[:, g["J"][:5]]
    res = A - C @ np.linalg.lstsq(C, A, rcond=None)[0]
    assert np.abs(res).max() <= 1e-10 * np.abs(A).max()


def test_permutation_scaling_and_sign_invariance():
    rng = np.random.default_rng(10)
    A = rng.standard_normal((80, 70))
    g = orc.greedy(A, 9)
    pr, pc = rng.permutation(80), rng.permutation(70)
    gp = orc.greedy(A[pr][:, pc], 9)
    np.testing.assert_array_equal(pr[gp["order_I"]], g["order_I"])
    np.testing.assert_array_equal(pc[gp["order_J"]], g["order_J"])
    for B in (4.0 * A, -A, 0.125 * A):
        gb = orc.greedy(B, 9)
        np.testing.assert_array_equal(gb["order_I"], g["order_I"])
        np.testing.assert_array_equal(gb["order_J"], g["order_J"])
