"""Pins of the oracle's rectangular cross (r rows, c columns; Alg. 2 takes
the two counts separately, Sec. 1.1 defines U as the pseudo-inverse of
A(I,J)) against what linear algebra fixes independently of the code:
numpy's SVD-based pseudo-inverse and the four Moore-Penrose conditions, the
exact reproduction of a rank-k matrix by any cross whose intersection has
rank k, QR with column pivoting for the norm-greedy order, the brute-force
argmax for one row and one column, and the row/column symmetry of Alg. 2."""
import numpy as np
import pytest
import scipy.linalg

from oracle import oracle as orc


def _rank_k(m, n, k, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, k)) @ rng.standard_normal((k, n))


@pytest.mark.parametrize("p,q,rank", [(7, 4, 4), (4, 7, 4), (9, 9, 9), (6, 5, 2), (3, 8, 1)])
def test_pinv_rect_moore_penrose(p, q, rank):
    rng = np.random.default_rng(p * 10 + q)
    G = rng.standard_normal((p, rank)) @ rng.standard_normal((rank, q))
    P = orc.pinv_rect(G)
    assert P.shape == (q, p)
    scale = np.abs(np.linalg.pinv(G)).max()
    np.testing.assert_allclose(P, np.linalg.pinv(G), rtol=0, atol=1e-10 * scale)
    tol = 1e-10 * max(1.0, np.abs(G).max() * scale)
    assert np.abs(G @ P @ G - G).max() <= tol * np.abs(G).max()
    assert np.abs(P @ G @ P - P).max() <= tol * scale
    assert np.abs((G @ P) - (G @ P).T).max() <= tol
    assert np.abs((P @ G) - (P @ G).T).max() <= tol


def test_pinv_rect_square_is_the_square_pinv():
    G = np.random.default_rng(3).standard_normal((12, 12))
    np.testing.assert_array_equal(orc.pinv_rect(G), orc.pinv(G))


@pytest.mark.parametrize("r,c", [(7, 9), (9, 7), (5, 5), (12, 6)])
def test_rank_k_matrix_is_reproduced(r, c):
    """rank A = k and rank A(I,J) = k give A = C A(I,J)^+ R exactly, for any
    r, c >= k: the residual is rounding only."""
    A = _rank_k(60, 50, 5, 11)
    rng = np.random.default_rng(r * 100 + c)
    I = np.sort(rng.choice(60, r, replace=False))
    J = np.sort(rng.choice(50, c, replace=False))
    assert np.linalg.matrix_rank(A[np.ix_(I, J)]) == 5
    C, U, R = orc.assemble_rect(A, I, J)
    assert C.shape == (60, c) and U.shape == (c, r) and R.shape == (r, 50)
    np.testing.assert_array_equal(C, A[:, J])
    np.testing.assert_array_equal(R, A[I, :])
    cheb, fro = orc.residual_rect(A, C, U, R)
    amax = np.abs(A).max()
    assert cheb <= 1e-10 * amax and fro <= 1e-10
    # with U = 0 the residual is A itself
    cheb0, fro0 = orc.residual_rect(A, C, np.zeros_like(U), R)
    assert cheb0 == amax and fro0 == pytest.approx(1.0, rel=1e-15)


def test_rect_functions_equal_the_square_ones_when_r_equals_c():
    A = np.random.default_rng(4).standard_normal((40, 30))
    I = np.array([1, 5, 9, 20, 33])
    J = np.array([0, 3, 4, 17, 29])
    C, U, R = orc.assemble_rect(A, I, J)
    C2, U2, R2, _ = orc.assemble(A, I, J)
    np.testing.assert_array_equal(C, C2)
    np.testing.assert_array_equal(R, R2)
    assert orc.residual_rect(A, C, U2, R) == orc.residual(A, C2, U2, R2)


def test_greedy_rc_orders_are_qr_pivots():
    """The norm-greedy order on columns is the column order of QR with
    column pivoting (largest remaining norm, projected out), on rows that of
    A^T; the counts only cut the orders."""
    A = np.random.default_rng(5).standard_normal((30, 24))
    g = orc.greedy_rc(A, 6, 11)
    piv_c = scipy.linalg.qr(A, pivoting=True)[2]
    piv_r = scipy.linalg.qr(A.T, pivoting=True)[2]
    np.testing.assert_array_equal(g["order_J"], piv_c[:11])
    np.testing.assert_array_equal(g["order_I"], piv_r[:6])
    sq = orc.greedy(A, 6)
    np.testing.assert_array_equal(g["order_I"], sq["order_I"])
    np.testing.assert_array_equal(g["order_J"][:6], sq["order_J"])
    assert g["status"] == orc.OK and len(g["I"]) == 6 and len(g["J"]) == 11


@pytest.mark.parametrize("method", [0, 1])
def test_select_rect_one_row_one_column_is_the_largest_entry(method):
    """r = c = 1: the maximal-volume trees reduce to the argmax of |A|; the
    norm-greedy rule picks the row and the column of largest norm."""
    A = np.random.default_rng(6).standard_normal((70, 90))
    s = orc.select_rect(A, 1, 1, method=method)
    if method == 0:
        i, j = np.unravel_index(np.argmax(np.abs(A)), A.shape)
    else:
        i, j = np.argmax((A * A).sum(axis=1)), np.argmax((A * A).sum(axis=0))
    assert s["I"].tolist() == [i] and s["J"].tolist() == [j]


@pytest.mark.parametrize("method", [0, 1])
def test_select_rect_row_column_symmetry(method):
    """Alg. 2 chooses rows and columns by the same rule along each axis, so
    transposing A exchanges the two index sets (and the two counts)."""
    A = np.random.default_rng(7).standard_normal((150, 130))
    a = orc.select_rect(A, 9, 14, method=method)
    b = orc.select_rect(np.ascontiguousarray(A.T), 14, 9, method=method)
    np.testing.assert_array_equal(a["I"], b["J"])
    np.testing.assert_array_equal(a["J"], b["I"])
    assert len(a["I"]) == 9 and len(a["J"]) == 14 and a["status"] == orc.OK


def test_select_rect_rank_short_axis():
    """A rank-3 matrix: a count above 3 on either axis is rank-short."""
    A = _rank_k(80, 70, 3, 8)
    assert orc.select_rect(A, 3, 3)["status"] == orc.OK
    assert orc.select_rect(A, 3, 5)["status"] == orc.ERR_RANK
    assert orc.select_rect(A, 4, 3, method=1)["status"] == orc.ERR_RANK
