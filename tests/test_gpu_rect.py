"""The rectangular cross on the GPU (Alg. 2 with a row count r and a column
count c, U = A(I,J)^+) through the C ABI, against the oracle:
- cur_select_rect: method 0 (the column-block maximal-volume tree on A for J,
  the same tree on A^T for I) equal to the oracle's index sets and status;
  method 1 (norm-greedy) equal at every step whose margin exceeds the
  rounding bound of the lane-strided sums (all steps of these matrices);
- cur_assemble_rect: C and R exact, U (one-sided Jacobi in the oracle's
  operation order) bit for bit;
- cur_residual_rect: within 1e-10 max|A| of the oracle's FP64 residual (the
  products are summed in another order on MFMA)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2502_11017_amd as cur  # noqa: E402
from paper_2502_11017_amd import workloads as W  # noqa: E402
from tests.helpers import greedy_first_near_tie  # noqa: E402

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = [
    # (m, n, r, c, seed, dtype): one rank bucket; two buckets (run one after the other);
    # r > c and r < c; ragged shapes; FP32 input (selected in FP64 on the exact upcast)
    (300, 260, 9, 14, 1, torch.float64),
    (513, 700, 20, 7, 2, torch.float64),
    (1000, 640, 16, 40, 3, torch.float64),
    (640, 1000, 40, 16, 4, torch.float32),
    (257, 257, 1, 5, 5, torch.float64),
]


def _matrix(m, n, seed, dt):
    """Decaying spectrum with noise (a unique maximal-volume path is not
    needed: the oracle runs the same steps)."""
    Ah = W.spectral(m, n, 0.8 ** np.arange(min(m, n)), seed, 1e-8, "cpu", torch.float64).numpy()
    return Ah, torch.from_numpy(Ah).to(dt).to(DEV)


@pytest.mark.parametrize("m,n,r,c,seed,dt", CASES)
def test_select_rect_maxvol_matches_oracle(orc, m, n, r, c, seed, dt):
    Ah, A = _matrix(m, n, seed, dt)
    say(f"case select_rect maxvol m={m} n={n} r={r} c={c} {dt}")
    g = cur.select_rect(A, r, c)
    o = orc.select_rect(A.cpu().numpy().astype(np.float64), r, c)
    assert g["status"] == o["status"]
    np.testing.assert_array_equal(g["I"].cpu().numpy(), o["I"])
    np.testing.assert_array_equal(g["J"].cpu().numpy(), o["J"])
    assert g["rank"] == min(o["rows"]["rank"], o["cols"]["rank"])
    assert g["swaps"] == o["rows"]["swaps"] + o["cols"]["swaps"]


@pytest.mark.parametrize("m,n,r,c,seed,dt", CASES)
def test_select_rect_greedy_matches_oracle(orc, m, n, r, c, seed, dt):
    A = torch.from_numpy(W.gaussian(m, n, 40 + seed)).to(dt).to(DEV)
    say(f"case select_rect greedy m={m} n={n} r={r} c={c} {dt}")
    g = cur.select_rect(A, r, c, method=cur.METHOD_GREEDY)
    o = orc.select_rect(A.cpu().numpy().astype(np.float64), r, c, method=1)["greedy"]
    for gaps, length, q in ((o["gap_I"], n, o["rank_rows"]), (o["gap_J"], m, o["rank_cols"])):
        assert greedy_first_near_tie(gaps, q, length) == q
    assert g["status"] == o["status"]
    np.testing.assert_array_equal(g["I"].cpu().numpy(), o["I"])
    np.testing.assert_array_equal(g["J"].cpu().numpy(), o["J"])


@pytest.mark.parametrize("m,n,r,c,seed,dt", CASES)
def test_assemble_and_residual_rect_match_oracle(orc, m, n, r, c, seed, dt):
    Ah, A = _matrix(m, n, seed, dt)
    say(f"case assemble/residual rect m={m} n={n} r={r} c={c} {dt}")
    g = cur.select_rect(A, r, c)
    C, U, R = cur.assemble_rect(A, g["I"], g["J"])
    A64 = A.cpu().numpy().astype(np.float64)
    oC, oU, oR = orc.assemble_rect(A64, g["I"].cpu().numpy(), g["J"].cpu().numpy())
    np.testing.assert_array_equal(C.cpu().numpy().astype(np.float64), oC)
    np.testing.assert_array_equal(R.cpu().numpy().astype(np.float64), oR)
    np.testing.assert_array_equal(U.cpu().numpy(), oU)
    cheb, fro = cur.residual_rect(A, C, U, R)
    ocheb, ofro = orc.residual_rect(A64, oC, oU, oR)
    amax = float(np.abs(A64).max())
    say(f"  cheb {cheb:.6e} oracle {ocheb:.6e} fro {fro:.6e} oracle {ofro:.6e}")
    assert abs(cheb - ocheb) <= 1e-10 * amax
    assert abs(fro - ofro) <= 1e-10 * max(1.0, ofro)


def test_rank_k_matrix_reproduced_on_the_gpu():
    """A rank-6 matrix and a cross of rank 6 (r = 10 rows, c = 8 columns):
    C A(I,J)^+ R reproduces A to rounding."""
    rng = np.random.default_rng(9)
    Ah = rng.standard_normal((400, 6)) @ rng.standard_normal((6, 300))
    A = torch.from_numpy(Ah).to(DEV)
    I = torch.from_numpy(np.sort(rng.choice(400, 10, replace=False))).to(DEV)
    J = torch.from_numpy(np.sort(rng.choice(300, 8, replace=False))).to(DEV)
    C, U, R = cur.assemble_rect(A, I, J)
    cheb, fro = cur.residual_rect(A, C, U, R)
    say(f"case rank-6 reproduction: cheb {cheb:.3e} fro {fro:.3e}")
    assert cheb <= 1e-10 * np.abs(Ah).max() and fro <= 1e-10


@pytest.mark.parametrize("method", [cur.METHOD_MAXVOL, cur.METHOD_GREEDY])
def test_transpose_exchanges_rows_and_columns(method):
    Ah, A = _matrix(420, 380, 12, torch.float64)
    a = cur.select_rect(A, 12, 24, method=method)
    b = cur.select_rect(A.t().contiguous(), 24, 12, method=method)
    np.testing.assert_array_equal(a["I"].cpu().numpy(), b["J"].cpu().numpy())
    np.testing.assert_array_equal(a["J"].cpu().numpy(), b["I"].cpu().numpy())


def test_square_rect_selection_columns_equal_square_selection(orc):
    """With r = c the column set is the square selection's (the same column
    tree); the row set comes from the row tree instead of the column tree's
    rows."""
    Ah, A = _matrix(500, 450, 13, torch.float64)
    g = cur.select_rect(A, 16, 16)
    s = cur.select(A, 16)
    np.testing.assert_array_equal(g["J"].cpu().numpy(), s["J"].cpu().numpy())
    t = cur.select(A.t().contiguous(), 16)
    np.testing.assert_array_equal(g["I"].cpu().numpy(), t["J"].cpu().numpy())
