"""GPU parity of the whole-matrix polish (cur_opts.polish = 1) against the
oracle's oracle_cur_select_polish: after the tree, the swap loop once more
with every column a candidate, from the root's cross (Sec. 1.1's dominance
condition on all of A).  Index sets, statuses, counters and every trace
record must equal the oracle's exactly, as for the plain selection; the
volumes agree to the rounding of log.  Dominance over the whole matrix is
checked on the result with numpy solves, independently of both."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2502_11017_amd as cur  # noqa: E402
from paper_2502_11017_amd import workloads as W  # noqa: E402

from tests.helpers import col_interp, rand, row_interp  # noqa: E402

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def both(orc, A, r, w=0, tau=0.0, max_swaps=0):
    Ah = A.detach().cpu().numpy().astype(np.float64)
    say(f"polish case m={Ah.shape[0]} n={Ah.shape[1]} r={r} w={w} dtype={A.dtype}")
    g = cur.select(A, r, col_block=w, tau=tau, max_swaps=max_swaps, trace=True, polish=True)
    o = orc.select(Ah, r, w=w, tau=tau, max_swaps=max_swaps, trace=True, polish=True)
    return g, o, Ah


def same(g, o):
    assert g["status"] == o["status"], (g["status"], o["status"])
    assert g["rank"] == o["rank"]
    np.testing.assert_array_equal(g["I"].cpu().numpy(), o["I"])
    np.testing.assert_array_equal(g["J"].cpu().numpy(), o["J"])
    for key in ("nodes", "phases", "refreshes", "swaps"):
        assert g[key] == o[key], (key, g[key], o[key])
    gt, ot = g["trace"], o["trace"]
    assert len(gt["meta"]) == len(ot["meta"])
    np.testing.assert_array_equal(gt["meta"], ot["meta"])
    np.testing.assert_array_equal(gt["I"], ot["I"])
    np.testing.assert_array_equal(gt["J"], ot["J"])
    np.testing.assert_array_equal(gt["vol_m"], ot["vol_m"])
    if np.isfinite(o["logvol"]):
        assert abs(g["logvol"] - o["logvol"]) <= 1e-12 * max(1.0, abs(o["logvol"]))
    else:
        assert not np.isfinite(g["logvol"])


def dominant(Ah, I, J, tau=1e-13):
    n = Ah.shape[1]
    assert np.abs(row_interp(Ah, I, J)).max() <= 1 + tau + 1e-9
    assert np.abs(col_interp(Ah, I, J, np.arange(n))).max() <= 1 + tau + 1e-9


def lowrank(m, n, k, seed):
    A = rand(m, k, seed) @ np.diag(0.7 ** np.arange(k)) @ rand(k, n, seed + 10) + 1e-3 * rand(m, n, seed + 20)
    return torch.from_numpy(A).to(DEV)


# (m, n, r, w, seed): several leaves, ragged tails, candidate sets beyond the
# controller's LDS (r nc > 8192 doubles, nc > 4096 flags), r in each bucket
CASES = [
    (200, 512, 16, 64, 2),
    (513, 700, 16, 32, 3),
    (300, 1000, 5, 64, 4),
    (1000, 5000, 64, 64, 5),
    (600, 900, 100, 128, 6),
    (777, 129, 1, 0, 7),
]


@pytest.mark.parametrize("m,n,r,w,seed", CASES)
def test_polish_matches_oracle(orc, m, n, r, w, seed):
    A = torch.from_numpy(W.gaussian(m, n, seed)).to(DEV)
    g, o, Ah = both(orc, A, r, w)
    same(g, o)
    assert g["status"] == cur.OK
    dominant(Ah, g["I"].cpu().numpy(), g["J"].cpu().numpy())


def test_polish_low_rank_plus_noise(orc):
    # the tree's cross is not dominant over all columns here, so the polish swaps
    A = lowrank(200, 512, 20, 2)
    g, o, Ah = both(orc, A, 16, 64)
    same(g, o)
    base = cur.select(A, 16, col_block=64)
    assert g["swaps"] > base["swaps"] and g["nodes"] == base["nodes"] + 1
    assert g["logvol"] > base["logvol"]
    dominant(Ah, g["I"].cpu().numpy(), g["J"].cpu().numpy())


def test_polish_c2_recipe_small(orc):
    A = W.c2(31, device=DEV, n=2048)
    g, o, _ = both(orc, A, 64)
    same(g, o)


def test_polish_f32_input_matches_oracle_on_upcast(orc):
    A = torch.from_numpy(W.gaussian(300, 700, 8)).to(torch.float32).to(DEV)
    g, o, _ = both(orc, A, 8, 32)
    same(g, o)


def test_polish_single_leaf_root_is_already_dominant(orc):
    A = W.c1(1).to(DEV)
    g, o, _ = both(orc, A, 16, A.shape[1])
    same(g, o)
    assert g["trace"]["meta"][-1][6] == 0  # the polish record: no swap


def test_polish_rank_short_root_is_returned_as_is(orc):
    Ah = rand(40, 3, 5) @ rand(3, 60, 6)  # rank 3
    A = torch.from_numpy(Ah).to(DEV)
    g, o, _ = both(orc, A, 5, 8)
    same(g, o)
    assert g["status"] == cur.ERR_RANK
    base = cur.select(A, 5, col_block=8, trace=True)
    assert g["nodes"] == base["nodes"]
    np.testing.assert_array_equal(g["trace"]["meta"], base["trace"]["meta"])


def test_polish_with_a_swap_budget(orc):
    # the budget per node (max_swaps) also bounds the polish; both sides stop
    # at the same swap and report WARN_NOCONV alike
    A = lowrank(300, 800, 24, 9)
    g, o, _ = both(orc, A, 16, 32, max_swaps=3)
    same(g, o)


def test_polish_then_plain_selection_reuses_the_context(orc):
    # a polish call between two plain ones leaves the context's state intact
    A = torch.from_numpy(W.gaussian(400, 600, 10)).to(DEV)
    a = cur.select(A, 12, col_block=32)
    cur.select(A, 12, col_block=32, polish=True)
    b = cur.select(A, 12, col_block=32)
    np.testing.assert_array_equal(a["I"].cpu().numpy(), b["I"].cpu().numpy())
    np.testing.assert_array_equal(a["J"].cpu().numpy(), b["J"].cpu().numpy())


# the symmetric form of Alg. 2 (cur_select_rect, r == c) with the polish:
# I from the row tree, J from the column tree, then the swap loop on their
# cross over every column
RECT_CASES = [
    (300, 500, 12, 32, 21, torch.float64),
    (500, 300, 20, 40, 22, torch.float64),
    (400, 700, 8, 32, 23, torch.float32),
    (1000, 1500, 64, 64, 24, torch.float64),
    (600, 900, 100, 128, 25, torch.float64),
]


@pytest.mark.parametrize("m,n,r,w,seed,dt", RECT_CASES)
def test_rect_polish_matches_oracle(orc, m, n, r, w, seed, dt):
    A = torch.from_numpy(W.gaussian(m, n, seed)).to(dt).to(DEV)
    Ah = A.cpu().numpy().astype(np.float64)
    say(f"rect polish case m={m} n={n} r=c={r} w={w} dtype={dt}")
    g = cur.select_rect(A, r, r, col_block=w, polish=True)
    o = orc.select_rect(Ah, r, r, w=w, polish=True)
    assert g["status"] == o["status"] == cur.OK
    np.testing.assert_array_equal(g["I"].cpu().numpy(), o["I"])
    np.testing.assert_array_equal(g["J"].cpu().numpy(), o["J"])
    ps = o["polish"]
    assert g["nodes"] == o["rows"]["nodes"] + o["cols"]["nodes"] + 1
    for key in ("swaps", "phases", "refreshes"):
        assert g[key] == o["rows"][key] + o["cols"][key] + ps[key], key
    assert abs(g["logvol"] - o["logvol"]) <= 1e-12 * max(1.0, abs(o["logvol"]))
    dominant(Ah, o["I"], o["J"])


def test_rect_polish_skipped_on_a_rank_short_axis(orc):
    Ah = rand(40, 3, 7) @ rand(3, 60, 8)  # rank 3
    A = torch.from_numpy(Ah).to(DEV)
    g = cur.select_rect(A, 5, 5, col_block=8, polish=True)
    base = cur.select_rect(A, 5, 5, col_block=8)
    o = orc.select_rect(Ah, 5, 5, w=8, polish=True)
    assert g["status"] == base["status"] == o["status"] == cur.ERR_RANK
    assert "polish" not in o
    np.testing.assert_array_equal(g["I"].cpu().numpy(), base["I"].cpu().numpy())
    np.testing.assert_array_equal(g["J"].cpu().numpy(), base["J"].cpu().numpy())
    assert g["nodes"] == base["nodes"] and not np.isfinite(g["logvol"])


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_polish_of_a_padded_matrix(orc, dt):
    # lda > n: the polish's A^T panel is then a packed copy of A's rows
    # (with lda == n it is A itself); both selection paths must equal the
    # oracle on the packed matrix
    m, n, pad = 600, 900, 13
    Ah = W.gaussian(m, n, 44)
    big = torch.zeros((m, n + pad), dtype=dt, device=DEV)
    big[:, :n] = torch.from_numpy(Ah).to(dt).to(DEV)
    A = big[:, :n]
    assert A.stride(0) == n + pad
    Ap = A.contiguous().cpu().numpy().astype(np.float64)
    say(f"padded polish case m={m} n={n} lda={n + pad} dtype={dt}")
    g = cur.select(A, 16, col_block=64, polish=True, trace=True)
    o = orc.select(Ap, 16, w=64, polish=True, trace=True)
    same(g, o)
    g = cur.select_rect(A, 16, 16, col_block=64, polish=True)
    o = orc.select_rect(Ap, 16, 16, w=64, polish=True)
    assert g["status"] == o["status"]
    np.testing.assert_array_equal(g["I"].cpu().numpy(), o["I"])
    np.testing.assert_array_equal(g["J"].cpu().numpy(), o["J"])
    assert abs(g["logvol"] - o["logvol"]) <= 1e-12 * max(1.0, abs(o["logvol"]))


def test_batched_polish_equals_single_calls(orc):
    # one engine run for trees of different depths, shapes, dtypes and rank
    # buckets, each with its polish level (at different level indices), and a
    # rank-short item whose polish does nothing
    shapes = [(300, 500, 12, torch.float64), (700, 260, 20, torch.float64), (256, 1100, 8, torch.float32),
              (500, 700, 40, torch.float64), (640, 900, 70, torch.float64)]
    As = [torch.from_numpy(W.gaussian(m, n, 60 + k)).to(dt).to(DEV) for k, (m, n, r, dt) in enumerate(shapes)]
    rs = [r for (_, _, r, _) in shapes]
    As.append(torch.from_numpy(rand(50, 3, 61) @ rand(3, 80, 62)).to(DEV))  # rank 3
    rs.append(6)
    say(f"batched polish: {len(As)} items")
    outs, _ = cur.select_batched(As, rs, polish=True)
    for k, (A, r) in enumerate(zip(As, rs)):
        g = cur.select(A, r, polish=True)
        I, J, st = outs[k]
        assert st == g["status"], (k, st, g["status"])
        np.testing.assert_array_equal(I.cpu().numpy(), g["I"].cpu().numpy())
        np.testing.assert_array_equal(J.cpu().numpy(), g["J"].cpu().numpy())
        if k in (0, 2, 5):
            o = orc.select(A.cpu().numpy().astype(np.float64), r, polish=True)
            assert o["status"] == st
            np.testing.assert_array_equal(I.cpu().numpy()[:o["rank"]], o["I"][:o["rank"]])
