"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle.

Selection: index sets, statuses and every per-node counter of the selection
tree must equal the oracle's exactly; the volumes agree to rounding of log.
FP32 input is widened exactly and the selection computes in FP64, so it must
equal the oracle's selection of the upcast matrix in the same way.
Assembly: C and R are gathers (bit-exact); U is bit-exact when the LU inverse
is used.  Residual: |cheb_gpu - cheb_oracle| <= 1e-10 ||A||_C and the same
bound for the Frobenius relative error (rounding of an r-term dot product with
|B| <= 1 is ~ r eps ||A||_C, far below it).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2502_11017_amd as cur  # noqa: E402
from paper_2502_11017_amd import workloads as W  # noqa: E402
import os  # noqa: E402

from tests.helpers import check_tree_golden, greedy_first_near_tie, read_tree_golden, row_interp  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_both(orc, A, r, w=0, tau=0.0, max_swaps=0):
    Ah = A.detach().cpu().numpy()
    say(f"case m={Ah.shape[0]} n={Ah.shape[1]} r={r} w={w} dtype={A.dtype}")
    g = cur.select(A, r, col_block=w, tau=tau, max_swaps=max_swaps, trace=True)
    o = orc.select(Ah, r, w=w, tau=tau, max_swaps=max_swaps, trace=True)
    return g, o, Ah


def assert_same_selection(g, o):
    gI, gJ = g["I"].cpu().numpy(), g["J"].cpu().numpy()
    assert g["status"] == o["status"], (g["status"], o["status"])
    assert g["rank"] == o["rank"]
    np.testing.assert_array_equal(gI, o["I"])
    np.testing.assert_array_equal(gJ, o["J"])
    for key in ("nodes", "phases", "refreshes", "swaps"):
        assert g[key] == o[key], (key, g[key], o[key])
    gt, ot = g["trace"], o["trace"]
    np.testing.assert_array_equal(gt["meta"], ot["meta"])
    np.testing.assert_array_equal(gt["I"], ot["I"])
    np.testing.assert_array_equal(gt["J"], ot["J"])
    np.testing.assert_array_equal(gt["vol_m"], ot["vol_m"])  # same rounded products
    if np.isfinite(o["logvol"]):
        assert abs(g["logvol"] - o["logvol"]) <= 1e-12 * max(1.0, abs(o["logvol"]))


CASES_F64 = [
    # (m, n, r, w, seed): several tiles, ragged tails, odd node counts
    (200, 300, 8, 16, 1),
    (300, 1000, 5, 64, 2),     # last block takes the remainder (1000 = 15*64 + 40)
    (513, 700, 16, 32, 3),     # m not a multiple of the 256-row tile
    (1000, 97, 3, 3, 4),       # 32 leaves of width 3, last one 4
    (64, 64, 64, 64, 5),       # r = min(m, n): single leaf, full cross
    (777, 129, 1, 0, 6),       # r = 1
    (260, 2048, 32, 32, 7),    # 64 leaves
    (2000, 640, 96, 128, 8),   # r in the 128 bucket
    (600, 1100, 16, 300, 9),   # leaf blocks wider than 256 columns (300, 300, 500)
]


@pytest.mark.parametrize("m,n,r,w,seed", CASES_F64)
def test_select_f64_matches_oracle(orc, m, n, r, w, seed):
    A = torch.from_numpy(W.gaussian(m, n, seed)).to(DEV)
    g, o, _ = run_both(orc, A, r, w)
    assert_same_selection(g, o)


def test_select_f64_c1(orc):
    A = W.c1(1).to(DEV)
    g, o, Ah = run_both(orc, A, 16)
    assert g["status"] == 0
    assert_same_selection(g, o)
    assert np.abs(row_interp(Ah, o["I"], o["J"])).max() <= 1 + 1e-12


@pytest.mark.parametrize("n", [1024, 2048])
def test_select_f64_c2_recipe_small(orc, n):
    # the C2 construction (geometric 0.9 spectrum, 1e-6 floor, 1e-7 noise) at reduced size
    A = W.c2(20 + n, device=DEV, n=n)
    g, o, _ = run_both(orc, A, 64)
    assert_same_selection(g, o)


def test_select_is_deterministic_across_calls(orc):
    # repeated selections of one matrix (arena reused, assembly interleaved)
    # must return identical indices and counters, equal to the oracle's
    A = W.c2(7, device=DEV, n=2048)
    say("case determinism c2-recipe n=2048 x6")
    o = orc.select(A.cpu().numpy(), 64)
    for k in range(6):
        g = cur.select(A, 64)
        np.testing.assert_array_equal(g["I"].cpu().numpy(), o["I"])
        np.testing.assert_array_equal(g["J"].cpu().numpy(), o["J"])
        assert (g["swaps"], g["phases"], g["refreshes"]) == (o["swaps"], o["phases"], o["refreshes"])
        if k % 2:
            C, U, R = cur.assemble(A, g["I"], g["J"])
            cur.residual(A, C, U, R)


def test_select_f64_rank_short(orc):
    rng = np.random.default_rng(9)
    A = torch.from_numpy(rng.standard_normal((300, 3)) @ rng.standard_normal((3, 400))).to(DEV)
    g, o, _ = run_both(orc, A, 6, 32)
    assert o["status"] == orc.ERR_RANK
    assert_same_selection(g, o)


def test_select_f64_noconv(orc):
    A = torch.from_numpy(W.gaussian(300, 256, 10)).to(DEV)
    g, o, _ = run_both(orc, A, 8, 16, max_swaps=1)
    assert o["status"] == orc.WARN_NOCONV
    assert_same_selection(g, o)


def test_select_hilbert_and_recip(orc):
    A = torch.from_numpy(W.hilbert(256)).to(DEV)
    g, o, _ = run_both(orc, A, 6)
    assert_same_selection(g, o)
    A = torch.from_numpy(W.recip_lowrank(512, 20)).to(DEV)
    g, o, _ = run_both(orc, A, 20)
    assert o["status"] == orc.ERR_RANK
    assert_same_selection(g, o)


def test_select_errors():
    say("case error paths")
    A = torch.zeros((40, 50), dtype=torch.float64, device=DEV)
    g = cur.select(A, 3)
    assert g["status"] == cur.ERR_RANK and g["rank"] == 0
    assert (g["I"].cpu() == -1).all()
    A = torch.from_numpy(W.gaussian(40, 50, 1)).to(DEV)
    A[3, 7] = float("nan")
    with pytest.raises(cur.CurError) as ei:
        cur.select(A, 3)
    assert ei.value.status == cur.ERR_NONFINITE
    with pytest.raises(cur.CurError) as ei:
        cur.select(A, 0)
    assert ei.value.status == cur.ERR_ARG
    with pytest.raises(cur.CurError) as ei:
        cur.select(A, 5, col_block=4)
    assert ei.value.status == cur.ERR_ARG


@pytest.mark.parametrize("m,n,r,w,seed", [(400, 600, 12, 32, 11), (1500, 900, 40, 64, 12), (700, 1000, 20, 300, 13),
                                          (333, 777, 64, 64, 14)])
def test_select_f32_matches_oracle_on_upcast(orc, m, n, r, w, seed):
    """FP32 input: the selection computes in FP64 on the exactly widened values,
    so indices, status and every per-node counter equal the oracle's on the
    upcast matrix, bit for bit (volume ratio 1)."""
    A64 = W.c2(seed, n=max(m, n))[:m, :n].contiguous()
    A = A64.to(torch.float32).to(DEV)
    g, o, _ = run_both(orc, A, r, w)
    assert g["status"] in (cur.OK, cur.WARN_NOCONV)
    assert_same_selection(g, o)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_assemble_and_residual_match_oracle(orc, dtype):
    A = W.c1(1).to(dtype).to(DEV)
    Ah = A.cpu().numpy().astype(np.float64)
    o = orc.select(Ah, 16)
    I = torch.from_numpy(o["I"]).to(DEV)
    J = torch.from_numpy(o["J"]).to(DEV)
    say(f"case assemble/residual c1 {dtype}")
    C, U, R = cur.assemble(A, I, J)
    oC, oU, oR, used = orc.assemble(Ah, o["I"], o["J"])
    assert not used
    np.testing.assert_array_equal(C.cpu().numpy().astype(np.float64), oC)
    np.testing.assert_array_equal(R.cpu().numpy().astype(np.float64), oR)
    np.testing.assert_array_equal(U.cpu().numpy(), oU)
    cheb, fro = cur.residual(A, C, U, R)
    ocheb, ofro = orc.residual(Ah, oC, oU, oR)
    amax = np.abs(Ah).max()
    assert abs(cheb - ocheb) <= 1e-10 * amax
    assert abs(fro - ofro) <= 1e-10


def test_assemble_pinv_branch(orc):
    # a repeated column makes A(I,J) singular: the pseudo-inverse branch
    rng = np.random.default_rng(5)
    Ah = rng.standard_normal((30, 20))
    Ah[:, 7] = Ah[:, 3]
    I = np.array([1, 4, 9, 16])
    J = np.array([2, 3, 7, 11])
    A = torch.from_numpy(Ah).to(DEV)
    say("case assemble pinv")
    C, U, R = cur.assemble(A, torch.from_numpy(I).to(DEV), torch.from_numpy(J).to(DEV))
    _, oU, _, used = orc.assemble(Ah, I, J)
    assert used
    np.testing.assert_allclose(U.cpu().numpy(), oU, rtol=0, atol=1e-10 * np.abs(oU).max())


# The residual runs 128 x 128 tiles: interior tiles without bounds tests, the
# ragged right and bottom strips with them, and k in chunks of 32 whose ragged
# last chunk is padded with zeros to a multiple of 4.  The shapes cover: both
# strips (1000 x 700), a thin right strip and a 4-wide last chunk (3000 x 257,
# r = 100), interior tiles only with r % 4 != 0 (256 x 384, r = 37), one-row /
# one-column strips with r = 7 (129 x 130), no interior tile at all (100 x 90),
# and FP32 input through the same tiles.
@pytest.mark.parametrize("m,n,r,dt", [(1000, 700, 24, torch.float64), (3000, 257, 100, torch.float64),
                                      (256, 384, 37, torch.float64), (129, 130, 7, torch.float64),
                                      (100, 90, 5, torch.float64), (640, 515, 33, torch.float32)])
def test_residual_ragged(orc, m, n, r, dt):
    Ah = W.gaussian(m, r, 3) @ W.gaussian(r, n, 4) + 1e-3 * W.gaussian(m, n, 5)
    A = torch.from_numpy(Ah).to(dt).to(DEV)
    Ah = A.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(6)
    I = np.sort(rng.choice(m, r, replace=False))
    J = np.sort(rng.choice(n, r, replace=False))
    say(f"case residual m={m} n={n} r={r} {dt}")
    C, U, R = cur.assemble(A, torch.from_numpy(I).to(DEV), torch.from_numpy(J).to(DEV))
    cheb, fro = cur.residual(A, C, U, R)
    oC, oU, oR, _ = orc.assemble(Ah, I, J)
    ocheb, ofro = orc.residual(Ah, oC, oU, oR)
    amax = np.abs(Ah).max()
    assert abs(cheb - ocheb) <= 1e-10 * amax
    assert abs(fro - ofro) <= 1e-10


@pytest.mark.parametrize("case", ["exact_rank5", "steep_spectrum", "steep_batch"])
def test_f32_rank_verdict_is_the_oracles(orc, case):
    """FP32 input near and below its own resolution: the selection computes in
    FP64 on the widened input with the oracle's threshold, so its rank verdict
    (status, pivots found) and indices equal the oracle's on the upcast
    matrix."""
    rng = np.random.default_rng(60)
    if case == "exact_rank5":  # small integers: exact in FP32, rank exactly 5
        mats = [(np.round(4 * rng.standard_normal((500, 5))) @ np.round(4 * rng.standard_normal((5, 700))), 8)]
    else:  # spectra falling below FP32 resolution within r steps, as in the uneven batch
        mats = [(W.spectral(700, 900, 0.78 ** np.arange(700, dtype=np.float64), 61, 0.0, "cpu",
                            torch.float64).numpy(), 64)]
        if case == "steep_batch":
            mats.append((W.spectral(400, 1300, 0.8 ** np.arange(400, dtype=np.float64), 62, 0.0, "cpu",
                                    torch.float64).numpy(), 32))
    As = [torch.from_numpy(Ah).to(torch.float32).to(DEV) for Ah, _ in mats]
    rs = [r for _, r in mats]
    say(f"case f32 rank verdict {case}")
    if case == "steep_batch":
        outs, _ = cur.select_batched(As, rs)
        res = [(I, J, st) for I, J, st in outs]
    else:
        g = cur.select(As[0], rs[0])
        res = [(g["I"], g["J"], g["status"])]
    for (I, J, st), A, r in zip(res, As, rs):
        Ah = A.cpu().numpy().astype(np.float64)
        o = orc.select(Ah, r)
        say(f"  {Ah.shape} r={r}: status {st}, oracle {o['status']} rank {o['rank']}")
        assert st == o["status"]
        np.testing.assert_array_equal(I.cpu().numpy(), o["I"])
        np.testing.assert_array_equal(J.cpu().numpy(), o["J"])


@pytest.mark.parametrize("dt,prec", [(torch.float64, cur.PREC_NATIVE), (torch.float32, cur.PREC_NATIVE),
                                     (torch.float32, cur.PREC_BF16X3), (torch.float32, cur.PREC_FP8)])
def test_residual_nonfinite_is_reported(orc, dt, prec):
    """A NaN in A reaches the residual's maximum (no NaN-dropping max): the call
    returns ERR_NONFINITE, as the oracle does."""
    Ah = W.gaussian(300, 200, 12)
    I, J = np.array([3, 50, 99, 200]), np.array([1, 17, 150, 199])
    A = torch.from_numpy(Ah).to(dt).to(DEV)
    say(f"case residual nonfinite {dt} prec={prec}")
    C, U, R = cur.assemble(A, torch.from_numpy(I).to(DEV), torch.from_numpy(J).to(DEV))
    A[250, 100] = float("nan")
    with pytest.raises(cur.CurError) as ei:
        cur.residual(A, C, U, R, prec)
    assert ei.value.status == cur.ERR_NONFINITE
    rc, _, _ = orc.residual_raw(A.cpu().numpy(), C.cpu().numpy(), U.cpu().numpy(), R.cpu().numpy())
    assert rc == orc.ERR_NONFINITE


def test_select_batched_matches_single(orc):
    say("case batched")
    As = [torch.from_numpy(W.gaussian(m, n, s)).to(DEV) for (m, n, s) in [(300, 200, 1), (128, 500, 2), (700, 64, 3)]]
    rs = [8, 16, 4]
    outs, rc = cur.select_batched(As, rs)
    assert rc == cur.OK
    for (I, J, st), A, r in zip(outs, As, rs):
        o = orc.select(A.cpu().numpy(), r)
        assert st == o["status"]
        np.testing.assert_array_equal(I.cpu().numpy(), o["I"])
        np.testing.assert_array_equal(J.cpu().numpy(), o["J"])


def test_select_batched_mixed_trees_match_single(orc):
    """Trees of different depths, ranks (all three register buckets), dtypes,
    and an all-zero item, run as one batch: every item equals its own
    single-matrix selection bit for bit, and the FP64 items equal the oracle."""
    say("case batched mixed")
    specs = [(600, 512, 8, 11, torch.float64), (257, 96, 16, 12, torch.float64), (1500, 1024, 33, 13, torch.float64),
             (800, 700, 64, 14, torch.float64), (900, 300, 100, 15, torch.float64), (1200, 640, 16, 16, torch.float32),
             (333, 777, 64, 17, torch.float32), (400, 256, 8, 0, torch.float64)]
    As, rs = [], []
    for m, n, r, seed, dt in specs:
        A = torch.zeros(m, n, dtype=dt, device=DEV) if seed == 0 else \
            torch.from_numpy(W.gaussian(m, n, seed)).to(DEV).to(dt)
        As.append(A)
        rs.append(r)
    outs, rc = cur.select_batched(As, rs)
    for (I, J, st), A, r, (m, n, _, seed, dt) in zip(outs, As, rs, specs):
        say(f"  item m={m} n={n} r={r} seed={seed} {dt} status {st}")
        g = cur.select(A, r, allow=(cur.OK, cur.WARN_NOCONV, cur.ERR_RANK))
        assert st == g["status"]
        np.testing.assert_array_equal(I.cpu().numpy(), g["I"].cpu().numpy())
        np.testing.assert_array_equal(J.cpu().numpy(), g["J"].cpu().numpy())
        if dt == torch.float64 and seed != 0:
            o = orc.select(A.cpu().numpy(), r)
            assert st == o["status"]
            np.testing.assert_array_equal(I.cpu().numpy(), o["I"])
            np.testing.assert_array_equal(J.cpu().numpy(), o["J"])
        if seed == 0:
            assert st == cur.ERR_RANK
    # a second call of the same batch (workspace, streams and tuner entries
    # reused) gives the same results
    outs2, rc2 = cur.select_batched(As, rs)
    assert rc2 == rc
    for (I, J, st), (I2, J2, st2) in zip(outs, outs2):
        assert st2 == st
        np.testing.assert_array_equal(I2.cpu().numpy(), I.cpu().numpy())
        np.testing.assert_array_equal(J2.cpu().numpy(), J.cpu().numpy())


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_node_groups_do_not_change_the_selection(orc, dt):
    """Splitting each tree level into 1, 2 or 3 node groups on their own
    streams, fixed or chosen by the autotuner (whose first calls try each
    count), gives the same selection bit for bit; 24 leaves make levels of
    24, 12, 6, 3, 2, 1 nodes, so a promoted odd node lands in a group."""
    m, n, r, seed = 1024, 1536, 32, 21
    say(f"case node groups m={m} n={n} r={r} seed={seed} {dt}")
    A = torch.from_numpy(W.gaussian(m, n, seed)).to(DEV).to(dt)
    ref = cur.select(A, r, groups=1)
    for groups in (2, 3, 0, 0, 0, 0):
        g = cur.select(A, r, groups=groups)
        assert g["status"] == ref["status"]
        np.testing.assert_array_equal(g["I"].cpu().numpy(), ref["I"].cpu().numpy())
        np.testing.assert_array_equal(g["J"].cpu().numpy(), ref["J"].cpu().numpy())
    if dt == torch.float64:
        o = orc.select(A.cpu().numpy(), r)
        np.testing.assert_array_equal(ref["I"].cpu().numpy(), o["I"])
        np.testing.assert_array_equal(ref["J"].cpu().numpy(), o["J"])
    outs1, _ = cur.select_batched([A, A[:700, :900].contiguous()], [r, 16], groups=1)
    outs3, _ = cur.select_batched([A, A[:700, :900].contiguous()], [r, 16], groups=3)
    for (I1, J1, s1), (I3, J3, s3) in zip(outs1, outs3):
        assert s1 == s3
        assert torch.equal(I1, I3) and torch.equal(J1, J3)


def test_tune_cache_round_trip():
    """Three autotuned calls on one shape explore 1, 2 and 3 node groups; the
    exported cache then names the fastest.  An imported choice is used as is
    and the selection stays the same."""
    say("case tune cache")
    A = torch.from_numpy(W.gaussian(700, 1100, 22)).to(DEV)
    ref = cur.select(A, 16, groups=1)
    cur.tune_import([])
    for _ in range(3):
        cur.select(A, 16)
    t = cur.tune_export()
    assert t and all(e["tried"] == 3 and e["groups"] in (1, 2, 3) for e in t)
    forced = [dict(e, groups=2) for e in t]
    cur.tune_import(forced)
    g = cur.select(A, 16)
    assert torch.equal(g["I"], ref["I"]) and torch.equal(g["J"], ref["J"])
    assert [e["groups"] for e in cur.tune_export()] == [2] * len(t)
    cur.tune_import([])


def test_profile_counters_count_the_pass_bytes():
    """Level 1 times the streaming pass only, level 2 adds the fresh kernel;
    the algorithmic bytes of one selection are a fixed sum over its launches,
    and a busy launch is one that moved bytes.  The fresh kernel is launched
    only in iterations after a controller launch that admits factorization
    steps, so it has at most as many launches as the pass."""
    say("case profile counters")
    A = torch.from_numpy(W.gaussian(1000, 640, 23)).to(DEV)
    cur.select(A, 16, groups=1)
    cur.profile_enable(1)
    cur.select(A, 16, groups=1)
    p1 = cur.profile_read()
    cur.profile_enable(2)
    cur.select(A, 16, groups=1)
    p2 = cur.profile_read()
    cur.profile_enable(0)
    assert p1["launches"] > 0 and 0 < p1["busy"] <= p1["launches"]
    assert p1["bytes"] > 0 and p1["seconds"] > 0
    assert p1["fresh_launches"] == 0 and p1["fresh_bytes"] == 0
    assert p2["bytes"] == p1["bytes"] and p2["launches"] == p1["launches"]
    assert 0 < p2["fresh_busy"] <= p2["fresh_launches"] <= p2["launches"]
    assert 0 < p1["busy_seconds"] <= p1["seconds"] and 0 < p2["fresh_busy_seconds"] <= p2["fresh_seconds"]
    assert p2["fresh_bytes"] > 0


GREEDY_CASES = [
    # (m, n, r, seed, dtype)
    (200, 300, 8, 31, torch.float64),
    (513, 700, 16, 32, torch.float64),   # m not a multiple of 64
    (64, 64, 64, 33, torch.float64),     # r = min(m, n)
    (777, 129, 1, 34, torch.float64),    # r = 1
    (600, 900, 24, 35, torch.float32),   # FP32 input, exact upcast for the oracle
]


def greedy_both(orc, A, r):
    """GPU and oracle norm-greedy selections with the GPU's choice orders."""
    g = cur.select(A, r, method=cur.METHOD_GREEDY, trace=True)
    o = orc.greedy(A.cpu().numpy(), r)
    return g, o


def assert_greedy_agrees(g, o, m, n, r):
    """The GPU sums a vector in lane-strided order, the oracle in plain
    ascending order.  At every step whose margin (best - runner-up squared
    norm) exceeds the rounding bound of helpers.greedy_margin_bound both must
    choose the same vector; the comparison ends at the first near-tie, and the
    test matrices are chosen so that none occurs (asserted)."""
    tr = g["trace"]
    gI, gJ = tr["I"][0], tr["J"][0]
    for order, gaps, length, q in ((gI, o["gap_I"], n, o["rank_rows"]), (gJ, o["gap_J"], m, o["rank_cols"])):
        stop = greedy_first_near_tie(gaps, q, length)
        assert stop == q, f"near-tie at step {stop} of {q}: margin {gaps[stop]:.3e}"
        ref = o["order_I"] if order is gI else o["order_J"]
        np.testing.assert_array_equal(order[:q], ref[:q])
    assert g["status"] == o["status"]
    np.testing.assert_array_equal(g["I"].cpu().numpy(), o["I"])
    np.testing.assert_array_equal(g["J"].cpu().numpy(), o["J"])


@pytest.mark.parametrize("m,n,r,seed,dt", GREEDY_CASES)
def test_greedy_matches_oracle(orc, m, n, r, seed, dt):
    """Norm-greedy rows and columns (Alg. 2 with Alg. 3): the same choice at
    every step whose margin exceeds the rounding bound (all steps here), so
    the same index sets and status."""
    A = torch.from_numpy(W.gaussian(m, n, seed)).to(dt).to(DEV)
    say(f"case greedy m={m} n={n} r={r} seed={seed} {dt}")
    g, o = greedy_both(orc, A, r)
    assert_greedy_agrees(g, o, m, n, r)
    assert np.isnan(g["logvol"])


def test_greedy_rank_short_and_c2_recipe(orc):
    rng = np.random.default_rng(36)
    A = torch.from_numpy(rng.standard_normal((400, 6)) @ rng.standard_normal((6, 500))).to(DEV)
    say("case greedy rank-short")
    g, o = greedy_both(orc, A, 10)
    assert g["status"] == o["status"] == cur.ERR_RANK and g["rank"] == 6
    assert_greedy_agrees(g, o, 400, 500, 10)
    A = W.c2(37, device=DEV, n=1024)
    say("case greedy c2-recipe n=1024 r=64")
    g, o = greedy_both(orc, A, 64)
    assert_greedy_agrees(g, o, 1024, 1024, 64)
    B = A.clone()
    B[5, 9] = float("nan")
    with pytest.raises(cur.CurError) as ei:
        cur.select(B, 8, method=cur.METHOD_GREEDY)
    assert ei.value.status == cur.ERR_NONFINITE


@pytest.mark.parametrize("name,n", [("hilbert", 256), ("hilbert", 512), ("recip", 256), ("recip", 512)])
def test_error_curve_points_match_oracle(orc, name, n):
    """The paper's closed-form workloads (Sec. 3.1): Hilbert matrices for
    r = 1..20 and products of the 1/(i+j) factors for r = 5..20, each point of
    the error curve (paper_2502_11017_amd.curves.point) against the oracle:
    same status, rank reached and FP64 index sets; Chebyshev and Frobenius
    errors within 1e-10 ||A||_C plus the rounding of the 2q-term products
    C U R in two evaluation orders, 2 gamma_2q max(|C| |U| |R|): the crosses
    of the largest r are so ill-conditioned (Hilbert, r >= 17) that this term,
    not 1e-10 ||A||_C, is what two correct evaluations can differ by.  The
    Frobenius error also falls with r up to r = 8."""
    from paper_2502_11017_amd import curves

    Ah = W.hilbert(n) if name == "hilbert" else W.recip_lowrank(n, 20)
    A = torch.from_numpy(Ah).to(DEV)
    amax = float(np.abs(Ah).max())
    rs = range(1, 21) if name == "hilbert" else range(5, 21)
    fros = {}
    for r in rs:
        say(f"case curve {name} n={n} r={r}")
        g = cur.select(A, r)
        o = orc.select(Ah, r)
        assert g["status"] == o["status"] and g["rank"] == o["rank"], (r, g["status"], o["status"])
        np.testing.assert_array_equal(g["I"].cpu().numpy(), o["I"])
        np.testing.assert_array_equal(g["J"].cpu().numpy(), o["J"])
        q, fro, cheb = curves.point(A, r, cur.METHOD_MAXVOL)
        oq = r if o["status"] in (orc.OK, orc.WARN_NOCONV) else o["rank"]
        assert q == oq
        oC, oU, oR, _ = orc.assemble(Ah, o["I"][:q], o["J"][:q])
        ocheb, ofro = orc.residual(Ah, oC, oU, oR)
        gam = 2 * q * 2.0 ** -52 / (1 - 2 * q * 2.0 ** -52)
        prod = float((np.abs(oC) @ np.abs(oU) @ np.abs(oR)).max())
        tol = 1e-10 * amax + 2 * gam * prod
        assert abs(cheb - ocheb) <= tol, (r, cheb, ocheb, tol)
        afro = float(np.linalg.norm(Ah))
        assert abs(fro - ofro) <= 1e-10 + 2 * gam * prod * np.sqrt(Ah.size) / afro, (r, fro, ofro)
        fros[r] = fro
    if name == "hilbert":
        assert fros[1] < 1.0 and fros[2] > fros[4] > fros[8]


@pytest.mark.parametrize("case", read_tree_golden(os.path.join(GOLDEN, "tree_shape.txt")),
                         ids=lambda c: c["name"])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_tree_shape_and_merge_tie_golden(case, dt):
    """The hand-derived tree tables (5 and 12 leaves, merge tie to the left
    child, two identical blocks) hold on the GPU too, in both dtypes (the
    entries are small integers, exact in FP32)."""
    say(f"case golden tree {case['name']} {dt}")
    A = torch.from_numpy(case["A"]).to(dt).to(DEV)
    g = cur.select(A, case["r"], col_block=case["w"], trace=True)
    assert g["status"] == cur.OK
    check_tree_golden(case, g["I"].cpu().numpy(), g["J"].cpu().numpy(), g["trace"], g["logvol"])


def test_gate_periods_do_not_change_the_selection(orc):
    """The controller's factorization steps run only in one launch of P; the
    period changes when they run, never their operands or order.  Selections
    in child processes with no gating and with other periods equal the
    oracle's (the variable is read once per process)."""
    import json
    import subprocess

    import tempfile

    n = 1536
    Ah = W.c2(40, device=DEV, n=n).cpu().numpy()
    o = orc.select(Ah, 32)
    tmp = tempfile.NamedTemporaryFile(suffix=".npy", delete=False)
    tmp.close()
    np.save(tmp.name, Ah)
    code = ("import json, sys, numpy, torch; sys.path.insert(0, %r); import paper_2502_11017_amd as cur; "
            "A = torch.from_numpy(numpy.load(%r)).to('cuda:0'); "
            "g = cur.select(A, 32, groups=2); print(json.dumps({'I': g['I'].tolist(), 'J': g['J'].tolist(), "
            "'swaps': g['swaps'], 'phases': g['phases'], 'refreshes': g['refreshes']}))"
            % (os.path.dirname(os.path.dirname(os.path.abspath(__file__))), tmp.name))
    for gate in ("1", "24,16,8,2", "3"):
        say(f"  child process with CUR_GATE={gate}")
        env = dict(os.environ, CUR_GATE=gate)
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=240)
        assert out.returncode == 0, out.stderr[-2000:]
        g = json.loads(out.stdout.strip().splitlines()[-1])
        np.testing.assert_array_equal(np.array(g["I"]), o["I"])
        np.testing.assert_array_equal(np.array(g["J"]), o["J"])
        for key in ("swaps", "phases", "refreshes"):
            assert g[key] == o[key], (gate, key, g[key], o[key])
    os.unlink(tmp.name)


def test_compute_unit_mask_does_not_change_selection(orc):
    """The compute-unit sweep (strong scaling over CUs, after the scalability
    experiment of Sec. 3.2) runs each count in a child process restricted by
    the runtime's CU mask.  The CUs a selection runs on change its time,
    never its result: every count's I, J equal the oracle's."""
    import hashlib
    import shutil
    import tempfile

    from paper_2502_11017_amd import cusweep

    n, r = 1536, 32
    Ah = W.c2(41, device=DEV, n=n).cpu().numpy()
    o = orc.select(Ah, r)
    want = hashlib.sha256(np.asarray(o["I"], dtype=np.int64).tobytes()
                          + np.asarray(o["J"], dtype=np.int64).tobytes()).hexdigest()[:16]
    work = tempfile.mkdtemp(prefix="cusweep_test_")
    try:
        np.save(os.path.join(work, f"c2_{n}.npy"), Ah)  # the sweep's own file name: no generation step
        say(f"case cu sweep n={n} r={r} cus=(32, 256)")
        rows = cusweep.sweep(n=n, r=r, cus=(32, 256), steps=1, warmup=1, workdir=work)
    finally:
        shutil.rmtree(work, ignore_errors=True)
    assert [x["cus"] for x in rows] == [32, 256]
    for x in rows:
        assert x["status"] == cur.OK, x
        assert x["swaps"] == o["swaps"], (x, o["swaps"])
        assert x["digest"] == want, (x, want)
