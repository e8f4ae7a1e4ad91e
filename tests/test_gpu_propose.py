"""The learned candidate proposal on the GPU, through the C ABI, against the
FP64 references of oracle/mlp_oracle.py (network, gradient, Adam, features)
and the oracle's plain selection (volume ratio), plus the dominance of every
learned selection, which the verification pass guarantees whatever the
network's weights."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2502_11017_amd as cur  # noqa: E402
from oracle import mlp_oracle as mo  # noqa: E402
from paper_2502_11017_amd import learn  # noqa: E402
from paper_2502_11017_amd import workloads as W  # noqa: E402
from tests.helpers import col_interp, row_interp  # noqa: E402

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _problem(seed, n=1000):
    rng = np.random.default_rng(seed)
    p = (rng.standard_normal(mo.NPARAMS) * 0.3).astype(np.float32)
    X = np.column_stack([-np.abs(rng.standard_normal(n)) * 8, rng.standard_normal(n) * 3, rng.random(n),
                         rng.random(n)]).astype(np.float32)
    y = (rng.random(n) < 0.25).astype(np.float32)
    return p, X, y


def test_forward_and_gradient_match_fp64_reference():
    """Scores and the loss gradient (FP32 on the device, FP16 weights) against
    the FP64 chain rule on the same FP16-rounded weights: the FP32 sums of at
    most 128 products and of 1000 rows stay within 1e-4 of the scale."""
    p, X, y = _problem(1)
    say("case mlp forward/grad n=1000")
    blob = cur.mlp_pack(torch.from_numpy(p).to(DEV))
    Xd, yd = torch.from_numpy(X).to(DEV), torch.from_numpy(y).to(DEV)
    pr = mo.device_weights(p)
    s_ref, _ = mo.forward(pr, X)
    s = cur.mlp_forward(blob, Xd).cpu().numpy()
    np.testing.assert_allclose(s, s_ref, rtol=1e-4, atol=1e-4)
    for pw in (1.0, 3.0):
        g, loss = cur.mlp_grad(blob, Xd, yd, pos_weight=pw)
        g = g.cpu().numpy().astype(np.float64)
        g_ref = mo.grad(pr, X, y, pw)
        assert loss == pytest.approx(mo.loss(pr, X, y, pw), rel=1e-5)
        err = np.abs(g - g_ref).max()
        say(f"  pw={pw}: max |g - g_ref| {err:.3e}, max |g_ref| {np.abs(g_ref).max():.3e}")
        assert err <= 1e-4 * np.abs(g_ref).max() + 1e-7


def test_adam_matches_fp64_reference():
    rng = np.random.default_rng(2)
    p = (rng.standard_normal(mo.NPARAMS) * 0.3).astype(np.float32)
    g = (rng.standard_normal(mo.NPARAMS) * 1e-2).astype(np.float32)
    m1 = (rng.standard_normal(mo.NPARAMS) * 1e-3).astype(np.float32)
    m2 = (rng.random(mo.NPARAMS) * 1e-5).astype(np.float32)
    pd, m1d, m2d = (torch.from_numpy(x.copy()).to(DEV) for x in (p, m1, m2))
    blob = cur.mlp_pack(pd)
    cur.mlp_adam(blob, pd, m1d, m2d, torch.from_numpy(g).to(DEV), 3, 1e-3)
    # the device takes the hyper-parameters as FP32; the reference uses the same values in FP64,
    # so what remains is the FP32 rounding of the two products and the sum of each moment:
    # a few units in the last place (2^-24 relative) of its larger term
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    p_ref, m1_ref, m2_ref = mo.adam(p.astype(np.float64), m1.astype(np.float64), m2.astype(np.float64),
                                    g.astype(np.float64), 3, f32(1e-3), f32(0.9), f32(0.999), f32(1e-8))
    ulp = 2.0 ** -24
    t1 = np.maximum(np.abs(0.9 * m1), np.abs(0.1 * g)).astype(np.float64)
    t2 = np.maximum(np.abs(0.999 * m2), np.abs(1e-3 * g * g)).astype(np.float64)
    np.testing.assert_allclose(pd.cpu().numpy(), p_ref, rtol=0, atol=1e-6)
    assert (np.abs(m1d.cpu().numpy() - m1_ref) <= 4 * ulp * t1).all()
    assert (np.abs(m2d.cpu().numpy() - m2_ref) <= 4 * ulp * t2).all()
    # the blob now holds the updated weights: its scores are those of the reference network
    X = np.random.default_rng(3).standard_normal((200, 4)).astype(np.float32)
    s = cur.mlp_forward(blob, torch.from_numpy(X).to(DEV)).cpu().numpy()
    np.testing.assert_allclose(s, mo.forward(mo.device_weights(pd.cpu().numpy()), X)[0], rtol=1e-4, atol=1e-4)


@pytest.mark.parametrize("m,n,r,w", [(700, 330, 8, 64), (50, 130, 8, 64), (300, 200, 32, 40), (1000, 300, 64, 64)])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_features_match_reference(dt, m, n, r, w):
    """f0, f1 and f2 against the FP64 definitions (leverage from numpy's QR of
    the same sketch, drawn by the oracle's own copy of the counter-based
    generator; ridge block leverage from numpy's solve).  The rank feature f3
    is checked twice: exactly against the histogram rank of the device's own
    f2 (its FP32 binning re-done on the host), and against the exact rank of
    the reference's f2 within the rows one bin width away (a value near a bin
    edge may land in the neighbouring bin, which moves the rank of every row
    below it by a count).  Shapes: several leaves with a wider last one, fewer
    rows than a leaf has columns (a rank-deficient block Gram, held by the
    ridge), leaves narrower than 64, and the widest sketch (2r = 128
    columns)."""
    seed = 12345
    Ah = W.gaussian(m, 40, 4) @ W.gaussian(40, n, 5) + 0.01 * W.gaussian(m, n, 6)
    A = torch.from_numpy(Ah).to(dt).to(DEV)
    say(f"case features m={m} n={n} r={r} w={w} {dt}")
    F = cur.mlp_features(A, r, col_block=w, seed=seed).cpu().numpy().astype(np.float64)
    Fr = mo.features(A.cpu().numpy().astype(np.float64), r, w, seed)
    assert F.shape == Fr.shape
    d = np.abs(F[:, :3] - Fr[:, :3]).max(axis=0)
    say(f"  max |F - F_ref|: f0 {d[0]:.2e} f1 {d[1]:.2e} f2 {d[2]:.2e}")
    tol = (1e-4, 2e-3, 2e-3)
    for c in range(3):
        np.testing.assert_allclose(F[:, c], Fr[:, c], rtol=0, atol=tol[c])
    b = F.shape[0] // m
    bw = 96.0 / 1024.0
    for k in range(b):
        f2, f3, f2r = F[k * m:(k + 1) * m, 2], F[k * m:(k + 1) * m, 3], Fr[k * m:(k + 1) * m, 2]
        # the device's binning in FP32: bin = trunc(clamp((v + 64) (1024 / 96))), rank = (above + c / 2) / m
        t = (f2.astype(np.float32) + np.float32(64.0)) * np.float32(1024.0 / 96.0)
        bins = np.clip(t, 0, 1023).astype(np.int64)
        cnt = np.bincount(bins, minlength=1024)
        above = np.concatenate([np.cumsum(cnt[::-1])[::-1][1:], [0]])
        rank = ((above.astype(np.float32) + np.float32(0.5) * cnt.astype(np.float32)) / np.float32(m))
        np.testing.assert_array_equal(f3.astype(np.float32), rank[bins])
        srt = np.sort(f2r)
        above_exact = (m - np.searchsorted(srt, f2r, side="right")) / m
        near = (np.searchsorted(srt, f2r + bw + 2 * tol[2], side="right")
                - np.searchsorted(srt, f2r - bw - 2 * tol[2], side="left")) / m
        assert (np.abs(f3 - above_exact) <= 1.5 * near + 1e-6).all()


def _cur(Ah, I, J):
    """C, U = A(I, J)^-1, R of a cross, in FP64 on the host."""
    I, J = np.asarray(I), np.asarray(J)
    return Ah[:, J], np.linalg.inv(Ah[np.ix_(I, J)]), Ah[I, :]


def _weights():
    if os.path.exists(learn.WEIGHTS):
        return learn.load_blob(device=DEV), "trained"
    return cur.mlp_pack(torch.from_numpy(learn.init_params()).to(DEV)), "untrained"


@pytest.mark.parametrize("n,r", [(1024, 32), (2048, 64), (1500, 20)])
def test_learned_selection_is_dominant_and_near_plain(orc, n, r):
    """The learned start ends in the ordinary swap loop: the root cross is
    dominant over all m rows and over its candidate columns, whatever the
    weights.  Another start may end in another dominant cross (a different
    local maximum of the volume, larger or smaller); with the trained network
    the approximation it gives is within 1.5 times the Frobenius error of the
    oracle's plain selection."""
    A = W.c2(80 + n, device=DEV, n=n)
    Ah = A.cpu().numpy()
    blob, kind = _weights()
    say(f"case learned selection n={n} r={r} ({kind} weights)")
    g = cur.select(A, r, mlp=blob, seed=7, trace=True)
    assert g["status"] in (cur.OK, cur.WARN_NOCONV)
    I, J = g["I"].cpu().numpy(), g["J"].cpu().numpy()
    assert np.abs(row_interp(Ah, I, J)).max() <= 1 + 1e-12
    tr = g["trace"]
    meta = tr["meta"]
    top = meta[:, 0].max()
    if top > 0:
        kids = np.where(meta[:, 0] == top - 1)[0][:2]
        Jc = np.sort(np.concatenate([tr["J"][k][:meta[k, 2]] for k in kids]))
        assert np.abs(col_interp(Ah, I, J, Jc)).max() <= 1 + 1e-12
    o = orc.select(Ah, r)
    ratio = np.exp(orc.logvol(Ah, I, J) - o["logvol"])
    _, fro = orc.residual(Ah, *_cur(Ah, I, J))
    _, fro_plain = orc.residual(Ah, *_cur(Ah, o["I"], o["J"]))
    say(f"  volume ratio to the oracle's plain selection {ratio:.6f}; relative Frobenius error {fro:.4e} "
        f"(plain {fro_plain:.4e})")
    if kind == "trained":
        assert fro <= 1.5 * fro_plain


def test_training_lowers_the_loss():
    """A short run of the library's training kernels (8 matrices at 1024 x
    1024, r = 16) lowers the loss and raises the held-out recall."""
    out = []
    p, hist = learn.train(matrices=8, r=16, n=1024, steps_per_matrix=12, batch=4096, held_out=1,
                          log=lambda s: out.append(s))
    for s in out:
        say("  " + s)
    assert np.isfinite(p).all()
    blob0 = cur.mlp_pack(torch.from_numpy(learn.init_params()).to(DEV))
    A = W.c5_train(99, device=DEV, n=1024)
    X, y, F, Y = learn.labelled_rows(A, 16, 64, 5, np.random.default_rng(0))
    _, l0 = cur.mlp_grad(blob0, X, y, pos_weight=3.0)
    _, l1 = cur.mlp_grad(cur.mlp_pack(torch.from_numpy(p).to(DEV)), X, y, pos_weight=3.0)
    say(f"  loss on a fresh matrix: initial {l0:.4f}, trained {l1:.4f}")
    assert l1 < l0


def test_gain_at_full_size():
    """The benchmark's shape (8192 x 8192 FP64, r = 64, leaves of 64 columns)
    with the shipped weights: the learned selection's root cross is dominant
    over all 8192 rows (|A(:, J) A(I, J)^-1| <= 1 + 1e-12, host LAPACK solve),
    its volume is at least 0.99 of the plain selection's, and both times are
    reported."""
    import time

    if not os.path.exists(learn.WEIGHTS):
        pytest.skip("no shipped weights")
    A = W.c2(2, device=DEV)
    r = 64
    blob = learn.load_blob(device=DEV)
    say("case learned gain c2 8192 r=64")
    res = {}
    for name, kw in (("plain", {}), ("learned", dict(mlp=blob, seed=7))):
        cur.select(A, r, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter()
        g = cur.select(A, r, **kw)
        torch.cuda.synchronize()
        res[name] = (g, 1e3 * (time.perf_counter() - t))
    (gp, tp), (gl, tl) = res["plain"], res["learned"]
    ratio = float(np.exp(gl["logvol"] - gp["logvol"]))
    say(f"  plain {tp:.1f} ms, learned {tl:.1f} ms; volume ratio {ratio:.4f}; swaps {gp['swaps']} -> {gl['swaps']}")
    assert gl["status"] == cur.OK
    Ah = A.cpu().numpy()
    I, J = gl["I"].cpu().numpy(), gl["J"].cpu().numpy()
    assert np.abs(row_interp(Ah, I, J)).max() <= 1 + 1e-12
    assert ratio >= 0.99
