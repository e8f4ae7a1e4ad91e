"""Training of the learned candidate proposal (cur_opts.propose = 1) on the GPU.

    python -m paper_2502_11017_amd.learn --matrices 400 --out paper_2502_11017_amd/mlp_weights.f32

Training matrices are generated as they are consumed (workloads.c5_train:
4096 x 4096 FP64, the 64-direction geometric spectrum of the 8192 x 8192
benchmark matrix with noise), one per seed.  For each matrix the plain
maximal-volume selection with r = 32 or 64 (alternating) and leaf blocks of
64 columns (cur_select with a per-node trace) labels, in every leaf, the r rows that
leaf's swap loop ends with; the library's feature kernel gives every (leaf,
row) its four features.  Each leaf contributes its r positive rows and 3 r
rows drawn uniformly from the others.  The network is trained with the
library's own gradient (cur_mlp_grad, the weighted logistic loss with the
positives weighted 3:1 to balance the sampling) and Adam (cur_mlp_adam) on
minibatches drawn from the rows of the most recent matrices.  Held-out
matrices measure the recall of the proposal: the share of the leaf-selected
rows that fall among the leaf's 4r best-scored rows.

Output: the FP32 parameter vector (CUR_MLP_PARAMS floats, raw little-endian),
from which ``load_blob`` packs the device weight blob.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "mlp_weights.f32")


def init_params(seed: int = 0) -> np.ndarray:
    """He-scaled Gaussian weights, zero biases (parameter order W1, b1, W2, b2, w3, b3)."""
    import paper_2502_11017_amd as cur

    F, H = cur.MLP_FEATURES, cur.MLP_HIDDEN
    rng = np.random.default_rng(seed)
    p = np.zeros(cur.MLP_PARAMS, dtype=np.float32)
    o = 0
    p[o:o + H * F] = rng.standard_normal(H * F) * np.sqrt(2.0 / F)
    o += H * F + H
    p[o:o + H * H] = rng.standard_normal(H * H) * np.sqrt(2.0 / H)
    o += H * H + H
    p[o:o + H] = rng.standard_normal(H) * np.sqrt(1.0 / H)
    return p


def load_blob(path: str = WEIGHTS, device="cuda:0"):
    """The device weight blob of a saved parameter vector."""
    import torch

    import paper_2502_11017_amd as cur

    p = np.fromfile(path, dtype=np.float32)
    if p.size != cur.MLP_PARAMS:
        raise ValueError(f"{path}: {p.size} parameters, expected {cur.MLP_PARAMS}")
    return cur.mlp_pack(torch.from_numpy(p).to(device))


def labelled_rows(A, r, w, seed, rng, negatives=3):
    """(features, labels) of one matrix: every leaf's selected rows and
    `negatives` r others per leaf; and the full feature/label arrays."""
    import torch

    import paper_2502_11017_amd as cur

    m, n = A.shape
    b = max(1, n // w)
    g = cur.select(A, r, col_block=w, trace=True)
    meta, TI = g["trace"]["meta"], g["trace"]["I"]
    Y = np.zeros((b, m), dtype=np.float32)
    for k in range(b):
        q = int(meta[k, 2])
        Y[k, TI[k][:q]] = 1.0
    F = cur.mlp_features(A, r, col_block=w, seed=seed)
    pick = []
    for k in range(b):
        pos = np.flatnonzero(Y[k])
        neg = rng.choice(np.flatnonzero(Y[k] == 0), negatives * len(pos), replace=False)
        pick.append(k * m + np.concatenate([pos, neg]))
    pick = torch.from_numpy(np.concatenate(pick)).to(F.device)
    return F[pick], torch.from_numpy(Y.reshape(-1)).to(F.device)[pick], F, Y


def recall(blob, F, Y, r):
    """Share of the leaf-selected rows among each leaf's 4r best-scored rows."""
    import paper_2502_11017_amd as cur

    b, m = Y.shape
    s = cur.mlp_forward(blob, F).reshape(b, m).cpu().numpy()
    top = np.argsort(-s, axis=1, kind="stable")[:, :4 * r]
    hit = sum(int(Y[k, top[k]].sum()) for k in range(b))
    return hit / max(1.0, float(Y.sum()))


def recall_of(score, Y, r):
    """recall() for given scores (b m) instead of the network's."""
    b, m = Y.shape
    s = score.reshape(b, m)
    top = np.argsort(-s, axis=1, kind="stable")[:, :4 * r]
    return sum(int(Y[k, top[k]].sum()) for k in range(b)) / max(1.0, float(Y.sum()))


def train(matrices=400, r=(32, 64), w=64, n=4096, steps_per_matrix=4, batch=16384, lr=2e-3, seed0=50000,
          held_out=4, log=print, device="cuda:0"):
    """Matrix i is labelled with rank r[i % len(r)] (every rank the same leaf
    width w); the held-out matrices are labelled with every rank."""
    import torch

    import paper_2502_11017_amd as cur
    from paper_2502_11017_amd import workloads as W

    dev = torch.device(device)
    rng = np.random.default_rng(7)
    p = torch.from_numpy(init_params()).to(dev)
    m1 = torch.zeros_like(p)
    m2 = torch.zeros_like(p)
    blob = cur.mlp_pack(p)
    rs = (r,) if isinstance(r, int) else tuple(r)
    val = []
    for k in range(held_out):
        A = W.c5_train(seed0 + 10_000_000 + k, device=dev, n=n)
        for rk in rs:
            _, _, F, Y = labelled_rows(A, rk, w, k + 1, rng)
            val.append((F, Y, rk))
    # a reference point: the recall of the block leverage (feature 2) alone
    base = float(np.mean([recall_of(F[:, 2].cpu().numpy(), Y, rk) for F, Y, rk in val]))
    log(f"held-out recall of the 4r rows of largest block leverage: {base:.4f}")
    Xs, Ys = [], []
    step = 0
    t0 = time.time()
    hist = []
    for i in range(matrices):
        A = W.c5_train(seed0 + i, device=dev, n=n)
        X, y, _, _ = labelled_rows(A, rs[i % len(rs)], w, i + 101, rng)
        Xs.append(X)
        Ys.append(y)
        if len(Xs) > 16:  # the rows of the 16 most recent matrices
            Xs.pop(0)
            Ys.pop(0)
        Xb, Yb = torch.cat(Xs), torch.cat(Ys)
        for _ in range(steps_per_matrix):
            idx = torch.from_numpy(rng.choice(Xb.shape[0], min(batch, Xb.shape[0]), replace=False)).to(dev)
            gr, loss = cur.mlp_grad(blob, Xb[idx].contiguous(), Yb[idx].contiguous(), pos_weight=3.0)
            step += 1
            cur.mlp_adam(blob, p, m1, m2, gr, step, lr)
        if (i + 1) % 25 == 0 or i == matrices - 1:
            rc = float(np.mean([recall(blob, F, Y, rk) for F, Y, rk in val]))
            hist.append((i + 1, step, loss, rc))
            log(f"matrices {i + 1}, steps {step}: loss {loss:.4f}, held-out recall of the 4r candidates {rc:.4f} "
                f"({time.time() - t0:.0f} s)")
    return p.cpu().numpy(), hist


def main(argv=None):
    ap = argparse.ArgumentParser(prog="learn")
    ap.add_argument("--matrices", type=int, default=400)
    ap.add_argument("--steps-per-matrix", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--ranks", default="32,64", help="comma-separated ranks the matrices are labelled with")
    ap.add_argument("--out", default=WEIGHTS)
    a = ap.parse_args(argv)
    p, _ = train(a.matrices, r=tuple(int(x) for x in a.ranks.split(",")), steps_per_matrix=a.steps_per_matrix,
                 lr=a.lr, log=lambda s: print(s, flush=True))
    p.astype(np.float32).tofile(a.out)
    print(f"wrote {a.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
