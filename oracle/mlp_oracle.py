"""FP64 reference of the learned proposal's network, features and training step.

TEST INFRASTRUCTURE ONLY: the tests are the only callers; nothing here is
imported by the HIP library or its binding.  Plain numpy in FP64, written from
the definitions (no blocking or fusion):

  score(f) = w3 . relu(W2 relu(W1 f + b1) + b2) + b3          (W1 128x4, W2 128x128)
  loss     = (1/N) sum_i [ pw y_i softplus(-s_i) + (1 - y_i) softplus(s_i) ]
  Adam     m1 = b1 m1 + (1 - b1) g, m2 = b2 m2 + (1 - b2) g^2,
           p -= lr (m1 / (1 - b1^t)) / (sqrt(m2 / (1 - b2^t)) + eps)

The weights the device uses are FP16 (biases FP32): `device_weights` rounds
the weight parts of a parameter vector to FP16 (round to nearest even, as the
device's conversion does) so that both sides evaluate the same network.

Features (for each leaf block B of w_B columns, row i):
  f0 = log2 ||A(i, B)||^2 - log2 max_i ||A(i, B)||^2
  f1 = log2(l_i m / s), l_i the leverage of row i in the column space of
       Y = A Omega (Omega n x s, s = 2r), here from numpy's QR of Y
  f2 = log2(lb_i m / w_B), lb_i = a_i^T (A_B^T A_B + lambda I)^-1 a_i the ridge
       leverage of row a_i = A(i, B) in the block A_B = A(:, B), with
       lambda = 2^-20 max_j (A_B^T A_B)_jj, here from numpy's solve
  f3 = the 1024-bin histogram rank of f2 within the leaf:
       bin(v) = clamp(floor((v + 64) 1024 / 96), 0, 1023), rank(bin) =
       (rows in higher bins + half the rows in the bin) / m.
Omega's entries come from the counter-based generator `gauss(seed, idx)`:
SplitMix64 of seed ^ 2 idx and seed ^ (2 idx + 1), two 53-bit uniforms,
Box-Muller; the device implements the same published definition.
"""
from __future__ import annotations

import numpy as np

F, H = 4, 128
P_W1, P_B1 = 0, H * F
P_W2 = P_B1 + H
P_B2 = P_W2 + H * H
P_W3 = P_B2 + H
P_B3 = P_W3 + H
NPARAMS = P_B3 + 1

_M64 = (1 << 64) - 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return (p[P_W1:P_B1].reshape(H, F), p[P_B1:P_W2], p[P_W2:P_B2].reshape(H, H), p[P_B2:P_W3],
            p[P_W3:P_B3], float(p[P_B3]))


def device_weights(p):
    """The parameter vector as the device evaluates it: weights rounded to FP16."""
    q = np.asarray(p, dtype=np.float32).astype(np.float64)
    for a, b in ((P_W1, P_B1), (P_W2, P_B2), (P_W3, P_B3)):
        q[a:b] = q[a:b].astype(np.float16).astype(np.float64)
    return q


def forward(p, X):
    """Scores and the hidden activations (pre-activations a1, a2)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    return h2 @ w3 + b3, (a1, h1, a2, h2)


def softplus(x):
    return np.where(x > 0, x + np.log1p(np.exp(-np.abs(x))), np.log1p(np.exp(-np.abs(x))))


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def loss(p, X, y, pw):
    s, _ = forward(p, X)
    y = np.asarray(y, dtype=np.float64)
    return float(np.mean(pw * y * softplus(-s) + (1.0 - y) * softplus(s)))


def grad(p, X, y, pw):
    """Gradient of `loss` by the chain rule, layer by layer (relu'(0) = 0)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = X.shape[0]
    s, (a1, h1, a2, h2) = forward(p, X)
    ds = (-pw * y * sigmoid(-s) + (1.0 - y) * sigmoid(s)) / n
    g = np.zeros(NPARAMS)
    g[P_W3:P_B3] = h2.T @ ds
    g[P_B3] = ds.sum()
    g2 = np.outer(ds, w3) * (a2 > 0)
    g[P_W2:P_B2] = (g2.T @ h1).ravel()
    g[P_B2:P_W3] = g2.sum(axis=0)
    g1 = (g2 @ W2) * (a1 > 0)
    g[P_W1:P_B1] = (g1.T @ X).ravel()
    g[P_B1:P_W2] = g1.sum(axis=0)
    return g


def adam(p, m1, m2, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    m1 = beta1 * m1 + (1.0 - beta1) * g
    m2 = beta2 * m2 + (1.0 - beta2) * g * g
    p = p - lr * (m1 / (1.0 - beta1 ** t)) / (np.sqrt(m2 / (1.0 - beta2 ** t)) + eps)
    return p, m1, m2


# ---------------------------------------------------------------- features
def _splitmix64(x):
    z = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def gauss(seed, count):
    """gauss(seed, idx) for idx = 0 .. count - 1 (Python integers: exact 64-bit arithmetic)."""
    out = np.empty(count)
    for i in range(count):
        a = _splitmix64(seed ^ (2 * i))
        b = _splitmix64(seed ^ (2 * i + 1))
        u1 = ((a >> 11) + 1.0) * 2.0 ** -53
        u2 = (b >> 11) * 2.0 ** -53
        out[i] = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return out


def _bin(v):
    return np.clip(np.floor((v + 64.0) * (1024.0 / 96.0)), 0, 1023).astype(np.int64)


def _rank_table(vals, m):
    cnt = np.bincount(_bin(vals), minlength=1024).astype(np.float64)
    above = np.concatenate([np.cumsum(cnt[::-1])[::-1][1:], [0.0]])
    return (above + 0.5 * cnt) / m


def features(A, r, w, seed):
    """(b m, 4) features, leaf-major, as defined in the module docstring."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    s = 2 * r
    b = max(1, n // w)
    Om = gauss(seed, n * s).reshape(n, s)
    Q, _ = np.linalg.qr(A @ Om)
    lev = (Q * Q).sum(axis=1)
    f1 = np.log2(np.maximum(lev * m / s, 1e-38))
    out = np.zeros((b * m, 4))
    for k in range(b):
        c0, c1 = k * w, (n if k == b - 1 else (k + 1) * w)
        Ab = A[:, c0:c1]
        E = (Ab ** 2).sum(axis=1)
        f0 = np.log2(np.maximum(E, 1e-38)) - np.log2(max(E.max(), 1e-38))
        G = Ab.T @ Ab
        G = G + 2.0 ** -20 * G.diagonal().max() * np.eye(c1 - c0)
        lb = (Ab * np.linalg.solve(G, Ab.T).T).sum(axis=1)
        f2 = np.log2(np.maximum(lb * m / (c1 - c0), 1e-38))
        out[k * m:(k + 1) * m, 0] = f0
        out[k * m:(k + 1) * m, 1] = f1
        out[k * m:(k + 1) * m, 2] = f2
        out[k * m:(k + 1) * m, 3] = _rank_table(f2, m)[_bin(f2)]
    return out
