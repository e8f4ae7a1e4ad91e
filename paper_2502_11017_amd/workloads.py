"""Seeded synthetic inputs for the CUR selection path.

This module only draws random numbers and builds test matrices from them; it
holds none of the selection, assembly or residual arithmetic, so both the HIP
path and the CPU oracle can consume its outputs.

The paper measures on closed-form matrices (Hilbert matrices and products of
1/(i+j) factors, Sec. 3.1) and on an unspecified 16384^2 matrix (Sec. 3.2);
there is no public dataset.  The workloads below are the synthetic spectra the
benchmarks of this library are defined on:

``spectral(m, n, s, seed)``
    A = Q1 diag(s) Q2^T, Q1 (m x k) and Q2 (n x k) the Q factors (signs fixed
    so that diag(R) > 0) of seeded standard Gaussian matrices, k = len(s).
    Random stream: ``numpy.random.default_rng(seed)`` draws G1 (m x k), then
    G2 (n x k), then (if ``noise`` > 0) the m x n noise matrix, whose entries
    are multiplied by ``noise`` (a standard deviation).

Named configurations (all sizes as stated):
  * ``c1``: 512 x 512, s_i = 2^-i (i < 16), 1e-8 * 2^-(i-16) (16 <= i < 512).
  * ``c2``: 8192 x 8192, s_i = 0.9^i (i < 64), 1e-6 afterwards, plus i.i.d.
    Gaussian noise of standard deviation 1e-7.
  * ``c3``: batch of matrices, m, n uniform in [256, 4096], r uniform in
    {8, 16, 32, 64}, s_i = q^i with q uniform in [0.8, 0.95].
  * ``c4``: 1,048,576 x 1024 FP32, G1 (m x 128) G2 (128 x n) with entries of
    variance 1/128 plus noise of standard deviation 1e-4.
  * ``c5_train(seed)``: the training matrices of the learned proposal, the c2
    construction at 4096 x 4096 with the flat 1e-6 floor of the spectrum
    replaced by i.i.d. Gaussian entries of the same size (standard deviation
    1e-6 / sqrt(n), whose singular values spread over [0, 2e-6]) merged with
    the noise of standard deviation 1e-7: only the 64 leading directions need
    Q factors (two reduced QRs of n x 64 instead of two full n x n ones), so
    the matrices can be generated as they are consumed.
  * ``hilbert(n)``: H(i,j) = 1/(i+j-1), 1-based (Sec. 3.1).
  * ``recip_lowrank(n, r)``: H = A B with A(i,j) = B(i,j) = 1/(i+j), 1-based,
    A n x r, B r x n (Sec. 3.1).
The QR factorisations and the products run with torch on ``device`` (the GPU
when given one), so the bits of a generated matrix depend on that device; any
comparison against the oracle uses a host copy of the same tensor.
"""
from __future__ import annotations

import numpy as np
import torch


def _haar_q(G: torch.Tensor) -> torch.Tensor:
    Q, R = torch.linalg.qr(G, mode="reduced")
    d = torch.sign(torch.diagonal(R))
    d = torch.where(d == 0, torch.ones_like(d), d)
    return Q * d.unsqueeze(0)


def spectral(m: int, n: int, s, seed: int, noise: float = 0.0, device="cpu",
             dtype=torch.float64) -> torch.Tensor:
    s = np.asarray(s, dtype=np.float64)
    k = len(s)
    rng = np.random.default_rng(seed)
    dev = torch.device(device)
    G1 = torch.from_numpy(rng.standard_normal((m, k))).to(dev)
    G2 = torch.from_numpy(rng.standard_normal((n, k))).to(dev)
    Q1 = _haar_q(G1)
    del G1
    Q2 = _haar_q(G2)
    del G2
    A = (Q1 * torch.from_numpy(s).to(dev).unsqueeze(0)) @ Q2.T
    del Q1, Q2
    if noise > 0.0:
        rows = max(1, (1 << 24) // n)
        for i0 in range(0, m, rows):
            i1 = min(m, i0 + rows)
            N = torch.from_numpy(rng.standard_normal((i1 - i0, n))).to(dev)
            A[i0:i1] += noise * N
    return A.to(dtype).contiguous()


def c1_spectrum(n: int = 512) -> np.ndarray:
    i = np.arange(n, dtype=np.float64)
    return np.where(i < 16, 2.0 ** (-i), 1e-8 * 2.0 ** (-(i - 16)))


def c2_spectrum(n: int = 8192) -> np.ndarray:
    i = np.arange(n, dtype=np.float64)
    return np.where(i < 64, 0.9 ** i, 1e-6)


def c1(seed: int = 1, device="cpu", dtype=torch.float64) -> torch.Tensor:
    return spectral(512, 512, c1_spectrum(512), seed, 0.0, device, dtype)


def c2(seed: int = 2, device="cpu", dtype=torch.float64, n: int = 8192) -> torch.Tensor:
    """C2 construction; ``n`` < 8192 gives the same recipe at a smaller size."""
    return spectral(n, n, c2_spectrum(n), seed, 1e-7, device, dtype)


def c3_specs(seed: int = 3, count: int = 256, lo: int = 256, hi: int = 4096):
    """Per-matrix (m, n, r, q, item_seed) for the uneven batch."""
    rng = np.random.default_rng(seed)
    out = []
    for idx in range(count):
        m = int(rng.integers(lo, hi + 1))
        n = int(rng.integers(lo, hi + 1))
        r = int(rng.choice([8, 16, 32, 64]))
        q = float(rng.uniform(0.8, 0.95))
        out.append((m, n, r, q, seed * 1_000_003 + idx))
    return out


def c3_matrix(spec, device="cpu", dtype=torch.float32) -> torch.Tensor:
    m, n, r, q, s = spec
    k = min(m, n)
    return spectral(m, n, q ** np.arange(k, dtype=np.float64), s, 0.0, device, dtype)


def c4(seed: int = 4, device="cpu", m: int = 1 << 20, n: int = 1024, k: int = 128,
       noise: float = 1e-4) -> torch.Tensor:
    """Tall FP32 low-rank-k product plus noise (generated in row chunks)."""
    rng = np.random.default_rng(seed)
    dev = torch.device(device)
    G2 = torch.from_numpy(rng.standard_normal((k, n)) / np.sqrt(k)).to(dev)
    A = torch.empty((m, n), dtype=torch.float32, device=dev)
    rows = max(1, (1 << 22) // n)
    for i0 in range(0, m, rows):
        i1 = min(m, i0 + rows)
        G1 = torch.from_numpy(rng.standard_normal((i1 - i0, k)) / np.sqrt(k)).to(dev)
        N = torch.from_numpy(rng.standard_normal((i1 - i0, n))).to(dev)
        A[i0:i1] = (G1 @ G2 + noise * N).to(torch.float32)
    return A


def c5_train(seed: int, device="cpu", n: int = 4096, dtype=torch.float64) -> torch.Tensor:
    rng = np.random.default_rng(seed)
    dev = torch.device(device)
    s = torch.from_numpy(0.9 ** np.arange(64, dtype=np.float64)).to(dev)
    Q1 = _haar_q(torch.from_numpy(rng.standard_normal((n, 64))).to(dev))
    Q2 = _haar_q(torch.from_numpy(rng.standard_normal((n, 64))).to(dev))
    sd = float(np.sqrt(1e-14 + 1e-12 / n))
    A = (Q1 * s.unsqueeze(0)) @ Q2.T
    A += sd * torch.from_numpy(rng.standard_normal((n, n))).to(dev)
    return A.to(dtype)


def hilbert(n: int) -> np.ndarray:
    i = np.arange(1, n + 1, dtype=np.float64)
    return 1.0 / (i[:, None] + i[None, :] - 1.0)


def recip_lowrank(n: int, r: int) -> np.ndarray:
    i = np.arange(1, n + 1, dtype=np.float64)
    k = np.arange(1, r + 1, dtype=np.float64)
    Af = 1.0 / (i[:, None] + k[None, :])
    Bf = 1.0 / (k[:, None] + i[None, :])
    return Af @ Bf


def gaussian(m: int, n: int, seed: int, dtype=np.float64) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal((m, n)).astype(dtype)
