"""Reduced-precision residual (BF16x3 and two-term FP8 on MFMA, both products
Bm = C U and P = Bm R) against the FP64 CPU oracle, on the tall
low-rank-plus-noise recipe at reduced height.

The GPU selection and assembly give C, U, R; the oracle computes the residual
of the same C, U, R in FP64.  Bounds, from the representations, with
S = max_i sum_k |Bm_ik| ||A||_C and S_CU = max_i sum_k (|C| |U|)_ik ||A||_C
(Bm = C U; |R| <= ||A||_C):
  native: |cheb - cheb_oracle| <= 1e-10 ||A||_C (FP64 arithmetic);
  BF16x3: bf16 has an 8-bit significand, so x = hi + lo + d with
          |d| <= 2^-16 |x|; a product hi hi + hi lo + lo hi misses at most
          3 * 2^-16 |x y| (the two residuals d and the dropped lo lo), and
          r-term FP32 sums of the three products add <= 3 r 2^-24 per term.
          C U carries that error into Bm, splitting the FP32 Bm adds
          2^-16 |Bm|, and Bm R adds the product error again:
          |dE| <= (3 * 2^-16 + 3 r 2^-24) S_CU + (4 * 2^-16 + 3 r 2^-24) S;
  FP8:    e4m3 has a 4-bit significand; the two terms q1 + q2 / 16 represent
          x / s (s = max|tile| / 448) to 2^-8 relative, plus a floor of
          2^-14 s from the subnormals; a product misses <= 3 * 2^-8 |x y|
          plus the floors, so |dE| <= 2^-6 (S + S_CU) covers both products,
          the split of Bm, the floors and the FP32 sums.
The Frobenius ratio is checked against the same bound divided by ||A||_F /
sqrt(m n) (every entry error is below the bound).
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

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def c4_small():
    m, n, r = 8192, 1024, 128
    print(f"case c4 recipe m={m} n={n} r={r} FP32", flush=True)
    A = W.c4(seed=4, device=DEV, m=m, n=n, k=128)
    res = cur.select(A, r)
    assert res["status"] in (0, 1)
    C, U, R = cur.assemble(A, res["I"], res["J"])
    Ah = A.cpu().numpy().astype(np.float64)
    Ch, Uh, Rh = C.cpu().numpy().astype(np.float64), U.cpu().numpy(), R.cpu().numpy().astype(np.float64)
    return A, C, U, R, Ah, Ch, Uh, Rh, r


@pytest.fixture(scope="module")
def oracle_resid(orc, c4_small):
    A, C, U, R, Ah, Ch, Uh, Rh, r = c4_small
    return orc.residual(Ah, Ch, Uh, Rh)


def _scale(c4_small):
    A, C, U, R, Ah, Ch, Uh, Rh, r = c4_small
    amax = float(np.abs(Ah).max())
    S = float(np.abs(Ch @ Uh).sum(axis=1).max()) * amax
    S_cu = float((np.abs(Ch) @ np.abs(Uh)).sum(axis=1).max()) * amax
    return amax, S, S_cu


def mp_bound(prec, r, S, S_cu):
    if prec == cur.PREC_BF16X3:
        return (3 * 2.0**-16 + 3 * r * 2.0**-24) * S_cu + (4 * 2.0**-16 + 3 * r * 2.0**-24) * S
    return 2.0**-6 * (S + S_cu)


def test_native_fp32_input_matches_oracle(c4_small, oracle_resid):
    A, C, U, R, Ah, *_ = c4_small
    amax, _, _ = _scale(c4_small)
    cheb, fro = cur.residual(A, C, U, R)
    ocheb, ofro = oracle_resid
    print(f"native cheb {cheb:.6e} oracle {ocheb:.6e} fro {fro:.6e} oracle {ofro:.6e}", flush=True)
    assert abs(cheb - ocheb) <= 1e-10 * amax
    assert abs(fro - ofro) <= 1e-10 * max(1.0, ofro)


@pytest.mark.parametrize("prec,name", [(cur.PREC_BF16X3, "bf16x3"), (cur.PREC_FP8, "fp8")])
def test_reduced_precision_within_bound(c4_small, oracle_resid, prec, name):
    A, C, U, R, Ah, Ch, Uh, Rh, r = c4_small
    amax, S, S_cu = _scale(c4_small)
    bound = mp_bound(prec, r, S, S_cu)
    cheb, fro = cur.residual(A, C, U, R, prec)
    ocheb, ofro = oracle_resid
    m, n = Ah.shape
    rms_a = float(np.sqrt((Ah * Ah).mean()))
    print(f"{name}: cheb {cheb:.6e} oracle {ocheb:.6e} |d| {abs(cheb - ocheb):.3e} bound {bound:.3e}; "
          f"fro {fro:.6e} oracle {ofro:.6e}", flush=True)
    sys.stdout.flush()
    assert abs(cheb - ocheb) <= bound
    assert abs(fro - ofro) <= bound / rms_a


@pytest.mark.parametrize("m,n,r,pad", [(1000, 515, 40, 0), (3001, 700, 100, 3), (513, 2049, 8, 1),
                                       (1000, 515, 64, 0), (640, 384, 32, 0)])
@pytest.mark.parametrize("prec", [cur.PREC_BF16X3, cur.PREC_FP8])
def test_reduced_precision_ragged(orc, m, n, r, pad, prec):
    """Ragged tiles (m, n not multiples of 128, r not a multiple of 32, r <= 64
    leaving half the column tiles of C U empty) and a leading dimension that is
    not a multiple of 4 (scalar loads of A instead of 16-byte ones), within
    the same bounds against the oracle.  r = 64 and r = 32 (multiples of 32)
    take the untested row blocks of C U, whose strips of U past r repeat the
    last one; 640 x 384 has interior tiles only."""
    Ah = W.gaussian(m, r, 70) @ W.gaussian(r, n, 71) / np.sqrt(r) + 1e-3 * W.gaussian(m, n, 72)
    full = torch.zeros((m, n + pad), dtype=torch.float32, device=DEV)
    full[:, :n] = torch.from_numpy(Ah).to(torch.float32).to(DEV)
    A = full[:, :n]
    rng = np.random.default_rng(73)
    I = torch.from_numpy(np.sort(rng.choice(m, r, replace=False))).to(DEV)
    J = torch.from_numpy(np.sort(rng.choice(n, r, replace=False))).to(DEV)
    print(f"case mp ragged m={m} n={n} r={r} lda={n + pad} prec={prec}", flush=True)
    C, U, R = cur.assemble(A, I, J)
    Ah = A.cpu().numpy().astype(np.float64)
    Ch, Uh, Rh = C.cpu().numpy().astype(np.float64), U.cpu().numpy(), R.cpu().numpy().astype(np.float64)
    ocheb, ofro = orc.residual(Ah, Ch, Uh, Rh)
    amax = float(np.abs(Ah).max())
    S = float(np.abs(Ch @ Uh).sum(axis=1).max()) * amax
    S_cu = float((np.abs(Ch) @ np.abs(Uh)).sum(axis=1).max()) * amax
    bound = mp_bound(prec, r, S, S_cu)
    cheb, fro = cur.residual(A, C, U, R, prec)
    rms_a = float(np.sqrt((Ah * Ah).mean()))
    print(f"  cheb {cheb:.6e} oracle {ocheb:.6e} |d| {abs(cheb - ocheb):.3e} bound {bound:.3e}", flush=True)
    assert abs(cheb - ocheb) <= bound
    assert abs(fro - ofro) <= bound / rms_a
