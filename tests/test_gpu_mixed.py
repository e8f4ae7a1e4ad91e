"""Reduced-precision residual (BF16x3 and two-term FP8 on MFMA) against the
FP64 CPU oracle, on the tall low-rank-plus-noise recipe at reduced height.

The GPU selection (FP32 path) and assembly give C, U, R; the oracle computes
the residual of the same C, U, R in FP64.  Bounds, from the representations:
with S = max_i sum_k |Bm_ik| * ||A||_C (Bm = C U; |R| <= ||A||_C),
  native: |cheb - cheb_oracle| <= 1e-10 ||A||_C (FP64 arithmetic);
  BF16x3: each factor is hi + lo with |x - hi - lo| <= 2^-17 |x|, the dropped
          lo*lo term is <= 2^-16 |xy|, and the FP32 sums add <= 3 r 2^-24 per
          term, so |dE| <= (3 * 2^-17 + 3 r 2^-24) S;
  FP8:    two e4m3 terms represent x / s to 2^-8 relative (plus the 2^-9 s
          subnormal floor), the dropped q2 q2 / 256 term is below 2^-8, so
          |dE| <= 2^-6 S covers the products and the FP32 sums.
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
    return amax, S


def test_native_fp32_input_matches_oracle(c4_small, oracle_resid):
    A, C, U, R, Ah, *_ = c4_small
    amax, _ = _scale(c4_small)
    cheb, fro = cur.residual(A, C, U, R)
    ocheb, ofro = oracle_resid
    print(f"native cheb {cheb:.6e} oracle {ocheb:.6e} fro {fro:.6e} oracle {ofro:.6e}", flush=True)
    assert abs(cheb - ocheb) <= 1e-10 * amax
    assert abs(fro - ofro) <= 1e-10 * max(1.0, ofro)


@pytest.mark.parametrize("prec,name", [(cur.PREC_BF16X3, "bf16x3"), (cur.PREC_FP8, "fp8")])
def test_reduced_precision_within_bound(c4_small, oracle_resid, prec, name):
    A, C, U, R, Ah, Ch, Uh, Rh, r = c4_small
    amax, S = _scale(c4_small)
    bound = (3 * 2.0**-17 + 3 * r * 2.0**-24) * S if prec == cur.PREC_BF16X3 else 2.0**-6 * S
    cheb, fro = cur.residual(A, C, U, R, prec)
    ocheb, ofro = oracle_resid
    m, n = Ah.shape
    rms_a = float(np.sqrt((Ah * Ah).mean()))
    print(f"{name}: cheb {cheb:.6e} oracle {ocheb:.6e} |d| {abs(cheb - ocheb):.3e} bound {bound:.3e}; "
          f"fro {fro:.6e} oracle {ofro:.6e}", flush=True)
    sys.stdout.flush()
    assert abs(cheb - ocheb) <= bound
    assert abs(fro - ofro) <= bound / rms_a
