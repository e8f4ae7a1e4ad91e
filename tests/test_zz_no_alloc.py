"""The residual entry point that allocates nothing (cur_residual_noalloc):
through the C ABI, its results equal cur_residual's (same kernels, so
bit-identical; the bar is the residual tolerance 1e-10 ||A||_C), on two calls
in a row, the second with a smaller input, in every precision form."""
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


def _factors(m, n, r, seed, dt):
    Ah = W.gaussian(m, r, seed) @ W.gaussian(r, n, seed + 1) + 1e-3 * W.gaussian(m, n, seed + 2)
    A = torch.from_numpy(Ah).to(dt).to(DEV)
    rng = np.random.default_rng(seed)
    I = torch.from_numpy(np.sort(rng.choice(m, r, replace=False))).to(DEV)
    J = torch.from_numpy(np.sort(rng.choice(n, r, replace=False))).to(DEV)
    C, U, R = cur.assemble(A, I, J)
    return A, C, U, R


@pytest.mark.parametrize("dt,prec", [(torch.float64, cur.PREC_NATIVE), (torch.float32, cur.PREC_NATIVE),
                                     (torch.float32, cur.PREC_BF16X3), (torch.float32, cur.PREC_FP8)])
def test_noalloc_residual_equals_residual(dt, prec):
    for (m, n, r, seed) in [(3000, 2100, 48, 40), (700, 515, 20, 43)]:  # second call smaller
        print(f"case noalloc {dt} prec={prec} m={m} n={n} r={r}", flush=True)
        sys.stdout.flush()
        A, C, U, R = _factors(m, n, r, seed, dt)
        cheb0, fro0 = cur.residual(A, C, U, R, prec)
        cheb1, fro1 = cur.residual_noalloc(A, C, U, R, prec)
        amax = float(A.abs().max())
        assert abs(cheb1 - cheb0) <= 1e-10 * amax, (cheb1, cheb0)
        assert abs(fro1 - fro0) <= 1e-10, (fro1, fro0)
        assert cheb1 == cheb0 and fro1 == fro0  # same kernels, same order


def test_noalloc_rejects_calls_beyond_its_scratch():
    A, C, U, R = _factors(300, 200, 8, 50, torch.float64)
    big = torch.empty((40000, 64), dtype=torch.float64, device=DEV)  # 8 m r = 20 MB > 16 MiB
    with pytest.raises(cur.CurError) as ei:
        cur.residual_noalloc(big, big[:, :64], torch.eye(64, dtype=torch.float64, device=DEV), big[:64])
    assert ei.value.status == cur.ERR_ARG and "CUR_NOALLOC_SCRATCH_BYTES" in str(ei.value)
    cheb0, _ = cur.residual(A, C, U, R)
    cheb1, _ = cur.residual_noalloc(A, C, U, R)
    assert cheb1 == cheb0
