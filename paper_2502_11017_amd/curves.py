"""Error curves on the closed-form matrices of the paper's experiments
(Sec. 3.1): the Frobenius relative error ||A - CUR||_F / ||A||_F and the
Chebyshev error max |A - CUR| of the library's selections against the rank r,
for the maximal-volume tree and for the norm-greedy method (Alg. 2 with
Alg. 3), in FP64.

    python -m paper_2502_11017_amd.curves [--sizes 256 512 1024] [--rmax 20]

Matrices: Hilbert H(i,j) = 1 / (i + j - 1) and the products of the 1/(i+j)
factors (i, j >= 1, exact rank k).  A selection that stops rank-short (the
matrix is numerically of lower rank than r) is evaluated at the rank it
reached, which is printed.
"""
from __future__ import annotations

import argparse
import sys


def point(A, r: int, method: int):
    """(rank reached, Frobenius relative error, Chebyshev error) of the CUR
    approximation from the library's selection of rank r."""
    import paper_2502_11017_amd as cur

    g = cur.select(A, r, method=method)
    q = r if g["status"] in (cur.OK, cur.WARN_NOCONV) else int(g["rank"])
    if q < 1:
        return 0, 1.0, float(A.abs().max())
    I, J = g["I"][:q].contiguous(), g["J"][:q].contiguous()
    C, U, R = cur.assemble(A, I, J)
    cheb, fro = cur.residual(A, C, U, R)
    return q, fro, cheb


def curves(sizes=(256, 512, 1024), rmax=20, lowrank_k=20, device="cuda:0"):
    """Rows (matrix, n, r, method, rank reached, frobenius, chebyshev)."""
    import torch

    import paper_2502_11017_amd as cur
    from paper_2502_11017_amd import workloads as W

    rows = []
    for n in sizes:
        for name, Ah in (("hilbert", W.hilbert(n)), (f"recip_rank{lowrank_k}", W.recip_lowrank(n, lowrank_k))):
            A = torch.from_numpy(Ah).to(device)
            rs = range(1, rmax + 1) if name == "hilbert" else range(5, rmax + 1)
            for r in rs:
                for mname, method in (("maxvol", cur.METHOD_MAXVOL), ("greedy", cur.METHOD_GREEDY)):
                    q, fro, cheb = point(A, r, method)
                    rows.append((name, n, r, mname, q, fro, cheb))
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(prog="curves")
    ap.add_argument("--sizes", type=int, nargs="+", default=[256, 512, 1024])
    ap.add_argument("--rmax", type=int, default=20)
    a = ap.parse_args(argv)
    print(f"{'matrix':<14} {'n':>5} {'r':>3} {'method':<7} {'rank':>4} {'fro_rel':>11} {'cheb':>11}")
    for name, n, r, m, q, fro, cheb in curves(a.sizes, a.rmax):
        print(f"{name:<14} {n:>5} {r:>3} {m:<7} {q:>4} {fro:>11.3e} {cheb:>11.3e}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
