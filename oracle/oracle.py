"""ctypes front end of the FP64 CPU oracle (``cur_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  Nothing here is
imported by the HIP library or its Python binding.

FP32 inputs are upcast to FP64 exactly before they reach the C code, so the
oracle of an FP32 matrix is the oracle of its exact FP64 value.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cur_oracle.c")
LIB = os.path.join(HERE, "libcur_oracle.so")

OK, WARN_NOCONV = 0, 1
ERR_ARG, ERR_RANK, ERR_NONFINITE, ERR_NOMEM, ERR_INTERNAL = -1, -2, -3, -5, -6
TRACE_META = 10
TRACE_FIELDS = ("level", "index", "q", "short", "promoted", "nocap", "swaps", "phases",
                "refreshes", "vol_e")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, explicit fma, no contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-mfma", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
               "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", LIB, SRC, "-lm"]
        subprocess.check_call(cmd)
    return LIB


class _Info(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("nodes", ctypes.c_int32), ("phases", ctypes.c_int32),
                ("refreshes", ctypes.c_int32), ("swaps", ctypes.c_int64), ("logvol", ctypes.c_double),
                ("status", ctypes.c_int32), ("pad", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.oracle_gepp.argtypes = [i32, P, P]
        L.oracle_gepp.restype = i32
        L.oracle_lu_inverse.argtypes = [i32, P, P, P]
        L.oracle_lu_inverse.restype = None
        L.oracle_volume.argtypes = [i32, P, P, P]
        L.oracle_volume.restype = None
        L.oracle_aca.argtypes = [P, i64, i64, P, i32, i32, dbl, P, P, P]
        L.oracle_aca.restype = i32
        L.oracle_swap_loop.argtypes = [P, i64, i64, i64, i32, P, P, P, i32, dbl, i32, P]
        L.oracle_swap_loop.restype = i32
        L.oracle_tree_size.argtypes = [i64]
        L.oracle_tree_size.restype = i32
        L.oracle_cur_select.argtypes = [P, i64, i64, i64, i32, i32, dbl, i32, P, P, P, P, P, P, P]
        L.oracle_cur_select.restype = i32
        L.oracle_cur_select_polish.argtypes = [P, i64, i64, i64, i32, i32, dbl, i32, P, P, P, P, P, P, P]
        L.oracle_cur_select_polish.restype = i32
        L.oracle_cur_select_theta.argtypes = [P, i64, i64, i64, i32, i32, dbl, i32, dbl, P, P, P]
        L.oracle_cur_select_theta.restype = i32
        L.oracle_sm_row_update.argtypes = [P, i64, i32, i64, i32, P]
        L.oracle_sm_row_update.restype = None
        L.oracle_sm_col_update.argtypes = [P, i32, i32, i32, i32, P, P]
        L.oracle_sm_col_update.restype = None
        L.oracle_pinv.argtypes = [i32, P, P]
        L.oracle_pinv.restype = None
        L.oracle_cur_assemble.argtypes = [P, i64, i64, i64, i32, P, P, P, P, P, P]
        L.oracle_cur_assemble.restype = i32
        L.oracle_cur_residual.argtypes = [P, i64, i64, i64, i32, P, P, P, P, P]
        L.oracle_cur_residual.restype = i32
        L.oracle_greedy_select.argtypes = [P, i64, i64, i64, i32, P, P, P, P, P, P, P, P]
        L.oracle_greedy_select_rc.argtypes = [P, i64, i64, i64, i32, i32, P, P, P, P, P, P, P, P]
        L.oracle_greedy_select_rc.restype = i32
        L.oracle_pinv_rect.argtypes = [i32, i32, P, P]
        L.oracle_pinv_rect.restype = None
        L.oracle_cur_assemble_rect.argtypes = [P, i64, i64, i64, i32, i32, P, P, P, P, P]
        L.oracle_cur_assemble_rect.restype = i32
        L.oracle_cur_residual_rect.argtypes = [P, i64, i64, i64, i32, i32, P, P, P, P, P]
        L.oracle_cur_residual_rect.restype = i32
        L.oracle_greedy_select.restype = i32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(A) -> np.ndarray:
    A = np.asarray(A)
    if A.dtype != np.float64:
        A = A.astype(np.float64)  # exact for float32 input
    return np.ascontiguousarray(A)


def gepp(G):
    """LU with partial pivoting; returns (LU, perm, ok)."""
    G = _f64(G).copy()
    r = G.shape[0]
    perm = np.zeros(r, dtype=np.int32)
    rc = lib().oracle_gepp(r, _p(G), _p(perm))
    return G, perm, rc == 0


def inverse(G):
    LU, perm, ok = gepp(G)
    if not ok:
        raise ZeroDivisionError("singular")
    r = LU.shape[0]
    X = np.zeros((r, r))
    lib().oracle_lu_inverse(r, _p(LU), _p(perm), _p(X))
    return X


def volume(G):
    """(mant, expo, log|det|) of the square G; log is -inf if singular."""
    LU, perm, ok = gepp(G)
    if not ok:
        return 0.0, 0, -np.inf
    m = ctypes.c_double()
    e = ctypes.c_int()
    lib().oracle_volume(LU.shape[0], _p(LU), ctypes.byref(m), ctypes.byref(e))
    return m.value, e.value, float(np.log(m.value) + e.value * np.log(2.0))


def logvol(A, I, J):
    A = np.asarray(A)
    return volume(A[np.ix_(np.asarray(I), np.asarray(J))])[2]


def aca(A, r, cols=None, theta=None):
    A = _f64(A)
    m, n = A.shape
    cols = np.arange(n, dtype=np.int64) if cols is None else np.ascontiguousarray(cols, dtype=np.int64)
    if theta is None:
        theta = max(m, n) * 2.0 ** -52 * float(np.abs(A).max())
    I = np.full(r, -1, dtype=np.int64)
    J = np.full(r, -1, dtype=np.int64)
    piv = np.zeros(r)
    q = lib().oracle_aca(_p(A), m, n, _p(cols), len(cols), r, float(theta), _p(I), _p(J), _p(piv))
    return I[:q], J[:q], piv[:q]


def swap_loop(A, I, J, Jc, tau=1e-13, smax=None):
    A = _f64(A)
    m, n = A.shape
    r = len(I)
    I = np.ascontiguousarray(I, dtype=np.int64).copy()
    J = np.ascontiguousarray(J, dtype=np.int64).copy()
    Jc = np.ascontiguousarray(np.sort(np.asarray(Jc, dtype=np.int64)))
    st = np.zeros(5, dtype=np.int32)
    rc = lib().oracle_swap_loop(_p(A), m, n, n, r, _p(I), _p(J), _p(Jc), len(Jc), float(tau),
                                64 * r if smax is None else int(smax), _p(st))
    return I, J, {"status": rc, "swaps": int(st[0]), "phases": int(st[1]),
                  "refreshes": int(st[2]), "nocap": int(st[3])}


def n_leaves(n: int, w: int) -> int:
    return max(1, n // w)


def select(A, r, w=0, tau=0.0, max_swaps=0, trace=False, polish=False):
    """Full partition-and-merge selection (with polish: then the swap loop on
    all columns from the root's cross, oracle_cur_select_polish). Returns dict
    with I, J, status, info (+trace)."""
    A = _f64(A)
    m, n = A.shape
    I = np.full(r, -1, dtype=np.int64)
    J = np.full(r, -1, dtype=np.int64)
    info = _Info()
    ww = w if w else max(64, r)
    args = [None, None, None, None]
    if trace and ww >= r:
        N = lib().oracle_tree_size(n_leaves(n, ww)) + (1 if polish else 0)
        tm = np.full((N, TRACE_META), -1, dtype=np.int64)  # rows left at level -1 were not written
        tv = np.zeros(N)
        tI = np.zeros((N, r), dtype=np.int64)
        tJ = np.zeros((N, r), dtype=np.int64)
        args = [_p(tm), _p(tv), _p(tI), _p(tJ)]
    fn = lib().oracle_cur_select_polish if polish else lib().oracle_cur_select
    rc = fn(_p(A), m, n, n, r, int(w), float(tau), int(max_swaps), _p(I), _p(J), ctypes.byref(info), *args)
    out = {"status": rc, "I": I, "J": J, "rank": info.rank, "nodes": info.nodes,
           "phases": info.phases, "refreshes": info.refreshes, "swaps": info.swaps,
           "logvol": info.logvol}
    if trace and ww >= r:
        k = int(np.count_nonzero(tm[:, 0] >= 0))  # records are written in order
        out["trace"] = {"meta": tm[:k], "vol_m": tv[:k], "I": tI[:k], "J": tJ[:k]}
    return out


def select_theta(A, r, theta_rel, w=0, tau=0.0, max_swaps=0):
    """The selection with pivot threshold theta_rel * max|A| (see
    oracle_cur_select_theta); dict with status, rank, I, J."""
    A = _f64(A)
    m, n = A.shape
    I = np.full(r, -1, dtype=np.int64)
    J = np.full(r, -1, dtype=np.int64)
    info = _Info()
    rc = lib().oracle_cur_select_theta(_p(A), m, n, n, r, int(w), float(tau), int(max_swaps), float(theta_rel),
                                       _p(I), _p(J), ctypes.byref(info))
    return {"status": rc, "I": I, "J": J, "rank": info.rank, "logvol": info.logvol}


def sm_row_update(B, i, k):
    B = _f64(B).copy()
    m, r = B.shape
    v = np.zeros(r)
    lib().oracle_sm_row_update(_p(B), m, r, int(i), int(k), _p(v))
    return B


def sm_col_update(Bc, k, c):
    Bc = _f64(Bc).copy()
    r, nc = Bc.shape
    w = np.zeros(r)
    rowk = np.zeros(nc)
    lib().oracle_sm_col_update(_p(Bc), r, nc, int(k), int(c), _p(w), _p(rowk))
    return Bc


def pinv(G):
    G = _f64(G)
    r = G.shape[0]
    P = np.zeros((r, r))
    lib().oracle_pinv(r, _p(G), _p(P))
    return P


def assemble(A, I, J):
    A = _f64(A)
    m, n = A.shape
    I = np.ascontiguousarray(I, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.int64)
    r = len(I)
    C = np.zeros((m, r))
    U = np.zeros((r, r))
    R = np.zeros((r, n))
    used = ctypes.c_int()
    rc = lib().oracle_cur_assemble(_p(A), m, n, n, r, _p(I), _p(J), _p(C), _p(U), _p(R),
                                   ctypes.byref(used))
    if rc != OK:
        raise ValueError(f"oracle_cur_assemble: {rc}")
    return C, U, R, bool(used.value)


def residual(A, C, U, R):
    A = _f64(A)
    C, U, R = _f64(C), _f64(U), _f64(R)
    m, n = A.shape
    r = U.shape[0]
    cheb = ctypes.c_double()
    fro = ctypes.c_double()
    rc = lib().oracle_cur_residual(_p(A), m, n, n, r, _p(C), _p(U), _p(R), ctypes.byref(cheb),
                                   ctypes.byref(fro))
    if rc != OK:
        raise ValueError(f"oracle_cur_residual: {rc}")
    return cheb.value, fro.value


def residual_raw(A, C, U, R):
    """(status, cheb, fro_rel) without raising: status ERR_NONFINITE (and cheb
    NaN) when A - C U R has a non-finite entry."""
    A = _f64(A)
    C, U, R = _f64(C), _f64(U), _f64(R)
    m, n = A.shape
    cheb = ctypes.c_double()
    fro = ctypes.c_double()
    rc = lib().oracle_cur_residual(_p(A), m, n, n, U.shape[0], _p(C), _p(U), _p(R), ctypes.byref(cheb),
                                   ctypes.byref(fro))
    return rc, cheb.value, fro.value


def select_raw(A, r, w=0, tau=0.0, max_swaps=0):
    """Status code only (for the error-path tests); A may be any float64 array."""
    A = _f64(A)
    m, n = A.shape
    I = np.full(max(r, 1), -1, dtype=np.int64)
    J = np.full(max(r, 1), -1, dtype=np.int64)
    info = _Info()
    rc = lib().oracle_cur_select(_p(A), m, n, n, r, int(w), float(tau), int(max_swaps), _p(I), _p(J),
                                 ctypes.byref(info), None, None, None, None)
    return rc, info, I, J


def greedy(A, r):
    """Norm-greedy selection of rows and columns (Alg. 2 with Alg. 3), see
    oracle_greedy_select: choice orders, ascending I and J, status, ranks, and
    each step's margin (best - runner-up squared norm) / (largest initial
    squared norm) as gap_I / gap_J (NaN past the rank reached)."""
    A = _f64(A)
    m, n = A.shape
    oI = np.full(r, -1, np.int64)
    oJ = np.full(r, -1, np.int64)
    I = np.full(r, -1, np.int64)
    J = np.full(r, -1, np.int64)
    qr = ctypes.c_int(0)
    qc = ctypes.c_int(0)
    gI = np.full(r, np.nan)
    gJ = np.full(r, np.nan)
    st = lib().oracle_greedy_select(_p(A), m, n, n, r, _p(oI), _p(oJ), _p(I), _p(J), ctypes.byref(qr),
                                    ctypes.byref(qc), _p(gI), _p(gJ))
    if st == ERR_ARG:
        raise ValueError("oracle_greedy_select: invalid argument")
    return {"order_I": oI, "order_J": oJ, "I": I, "J": J, "status": st, "rank_rows": qr.value,
            "rank_cols": qc.value, "gap_I": gI, "gap_J": gJ}


# ---------------------------------------------------------------- rectangular cross (r rows, c columns)
def pinv_rect(G):
    """G^+ (q x p) of the p x q G by oracle_pinv_rect."""
    G = _f64(G)
    p, q = G.shape
    P = np.zeros((q, p))
    lib().oracle_pinv_rect(p, q, _p(G), _p(P))
    return P


def assemble_rect(A, I, J):
    """C = A(:,J) (m x c), U = A(I,J)^+ (c x r), R = A(I,:) (r x n)."""
    A = _f64(A)
    m, n = A.shape
    I = np.ascontiguousarray(I, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.int64)
    r, c = len(I), len(J)
    C, U, R = np.zeros((m, c)), np.zeros((c, r)), np.zeros((r, n))
    rc = lib().oracle_cur_assemble_rect(_p(A), m, n, n, r, c, _p(I), _p(J), _p(C), _p(U), _p(R))
    if rc != OK:
        raise ValueError(f"oracle_cur_assemble_rect: {rc}")
    return C, U, R


def residual_rect(A, C, U, R):
    """(cheb, fro_rel) of A - (C U) R for C m x c, U c x r, R r x n."""
    A, C, U, R = _f64(A), _f64(C), _f64(U), _f64(R)
    m, n = A.shape
    c, r = U.shape
    cheb, fro = ctypes.c_double(), ctypes.c_double()
    rc = lib().oracle_cur_residual_rect(_p(A), m, n, n, r, c, _p(C), _p(U), _p(R), ctypes.byref(cheb),
                                        ctypes.byref(fro))
    if rc not in (OK, ERR_NONFINITE):
        raise ValueError(f"oracle_cur_residual_rect: {rc}")
    return cheb.value, fro.value


def greedy_rc(A, r, c):
    """Norm-greedy rows (r) and columns (c), oracle_greedy_select_rc."""
    A = _f64(A)
    m, n = A.shape
    oI, I = np.full(r, -1, np.int64), np.full(r, -1, np.int64)
    oJ, J = np.full(c, -1, np.int64), np.full(c, -1, np.int64)
    qr, qc = ctypes.c_int(0), ctypes.c_int(0)
    gI, gJ = np.full(r, np.nan), np.full(c, np.nan)
    st = lib().oracle_greedy_select_rc(_p(A), m, n, n, r, c, _p(oI), _p(oJ), _p(I), _p(J), ctypes.byref(qr),
                                       ctypes.byref(qc), _p(gI), _p(gJ))
    if st == ERR_ARG:
        raise ValueError("oracle_greedy_select_rc: invalid argument")
    return {"order_I": oI, "order_J": oJ, "I": I, "J": J, "status": st, "rank_rows": qr.value,
            "rank_cols": qc.value, "gap_I": gI, "gap_J": gJ}


def _worse(a, b):
    """The combined status of two selections: a rank shortfall, then a spent
    swap budget, then OK."""
    for s in (ERR_RANK, WARN_NOCONV):
        if s in (a, b):
            return s
    return a if a != OK else b


def select_rect(A, r, c, method=0, w=0, tau=0.0, max_swaps=0, polish=False):
    """Alg. 2 with separate counts: I (r rows) and J (c columns) chosen
    independently, each along its own axis.  method 0: J by the column-block
    maximal-volume tree on A with rank c, I by the same tree on A^T (row
    blocks of A) with rank r -- each tree's other index set is dropped;
    method 1: the norm-greedy rule on rows and on columns (greedy_rc).
    polish (method 0, r == c): then the swap loop on the cross (I, J) with
    every column a candidate (oracle_swap_loop), so that the square cross
    meets Sec. 1.1's dominance condition on all of A; skipped when either
    tree is rank-short or failed."""
    A = _f64(A)
    if method == 1:
        g = greedy_rc(A, r, c)
        return {"I": g["I"], "J": g["J"], "status": g["status"], "greedy": g}
    cols = select(A, c, w=w, tau=tau, max_swaps=max_swaps)
    rows = select(np.ascontiguousarray(A.T), r, w=w, tau=tau, max_swaps=max_swaps)
    out = {"I": rows["J"], "J": cols["J"], "status": _worse(rows["status"], cols["status"]),
           "rows": rows, "cols": cols}
    if polish and r == c and out["status"] in (OK, WARN_NOCONV):
        n = A.shape[1]
        I, J, st = swap_loop(A, out["I"], out["J"], np.arange(n), tau=tau if tau else 1e-13,
                             smax=max_swaps if max_swaps else 64 * r)
        out["polish"] = st
        out["I"], out["J"] = I, J
        out["status"] = _worse(out["status"], st["status"])
        out["logvol"] = logvol(A, I, J)
    return out
