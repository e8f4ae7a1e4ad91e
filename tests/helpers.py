"""Independent numpy checks used by the tests (no oracle or HIP code here)."""
import itertools

import numpy as np

EPS = 2.0 ** -52


def rand(m, n, seed):
    return np.random.default_rng(seed).standard_normal((m, n))


def brute_force_maxvol(A, r):
    """Exhaustive argmax over all r x r crosses of |det| (Sec. 1.2 objective)."""
    m, n = A.shape
    rows = list(itertools.combinations(range(m), r))
    cols = list(itertools.combinations(range(n), r))
    best, arg = -1.0, None
    for I in rows:
        sub = A[list(I)]
        stack = np.stack([sub[:, list(J)] for J in cols])
        v = np.abs(np.linalg.det(stack))
        k = int(np.argmax(v))
        if v[k] > best:
            best, arg = float(v[k]), (np.array(I), np.array(cols[k]))
    return arg[0], arg[1], best


def row_interp(A, I, J):
    """A(:,J) A(I,J)^{-1} with numpy's LAPACK solve."""
    G = A[np.ix_(I, J)]
    return np.linalg.solve(G.T, A[:, J].T).T


def col_interp(A, I, J, Jc):
    G = A[np.ix_(I, J)]
    return np.linalg.solve(G, A[np.ix_(I, Jc)])


def single_swap_gain(A, I, J, Jc=None):
    """Largest |det| ratio reachable by one row swap (any row) or one column
    swap (within Jc), by brute-force determinants."""
    m, n = A.shape
    r = len(I)
    base = abs(np.linalg.det(A[np.ix_(I, J)]))
    best = 0.0
    for k in range(r):
        for i in range(m):
            if i in I:
                continue
            I2 = I.copy()
            I2[k] = i
            best = max(best, abs(np.linalg.det(A[np.ix_(I2, J)])) / base)
    for k in range(r):
        for j in (Jc if Jc is not None else range(n)):
            if j in J:
                continue
            J2 = J.copy()
            J2[k] = j
            best = max(best, abs(np.linalg.det(A[np.ix_(I, J2)])) / base)
    return best


def cur_error(A, C, U, R):
    return A - C @ U @ R


def root_candidates(trace, r):
    """Candidate columns of the root: sorted union of its children's J."""
    meta = trace["meta"]
    levels = meta[:, 0]
    top = levels.max()
    if top == 0:
        return None
    kids = np.where(levels == top - 1)[0]
    Js = [trace["J"][k][: meta[k, 2]] for k in kids[:2]]
    return np.sort(np.concatenate(Js))


def trace_logvol(trace, k):
    return float(np.log(trace["vol_m"][k]) + trace["meta"][k, 9] * np.log(2.0))
