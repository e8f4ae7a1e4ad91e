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


def greedy_margin_bound(t, length):
    """Rounding bound on the margin (best - runner-up squared norm, relative to
    the largest initial squared norm) below which two evaluation orders of the
    norm-greedy rule may choose differently at step t: each of the t + 1
    projections and norms so far sums `length` products, each sum rounding by
    at most length * 2^-52 of the squared norms involved; the factor 4 is the
    margin taken over that first-order estimate."""
    return 4.0 * (t + 1) * length * EPS


def greedy_first_near_tie(gaps, q, length):
    """First step (< q) whose margin is within greedy_margin_bound, else q."""
    for t in range(q):
        if not gaps[t] > greedy_margin_bound(t, length):
            return t
    return q


def read_tree_golden(path):
    """Cases of tests/golden/tree_shape.txt: dicts with A, r, w, nodes
    [(level, index, promoted, I, J)], root (I, J) and logvol."""
    cases, cur = [], None
    with open(path) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "case":
                kv = dict(zip(t[2::2], (int(x) for x in t[3::2])))
                cur = {"name": t[1], "A": np.zeros((kv["m"], kv["n"])), "r": kv["r"], "w": kv["w"],
                       "nodes": []}
            elif t[0] == "entry":
                cur["A"][int(t[1]), int(t[2])] = float(t[3])
            elif t[0] == "node":
                r = cur["r"]
                v = [int(x) for x in t[1:]]
                cur["nodes"].append((v[0], v[1], v[2], v[3:3 + r], v[3 + r:3 + 2 * r]))
            elif t[0] == "root":
                r = cur["r"]
                cur["root"] = ([int(x) for x in t[1:1 + r]], [int(x) for x in t[1 + r:1 + 2 * r]])
                cur["logvol"] = float(t[-1])
            elif t[0] == "end":
                cases.append(cur)
    return cases


def check_tree_golden(case, I, J, trace, logvol):
    """Compare one selection (root I, J, its per-node trace and log-volume)
    with a golden tree case."""
    meta = trace["meta"]
    assert len(meta) == len(case["nodes"]), (len(meta), len(case["nodes"]))
    for k, (lev, idx, prom, nI, nJ) in enumerate(case["nodes"]):
        assert (meta[k, 0], meta[k, 1], meta[k, 4]) == (lev, idx, prom), (k, meta[k, :5])
        assert sorted(trace["I"][k]) == nI and sorted(trace["J"][k]) == nJ, (k, trace["I"][k], trace["J"][k])
    assert list(I) == case["root"][0] and list(J) == case["root"][1]
    assert abs(logvol - case["logvol"]) <= 1e-14 * abs(case["logvol"])
