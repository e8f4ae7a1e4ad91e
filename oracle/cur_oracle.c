/*
 * cur_oracle.c -- plain, slow, single-threaded FP64 CPU oracle for the
 * partition-and-merge maximal-volume CUR selection, assembly and residual.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's cpu_baseline leg may load or call this file.  It shares no code,
 * header, table or helper with the HIP library, and the HIP library never
 * loads it.
 *
 * What it follows (arXiv 2502.11017, "Scalable Binary CUR Low-Rank
 * Approximation Algorithm"):
 *   - CUR form C = A(:,J), U = A(I,J)^+, R = A(I,:)              (Sec. 1.1)
 *   - volume = |det| of the r x r cross                          (Def. 1)
 *   - maximal-volume objective                                    (Sec. 1.2)
 *   - Chebyshev-norm residual, Theorem 1 bound (r+1) sigma_{r+1}   (Thm 1, 2)
 *   - Adaptive Cross Approximation with complete pivoting         (Alg. 1)
 *   - column blocks, per-block local maxima, global maximum        (Alg. 3)
 *   - Frobenius relative error                                     (Sec. 3.1)
 *   - rectangular cross: r rows, c columns chosen independently,
 *     U = A(I,J)^+ (c x r)                          (Alg. 2 inputs, Sec. 1.1)
 * The maxvol swap rule itself is only cited by the paper (Sec. 1.2, the
 * maximal-volume reference); it is written here from the Sherman-Morrison
 * identity.  The binary-tree merge is the partition-and-merge reading of the
 * word "binary" in the title and in the overview of Sec. 2.1.
 *
 * Every multiply-add is an explicit fma() so the operation sequence is fully
 * stated; the file must be built with -ffp-contract=off.  Scan orders and
 * tie rules are part of the algorithm and are documented at each argmax.
 *
 * Parity status: every exported function is pinned by tests/test_oracle_*.py
 * (library routines, closed forms, brute force, invariants).  The particular
 * local optimum reached by the swap loop and the tree on large random inputs
 * has no independent pin ("parity unpinned"); it is the reference by
 * definition of the algorithm.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_WARN_NOCONV 1
#define ORC_ERR_ARG (-1)
#define ORC_ERR_RANK (-2)
#define ORC_ERR_NONFINITE (-3)
#define ORC_ERR_NOMEM (-5)
#define ORC_ERR_INTERNAL (-6)

#define TRACE_META 10 /* level,index,q,short,promoted,nocap,swaps,phases,refreshes,vol_e */

typedef struct {
  int32_t rank, nodes, phases, refreshes;
  int64_t swaps;
  double logvol;
  int32_t status, pad;
} orc_info;

/* ------------------------------------------------------------------------ */
/* small helpers                                                            */
/* ------------------------------------------------------------------------ */

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

static void sort_i64(int64_t* v, int n) { qsort(v, (size_t)n, sizeof(int64_t), cmp_i64); }

/*
 * Gaussian elimination with partial pivoting, in place on the r x r row-major
 * G.  Pivot of column k: the largest |G(a,k)|, a >= k; ties go to the smallest
 * a (strict '>' while scanning a upward).  After the call G holds L (unit,
 * strictly below the diagonal) and U (on and above it) of P*G = L*U, and
 * perm[k] is the original row now at position k.  Returns -1 if a pivot
 * column is entirely zero (G singular), else 0.
 */
int oracle_gepp(int r, double* G, int* perm) {
  for (int k = 0; k < r; ++k) perm[k] = k;
  for (int k = 0; k < r; ++k) {
    int piv = k;
    double best = fabs(G[(size_t)k * r + k]);
    for (int a = k + 1; a < r; ++a) {
      double v = fabs(G[(size_t)a * r + k]);
      if (v > best) { best = v; piv = a; }
    }
    if (best == 0.0) return -1;
    if (piv != k) {
      for (int c = 0; c < r; ++c) {
        double t = G[(size_t)k * r + c];
        G[(size_t)k * r + c] = G[(size_t)piv * r + c];
        G[(size_t)piv * r + c] = t;
      }
      int tp = perm[k]; perm[k] = perm[piv]; perm[piv] = tp;
    }
    double d = G[(size_t)k * r + k];
    for (int a = k + 1; a < r; ++a) {
      double l = G[(size_t)a * r + k] / d;
      G[(size_t)a * r + k] = l;
      for (int c = k + 1; c < r; ++c)
        G[(size_t)a * r + c] = fma(-l, G[(size_t)k * r + c], G[(size_t)a * r + c]);
    }
  }
  return 0;
}

/*
 * X = G^{-1} from the factors of oracle_gepp, one column at a time:
 * L y = P e_j by forward substitution (sum over k ascending), then
 * U x = y by back substitution (sum over k descending from r-1), x_i = s/U(i,i).
 */
void oracle_lu_inverse(int r, const double* LU, const int* perm, double* X) {
  double* y = (double*)malloc(sizeof(double) * (size_t)r);
  double* x = (double*)malloc(sizeof(double) * (size_t)r);
  for (int j = 0; j < r; ++j) {
    for (int i = 0; i < r; ++i) {
      double s = (perm[i] == j) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s = fma(-LU[(size_t)i * r + k], y[k], s);
      y[i] = s;
    }
    for (int i = r - 1; i >= 0; --i) {
      double s = y[i];
      for (int k = r - 1; k > i; --k) s = fma(-LU[(size_t)i * r + k], x[k], s);
      x[i] = s / LU[(size_t)i * r + i];
    }
    for (int i = 0; i < r; ++i) X[(size_t)i * r + j] = x[i];
  }
  free(y);
  free(x);
}

/*
 * Volume |det G| = prod_k |U(k,k)| (Def. 1), carried as mant * 2^expo with
 * mant in [0.5, 1) so that it neither underflows nor overflows for any r.
 * Each factor is split by frexp (exact), the mantissas are multiplied in k
 * order (one rounding per product) and renormalised by frexp (exact).
 */
void oracle_volume(int r, const double* LU, double* mant, int* expo) {
  double mt = 1.0;
  int e = 0;
  for (int k = 0; k < r; ++k) {
    int eu, em;
    double u = frexp(fabs(LU[(size_t)k * r + k]), &eu);
    mt = frexp(mt * u, &em);
    e += eu + em;
  }
  *mant = mt;
  *expo = e;
}

/* volume (m1,e1) strictly larger than (m2,e2) */
static int vol_greater(double m1, int e1, double m2, int e2) {
  if (e1 != e2) return e1 > e2;
  return m1 > m2;
}

/* G = A(I,J) for the given orders of I and J (row-major r x r) */
static void gather_cross(const double* A, int64_t lda, int r, const int64_t* I, const int64_t* J,
                         double* G) {
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < r; ++b) G[(size_t)a * r + b] = A[I[a] * lda + J[b]];
}

/*
 * Adaptive Cross Approximation with complete pivoting (Alg. 1), stopped after
 * at most r steps (Alg. 1 takes the target rank r as input; its loop bound is
 * read as r).  The working residual starts as A(:, cols) (m x nc).  Step t:
 *   (i,c) = argmax |R(i,c)|, scanning i ascending (outer) then c ascending
 *           (inner) and keeping the first strictly larger value;
 *   p = R(i,c); if |p| <= theta the block is rank-short and ACA stops;
 *   I += i, J += cols[c];  f_c' = R(i,c')/p;  R(a,c') -= R(a,c) * f_c';
 *   row i and column c of R are then set to exactly zero.
 * Returns the number q of pivots taken; pivot magnitudes go to piv (nullable).
 */
int oracle_aca(const double* A, int64_t m, int64_t lda, const int64_t* cols, int nc, int r,
               double theta, int64_t* I, int64_t* J, double* piv) {
  double* R = (double*)malloc(sizeof(double) * (size_t)m * (size_t)nc);
  double* f = (double*)malloc(sizeof(double) * (size_t)nc);
  if (!R || !f) { free(R); free(f); return -1; }
  for (int64_t i = 0; i < m; ++i)
    for (int c = 0; c < nc; ++c) R[i * nc + c] = A[i * lda + cols[c]];
  int steps = r;
  if (steps > nc) steps = nc;
  if ((int64_t)steps > m) steps = (int)m;
  int q = 0;
  for (int t = 0; t < steps; ++t) {
    int64_t bi = 0;
    int bc = 0;
    double best = -1.0;
    for (int64_t i = 0; i < m; ++i)
      for (int c = 0; c < nc; ++c) {
        double v = fabs(R[i * nc + c]);
        if (v > best) { best = v; bi = i; bc = c; }
      }
    double p = R[bi * nc + bc];
    if (fabs(p) <= theta) break;
    I[q] = bi;
    J[q] = cols[bc];
    if (piv) piv[q] = p;
    ++q;
    for (int c = 0; c < nc; ++c) f[c] = R[bi * nc + c] / p;
    for (int64_t a = 0; a < m; ++a) {
      double g = R[a * nc + bc];
      for (int c = 0; c < nc; ++c) R[a * nc + c] = fma(-g, f[c], R[a * nc + c]);
    }
    for (int c = 0; c < nc; ++c) R[bi * nc + c] = 0.0;
    for (int64_t a = 0; a < m; ++a) R[a * nc + bc] = 0.0;
  }
  free(R);
  free(f);
  return q;
}

/* ------------------------------------------------------------------------ */
/* maxvol swap phases                                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
  int swaps, phases, refreshes, nocap, err;
} node_stats;

/*
 * One ROW swap on B (m x r, row-major): row i* enters slot k*.
 * p = B(i*,k*); v_c = B(i*,c)/p (c != k*), v_k* = (p-1)/p;
 * B(a,c) -= B(a,k*) v_c for every a, c (B(a,k*) read before the row changes);
 * row i* := e_k*^T.  This is B * (I + e_k* (B(i*,:) - e_k*^T))^{-1}, the
 * Sherman-Morrison inverse of the rank-1 change of A(I,J).  v: r scratch.
 */
void oracle_sm_row_update(double* B, int64_t m, int r, int64_t bi, int bk, double* v) {
  double p = B[bi * r + bk];
  for (int c = 0; c < r; ++c) v[c] = B[bi * r + c] / p;
  v[bk] = (p - 1.0) / p;
  for (int64_t a = 0; a < m; ++a) {
    double g = B[a * r + bk];
    for (int c = 0; c < r; ++c) B[a * r + c] = fma(-g, v[c], B[a * r + c]);
  }
  for (int c = 0; c < r; ++c) B[bi * r + c] = (c == bk) ? 1.0 : 0.0;
}

/*
 * One COL swap on Bc (r x nc, row-major): candidate column c* enters slot k*.
 * p = Bc(k*,c*); w_a = Bc(a,c*)/p (a != k*), w_k* = (p-1)/p;
 * Bc(a,c) -= w_a Bc(k*,c) for every a, c with the old row k*;
 * column c* := e_k*.  w: r scratch, rowk: nc scratch.
 */
void oracle_sm_col_update(double* Bc, int r, int nc, int bk, int bc, double* w, double* rowk) {
  double p = Bc[(size_t)bk * nc + bc];
  for (int a = 0; a < r; ++a) w[a] = Bc[(size_t)a * nc + bc] / p;
  w[bk] = (p - 1.0) / p;
  for (int c = 0; c < nc; ++c) rowk[c] = Bc[(size_t)bk * nc + c];
  for (int a = 0; a < r; ++a)
    for (int c = 0; c < nc; ++c) Bc[(size_t)a * nc + c] = fma(-w[a], rowk[c], Bc[(size_t)a * nc + c]);
  for (int a = 0; a < r; ++a) Bc[(size_t)a * nc + bc] = (a == bk) ? 1.0 : 0.0;
}

/*
 * Fresh row interpolation matrix for the current orders of I and J:
 * B = A(:,J) * A(I,J)^{-1} (m x r, row-major), B(i,c) = sum_k A(i,J[k]) X(k,c)
 * with k ascending; rows I[k] are then set to exactly e_k^T.
 */
static int fresh_row(const double* A, int64_t m, int64_t lda, int r, const int64_t* I,
                     const int64_t* J, double* B, double* G, double* X, int* perm) {
  gather_cross(A, lda, r, I, J, G);
  if (oracle_gepp(r, G, perm) != 0) return -1;
  oracle_lu_inverse(r, G, perm, X);
  for (int64_t i = 0; i < m; ++i)
    for (int c = 0; c < r; ++c) {
      double s = 0.0;
      for (int k = 0; k < r; ++k) s = fma(A[i * lda + J[k]], X[(size_t)k * r + c], s);
      B[i * r + c] = s;
    }
  for (int k = 0; k < r; ++k)
    for (int c = 0; c < r; ++c) B[I[k] * r + c] = (c == k) ? 1.0 : 0.0;
  return 0;
}

/*
 * ROW phase: maxvol on the tall A(:,J) with J fixed.
 *   (i*,k*) = argmax |B(i,k)| over rows i not in I, scanning i ascending then
 *             k ascending, first strictly larger value wins;
 *   if |B(i*,k*)| <= 1+tau: if B has been updated since its last fresh
 *             computation, recompute it fresh (same orders of I, J) and scan
 *             again, else the phase ends;
 *   else (unless the node's swap budget is spent) swap row i* into slot k*:
 *             p = B(i*,k*); v_c = B(i*,c)/p (c != k*), v_k* = (p-1)/p;
 *             B(a,c) -= B(a,k*) v_c for all a, c; row i* := e_k*^T; I[k*] = i*.
 * The update is the Sherman-Morrison form of replacing row k* of A(I,J) by
 * row i* of A(:,J); |det| grows by the factor |p|.  Returns the swap count.
 */
static int row_phase(const double* A, int64_t m, int64_t lda, int r, int64_t* I, const int64_t* J,
                     double tau, int smax, node_stats* st) {
  if (m == r) return 0; /* no candidate rows */
  double* B = (double*)malloc(sizeof(double) * (size_t)m * (size_t)r);
  double* G = (double*)malloc(sizeof(double) * (size_t)r * r);
  double* X = (double*)malloc(sizeof(double) * (size_t)r * r);
  double* v = (double*)malloc(sizeof(double) * (size_t)r);
  int* perm = (int*)malloc(sizeof(int) * (size_t)r);
  char* sel = (char*)calloc((size_t)m, 1);
  int nsw = 0;
  if (!B || !G || !X || !v || !perm || !sel) { st->err = ORC_ERR_NOMEM; goto out; }
  for (int k = 0; k < r; ++k) sel[I[k]] = 1;
  if (fresh_row(A, m, lda, r, I, J, B, G, X, perm) != 0) { st->err = ORC_ERR_INTERNAL; goto out; }
  st->refreshes++;
  int since = 0;
  const double lim = 1.0 + tau;
  for (;;) {
    int64_t bi = 0;
    int bk = 0;
    double best = -1.0;
    for (int64_t i = 0; i < m; ++i) {
      if (sel[i]) continue;
      for (int k = 0; k < r; ++k) {
        double x = fabs(B[i * r + k]);
        if (x > best) { best = x; bi = i; bk = k; }
      }
    }
    if (best <= lim) {
      if (since == 0) break;
      if (fresh_row(A, m, lda, r, I, J, B, G, X, perm) != 0) { st->err = ORC_ERR_INTERNAL; break; }
      st->refreshes++;
      since = 0;
      continue;
    }
    if (st->swaps >= smax) { st->nocap = 1; break; }
    oracle_sm_row_update(B, m, r, bi, bk, v);
    sel[I[bk]] = 0;
    sel[bi] = 1;
    I[bk] = bi;
    ++nsw;
    st->swaps++;
    ++since;
  }
out:
  free(B); free(G); free(X); free(v); free(perm); free(sel);
  return nsw;
}

/*
 * Fresh column interpolation matrix Bc = A(I,J)^{-1} * A(I,Jc) (r x nc,
 * row-major), Bc(a,c) = sum_k X(a,k) A(I[k],Jc[c]) with k ascending; the
 * column holding J[k] is then set to exactly e_k.
 */
static int fresh_col(const double* A, int64_t lda, int r, const int64_t* I, const int64_t* J,
                     const int64_t* Jc, int nc, const int* posJ, double* Bc, double* G, double* X,
                     int* perm) {
  gather_cross(A, lda, r, I, J, G);
  if (oracle_gepp(r, G, perm) != 0) return -1;
  oracle_lu_inverse(r, G, perm, X);
  for (int a = 0; a < r; ++a)
    for (int c = 0; c < nc; ++c) {
      double s = 0.0;
      for (int k = 0; k < r; ++k) s = fma(X[(size_t)a * r + k], A[I[k] * lda + Jc[c]], s);
      Bc[(size_t)a * nc + c] = s;
    }
  for (int k = 0; k < r; ++k)
    for (int a = 0; a < r; ++a) Bc[(size_t)a * nc + posJ[k]] = (a == k) ? 1.0 : 0.0;
  return 0;
}

static int pos_in(const int64_t* Jc, int nc, int64_t j) {
  for (int c = 0; c < nc; ++c)
    if (Jc[c] == j) return c;
  return -1;
}

/*
 * COL phase: maxvol on A(I,Jc)^T with I fixed; the transpose of the ROW
 * phase.  Candidates are the positions c with Jc[c] not in J, scanned c
 * ascending (outer) then k ascending (inner), first strictly larger value.
 * Swap of candidate c* into slot k*: p = Bc(k*,c*); w_a = Bc(a,c*)/p (a != k*),
 * w_k* = (p-1)/p; Bc(a,c) -= w_a Bc(k*,c) for all a, c (old row k* used);
 * column c* := e_k*; J[k*] = Jc[c*].  Refresh and stop rules as in ROW.
 */
static int col_phase(const double* A, int64_t lda, int r, const int64_t* I, int64_t* J,
                     const int64_t* Jc, int nc, double tau, int smax, node_stats* st) {
  if (nc == r) return 0; /* no candidate columns */
  double* Bc = (double*)malloc(sizeof(double) * (size_t)r * (size_t)nc);
  double* G = (double*)malloc(sizeof(double) * (size_t)r * r);
  double* X = (double*)malloc(sizeof(double) * (size_t)r * r);
  double* w = (double*)malloc(sizeof(double) * (size_t)r);
  double* rowk = (double*)malloc(sizeof(double) * (size_t)nc);
  int* perm = (int*)malloc(sizeof(int) * (size_t)r);
  int* posJ = (int*)malloc(sizeof(int) * (size_t)r);
  char* insel = (char*)calloc((size_t)nc, 1);
  int nsw = 0;
  if (!Bc || !G || !X || !w || !rowk || !perm || !posJ || !insel) { st->err = ORC_ERR_NOMEM; goto out; }
  for (int k = 0; k < r; ++k) {
    posJ[k] = pos_in(Jc, nc, J[k]);
    if (posJ[k] < 0) { st->err = ORC_ERR_INTERNAL; goto out; }
    insel[posJ[k]] = 1;
  }
  if (fresh_col(A, lda, r, I, J, Jc, nc, posJ, Bc, G, X, perm) != 0) { st->err = ORC_ERR_INTERNAL; goto out; }
  st->refreshes++;
  int since = 0;
  const double lim = 1.0 + tau;
  for (;;) {
    int bc = 0, bk = 0;
    double best = -1.0;
    for (int c = 0; c < nc; ++c) {
      if (insel[c]) continue;
      for (int k = 0; k < r; ++k) {
        double x = fabs(Bc[(size_t)k * nc + c]);
        if (x > best) { best = x; bc = c; bk = k; }
      }
    }
    if (best <= lim) {
      if (since == 0) break;
      if (fresh_col(A, lda, r, I, J, Jc, nc, posJ, Bc, G, X, perm) != 0) { st->err = ORC_ERR_INTERNAL; break; }
      st->refreshes++;
      since = 0;
      continue;
    }
    if (st->swaps >= smax) { st->nocap = 1; break; }
    oracle_sm_col_update(Bc, r, nc, bk, bc, w, rowk);
    insel[posJ[bk]] = 0;
    insel[bc] = 1;
    posJ[bk] = bc;
    J[bk] = Jc[bc];
    ++nsw;
    st->swaps++;
    ++since;
  }
out:
  free(Bc); free(G); free(X); free(w); free(rowk); free(perm); free(posJ); free(insel);
  return nsw;
}

/*
 * Swap loop on candidate columns Jc (sorted ascending) starting from (I, J).
 * Phases alternate ROW, COL, ROW, ...; I and J are sorted ascending at the
 * start of every phase.  The loop stops after the first phase, other than the
 * very first, that makes no swap (both sides are then dominant), when the
 * node's swap budget smax is spent (nocap), or on an internal error.
 */
static void swap_loop(const double* A, int64_t m, int64_t lda, int r, int64_t* I, int64_t* J,
                      const int64_t* Jc, int nc, double tau, int smax, node_stats* st) {
  for (int phase = 0;; ++phase) {
    sort_i64(I, r);
    sort_i64(J, r);
    int nsw = (phase % 2 == 0) ? row_phase(A, m, lda, r, I, J, tau, smax, st)
                               : col_phase(A, lda, r, I, J, Jc, nc, tau, smax, st);
    st->phases++;
    if (st->nocap || st->err) break;
    if (phase >= 1 && nsw == 0) break;
  }
  sort_i64(I, r);
  sort_i64(J, r);
}

/* exported single-node swap loop (used by the pins) */
int oracle_swap_loop(const double* A, int64_t m, int64_t n, int64_t lda, int r, int64_t* I,
                     int64_t* J, const int64_t* Jc, int nc, double tau, int smax, int32_t* stats) {
  (void)n;
  node_stats st = {0, 0, 0, 0, 0};
  swap_loop(A, m, lda, r, I, J, Jc, nc, tau, smax, &st);
  stats[0] = st.swaps;
  stats[1] = st.phases;
  stats[2] = st.refreshes;
  stats[3] = st.nocap;
  stats[4] = st.err;
  return st.err ? st.err : (st.nocap ? ORC_WARN_NOCONV : ORC_OK);
}

/* ------------------------------------------------------------------------ */
/* the tree                                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
  int q, is_short, promoted;
  int64_t* I;
  int64_t* J;
  double vol_m;
  int vol_e;
  node_stats st;
} node_t;

static int node_volume(const double* A, int64_t lda, int r, node_t* nd) {
  double* G = (double*)malloc(sizeof(double) * (size_t)r * r);
  int* perm = (int*)malloc(sizeof(int) * (size_t)r);
  gather_cross(A, lda, r, nd->I, nd->J, G);
  int rc = oracle_gepp(r, G, perm);
  if (rc == 0) oracle_volume(r, G, &nd->vol_m, &nd->vol_e);
  free(G);
  free(perm);
  return rc;
}

/* ACA start on candidate columns, then the swap loop if ACA reached rank r */
static void aca_node(const double* A, int64_t m, int64_t lda, int r, const int64_t* cols, int nc,
                     double theta, double tau, int smax, node_t* nd) {
  int q = oracle_aca(A, m, lda, cols, nc, r, theta, nd->I, nd->J, NULL);
  if (q < 0) { nd->st.err = ORC_ERR_NOMEM; return; }
  nd->q = q;
  if (q < r) {
    nd->is_short = 1;
    sort_i64(nd->I, q);
    sort_i64(nd->J, q);
    return;
  }
  swap_loop(A, m, lda, r, nd->I, nd->J, cols, nc, tau, smax, &nd->st);
  if (!nd->st.err && node_volume(A, lda, r, nd) != 0) nd->st.err = ORC_ERR_INTERNAL;
}

static void merge_nodes(const double* A, int64_t m, int64_t lda, int r, double theta, double tau,
                        int smax, const node_t* L, const node_t* Rn, node_t* out) {
  int nc = L->q + Rn->q;
  int64_t* Jc = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nc > 0 ? nc : 1));
  for (int k = 0; k < L->q; ++k) Jc[k] = L->J[k];
  for (int k = 0; k < Rn->q; ++k) Jc[L->q + k] = Rn->J[k];
  sort_i64(Jc, nc);
  if (!L->is_short || !Rn->is_short) {
    const node_t* src;
    if (!L->is_short && !Rn->is_short)
      src = vol_greater(Rn->vol_m, Rn->vol_e, L->vol_m, L->vol_e) ? Rn : L;
    else
      src = L->is_short ? Rn : L;
    memcpy(out->I, src->I, sizeof(int64_t) * (size_t)r);
    memcpy(out->J, src->J, sizeof(int64_t) * (size_t)r);
    out->q = r;
    out->is_short = 0;
    swap_loop(A, m, lda, r, out->I, out->J, Jc, nc, tau, smax, &out->st);
    if (!out->st.err && node_volume(A, lda, r, out) != 0) out->st.err = ORC_ERR_INTERNAL;
  } else {
    aca_node(A, m, lda, r, Jc, nc, theta, tau, smax, out);
  }
  free(Jc);
}

static void record(const node_t* nd, int level, int index, int r, int64_t* tmeta, double* tvol,
                   int64_t* tI, int64_t* tJ, int slot) {
  int64_t* mt = tmeta + (size_t)slot * TRACE_META;
  mt[0] = level; mt[1] = index; mt[2] = nd->q; mt[3] = nd->is_short; mt[4] = nd->promoted;
  mt[5] = nd->st.nocap; mt[6] = nd->st.swaps; mt[7] = nd->st.phases; mt[8] = nd->st.refreshes;
  mt[9] = nd->is_short ? 0 : nd->vol_e;
  tvol[slot] = nd->is_short ? 0.0 : nd->vol_m;
  for (int k = 0; k < r; ++k) {
    tI[(size_t)slot * r + k] = (k < nd->q) ? nd->I[k] : -1;
    tJ[(size_t)slot * r + k] = (k < nd->q) ? nd->J[k] : -1;
  }
}

/* number of tree records for b leaves (every node of every level) */
int oracle_tree_size(int64_t b) {
  int64_t tot = 0, c = b;
  for (;;) {
    tot += c;
    if (c <= 1) break;
    c = (c + 1) / 2;
  }
  return (int)tot;
}

/*
 * Full selection.  A is m x n row-major (leading dimension lda), FP64.
 * w = leaf column-block width (0 -> max(64, r)); tau = swap threshold
 * (0 -> 1e-13); max_swaps = swap budget per node (0 -> 64 r).
 * Steps:
 *   1. validate; amax = max|A|; theta = max(m,n) * 2^-52 * amax;
 *   2. b = max(1, floor(n/w)) contiguous column blocks of width w, the last
 *      one taking the remainder (Alg. 3 block partition);
 *   3. every block: ACA start, then the swap loop on its columns;
 *   4. binary tree: nodes (2p, 2p+1) merge, an odd last node is promoted;
 *      merge candidates Jc = sorted union of the children's J; start from
 *      the child of larger volume (exact tie -> left); rank-short children
 *      handled as documented in merge_nodes;
 *   5. root I, J sorted ascending; info.logvol from its fresh GEPP.
 * Optional trace (all four trace pointers non-null): one record per node of
 * every level, level by level, index ascending.
 */
static int select_impl(const double* A, int64_t m, int64_t n, int64_t lda, int r, int w, double tau,
                       int max_swaps, double theta_rel, int polish, int64_t* I_out, int64_t* J_out,
                       orc_info* info, int64_t* tmeta, double* tvol, int64_t* tI, int64_t* tJ);

int oracle_cur_select(const double* A, int64_t m, int64_t n, int64_t lda, int r, int w, double tau,
                      int max_swaps, int64_t* I_out, int64_t* J_out, orc_info* info,
                      int64_t* tmeta, double* tvol, int64_t* tI, int64_t* tJ) {
  return select_impl(A, m, n, lda, r, w, tau, max_swaps, 0.0, 0, I_out, J_out, info, tmeta, tvol, tI, tJ);
}

/*
 * The selection followed by a polish of the root's cross over the whole
 * matrix: the same swap loop (row phase over all m rows, column phase over
 * the candidate set) with every column 0..n-1 as a candidate, started from
 * the root's (I, J).  When it ends without reaching the swap budget, the
 * cross is dominant over the whole matrix: every entry of A(:,J) A(I,J)^-1
 * and of A(I,J)^-1 A(I,:) is at most 1 + tau in magnitude, the maximal-volume
 * condition of Sec. 1.1 on all of A rather than on the root's candidates.
 * A rank-short root is returned as it is.  The trace, if given, holds one
 * more record (the polish, at the level after the root, index 0).
 */
int oracle_cur_select_polish(const double* A, int64_t m, int64_t n, int64_t lda, int r, int w, double tau,
                             int max_swaps, int64_t* I_out, int64_t* J_out, orc_info* info,
                             int64_t* tmeta, double* tvol, int64_t* tI, int64_t* tJ) {
  return select_impl(A, m, n, lda, r, w, tau, max_swaps, 0.0, 1, I_out, J_out, info, tmeta, tvol, tI, tJ);
}

/*
 * The same selection with the numerical-zero pivot threshold set to
 * theta_rel * max|A| instead of max(m,n) 2^-52 max|A| (theta_rel > 0).  Used
 * to check the rank verdicts of the GPU's FP32 path, whose threshold is
 * r 2^-23 max|A| (the rounding of r FP32 elimination steps), on the exactly
 * upcast matrix.
 */
int oracle_cur_select_theta(const double* A, int64_t m, int64_t n, int64_t lda, int r, int w, double tau,
                            int max_swaps, double theta_rel, int64_t* I_out, int64_t* J_out, orc_info* info) {
  if (!(theta_rel > 0.0)) return ORC_ERR_ARG;
  return select_impl(A, m, n, lda, r, w, tau, max_swaps, theta_rel, 0, I_out, J_out, info, NULL, NULL, NULL,
                     NULL);
}

static int select_impl(const double* A, int64_t m, int64_t n, int64_t lda, int r, int w, double tau,
                       int max_swaps, double theta_rel, int polish, int64_t* I_out, int64_t* J_out,
                       orc_info* info, int64_t* tmeta, double* tvol, int64_t* tI, int64_t* tJ) {
  if (info) memset(info, 0, sizeof(*info));
  if (!A || !I_out || !J_out || m < 1 || n < 1 || lda < n || r < 1 || (int64_t)r > m ||
      (int64_t)r > n || w < 0 || tau < 0.0 || max_swaps < 0)
    return ORC_ERR_ARG;
  if (w == 0) w = r > 64 ? r : 64;
  if (w < r) return ORC_ERR_ARG;
  if (tau == 0.0) tau = 1e-13;
  if (max_swaps == 0) max_swaps = 64 * r;
  for (int k = 0; k < r; ++k) { I_out[k] = -1; J_out[k] = -1; }

  double amax = 0.0;
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double v = A[i * lda + j];
      if (!isfinite(v)) return ORC_ERR_NONFINITE;
      if (fabs(v) > amax) amax = fabs(v);
    }
  if (amax == 0.0) {
    if (info) { info->rank = 0; info->status = ORC_ERR_RANK; }
    return ORC_ERR_RANK;
  }
  const double theta = theta_rel > 0.0 ? theta_rel * amax : (double)(m > n ? m : n) * 0x1p-52 * amax;

  int64_t b = n / w;
  if (b < 1) b = 1;
  int trace = tmeta && tvol && tI && tJ;
  node_t* cur = (node_t*)calloc((size_t)b, sizeof(node_t));
  int64_t* cols = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  for (int64_t j = 0; j < n; ++j) cols[j] = j;
  int status = ORC_OK, slot = 0;
  int32_t nodes = 0, phases = 0, refreshes = 0;
  int64_t swaps = 0;
  int anynocap = 0;

  for (int64_t k = 0; k < b; ++k) {
    node_t* nd = &cur[k];
    nd->I = (int64_t*)calloc((size_t)r, sizeof(int64_t));
    nd->J = (int64_t*)calloc((size_t)r, sizeof(int64_t));
    int64_t c0 = k * w, c1 = (k == b - 1) ? n : (k + 1) * w;
    aca_node(A, m, lda, r, cols + c0, (int)(c1 - c0), theta, tau, max_swaps, nd);
    nodes++;
    phases += nd->st.phases; refreshes += nd->st.refreshes; swaps += nd->st.swaps;
    anynocap |= nd->st.nocap;
    if (nd->st.err) status = nd->st.err;
    if (trace) record(nd, 0, (int)k, r, tmeta, tvol, tI, tJ, slot++);
  }
  int64_t cnt = b;
  int level = 0;
  while (cnt > 1 && status >= 0) {
    int64_t nxt = (cnt + 1) / 2;
    node_t* up = (node_t*)calloc((size_t)nxt, sizeof(node_t));
    ++level;
    for (int64_t p = 0; p < nxt; ++p) {
      node_t* nd = &up[p];
      if (2 * p + 1 < cnt) {
        nd->I = (int64_t*)calloc((size_t)r, sizeof(int64_t));
        nd->J = (int64_t*)calloc((size_t)r, sizeof(int64_t));
        merge_nodes(A, m, lda, r, theta, tau, max_swaps, &cur[2 * p], &cur[2 * p + 1], nd);
        nodes++;
        phases += nd->st.phases; refreshes += nd->st.refreshes; swaps += nd->st.swaps;
        anynocap |= nd->st.nocap;
        if (nd->st.err) status = nd->st.err;
      } else {
        *nd = cur[2 * p];
        cur[2 * p].I = NULL;
        cur[2 * p].J = NULL;
        memset(&nd->st, 0, sizeof(nd->st));
        nd->promoted = 1;
      }
      if (trace) record(nd, level, (int)p, r, tmeta, tvol, tI, tJ, slot++);
    }
    for (int64_t p = 0; p < cnt; ++p) { free(cur[p].I); free(cur[p].J); }
    free(cur);
    cur = up;
    cnt = nxt;
  }
  node_t* root = &cur[0];
  if (polish && status >= 0 && !root->is_short) {
    /* the polish: the swap loop on all n columns, from the root's cross */
    memset(&root->st, 0, sizeof(root->st));
    swap_loop(A, m, lda, r, root->I, root->J, cols, (int)n, tau, max_swaps, &root->st);
    nodes++;
    phases += root->st.phases; refreshes += root->st.refreshes; swaps += root->st.swaps;
    anynocap |= root->st.nocap;
    if (root->st.err) status = root->st.err;
    else if (node_volume(A, lda, r, root) != 0) status = ORC_ERR_INTERNAL;
    root->promoted = 0;
    ++level;
    if (trace) record(root, level, 0, r, tmeta, tvol, tI, tJ, slot++);
  }
  if (status >= 0) {
    for (int k = 0; k < root->q; ++k) { I_out[k] = root->I[k]; J_out[k] = root->J[k]; }
    if (root->is_short) status = ORC_ERR_RANK;
    else if (anynocap) status = ORC_WARN_NOCONV;
  }
  if (info) {
    info->rank = root->q;
    info->nodes = nodes;
    info->phases = phases;
    info->refreshes = refreshes;
    info->swaps = swaps;
    info->logvol = root->is_short ? -INFINITY : log(root->vol_m) + (double)root->vol_e * M_LN2;
    info->status = status;
  }
  for (int64_t p = 0; p < cnt; ++p) { free(cur[p].I); free(cur[p].J); }
  free(cur);
  free(cols);
  return status;
}

/* ------------------------------------------------------------------------ */
/* assembly and residual                                                    */
/* ------------------------------------------------------------------------ */

/*
 * Pseudo-inverse of the r x r row-major G by one-sided (Hestenes) Jacobi SVD:
 * cyclic sweeps over column pairs (p<q) rotate W = G*V until every pair is
 * orthogonal to 2^-52 relative (at most 60 sweeps); sigma_j = ||W(:,j)||,
 * u_j = W(:,j)/sigma_j; G^+ = V diag(1/sigma) U^T over sigma_j >
 * r * 2^-52 * max(sigma).  Output P is r x r row-major.
 */
void oracle_pinv(int r, const double* G, double* P) {
  double* W = (double*)malloc(sizeof(double) * (size_t)r * r);
  double* V = (double*)malloc(sizeof(double) * (size_t)r * r);
  double* sg = (double*)malloc(sizeof(double) * (size_t)r);
  memcpy(W, G, sizeof(double) * (size_t)r * r);
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < r; ++b) V[(size_t)a * r + b] = (a == b) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    int rotated = 0;
    for (int p = 0; p < r - 1; ++p)
      for (int q = p + 1; q < r; ++q) {
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = 0; i < r; ++i) {
          double wp = W[(size_t)i * r + p], wq = W[(size_t)i * r + q];
          al = fma(wp, wp, al);
          be = fma(wq, wq, be);
          ga = fma(wp, wq, ga);
        }
        if (ga == 0.0 || fabs(ga) <= 0x1p-52 * sqrt(al * be)) continue;
        rotated = 1;
        double zeta = (be - al) / (2.0 * ga);
        double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double c = 1.0 / sqrt(1.0 + t * t);
        double s = c * t;
        for (int i = 0; i < r; ++i) {
          double wp = W[(size_t)i * r + p], wq = W[(size_t)i * r + q];
          W[(size_t)i * r + p] = c * wp - s * wq;
          W[(size_t)i * r + q] = s * wp + c * wq;
          double vp = V[(size_t)i * r + p], vq = V[(size_t)i * r + q];
          V[(size_t)i * r + p] = c * vp - s * vq;
          V[(size_t)i * r + q] = s * vp + c * vq;
        }
      }
    if (!rotated) break;
  }
  double smax = 0.0;
  for (int j = 0; j < r; ++j) {
    double s = 0.0;
    for (int i = 0; i < r; ++i) s = fma(W[(size_t)i * r + j], W[(size_t)i * r + j], s);
    sg[j] = sqrt(s);
    if (sg[j] > smax) smax = sg[j];
  }
  const double cut = (double)r * 0x1p-52 * smax;
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < r; ++b) {
      double s = 0.0;
      for (int j = 0; j < r; ++j) {
        if (!(sg[j] > cut)) continue;
        /* V(a,j) * (1/sigma_j) * U(b,j), U(b,j) = W(b,j)/sigma_j */
        s = fma(V[(size_t)a * r + j], W[(size_t)b * r + j] / (sg[j] * sg[j]), s);
      }
      P[(size_t)a * r + b] = s;
    }
  free(W);
  free(V);
  free(sg);
}

/*
 * C = A(:,J) (m x r), R = A(I,:) (r x n), U = A(I,J)^+ (r x r), all
 * row-major FP64 (Sec. 1.1).  U is the GEPP inverse unless a pivot is zero or
 * min|u_kk| / max|u_kk| < r * 2^-52, in which case it is oracle_pinv.
 * *used_pinv (nullable) reports which.
 */
int oracle_cur_assemble(const double* A, int64_t m, int64_t n, int64_t lda, int r,
                        const int64_t* I, const int64_t* J, double* C, double* U, double* R,
                        int* used_pinv) {
  if (!A || !I || !J || !C || !U || !R || m < 1 || n < 1 || lda < n || r < 1 || (int64_t)r > m ||
      (int64_t)r > n)
    return ORC_ERR_ARG;
  for (int k = 0; k < r; ++k)
    if (I[k] < 0 || I[k] >= m || J[k] < 0 || J[k] >= n) return ORC_ERR_ARG;
  for (int64_t i = 0; i < m; ++i)
    for (int k = 0; k < r; ++k) C[i * r + k] = A[i * lda + J[k]];
  for (int k = 0; k < r; ++k)
    for (int64_t j = 0; j < n; ++j) R[(int64_t)k * n + j] = A[I[k] * lda + j];
  double* G = (double*)malloc(sizeof(double) * (size_t)r * r);
  int* perm = (int*)malloc(sizeof(int) * (size_t)r);
  gather_cross(A, lda, r, I, J, G);
  int sing = oracle_gepp(r, G, perm);
  int pinv = 1;
  if (sing == 0) {
    double umin = INFINITY, umax = 0.0;
    for (int k = 0; k < r; ++k) {
      double u = fabs(G[(size_t)k * r + k]);
      if (u < umin) umin = u;
      if (u > umax) umax = u;
    }
    pinv = (umin / umax < (double)r * 0x1p-52);
  }
  if (!pinv) {
    oracle_lu_inverse(r, G, perm, U);
  } else {
    gather_cross(A, lda, r, I, J, G);
    oracle_pinv(r, G, U);
  }
  if (used_pinv) *used_pinv = pinv;
  free(G);
  free(perm);
  return ORC_OK;
}

/*
 * Residual of the CUR approximation (Thm 1, Sec. 3.1):
 *   Bm = C * U (m x r; sums over l ascending),
 *   E(i,j) = A(i,j) - sum_k Bm(i,k) R(k,j) (k ascending),
 *   cheb = max |E(i,j)|, fro_rel = ||E||_F / ||A||_F.
 * C is m x r, U r x r, R r x n, all row-major FP64.  If some E(i,j) is NaN or
 * infinite, cheb is NaN and the status ORC_ERR_NONFINITE.
 */
int oracle_cur_residual(const double* A, int64_t m, int64_t n, int64_t lda, int r, const double* C,
                        const double* U, const double* R, double* cheb, double* fro_rel) {
  if (!A || !C || !U || !R || !cheb || m < 1 || n < 1 || lda < n || r < 1) return ORC_ERR_ARG;
  double* Bm = (double*)malloc(sizeof(double) * (size_t)r);
  double emax = 0.0, esq = 0.0, asq = 0.0;
  int nonfinite = 0;
  for (int64_t i = 0; i < m; ++i) {
    for (int k = 0; k < r; ++k) {
      double s = 0.0;
      for (int l = 0; l < r; ++l) s = fma(C[i * r + l], U[(size_t)l * r + k], s);
      Bm[k] = s;
    }
    for (int64_t j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k < r; ++k) s = fma(Bm[k], R[(int64_t)k * n + j], s);
      double a = A[i * lda + j];
      double e = a - s;
      if (!isfinite(e)) nonfinite = 1;
      else if (fabs(e) > emax) emax = fabs(e);
      esq = fma(e, e, esq);
      asq = fma(a, a, asq);
    }
  }
  free(Bm);
  *cheb = nonfinite ? NAN : emax;
  if (fro_rel) *fro_rel = (asq > 0.0) ? sqrt(esq) / sqrt(asq) : 0.0;
  return nonfinite ? ORC_ERR_NONFINITE : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Rectangular cross: r rows, c columns (Alg. 2 takes the two counts apart;  */
/* Sec. 1.1 and the overview define U as the pseudo-inverse of A(I,J))       */
/* ------------------------------------------------------------------------ */
/*
 * Pseudo-inverse of the p x q row-major G, written q x p row-major to P, by
 * one-sided (Hestenes) Jacobi on the columns of the taller of G and G^T:
 * for p >= q, W = G V with cyclic sweeps over column pairs (a < b) until
 * every pair is orthogonal to 2^-52 relative (at most 60 sweeps), sigma_j =
 * ||W(:,j)||, G^+ = V diag(1/sigma^2) W^T over sigma_j > max(p,q) 2^-52
 * sigma_max; for p < q, G^+ = ((G^T)^+)^T.  Sums run over the rows in
 * ascending order, one fma per term.  For p == q these are the operations of
 * oracle_pinv.
 */
void oracle_pinv_rect(int p, int q, const double* G, double* P) {
  if (p < q) {
    double* T = (double*)malloc(sizeof(double) * (size_t)p * q);
    double* Q = (double*)malloc(sizeof(double) * (size_t)p * q);
    for (int a = 0; a < p; ++a)
      for (int b = 0; b < q; ++b) T[(size_t)b * p + a] = G[(size_t)a * q + b];
    oracle_pinv_rect(q, p, T, Q); /* Q = (G^T)^+, p x q */
    for (int a = 0; a < p; ++a)
      for (int b = 0; b < q; ++b) P[(size_t)b * p + a] = Q[(size_t)a * q + b];
    free(T);
    free(Q);
    return;
  }
  double* W = (double*)malloc(sizeof(double) * (size_t)p * q);
  double* V = (double*)malloc(sizeof(double) * (size_t)q * q);
  double* sg = (double*)malloc(sizeof(double) * (size_t)q);
  memcpy(W, G, sizeof(double) * (size_t)p * q);
  for (int a = 0; a < q; ++a)
    for (int b = 0; b < q; ++b) V[(size_t)a * q + b] = (a == b) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    int rotated = 0;
    for (int a = 0; a < q - 1; ++a)
      for (int b = a + 1; b < q; ++b) {
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = 0; i < p; ++i) {
          double wa = W[(size_t)i * q + a], wb = W[(size_t)i * q + b];
          al = fma(wa, wa, al);
          be = fma(wb, wb, be);
          ga = fma(wa, wb, ga);
        }
        if (ga == 0.0 || fabs(ga) <= 0x1p-52 * sqrt(al * be)) continue;
        rotated = 1;
        double zeta = (be - al) / (2.0 * ga);
        double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double cs = 1.0 / sqrt(1.0 + t * t);
        double sn = cs * t;
        for (int i = 0; i < p; ++i) {
          double wa = W[(size_t)i * q + a], wb = W[(size_t)i * q + b];
          W[(size_t)i * q + a] = cs * wa - sn * wb;
          W[(size_t)i * q + b] = sn * wa + cs * wb;
        }
        for (int i = 0; i < q; ++i) {
          double va = V[(size_t)i * q + a], vb = V[(size_t)i * q + b];
          V[(size_t)i * q + a] = cs * va - sn * vb;
          V[(size_t)i * q + b] = sn * va + cs * vb;
        }
      }
    if (!rotated) break;
  }
  double smax = 0.0;
  for (int j = 0; j < q; ++j) {
    double sum = 0.0;
    for (int i = 0; i < p; ++i) sum = fma(W[(size_t)i * q + j], W[(size_t)i * q + j], sum);
    sg[j] = sqrt(sum);
    if (sg[j] > smax) smax = sg[j];
  }
  const double cut = (double)p * 0x1p-52 * smax;
  for (int a = 0; a < q; ++a)
    for (int b = 0; b < p; ++b) {
      double sum = 0.0;
      for (int j = 0; j < q; ++j) {
        if (!(sg[j] > cut)) continue;
        sum = fma(V[(size_t)a * q + j], W[(size_t)b * q + j] / (sg[j] * sg[j]), sum);
      }
      P[(size_t)a * p + b] = sum;
    }
  free(W);
  free(V);
  free(sg);
}

/*
 * C = A(:,J) (m x c), R = A(I,:) (r x n), U = A(I,J)^+ (c x r) by
 * oracle_pinv_rect, all row-major FP64.  I holds r rows, J c columns.
 */
int oracle_cur_assemble_rect(const double* A, int64_t m, int64_t n, int64_t lda, int r, int c,
                             const int64_t* I, const int64_t* J, double* C, double* U, double* R) {
  if (!A || !I || !J || !C || !U || !R || m < 1 || n < 1 || lda < n || r < 1 || c < 1 || (int64_t)r > m ||
      (int64_t)c > n)
    return ORC_ERR_ARG;
  for (int k = 0; k < r; ++k)
    if (I[k] < 0 || I[k] >= m) return ORC_ERR_ARG;
  for (int k = 0; k < c; ++k)
    if (J[k] < 0 || J[k] >= n) return ORC_ERR_ARG;
  for (int64_t i = 0; i < m; ++i)
    for (int k = 0; k < c; ++k) C[i * c + k] = A[i * lda + J[k]];
  for (int k = 0; k < r; ++k)
    for (int64_t j = 0; j < n; ++j) R[(int64_t)k * n + j] = A[I[k] * lda + j];
  double* G = (double*)malloc(sizeof(double) * (size_t)r * c);
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < c; ++b) G[(size_t)a * c + b] = A[I[a] * lda + J[b]];
  oracle_pinv_rect(r, c, G, U);
  free(G);
  return ORC_OK;
}

/*
 * Residual of the rectangular form: Bm = C U (m x r, sums over l < c
 * ascending), E(i,j) = A(i,j) - sum_k Bm(i,k) R(k,j) (k < r ascending);
 * cheb, fro_rel and the non-finite verdict as in oracle_cur_residual.  C is
 * m x c, U c x r, R r x n.
 */
int oracle_cur_residual_rect(const double* A, int64_t m, int64_t n, int64_t lda, int r, int c, const double* C,
                             const double* U, const double* R, double* cheb, double* fro_rel) {
  if (!A || !C || !U || !R || !cheb || m < 1 || n < 1 || lda < n || r < 1 || c < 1) return ORC_ERR_ARG;
  double* Bm = (double*)malloc(sizeof(double) * (size_t)r);
  double emax = 0.0, esq = 0.0, asq = 0.0;
  int nonfinite = 0;
  for (int64_t i = 0; i < m; ++i) {
    for (int k = 0; k < r; ++k) {
      double sum = 0.0;
      for (int l = 0; l < c; ++l) sum = fma(C[i * c + l], U[(size_t)l * r + k], sum);
      Bm[k] = sum;
    }
    for (int64_t j = 0; j < n; ++j) {
      double sum = 0.0;
      for (int k = 0; k < r; ++k) sum = fma(Bm[k], R[(int64_t)k * n + j], sum);
      double a = A[i * lda + j];
      double e = a - sum;
      if (!isfinite(e)) nonfinite = 1;
      else if (fabs(e) > emax) emax = fabs(e);
      esq = fma(e, e, esq);
      asq = fma(a, a, asq);
    }
  }
  free(Bm);
  *cheb = nonfinite ? NAN : emax;
  if (fro_rel) *fro_rel = (asq > 0.0) ? sqrt(esq) / sqrt(asq) : 0.0;
  return nonfinite ? ORC_ERR_NONFINITE : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Norm-greedy selection (Alg. 2 with Alg. 3)                                */
/* ------------------------------------------------------------------------ */
/*
 * Alg. 3 on one axis: r times, the candidate vector (column, or row) of
 * largest Euclidean norm is chosen (strict '>' in ascending index order, so
 * the first maximum wins) and projected out of every vector:
 *     v <- v - ((s . v) / (s . s)) s
 * (the division by the squared norm of s, the reading that makes this the
 * orthogonal projection; the listing's "maxNorm" is ambiguous).  Norms are
 * compared squared (same order), a chosen vector is no candidate again (its
 * projection is zero in exact arithmetic), and the selection stops early,
 * rank-short, once the largest remaining squared norm is at most
 * (max(m,n) 2^-52)^2 times the largest initial one.  The block partition of
 * Alg. 3 only distributes the argmax and the update; it does not change the
 * result, so the oracle works on the whole matrix.
 *
 * Sums over a vector (dot products, squared norms) run over the elements in
 * ascending index order, one fma per element, as the definition reads.  The
 * update of an element is one fma with the coefficient c = (s . v) / (s . s).
 */
int oracle_greedy_select_rc(const double* A, int64_t m, int64_t n, int64_t lda, int r, int c, int64_t* order_I,
                            int64_t* order_J, int64_t* I, int64_t* J, int* rank_rows, int* rank_cols,
                            double* gap_I, double* gap_J);

static double plain_dot(const double* a, const double* b, int64_t len) {
  double s = 0.0;
  for (int64_t i = 0; i < len; ++i) s = fma(a[i], b[i], s);
  return s;
}

/* Vectors W[v * len + i] (cnt of them, contiguous); order[t] receives the
 * chosen vector of step t.  If gap is non-NULL, gap[t] receives the margin of
 * step t's choice, (best - runner-up) / (largest initial squared norm), the
 * runner-up being the second largest squared norm among the candidates of
 * that step (+inf when there is none); entries past the last step are left
 * alone.  Returns the number chosen (<= r). */
static int greedy_axis(double* W, int64_t len, int64_t cnt, int r, int64_t* order, double* gap) {
  double* nrm = (double*)malloc(sizeof(double) * (size_t)cnt);
  char* sel = (char*)calloc((size_t)cnt, 1);
  double nmax0 = 0.0;
  for (int64_t v = 0; v < cnt; ++v) {
    nrm[v] = plain_dot(W + v * len, W + v * len, len);
    if (nrm[v] > nmax0) nmax0 = nrm[v];
  }
  const double eps = (double)(len > cnt ? len : cnt) * ldexp(1.0, -52);
  const double theta = eps * eps * nmax0;
  int t = 0;
  for (; t < r; ++t) {
    int64_t j = -1;
    double best = -1.0, second = -1.0;
    for (int64_t v = 0; v < cnt; ++v) {
      if (sel[v]) continue;
      if (nrm[v] > best) {
        second = best;
        best = nrm[v];
        j = v;
      } else if (nrm[v] > second) {
        second = nrm[v];
      }
    }
    if (j < 0 || !(best > theta)) break;
    if (gap) gap[t] = second < 0.0 ? INFINITY : (best - second) / nmax0;
    sel[j] = 1;
    order[t] = j;
    const double* s = W + j * len;
    const double ss = nrm[j];
    for (int64_t v = 0; v < cnt; ++v) {
      if (sel[v]) continue;
      double* w = W + v * len;
      const double c = plain_dot(s, w, len) / ss;
      for (int64_t i = 0; i < len; ++i) w[i] = fma(-c, s[i], w[i]);
      nrm[v] = plain_dot(w, w, len);
    }
  }
  free(nrm);
  free(sel);
  return t;
}

/*
 * Alg. 2 by Alg. 3: rows I and columns J chosen independently by the
 * norm-greedy rule.  A is m x n row-major (lda).  order_I / order_J (r each)
 * receive the choice order, I and J the same indices ascending; entries past
 * the rank reached are -1.  Returns ORC_OK, or ORC_ERR_RANK when either axis
 * stops short (*rank_rows / *rank_cols say where).  gap_I / gap_J (nullable,
 * r doubles each) receive each step's margin as described at greedy_axis.
 */
int oracle_greedy_select(const double* A, int64_t m, int64_t n, int64_t lda, int r, int64_t* order_I,
                         int64_t* order_J, int64_t* I, int64_t* J, int* rank_rows, int* rank_cols,
                         double* gap_I, double* gap_J) {
  return oracle_greedy_select_rc(A, m, n, lda, r, r, order_I, order_J, I, J, rank_rows, rank_cols, gap_I, gap_J);
}

/*
 * The same with a row count r and a column count c (Alg. 2 takes the two
 * separately): order_I / I hold r entries, order_J / J hold c.
 */
int oracle_greedy_select_rc(const double* A, int64_t m, int64_t n, int64_t lda, int r, int c, int64_t* order_I,
                            int64_t* order_J, int64_t* I, int64_t* J, int* rank_rows, int* rank_cols,
                            double* gap_I, double* gap_J) {
  if (!A || m < 1 || n < 1 || lda < n || r < 1 || c < 1 || r > m || c > n || r > n || c > m) return ORC_ERR_ARG;
  double* W = (double*)malloc(sizeof(double) * (size_t)(m * n));
  if (!W) return ORC_ERR_NOMEM;
  for (int64_t i = 0; i < r; ++i) order_I[i] = I[i] = -1;
  for (int64_t j = 0; j < c; ++j) order_J[j] = J[j] = -1;
  /* rows: vector i = A(i, :) */
  for (int64_t i = 0; i < m; ++i) memcpy(W + i * n, A + i * lda, sizeof(double) * (size_t)n);
  const int qr = greedy_axis(W, n, m, r, order_I, gap_I);
  /* columns: vector j = A(:, j) */
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j) W[j * m + i] = A[i * lda + j];
  const int qc = greedy_axis(W, m, n, c, order_J, gap_J);
  free(W);
  for (int t = 0; t < qr; ++t) I[t] = order_I[t];
  for (int t = 0; t < qc; ++t) J[t] = order_J[t];
  sort_i64(I, qr);
  sort_i64(J, qc);
  *rank_rows = qr;
  *rank_cols = qc;
  return (qr < r || qc < c) ? ORC_ERR_RANK : ORC_OK;
}
