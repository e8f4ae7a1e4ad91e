/* The CPU oracle under AddressSanitizer and UBSan: every exported function on
 * small seeded inputs (selection with and without a trace, rank-short and
 * non-finite inputs, argument errors, assembly on both branches, residual,
 * norm-greedy selection, the building blocks).  Built and run by
 * tests/test_sanitizers.py; prints OK and exits 0 when the calls return the
 * expected statuses.  The oracle's functions are declared here by hand (it
 * has no header by design). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t rank, nodes, phases, refreshes;
  int64_t swaps;
  double logvol;
  int32_t status, pad;
} orc_info;

int oracle_gepp(int r, double* G, int* perm);
void oracle_lu_inverse(int r, const double* LU, const int* perm, double* X);
void oracle_volume(int r, const double* LU, double* mant, int* expo);
int oracle_aca(const double* A, int64_t m, int64_t lda, const int64_t* cols, int nc, int r, double theta,
               int64_t* I, int64_t* J, double* piv);
int oracle_tree_size(int64_t b);
int oracle_cur_select(const double* A, int64_t m, int64_t n, int64_t lda, int r, int w, double tau, int max_swaps,
                      int64_t* I, int64_t* J, orc_info* info, int64_t* tmeta, double* tvol, int64_t* tI,
                      int64_t* tJ);
void oracle_pinv(int r, const double* G, double* P);
int oracle_cur_assemble(const double* A, int64_t m, int64_t n, int64_t lda, int r, const int64_t* I,
                        const int64_t* J, double* C, double* U, double* R, int* used_pinv);
int oracle_cur_residual(const double* A, int64_t m, int64_t n, int64_t lda, int r, const double* C,
                        const double* U, const double* R, double* cheb, double* fro_rel);
int oracle_greedy_select(const double* A, int64_t m, int64_t n, int64_t lda, int r, int64_t* order_I,
                         int64_t* order_J, int64_t* I, int64_t* J, int* rank_rows, int* rank_cols, double* gap_I,
                         double* gap_J);

static uint64_t rs = 88172645463325252ull;
static double urand(void) { /* xorshift64, uniform in (-1, 1) */
  rs ^= rs << 13; rs ^= rs >> 7; rs ^= rs << 17;
  return (double)(rs >> 11) * 0x1p-52 - 1.0;
}

int main(void) {
  int bad = 0;
  const int64_t m = 37, n = 53;
  const int r = 5, w = 8;
  double* A = malloc(sizeof(double) * m * n);
  for (int64_t k = 0; k < m * n; ++k) A[k] = urand();
  int64_t I[8], J[8], oI[8], oJ[8];
  orc_info info;
  int b = (int)(n / w), N = oracle_tree_size(b);
  int64_t* tm = malloc(sizeof(int64_t) * N * 10);
  double* tv = malloc(sizeof(double) * N);
  int64_t* tI = malloc(sizeof(int64_t) * N * r);
  int64_t* tJ = malloc(sizeof(int64_t) * N * r);
  bad |= oracle_cur_select(A, m, n, n, r, w, 0.0, 0, I, J, &info, tm, tv, tI, tJ) != 0;
  bad |= oracle_cur_select(A, m, n, n, r, 0, 0.0, 0, I, J, &info, NULL, NULL, NULL, NULL) != 0;
  bad |= oracle_cur_select(A, m, n, n, r, w, 0.0, 2, I, J, &info, NULL, NULL, NULL, NULL) < 0;
  /* argument errors */
  bad |= oracle_cur_select(A, m, n, n, 0, w, 0.0, 0, I, J, &info, NULL, NULL, NULL, NULL) != -1;
  bad |= oracle_cur_select(A, m, n, n - 1, r, w, 0.0, 0, I, J, &info, NULL, NULL, NULL, NULL) != -1;
  bad |= oracle_cur_select(A, m, n, n, r, 3, 0.0, 0, I, J, &info, NULL, NULL, NULL, NULL) != -1;
  /* assembly (LU branch), residual */
  double* C = malloc(sizeof(double) * m * r);
  double* U = malloc(sizeof(double) * r * r);
  double* R = malloc(sizeof(double) * r * n);
  int used = -1;
  bad |= oracle_cur_assemble(A, m, n, n, r, I, J, C, U, R, &used) != 0 || used != 0;
  double cheb = -1.0, fro = -1.0;
  bad |= oracle_cur_residual(A, m, n, n, r, C, U, R, &cheb, &fro) != 0 || !(cheb > 0.0);
  /* rank-deficient input: rank 2, asked for 4; assembly on the pseudo-inverse branch */
  double* L = malloc(sizeof(double) * m * n);
  double u[2][64], v[2][64];
  for (int t = 0; t < 2; ++t) {
    for (int64_t i = 0; i < m; ++i) u[t][i] = urand();
    for (int64_t j = 0; j < n; ++j) v[t][j] = urand();
  }
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j) L[i * n + j] = u[0][i] * v[0][j] + u[1][i] * v[1][j];
  bad |= oracle_cur_select(L, m, n, n, 4, w, 0.0, 0, I, J, &info, NULL, NULL, NULL, NULL) != -2;
  int64_t Ii[3] = {0, 1, 2}, Jj[3] = {0, 1, 2};
  bad |= oracle_cur_assemble(L, m, n, n, 3, Ii, Jj, C, U, R, &used) != 0 || used != 1;
  /* non-finite input */
  A[5 * n + 7] = NAN;
  bad |= oracle_cur_select(A, m, n, n, r, w, 0.0, 0, I, J, &info, NULL, NULL, NULL, NULL) != -3;
  bad |= oracle_cur_residual(A, m, n, n, 3, C, U, R, &cheb, &fro) != -3;
  A[5 * n + 7] = 0.25;
  /* norm-greedy */
  double gI[8], gJ[8];
  int qr = 0, qc = 0;
  bad |= oracle_greedy_select(A, m, n, n, r, oI, oJ, I, J, &qr, &qc, gI, gJ) != 0 || qr != r || qc != r;
  bad |= oracle_greedy_select(L, m, n, n, 4, oI, oJ, I, J, &qr, &qc, NULL, NULL) != -2 || qr != 2;
  /* building blocks */
  double G[25], X[25], P[25], mant;
  int perm[5], expo;
  for (int k = 0; k < 25; ++k) G[k] = urand();
  memcpy(P, G, sizeof(G));
  bad |= oracle_gepp(5, P, perm) != 0;
  oracle_lu_inverse(5, P, perm, X);
  oracle_volume(5, P, &mant, &expo);
  oracle_pinv(5, G, P);
  int64_t cols[8] = {0, 1, 2, 3, 4, 5, 6, 7};
  double piv[5];
  bad |= oracle_aca(A, m, n, cols, 8, 5, 1e-300, I, J, piv) != 5;
  free(A); free(L); free(C); free(U); free(R); free(tm); free(tv); free(tI); free(tJ);
  printf("%s\n", bad ? "FAIL" : "OK");
  return bad;
}
