/*
 * cur.h -- C ABI of libcur: maximal-volume CUR selection, assembly and
 * residual on one AMD Instinct MI355X (gfx950).
 *
 * Method (arXiv 2502.11017, "Scalable Binary CUR Low-Rank Approximation"):
 *   A (m x n) ~ C U R with C = A(:,J), U = A(I,J)^+, R = A(I,:)      (Sec. 1.1)
 *   I, J chosen so that |det A(I,J)| is near maximal                (Def. 1, Sec. 1.2)
 *   residual measured in the Chebyshev norm max|A - CUR|             (Thm 1, Thm 2)
 *   and as the Frobenius relative error ||A - CUR||_F / ||A||_F      (Sec. 3.1)
 * Selection: the columns are split into contiguous blocks (Alg. 3 block
 * partition); each block is started by adaptive cross approximation with
 * complete pivoting (Alg. 1) and refined by maxvol row/column swaps (the
 * maximal-volume search cited in Sec. 1.2); blocks are merged pairwise up a
 * binary tree, each merge re-running the swaps over the union of the
 * children's columns.
 *
 * Conventions common to every entry point
 *   - Matrices are row-major with a leading dimension counted in elements.
 *   - Every matrix and index pointer is a DEVICE pointer owned by the caller;
 *     the library never frees or retains it.  Outputs written by the library
 *     must not alias inputs.
 *   - Indices are 0-based int64 and are returned sorted ascending.
 *   - Argument errors (sizes, null pointers, bad options) are detected on the
 *     host before any device work and return CUR_ERR_ARG; a description of
 *     the last error of the calling thread is available from
 *     cur_last_error().
 *   - Data-dependent outcomes (non-finite input, rank shortfall, swap budget
 *     exhausted) are computed on the device; the calls are synchronous with
 *     respect to the context's stream and return them.
 *   - A context must not be used from two host threads at once.
 */
#ifndef CUR_H
#define CUR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cur_ctx_s* cur_ctx;

typedef enum {
  CUR_OK = 0,
  CUR_WARN_NOCONV = 1,    /* result valid; some node spent its swap budget, dominance not certified */
  CUR_ERR_ARG = -1,       /* invalid argument (host-side check)                                     */
  CUR_ERR_RANK = -2,      /* fewer than r pivots above the numerical-zero threshold                  */
  CUR_ERR_NONFINITE = -3, /* A holds NaN or Inf                                                      */
  CUR_ERR_DEVICE = -4,    /* a HIP call failed                                                       */
  CUR_ERR_NOMEM = -5,     /* device workspace allocation failed                                      */
  CUR_ERR_INTERNAL = -6   /* a cross that must be nonsingular was found singular                     */
} cur_status;

typedef enum { CUR_F64 = 0, CUR_F32 = 1 } cur_dtype;

/* Arithmetic of the residual GEMM E = A - (C U) R (cur_residual). */
typedef enum {
  CUR_PREC_NATIVE = 0, /* in the input dtype (FP64 or FP32)                                  */
  CUR_PREC_BF16X3 = 1, /* three BF16 products (hi*hi + hi*lo + lo*hi), FP32 accumulation    */
  CUR_PREC_FP8 = 2     /* two-term e4m3 split with per-tile scales, FP32 accumulation        */
} cur_prec;

/* Per-node record of the selection tree (optional, for inspection and tests).
 * Nodes are listed level by level (leaves first), index ascending; an odd
 * last node of a level is promoted to the next level unchanged. */
typedef struct {
  int32_t capacity;  /* number of records the arrays below can hold               */
  int32_t count;     /* written: number of records                                */
  int64_t* meta;     /* host, capacity x 10: level, index, q, short, promoted,
                        nocap, swaps, phases, refreshes, volume exponent          */
  double* vol_mant;  /* host, capacity: volume mantissa in [0.5,1) (0 if short)   */
  int64_t* I;        /* host, capacity x r (unused entries -1)                    */
  int64_t* J;        /* host, capacity x r                                        */
} cur_trace;

typedef struct {
  int32_t struct_size; /* sizeof(cur_opts), for ABI versioning                                   */
  int32_t col_block;   /* leaf column-block width w; 0 -> max(64, r); must be >= r               */
  double tau;          /* a swap happens iff |B| > 1 + tau; 0 -> 1e-13                           */
  int32_t max_swaps;   /* swap budget per tree node; 0 -> 64 r                                   */
  int32_t prec;        /* cur_prec of the assembly/residual GEMMs (selection itself is exact)    */
  int32_t propose;     /* 0: no candidate proposal; 1: learned proposal for the leaves (mlp, seed;
                          see "Learned candidate proposal" below; r <= 64, cur_select only)    */
  int32_t groups;      /* node groups per tree level, each iterating on a stream of its own:
                          0 -> autotuned per level shape (the first calls on a shape try 1, 2
                          and 3 groups once each, later calls use the fastest); 1..3 fixed.
                          The result does not depend on it.                                     */
  const void* mlp;     /* propose == 1: device weight blob (CUR_MLP_BLOB_BYTES); else NULL       */
  uint64_t seed;       /* propose == 1: seed of the Gaussian sketch of the leverage feature      */
  cur_trace* trace;    /* host pointer or NULL: per-node tree records                            */
  int32_t method;      /* 0: maximal-volume tree (Alg. 1 leaves, swap loops, binary merge);
                          1: norm-greedy rows and columns (Alg. 2 with Alg. 3): r times the
                          row (column) of largest norm, projected out of all rows (columns);
                          col_block, tau, max_swaps and groups do not apply, info->logvol is
                          NaN, cur_select_batched rejects it, and a trace (capacity >= 1)
                          receives one record whose I and J list the rows and columns in the
                          order chosen (q = rank reached, short = 1 if below r)               */
  int32_t polish;      /* method 0: 0 none; 1 after the tree, the same swap loop
                          once more on the whole matrix: every column is a candidate and the
                          start is the root's cross, so that on return (status CUR_OK) every
                          entry of A(:,J) A(I,J)^-1 and of A(I,J)^-1 A(I,:) is at most 1 + tau
                          in magnitude (Sec. 1.1's condition on all of A).  Costs one more
                          tree level with an m x n copy of A in the workspace; needs
                          r * n < 2^31.  A trace gets one more record (the level after the
                          root, index 0).  A rank-short root is returned as it is, with no
                          further record and no node counted.  cur_select_rect with r == c:
                          the same loop on the cross (I, J) of its two trees (the symmetric
                          form of Alg. 2), skipped if either tree falls short; info.logvol
                          is then that cross's.  cur_select_batched: every item's tree
                          gets its polish level.                                         */
} cur_opts;

typedef struct {
  int32_t rank;      /* r, or the number q < r of pivots found (CUR_ERR_RANK)  */
  int32_t nodes;     /* leaves + merges processed                             */
  int32_t phases;    /* swap phases over all nodes                            */
  int32_t refreshes; /* fresh interpolation-matrix computations              */
  int64_t swaps;     /* row + column swaps over all nodes                     */
  double logvol;     /* log|det A(I,J)| of the result (fresh LU)              */
} cur_info;

/* Fill *opts with the defaults (struct_size set, everything else zero). */
void cur_opts_init(cur_opts* opts);

/* Create a context on HIP device `device`.  `hip_stream` (a hipStream_t) is
 * used for all work; NULL means the device's default (null) stream, as a NULL
 * hipStream_t does in every HIP call, so work is ordered with everything else
 * issued there (PyTorch's default stream is that null stream).  A caller that
 * wants the library on a private stream creates one and passes it.  The
 * context owns a device workspace that grows on demand. */
cur_status cur_create(cur_ctx* out, int device, void* hip_stream);
cur_status cur_destroy(cur_ctx ctx);
const char* cur_strerror(cur_status s);
/* Description of the last error returned to the calling thread ("" if none). */
const char* cur_last_error(void);

/*
 * Selection (Def. 1 objective, Alg. 1 leaf start, Alg. 3 block partition,
 * binary merge tree).
 *   dtype  a cur_dtype value (passed as int32_t so that any integer a caller
 *          passes is a valid argument; others are CUR_ERR_ARG)
 *   A      device, m x n, row-major, leading dimension lda >= n, dtype `dtype`
 *   r      1 <= r <= min(m, n) and r <= 128; m x 8 bytes must be below
 *          4 GiB (the row kernels address one FP64 column with 32-bit
 *          offsets), CUR_ERR_ARG otherwise
 *   opts   NULL for defaults
 *   I, J   device int64[r]: selected rows and columns, ascending.  On
 *          CUR_ERR_RANK the first info->rank entries hold the pivots found and
 *          the rest are -1.
 *   info   host, nullable
 * The FP64 path computes exactly the sequence of decisions of the documented
 * algorithm (bit-identical arithmetic in every decision-relevant quantity).
 * FP32 input is widened exactly and the selection computes in FP64 (the
 * candidate panels stay FP32), so it makes the decisions of the FP64 path on
 * the widened values: the same result as the FP64 call on A converted to
 * double.
 * Workspace (grown on demand, kept by the context): per tree node, an m x |Jc|
 * candidate panel in the input's element type, an FP64 working matrix of
 * m x max(|Jc|, r) and 4 FP64 m-element columns of pending row-swap history,
 * plus O(r^2) doubles (8192 x 8192 FP64 with r = 64: ~8.3 MiB per leaf,
 * ~3 GiB in all).
 */
cur_status cur_select(cur_ctx ctx, int32_t dtype, const void* A, int64_t m, int64_t n, int64_t lda,
                      int32_t r, const cur_opts* opts, int64_t* I, int64_t* J, cur_info* info);

/*
 * Assembly (Sec. 1.1): C = A(:,J) (m x r, ld r, dtype), R = A(I,:) (r x n,
 * ld n, dtype), U = A(I,J)^+ (r x r, ld r, FP64).  U is the inverse from LU
 * with partial pivoting, or, when a pivot is zero or min|u_kk|/max|u_kk| <
 * r 2^-52, the pseudo-inverse from a one-sided Jacobi SVD with singular values
 * below r 2^-52 sigma_max dropped.  I, J: device int64[r], each in range.
 */
cur_status cur_assemble(cur_ctx ctx, int32_t dtype, const void* A, int64_t m, int64_t n, int64_t lda,
                        int32_t r, const int64_t* I, const int64_t* J, void* C, double* U, void* R);

/*
 * Residual (Thm 1 Chebyshev norm, Sec. 3.1 Frobenius error) of the factors of
 * cur_assemble: E = A - (C U) R, never stored.
 *   cheb     host: max |E(i,j)|
 *   fro_rel  host, nullable: ||E||_F / ||A||_F
 *   prec     cur_prec of the GEMM (NATIVE for FP64 input; NATIVE, BF16X3 or
 *            FP8 for FP32 input).  U is always FP64; C U is formed in FP64.
 * Returns CUR_ERR_NONFINITE (with *cheb NaN or infinite) when some entry of
 * A - C U R is NaN or infinite, e.g. from a non-finite input.
 */
cur_status cur_residual(cur_ctx ctx, int32_t dtype, const void* A, int64_t m, int64_t n, int64_t lda,
                        int32_t r, const void* C, const double* U, const void* R, int32_t prec,
                        double* cheb, double* fro_rel);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): cur_residual
 * with the same arguments, results and kernels, but every temporary (the
 * m x r product C U in FP64, the split operands of the BF16X3 / FP8 forms, the
 * per-tile partial sums) placed in a fixed device array of
 * CUR_NOALLOC_SCRATCH_BYTES that the library holds on each GPU, instead of the
 * context's growable workspace.  The call allocates nothing (no hipMalloc, no
 * hipFree); the array is set up by cur_create on each device (with that device
 * current) and lives until the process ends.
 *   Limit: the call needs, with align() rounding up to 256 bytes and
 *   T = ceil(m/128) ceil(n/128) tiles,
 *     align(8 m r) + align(24 T) + align(24576) + 256 bytes (NATIVE);
 *     align(24 T) + align(24576) + 2 align(s m r32) + 2 align(s n r32)
 *       + 2 align(s r32 r32) + align(4 ceil(m/16)) + align(4 ceil(n/16))
 *       + align(4 r32/16) + 512 bytes (BF16X3: s = 2, FP8: s = 1),
 *   r32 = r rounded up to a multiple of 32.  A call needing more than
 *   CUR_NOALLOC_SCRATCH_BYTES returns CUR_ERR_ARG before any device work
 *   (e.g. FP64 with m = n = 8192, r = 64 needs 4.1 MiB; NATIVE fits m r up to
 *   about 2 million).
 *   Sharing: every call on one GPU, from any context or thread, uses that
 *   GPU's one array, which keeps the last call's contents.  Calls that overlap
 *   in time on one GPU (two streams, two host threads) race on it and may
 *   return wrong results: serialize them.  Nothing in it needs to start at
 *   zero.
 */
#define CUR_NOALLOC_SCRATCH_BYTES (16u << 20)
cur_status cur_residual_noalloc(cur_ctx ctx, int32_t dtype, const void* A, int64_t m, int64_t n, int64_t lda,
                                int32_t r, const void* C, const double* U, const void* R, int32_t prec,
                                double* cheb, double* fro_rel);

/* One independent selection of a batch. */
typedef struct {
  int32_t dtype; /* cur_dtype                        */
  int32_t r;
  const void* A; /* device                           */
  int64_t m, n, lda;
  int64_t* I;    /* device int64[r]                  */
  int64_t* J;    /* device int64[r]                  */
} cur_item;

/*
 * Batched selection of `count` independent matrices of any shapes and ranks
 * (same rules as cur_select for each item).  per_item: host cur_status[count]
 * (nullable); the return value is the worst status (errors before warnings).
 * opts->trace must be NULL.
 */
cur_status cur_select_batched(cur_ctx ctx, int32_t count, const cur_item* items, const cur_opts* opts,
                              cur_status* per_item);

/*
 * Rectangular cross (Alg. 2 takes a row count r and a column count c and
 * chooses I and J independently, each along its own axis; Sec. 1.1 and the
 * overview define U as the pseudo-inverse of A(I,J)).
 *
 * cur_select_rect: I (device int64[r], ascending) and J (device int64[c],
 * ascending).  opts->method 0: J from the column-block maximal-volume tree on
 * A with rank c, I from the same tree on A^T (the row blocks of A) with rank
 * r, each tree's other index set dropped; col_block (0 -> max(64, r, c), and
 * >= max(r, c)), tau, max_swaps and groups apply to both trees.  method 1: the
 * norm-greedy rule (Alg. 3) on rows (r) and on columns (c).  Requires
 * 1 <= r, c <= min(m, n) and r, c <= 128; no trace, no learned proposal.
 * Status: CUR_ERR_RANK if either axis is rank-short (entries past the rank
 * reached are -1), else CUR_WARN_NOCONV if either tree spent its swap budget.
 * info (nullable): rank = the smaller of the two ranks reached, swaps /
 * phases / refreshes / nodes summed over both trees, logvol NaN.
 * opts->polish = 1 (method 0, r == c only, else CUR_ERR_ARG): then the swap
 * loop on the square cross (I, J) of the two trees with every column a
 * candidate, one more node whose counters are added to info; logvol is then
 * log |det A(I,J)| of the result.  Skipped when either tree is rank-short.
 */
cur_status cur_select_rect(cur_ctx ctx, int32_t dtype, const void* A, int64_t m, int64_t n, int64_t lda, int32_t r,
                           int32_t c, const cur_opts* opts, int64_t* I, int64_t* J, cur_info* info);
/* C = A(:,J) (device, m x c row-major, element dtype), R = A(I,:) (r x n),
 * U = A(I,J)^+ (device FP64, c x r row-major) by one-sided Jacobi on the
 * taller of A(I,J) and its transpose, cut-off max(r, c) 2^-52 sigma_max.
 * Requires min(r, c) <= 64 and max(r, c) <= 128. */
cur_status cur_assemble_rect(cur_ctx ctx, int32_t dtype, const void* A, int64_t m, int64_t n, int64_t lda,
                             int32_t r, int32_t c, const int64_t* I, const int64_t* J, void* C, double* U, void* R);
/* Residual max |A - C U R| and ||A - C U R||_F / ||A||_F of the factors of
 * cur_assemble_rect (C m x c, U c x r, R r x n), in the input's arithmetic
 * (FP64 products on MFMA); CUR_ERR_NONFINITE as for cur_residual. */
cur_status cur_residual_rect(cur_ctx ctx, int32_t dtype, const void* A, int64_t m, int64_t n, int64_t lda, int32_t r,
                             int32_t c, const void* C, const double* U, const void* R, double* cheb, double* fro_rel);

/*
 * Learned candidate proposal (cur_opts.propose = 1).
 * A small MLP scores every row of every leaf block from four features; the
 * leaf's 4r best rows are the candidates of a restricted start (adaptive
 * cross approximation, Alg. 1, on the 4r candidate rows x the block's
 * columns, held on chip) that replaces the r elimination passes over all m
 * rows.  The leaf then runs the ordinary swap loop from that start: its first
 * row phase forms A(:,J) A(I,J)^-1 over all m rows (verification) and swaps
 * in every row of |B| > 1 + tau (fallback to plain maxvol), so every node
 * still ends dominant; the selection may reach another dominant cross than
 * the plain method.  A leaf whose candidate elimination finds a pivot at or
 * below the rank threshold, or whose 4r x |block| submatrix exceeds
 * 16384 doubles, keeps the plain start.
 * Features of row i in leaf k, FP32, four per (leaf, row), leaf-major
 * (F[(k m + i) 4 + f]):
 *   f0 = log2 ||A(i, block_k)||^2 - log2 max_i ||A(i, block_k)||^2
 *   f1 = log2(l_i m / s), l_i the leverage of row i in the column space of the
 *        Gaussian sketch A Omega (Omega n x s, s = 2r, entries from a
 *        counter-based generator of `seed`), by CholeskyQR2
 *   f2 = log2(lb_i m / w_k), lb_i = a_i^T (A_k^T A_k + lambda I)^-1 a_i the
 *        ridge leverage of a_i = A(i, block_k) in A_k = A(:, block_k) (width
 *        w_k), lambda = 2^-20 max_j ||A_k(:, j)||^2
 *   f3 = share of the leaf's rows with a larger f2 (1024-bin histogram)
 * Network: score = w3 . relu(W2 relu(W1 f + b1) + b2) + b3, W1 128 x 4,
 * W2 128 x 128, w3 128, FP16; biases FP32; FP32 accumulation.  Blob layout
 * (bytes): W1 at 0 (row-major [128][4] FP16), W2 at 1024 ([128][128] FP16),
 * w3 at 33792 (FP16), b1 at 34048 (FP32 [128]), b2 at 34560, b3 at 35072.
 * Parameter vector (FP32, CUR_MLP_PARAMS): W1, b1, W2, b2, w3, b3 in that
 * order, each row-major.
 */
#define CUR_MLP_FEATURES 4
#define CUR_MLP_HIDDEN 128
#define CUR_MLP_PARAMS 17281
#define CUR_MLP_BLOB_BYTES 35328
/* Features of every (leaf, row) of A for blocks of width col_block (0 ->
 * max(64, r)): F device float[b m 4] with b = max(1, n / col_block). */
cur_status cur_mlp_features(cur_ctx ctx, int32_t dtype, const void* A, int64_t m, int64_t n, int64_t lda, int32_t r,
                            int32_t col_block, uint64_t seed, float* F);
/* Scores of count feature rows (F device float[count 4] -> score device float[count]). */
cur_status cur_mlp_forward(cur_ctx ctx, const void* blob, const float* F, int64_t count, float* score);
/* Gradient of the mean weighted logistic loss
 *   (1/count) sum_i [ pos_weight y_i softplus(-s_i) + (1 - y_i) softplus(s_i) ]
 * with respect to the parameter vector: grad device float[CUR_MLP_PARAMS];
 * y device float[count] in [0, 1]; loss host (nullable).  Deterministic. */
cur_status cur_mlp_grad(cur_ctx ctx, const void* blob, const float* F, const float* y, int64_t count,
                        float pos_weight, float* grad, double* loss);
/* One Adam step (bias-corrected, step >= 1) on the FP32 parameter vector
 * params with moments m1, m2 (device float[CUR_MLP_PARAMS] each); writes the
 * updated weights into blob (FP16 weights, FP32 biases).  With lr = 0 it only
 * packs params into blob. */
cur_status cur_mlp_adam(cur_ctx ctx, void* blob, float* params, float* m1, float* m2, const float* grad, int32_t step,
                        float lr, float beta1, float beta2, float eps);

/* Measurement counters of the selection's row kernels.  While enabled,
 * cur_select and cur_select_batched bracket every launch of the two row
 * kernels with HIP events on the stream it is issued on, and count on the
 * device two byte figures per launch:
 *   bytes          what this implementation must move: every element of the
 *                  working and history columns it reads plus every element
 *                  it writes, once (row swaps are applied lazily, so a swap
 *                  pass reads r + S columns and writes one);
 *   bytes_inplace  what the plain in-place algorithm moves for the same
 *                  steps: an elimination step with t pivots reads and writes
 *                  the nc - t active columns, a row swap reads and writes the
 *                  m x r matrix B, a fresh B reads A(:, J) and writes B, all
 *                  in the input's element size.
 * for the two kernels:
 *   pass   the streaming sweep: ACA rank-1 updates and Sherman-Morrison row
 *          swaps over the m x (active columns) working matrix;
 *   fresh  fresh interpolation matrices B = A(:, J) A(I, J)^-1.
 * A launch is "busy" when at least one node of it moved bytes; the others
 * found no node in their state and returned at once. */
typedef struct {
  int64_t launches;        /* pass launches timed                                 */
  int64_t busy;            /* pass launches in which some node had work           */
  double seconds;          /* summed event time of the pass launches              */
  double bytes;            /* summed bytes of the pass launches (implementation)  */
  int64_t fresh_launches;  /* the same figures for the fresh kernel               */
  int64_t fresh_busy;
  double fresh_seconds;
  double fresh_bytes;
  double bytes_inplace;        /* summed in-place-algorithm bytes, pass launches  */
  double fresh_bytes_inplace;  /* the same for the fresh launches                 */
  double busy_seconds;         /* summed event time of the busy pass launches     */
  double fresh_busy_seconds;   /* the same for the fresh launches                 */
} cur_profile;

/* The launch-shape autotuner cache of a context (cur_opts.groups == 0).  One
 * entry per tree-level shape: key = {FP64 (1) or FP32 (0), r bucket (32, 64
 * or 128), nodes in the level, row tiles per node, rows, leaf level (1/0)};
 * ms = wall time measured for 1, 2 and 3 node groups (tried of them so far);
 * groups = the count in use: the fastest once all three are measured, an
 * imported choice, or 0 while still exploring.  Export copies up to `cap`
 * entries to a host array (count = entries in the cache); import replaces the
 * cache, and an entry with groups > 0 is then used as is, with no exploring.
 * Lets a caller keep tuned choices across processes. */
typedef struct {
  int64_t key[6];
  double ms[3];
  int32_t tried;
  int32_t groups;
} cur_tune_entry;
cur_status cur_tune_export(cur_ctx ctx, cur_tune_entry* out, int32_t cap, int32_t* count);
cur_status cur_tune_import(cur_ctx ctx, const cur_tune_entry* in, int32_t count);

/* Set the counters: 0 off, 1 the pass kernel, 2 the pass and fresh kernels
 * (each timed launch adds two events to its stream); any call clears them. */
cur_status cur_profile_enable(cur_ctx ctx, int enable);
/* Copy the counters accumulated since enabling (host struct). */
cur_status cur_profile_read(cur_ctx ctx, cur_profile* out);

#ifdef __cplusplus
}
#endif
#endif /* CUR_H */
