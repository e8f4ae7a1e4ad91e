// Internal declarations of libcur (HIP, gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/cur.h"

namespace cur {

constexpr int kThreads = 256;      // threads per workgroup of every kernel here
constexpr int kTileRows = 256;     // rows of a row-pass tile (one row per thread)
constexpr int kMetaFields = 10;    // fields of a cur_trace meta record
constexpr int kDbgRing = 64;       // swap decisions remembered per node
// Row swaps whose Sherman-Morrison updates a pass applies on the fly instead
// of holding them in the working matrix (the pass after the last of them
// writes the matrix out again).
constexpr int kLz = 4;

// Per-node state machine.  A node is a leaf (one column block), a merge of two
// children, or a promoted copy of an odd last child.
enum NodeState : int32_t {
  ST_DONE = 0,
  ST_ACA = 1,        // next pass: ACA step (apply pending pivot, then argmax)
  ST_ROW_FRESH = 2,  // next pass: B = A(:,J) X fresh, then argmax
  ST_ROW_SWAP = 3,   // next pass: apply pending row swap to B, then argmax
  ST_START_SWAP = 4, // next ctl: start the swap loop (ROW phase start)
  ST_DEFER = 5,      // a controller step with an r x r factorization (or a column phase) is
                     // due (pend_mode); it waits for a launch that admits such steps
};

// KIND_POLISH: one node after a tree's root whose candidates are all n columns,
// started from the root's cross (cur_opts.polish).
enum NodeKind : int32_t { KIND_LEAF = 0, KIND_MERGE = 1, KIND_PROMOTED = 2, KIND_POLISH = 3 };

// Winner of one row tile in a pass.
struct Partial {
  double val;   // |x| (the magnitude compared)
  double sval;  // x   (signed value in the working precision, widened)
  int64_t key;  // scan-order key: smaller wins ties
  int64_t row;  // row index
  int32_t pos;  // column position in the working layout
  int32_t seq;  // the node's pass sequence number when written
};

struct Node {
  // ---- geometry and buffers (set by the host) ----
  int64_t m;         // rows of A
  int32_t r;         // rank
  int32_t ncmax;     // capacity of the candidate arrays
  int32_t ntiles;    // row tiles of a pass
  int32_t smax;      // swap budget
  int32_t kind;      // NodeKind
  int32_t child0, child1;  // indices into the previous level's node table (-1: none)
  int32_t seq;       // pass sequence number: stamps the tile winners of a pass
  double tau;        // swap iff |B| > 1 + tau
  double theta;      // numerical-zero pivot threshold of ACA
  void* panel;       // m x ncmax, column-major (ld m), element T: A(:, Jc)
  void* work;        // m x max(ncmax, r), column-major, FP64: ACA residual, then B
  double* X;         // r x r row-major: A(I,J)^{-1}
  double* Bc;        // r x ncmax row-major: column interpolation matrix
  double* vec;       // max(ncmax, r): pivot-row factors f (ACA) or v (row swap)
  Partial* part;     // ntiles
  int64_t* Jc;       // ncmax: original column index of each candidate (ascending)
  int32_t* colmap;   // ncmax: ACA layout position -> candidate position
  int32_t* srcpos;   // ncmax: merge: (child << 24) | position in the child's panel
  uint8_t* insel;    // ncmax: candidate currently in J
  int64_t* I;        // r: selected rows (current order)
  int32_t* Jp;       // r: selected candidate positions (current order)
  double* dbg;       // 4 x kDbgRing swap log (kind, index, slot, pivot) for diagnostics
  void* lzg;         // kLz x m, column s (ld m), FP64: the column g_s = B(:, k_s)
                     // before row swap s of the pending history
  double* lzv;       // kLz x r row-major: the factors v_s of those swaps
  const void* src;   // leaves: the matrix A this tree selects from (element T)
  int64_t lda;       // leaves: its leading dimension
  int32_t trans;     // leaves: the tree selects from A^T (its rows are the columns of src)
  int64_t col0;      // leaves: first column of the block
  void* panel_alt;   // polish node: A^T column-major (n x m, ld n), element T; the panel of
                     // its column phases, which run as row phases of A^T (panel and panel_alt,
                     // m and m_alt, ntiles and ntiles_alt trade places at each phase change)
  int64_t m_alt;     // polish node: rows of the other orientation's panel
  int32_t ntiles_alt;  // polish node: row tiles of the other orientation
  int64_t tclk[8];   // wall-clock ticks spent in controller steps (diagnostics):
                     // build, col phase, col fresh, col swaps, sort, whole ctl, LU, inverse
  // ---- dynamic state (device) ----
  int32_t nc;        // number of candidates
  int32_t st;        // NodeState
  int32_t t;         // ACA pivots accepted
  int32_t q;         // pivots held (r unless rank-short)
  int32_t steps;     // ACA step limit min(r, nc, m)
  int32_t na;        // ACA: active columns of the layout the next pass reads
  int32_t is_short, nocap, err, phase;
  int32_t phase_swaps, since, swaps, phases, refreshes;
  int32_t pend_k;    // pending pivot column position (ACA) / slot k* (row swap)
  int64_t pend_i;    // pending pivot row
  double pend_p;     // pending pivot value
  double vol_m;      // volume mantissa (finished nodes)
  int32_t vol_e;     // volume exponent
  int32_t lz;        // row swaps pending in the history (their updates are not in `work`)
  int32_t flipped;   // polish node: 1 while in the A^T orientation (I holds J, Jp holds I)
  int32_t pend_mode; // ST_DEFER: the controller step to resume
  int64_t lzi[kLz];  // row swapped in by each pending swap
  int32_t lzk[kLz];  // its slot k
};

// Host-side error reporting (thread-local last error).
void set_error(const std::string& msg);
const char* last_error();

#define CUR_HIP_CHECK(expr)                                                           \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      ::cur::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));            \
      return CUR_ERR_DEVICE;                                                          \
    }                                                                                 \
  } while (0)

}  // namespace cur

// Context (opaque to callers).
namespace cur {
// One entry of the launch-shape autotuner: a tree level's shape and the wall
// time measured for each node-group count tried on it.
struct TuneEntry {
  int64_t key[6];  // FP64, r bucket, nodes, row tiles, rows, leaf level
  double ms[3];    // wall time per candidate group count (1, 2, 3)
  int tried;       // candidates measured so far
  int fixed;       // > 0: use this group count (an imported choice)
};
}  // namespace cur

struct cur_ctx_s {
  int device;
  hipStream_t stream;
  bool own_stream;
  void* arena;          // device workspace
  size_t arena_bytes;
  int32_t* host_flag;   // pinned host word for polling
  int cu_count;
  int last_pinv;        // cur_assemble used the pseudo-inverse
  int64_t* rect_discard;  // device, 256 entries: the index sets cur_select_rect does not return
  // measurement counters (cur_profile_*)
  int prof_on;
  unsigned long long* prof_bytes;   // device byte slots, one per timed launch
  std::vector<hipEvent_t>* prof_ev; // event pairs of the current selection
  std::vector<int>* prof_kind;      // per pair: 0 pass, 1 fresh
  cur_profile prof;
  // node groups of a tree level, each iterating on a stream of its own
  // (created on first use, default priority)
  int groups_ready;
  hipStream_t gstream[4];
  hipEvent_t gfork;
  hipEvent_t gjoin[4];
  std::vector<cur::TuneEntry>* tune;  // autotuner cache of this context
};

namespace cur {
// Bump allocator over the context arena; sizes are rounded to 256 bytes.
struct Arena {
  char* base;
  size_t cap;
  size_t off;
  void* take(size_t bytes) {
    size_t b = (bytes + 255) & ~size_t(255);
    if (off + b > cap) return nullptr;
    void* p = base + off;
    off += b;
    return p;
  }
};
cur_status ensure_arena(cur_ctx ctx, size_t bytes);

// The row kernels over every node of a level in their state (pass.hip): the
// fresh interpolation matrix, and the streaming pass (ACA step or row swap).
// rb is the register bucket of r (32, 64 or 128), prof the launch's device
// byte slot or null.
constexpr int kProfSlots = 1 << 16;  // timed launches per selection call
int tune_best(const TuneEntry& e);  // fastest group count of an explored entry
cur_status ensure_groups(cur_ctx ctx);  // group streams and events of the context (select.hip)
// Norm-greedy selection of rows and columns (greedy.hip).
cur_status greedy_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n, int64_t lda, int r,
                           int64_t* I, int64_t* J, cur_info* info, cur_trace* trace);
void fresh_launch(bool f64, int rb, Node* nodes, int count, int tiles, unsigned long long* prof, hipStream_t s);
void pass_launch(bool f64, int rb, Node* nodes, int count, int tiles, unsigned long long* prof, hipStream_t s);

// Reduced-precision residual (residual_mp.hip): scratch bytes, tile count, and
// the launches that form Bm = C U and P = Bm R on MFMA and reduce E into tile
// partials.
size_t residual_mp_scratch(int64_t m, int64_t n, int r, int prec);
int64_t residual_mp_tiles(int64_t m, int64_t n);
cur_status residual_mp_launch(cur_ctx ctx, const float* A, int64_t m, int64_t n, int64_t lda, int r, const float* C,
                              const double* U, const float* R, int prec, char* scratch, size_t scratch_bytes,
                              double* part, int64_t* nb);

// Independent selections of several matrices, run together per dtype and
// rank bucket; per_item receives every item's status.
cur_status select_batched_dispatch(cur_ctx ctx, int32_t count, const cur_item* items,
                                   const std::vector<cur_opts>& opts, cur_status* per_item);

cur_status select_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n,
                           int64_t lda, int r, const cur_opts& o, int64_t* I, int64_t* J,
                           cur_info* info);
cur_status assemble_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n,
                             int64_t lda, int r, const int64_t* I, const int64_t* J, void* C,
                             double* U, void* R);
// Learned candidate proposal (propose.hip).
size_t propose_scratch(int64_t m, int64_t n, int r, int b);
template <typename T>
cur_status propose_leaves(cur_ctx ctx, const T* A, int64_t m, int64_t n, int64_t lda, int r, int w, int b,
                          const void* mlp, uint64_t seed, Node* leaves, char* scratch);
cur_status propose_features(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n, int64_t lda, int r, int w,
                            uint64_t seed, float* F);
cur_status mlp_forward_dispatch(cur_ctx ctx, const void* blob, const float* F, int64_t count, float* score);
cur_status mlp_grad_dispatch(cur_ctx ctx, const void* blob, const float* F, const float* Y, int64_t count, float pw,
                             float* grad, double* loss);
cur_status mlp_adam_dispatch(cur_ctx ctx, void* blob, float* p, float* m1, float* m2, const float* g, int t, float lr,
                             float beta1, float beta2, float eps);

// The residual entry point that allocates nothing (residual.hip): its
// scratch is a fixed device array whose address on `device` noalloc_init looks
// up (once per device, with that device current).
cur_status noalloc_init(int device);
size_t residual_noalloc_need(int64_t m, int64_t n, int r, int prec);
cur_status residual_noalloc_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n, int64_t lda,
                                     int r, const void* C, const double* U, const void* R, int prec, double* cheb,
                                     double* fro_rel);
cur_status residual_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n,
                             int64_t lda, int r, const void* C, const double* U, const void* R,
                             int prec, double* cheb, double* fro_rel);

// Rectangular cross, r rows and c columns (select.hip, greedy.hip,
// assemble.hip, residual.hip).  `discard` (device, 2 max(r, c) entries)
// receives the index sets of the two trees that are not returned.
cur_status select_rect_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n, int64_t lda,
                                int r, int c, const cur_opts& o, int64_t* I, int64_t* J, int64_t* discard,
                                cur_info* info);
cur_status greedy_rect_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n, int64_t lda,
                                int r, int c, int64_t* I, int64_t* J, cur_info* info);
cur_status assemble_rect_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n, int64_t lda,
                                  int r, int c, const int64_t* I, const int64_t* J, void* C, double* U, void* R);
cur_status residual_rect_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n, int64_t lda,
                                  int r, int c, const void* C, const double* U, const void* R, double* cheb,
                                  double* fro_rel);
}  // namespace cur
