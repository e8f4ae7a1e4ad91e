// Maximal-volume CUR selection on gfx950: column-block leaves started by
// adaptive cross approximation (Alg. 1), maxvol row/column swap phases, and a
// binary merge tree over the blocks (Alg. 3 block partition, merged pairwise).
//
// Execution model.  A tree level is a table of nodes.  The host repeats two
// launches until every node of the level is finished:
//   k_pass  grid (row tiles x nodes), in pass.hip: the bandwidth-bound sweep
//           over a node's m x (active columns) working matrix -- an ACA rank-1
//           update, a row swap (Sherman-Morrison) update, or a fresh
//           B = A(:,J) A(I,J)^-1 -- fused with the per-tile argmax of the next
//           decision;
//   k_ctl   one workgroup per node: reduces the tile winners (the global
//           maximum of Alg. 3), takes the decision of the documented algorithm
//           and does the small serial work (r x r LU and inverse, the column
//           phase on the r x |Jc| matrix, sorting, the final volume).
// No kernel waits on another workgroup, so every launch ends by construction;
// the host bounds the number of iterations.
//
// Layouts: every node keeps its candidate columns A(:, Jc) as a compact
// column-major panel (m x |Jc|, leading dimension m) so that every pass reads
// and writes whole columns with unit stride across a wavefront.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <array>
#include <vector>

#include "cur_device.hpp"
#include "cur_internal.hpp"

namespace cur {

// Rows per thread block of the transposing panel copy.
constexpr int kTR = 64;

// ---------------------------------------------------------------- a0: input scan
// max|A| and a non-finite flag of every matrix of a call in one launch:
// grid.y = matrix, workgroups stride over its rows, threads over a row's
// columns (coalesced, no index division).  out[2 j]: max bits of matrix j
// (non-negative doubles order like their bit patterns), out[2 j + 1]: its
// non-finite flag.
struct ScanItem {
  const void* A;
  int64_t m, n, lda;
};

template <typename T>
__global__ __launch_bounds__(kThreads) void k_amax(const ScanItem* __restrict__ items, unsigned long long* out) {
  const ScanItem it = items[blockIdx.y];
  const T* A = (const T*)it.A;
  double mx = 0.0;
  int bad = 0;
  for (int64_t i = blockIdx.x; i < it.m; i += gridDim.x) {
    const T* row = A + i * it.lda;
    for (int64_t j = threadIdx.x; j < it.n; j += kThreads) {
      const double v = (double)row[j];
      if (!isfinite(v)) bad = 1;
      else mx = fmax(mx, fabs(v));
    }
  }
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, s, 64));
    bad |= __shfl_xor(bad, s, 64);
  }
  __shared__ double smx[kThreads / 64];
  __shared__ int sbad[kThreads / 64];
  if ((threadIdx.x & 63) == 0) {
    smx[threadIdx.x >> 6] = mx;
    sbad[threadIdx.x >> 6] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / 64; ++w) {
      mx = fmax(mx, smx[w]);
      bad |= sbad[w];
    }
    atomicMax(&out[2 * blockIdx.y], (unsigned long long)__double_as_longlong(mx));
    if (bad) atomicOr(&out[2 * blockIdx.y + 1], 1ull);
  }
}

// ---------------------------------------------------------------- leaf set-up
// panel(:, c) = A(:, c0 + c) for each leaf's block (the leaf's own matrix; a
// polish node's block is every column),
// transposed through LDS.  grid (row tiles, column tiles of 64, leaves).  A
// tree over A^T (trans) reads panel column c from row c0 + c of the source,
// which is already contiguous (lanes along it).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_panel_from_A(Node* nodes) {
  Node& nd = nodes[blockIdx.z];
  if (nd.kind != KIND_LEAF && nd.kind != KIND_POLISH) return;
  const int64_t m = nd.m;
  const int nc = nd.nc;
  const int64_t r0 = (int64_t)blockIdx.x * kTR;
  const int cb = blockIdx.y * 64;
  if (r0 >= m || cb >= nc) return;
  __shared__ T tile[kTR][65];
  const T* A = (const T*)nd.src;
  const int64_t lda = nd.lda, c0 = nd.col0;
  if (nd.trans) {
    T* P = (T*)nd.panel;
    for (int idx = threadIdx.x; idx < kTR * 64; idx += kThreads) {
      const int cc = idx / kTR, rr = idx % kTR;
      const int64_t i = r0 + rr;
      if (i < m && cb + cc < nc) P[(int64_t)(cb + cc) * m + i] = A[(c0 + cb + cc) * lda + i];
    }
    return;
  }
  // read kTR rows x 64 columns, lanes along the row
  for (int idx = threadIdx.x; idx < kTR * 64; idx += kThreads) {
    const int rr = idx >> 6, cc = idx & 63;
    const int64_t i = r0 + rr;
    if (i < m && cb + cc < nc) tile[rr][cc] = A[i * lda + c0 + cb + cc];
  }
  __syncthreads();
  T* P = (T*)nd.panel;
  for (int idx = threadIdx.x; idx < kTR * 64; idx += kThreads) {
    const int cc = idx / kTR, rr = idx % kTR;
    const int64_t i = r0 + rr;
    if (i < m && cb + cc < nc) P[(int64_t)(cb + cc) * m + i] = tile[rr][cc];
  }
}

// Leaf candidate lists: Jc = c0 + [0, nc), identity layout map.
__global__ void k_leaf_init(Node* nodes) {
  Node& nd = nodes[blockIdx.x];
  for (int c = threadIdx.x; c < nd.nc; c += blockDim.x) {
    nd.Jc[c] = nd.col0 + c;
    nd.colmap[c] = c;
  }
}

// A node that starts from a given cross (r original row and column indices;
// its candidate list is the identity, so J's positions are the indices).
__global__ void k_start_cross(Node* nd, const int64_t* __restrict__ I, const int64_t* __restrict__ J) {
  for (int k = threadIdx.x; k < nd->r; k += blockDim.x) {
    nd->I[k] = I[k];
    nd->Jp[k] = (int32_t)J[k];
  }
}

// ---------------------------------------------------------------- merge set-up
// One workgroup per node of the new level.  Promoted nodes copy their child.
// Merges form Jc as the sorted union of the children's selected columns, the
// source map of the panel, and the starting (I, J) from the child of larger
// volume (exact tie: left), or prepare an ACA start when both children are
// rank-short.
__global__ __launch_bounds__(kThreads) void k_merge_init(Node* nodes, const Node* prev) {
  Node& nd = nodes[blockIdx.x];
  const int tid = threadIdx.x;
  const int r = nd.r;
  if (nd.kind == KIND_POLISH) {
    // candidates: every column (Jc the identity); start: the root's cross,
    // J as positions in Jc, i.e. original indices; a rank-short or failed
    // root is passed on unchanged
    const Node& c = prev[nd.child0];
    for (int cc = tid; cc < nd.nc; cc += blockDim.x) {
      nd.Jc[cc] = cc;
      nd.colmap[cc] = cc;
    }
    const int q = c.q;
    for (int k = tid; k < q; k += blockDim.x) {
      nd.I[k] = c.I[k];
      nd.Jp[k] = (int32_t)c.Jc[c.Jp[k]];
    }
    if (tid == 0) {
      nd.q = q;
      nd.t = q;
      nd.is_short = c.is_short;
      nd.vol_m = c.vol_m;
      nd.vol_e = c.vol_e;
      nd.err = c.err;
      nd.swaps = nd.phases = nd.refreshes = 0;
      nd.nocap = 0;
      nd.phase = nd.phase_swaps = nd.since = 0;
      nd.st = (c.is_short || c.err) ? ST_DONE : ST_START_SWAP;
    }
    return;
  }
  if (nd.kind == KIND_PROMOTED) {
    const Node& c = prev[nd.child0];
    for (int k = tid; k < r; k += blockDim.x) {
      nd.I[k] = c.I[k];
      nd.Jp[k] = c.Jp[k];
    }
    if (tid == 0) {
      nd.nc = c.nc;
      nd.q = c.q;
      nd.t = c.t;
      nd.is_short = c.is_short;
      nd.vol_m = c.vol_m;
      nd.vol_e = c.vol_e;
      nd.err = c.err;
      nd.st = ST_DONE;  // counted by the level's start-up controller launch
    }
    return;
  }
  const Node& L = prev[nd.child0];
  const Node& R = prev[nd.child1];
  // The merged list is the sorted union of two ascending lists of original
  // column indices (the children's J, at most 128 each).  Each entry's place
  // is its rank in its own list plus the number of entries of the other list
  // placed before it, the serial merge's rule (equal indices: the right
  // child's first), counted over copies staged in LDS by all threads at once.
  __shared__ int64_t sjl[128], sjr[128];
  __shared__ int s_src;
  const int qL = L.q, qR = R.q;
  for (int a = tid; a < qL; a += blockDim.x) sjl[a] = L.Jc[L.Jp[a]];
  for (int b = tid; b < qR; b += blockDim.x) sjr[b] = R.Jc[R.Jp[b]];
  if (tid == 0) {
    // the starting cross: from the child of larger volume (exact tie: left),
    // or an ACA start (src = -1) when both children are rank-short
    int src = -1;
    if (!L.is_short && !R.is_short) {
      const bool rg = (R.vol_e != L.vol_e) ? (R.vol_e > L.vol_e) : (R.vol_m > L.vol_m);
      src = rg ? 1 : 0;
    } else if (!L.is_short || !R.is_short) {
      src = L.is_short ? 1 : 0;
    }
    s_src = src;
  }
  __syncthreads();
  const int src = s_src;
  for (int a = tid; a < qL; a += blockDim.x) {
    const int64_t ja = sjl[a];
    int before = 0;
    for (int b = 0; b < qR; ++b) before += sjr[b] <= ja;
    const int cc = a + before;
    nd.Jc[cc] = ja;
    nd.srcpos[cc] = (0 << 24) | L.Jp[a];
    nd.colmap[cc] = src < 0 ? cc : a;
    if (src == 0) nd.Jp[a] = cc;
  }
  for (int b = tid; b < qR; b += blockDim.x) {
    const int64_t jb = sjr[b];
    int before = 0;
    for (int a = 0; a < qL; ++a) before += sjl[a] < jb;
    const int cc = b + before;
    nd.Jc[cc] = jb;
    nd.srcpos[cc] = (1 << 24) | R.Jp[b];
    nd.colmap[cc] = src < 0 ? cc : ((1 << 24) | b);
    if (src == 1) nd.Jp[b] = cc;
  }
  if (src >= 0) {
    const Node& S = src ? R : L;
    for (int k = tid; k < r; k += blockDim.x) nd.I[k] = S.I[k];
  }
  if (tid == 0) {
    const int c = qL + qR;
    nd.nc = c;
    nd.swaps = nd.phases = nd.refreshes = 0;
    nd.nocap = nd.err = 0;
    nd.phase = nd.phase_swaps = nd.since = 0;
    nd.vol_m = 0.0;
    nd.vol_e = 0;
    if (src >= 0) {
      nd.is_short = 0;
      nd.q = r;
      nd.t = r;
      nd.st = ST_START_SWAP;
    } else {
      nd.steps = min(r, c);
      if ((int64_t)nd.steps > nd.m) nd.steps = (int)nd.m;
      nd.is_short = 0;
      nd.q = 0;
      nd.t = 0;
      nd.na = c;
      if (nd.steps == 0) {
        nd.is_short = 1;
        nd.st = ST_DONE;  // counted by the level's start-up controller launch
      } else {
        nd.st = ST_ACA;
      }
    }
  }
}

// parent panel column c = child panel column (srcpos), for all merge nodes
template <typename T>
__global__ __launch_bounds__(kThreads) void k_panel_build(Node* nodes, const Node* prev) {
  Node& nd = nodes[blockIdx.z];
  if (nd.kind != KIND_MERGE) return;
  const int c = blockIdx.y;
  if (c >= nd.nc) return;
  const int sp = nd.srcpos[c];
  const Node& ch = prev[(sp >> 24) ? nd.child1 : nd.child0];
  const T* src = (const T*)ch.panel + (int64_t)(sp & 0xffffff) * nd.m;
  T* dst = (T*)nd.panel + (int64_t)c * nd.m;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nd.m;
       i += (int64_t)gridDim.x * kThreads)
    dst[i] = src[i];
}

// ---------------------------------------------------------------- the controller
enum CtlMode : int32_t {
  M_EXIT = 0,
  M_ROW_START = 100,
  M_ROW_END = 101,
  M_COL = 102,
  M_FINISH = 103,
  M_FINISH_SHORT = 104,
  M_REFRESH = 105,
  M_SWAPVEC = 106,
  M_FLIP = 108,      // polish node: change orientation, then the next phase as a row phase
};

struct CtlShared {
  int mode;
  int pend_mode;
  int stale;
  int st, t, q, na, steps, nc;
  int is_short, nocap, err, phase, phase_swaps, since, swaps, phases, refreshes;
  int pend_k;
  int64_t pend_i;
  double pend_p;
  double vol_m;
  int vol_e;
  int lz;
  int spiv;
  int wtile;
  Cand win;
};

// LDS of the register LU, present only where it is used.
template <int RMAX, bool REG = (RMAX <= 64)>
struct LuLds : LuScratch {};
template <int RMAX>
struct LuLds<RMAX, false> {};

template <typename T, int RMAX>
struct CtlLds {
  static constexpr int CH = RMAX <= 64 ? RMAX : 16;     // inverse column chunk
  static constexpr int BCCAP = RMAX <= 64 ? 8192 : 1;  // doubles of Bc kept in LDS
  static constexpr int INSCAP = 4096;                  // candidate flags kept in LDS
  double A[RMAX * RMAX];   // G / LU, later X
  double B[RMAX * CH];     // inverse chunk, later columns of A(I, Jc)
  double Bcl[BCCAP];       // column interpolation matrix when it fits
  double lk[RMAX];         // LU multipliers of one elimination step
  int64_t sI[RMAX];        // working copies of I and Jp
  int32_t sJp[RMAX];
  int perm[RMAX];
  int64_t tmp64[RMAX];
  int tmp32[RMAX];
  static constexpr int ROWKCAP = 256;
  uint8_t insel[INSCAP];
  int slot[kThreads];      // column phase: slot k of a selected candidate, -1 otherwise
  double wv[RMAX];
  double rowk[ROWKCAP];
  Cand sc[kThreads / 64];
  CtlShared s;
  LuLds<RMAX> lu;          // register LU hand-off (r <= 64)
};

// Append one swap decision to the node's diagnostic ring (thread 0 only).
__device__ __forceinline__ void dbg_log(Node& nd, int count, double kind, double idx, double slot, double piv) {
  double* d = nd.dbg + 4 * (count % kDbgRing);
  d[0] = kind;
  d[1] = idx;
  d[2] = slot;
  d[3] = piv;
}

// Reduce the tile winners of the last pass (the global argmax of the node).
template <typename T, int RMAX>
__device__ void ctl_reduce(Node& nd, CtlLds<T, RMAX>& L) {
  Cand b = cand_none();
  const int seq = nd.seq;
  int stale = 0;
  for (int tl = threadIdx.x; tl < nd.ntiles; tl += kThreads) {
    const Partial p = nd.part[tl];
    stale |= (p.seq != seq);  // a tile winner this pass did not write
    Cand o;
    o.val = p.val;
    o.sval = p.sval;
    o.key = p.key;
    o.row = p.row;
    o.pos = p.pos;
    cand_take(b, o);
  }
  b = block_argmax(b, L.sc);
  stale = __syncthreads_or(stale);
  if (threadIdx.x == 0) {
    L.s.stale = stale;
    L.s.win = b;
    L.s.wtile = b.row >= 0 ? (int)(b.row / kTileRows) : -1;
    if (L.s.stale) L.s.err = 120;
  }
  __syncthreads();
}

// G = A(I, J) for the current orders, LU, X = G^{-1} to nd.X (and, for
// r <= 64, to L.A); optionally the volume instead of X.  Returns false on a
// singular G.
template <typename T, int RMAX>
__device__ bool ctl_build_impl(Node& nd, CtlLds<T, RMAX>& L, bool want_X, bool want_vol) {
  const int r = nd.r;
  const int64_t m = nd.m;
  const T* P = (const T*)nd.panel;
  // In the A^T orientation (a polish node's column phase) the panel is A^T
  // and sI / sJp hold J / I, so G = A(I, J) is gathered transposed, and the
  // fresh kernel is handed X^T: B^T = X A(I, :) row for row.
  const bool fl = nd.flipped != 0;
  if constexpr (RMAX <= 64) {
    const int64_t tg = wall_clock64();
    LuRegs<RMAX> R;
    const GPtr<const T> Pg = (GPtr<const T>)P;
    const bool okg = lu_fwd_reg<RMAX>(
        [&](int p, int c) {
          const int64_t i = fl ? L.sI[c] : L.sI[p];
          const int64_t j = fl ? L.sJp[p] : L.sJp[c];
          return (double)Pg[j * m + i];
        },
        r, R, L.B, L.lu);
    if (threadIdx.x == 0) nd.tclk[6] += wall_clock64() - tg;
    if (!okg) return false;
    if (want_vol && threadIdx.x == 0) lu_volume(L.lu.diag, 1, r, &L.s.vol_m, &L.s.vol_e);
    const int64_t ti = wall_clock64();
    if (want_X) lu_back_reg<RMAX>(r, R, L.B, L.lu, nd.X, L.A);
    __syncthreads();
    if (want_X && fl) {
      // X(a, k) is L.A[k RMAX + a]: row k of X^T
      block_global_sync();
      for (int idx = threadIdx.x; idx < r * r; idx += kThreads) {
        const int k = idx / r, a = idx % r;
        nd.X[idx] = L.A[k * RMAX + a];
      }
      block_global_sync();
    }
    if (threadIdx.x == 0) nd.tclk[7] += wall_clock64() - ti;
  } else {
    for (int idx = threadIdx.x; idx < r * r; idx += kThreads) {
      const int a = idx / r, b = idx % r;
      L.A[idx] = fl ? (double)P[(int64_t)L.sJp[a] * m + L.sI[b]] : (double)P[(int64_t)L.sJp[b] * m + L.sI[a]];
    }
    __syncthreads();
    const int64_t tg = wall_clock64();
    const bool okg = block_gepp(L.A, r, L.perm, L.lk, &L.s.spiv);
    if (threadIdx.x == 0) nd.tclk[6] += wall_clock64() - tg;
    if (!okg) return false;
    if (want_vol && threadIdx.x == 0) lu_volume(L.A, r + 1, r, &L.s.vol_m, &L.s.vol_e);
    const int64_t ti = wall_clock64();
    if (want_X) block_lu_inverse<CtlLds<T, RMAX>::CH>(L.A, L.perm, r, L.B, nd.X);
    __syncthreads();
    if (want_X && fl) {  // X (row-major in nd.X) -> X^T, through L.A
      block_global_sync();
      for (int idx = threadIdx.x; idx < r * r; idx += kThreads) L.A[idx] = nd.X[idx];
      __syncthreads();
      for (int idx = threadIdx.x; idx < r * r; idx += kThreads) {
        const int k = idx / r, a = idx % r;
        nd.X[idx] = L.A[a * r + k];
      }
      block_global_sync();
    }
    if (threadIdx.x == 0) nd.tclk[7] += wall_clock64() - ti;
  }
  return true;
}

// Polish node: trade the A and A^T orientations (I and J, the two panels,
// their row counts and tile counts).  Every thread reads the orientation
// before thread 0 changes it.
template <typename T, int RMAX>
__device__ void ctl_flip(Node& nd, CtlLds<T, RMAX>& L, int r) {
  __syncthreads();
  for (int k = threadIdx.x; k < r; k += kThreads) {
    const int64_t a = L.sI[k];
    const int32_t b = L.sJp[k];
    L.sI[k] = b;
    L.sJp[k] = (int32_t)a;
  }
  if (threadIdx.x == 0) {
    void* p = nd.panel;
    nd.panel = nd.panel_alt;
    nd.panel_alt = p;
    const int64_t mm = nd.m;
    nd.m = nd.m_alt;
    nd.m_alt = mm;
    const int32_t nt = nd.ntiles;
    nd.ntiles = nd.ntiles_alt;
    nd.ntiles_alt = nt;
    nd.flipped ^= 1;
  }
  block_global_sync();
}

template <typename T, int RMAX>
__device__ bool ctl_build(Node& nd, CtlLds<T, RMAX>& L, bool want_X, bool want_vol) {
  const int64_t t0 = wall_clock64();
  const bool ok = ctl_build_impl(nd, L, want_X, want_vol);
  if (threadIdx.x == 0) nd.tclk[0] += wall_clock64() - t0;
  return ok;
}

template <typename T, int RMAX>
__device__ void ctl_sort_IJ(Node& nd, CtlLds<T, RMAX>& L, int n) {
  const int64_t t0 = wall_clock64();
  block_sort<int64_t>(L.sI, n, L.tmp64);
  block_sort<int32_t>(L.sJp, n, L.tmp32);
  if (threadIdx.x == 0) nd.tclk[4] += wall_clock64() - t0;
}

// X(a, k) in L.A: column-major (ld RMAX) from the register LU, row-major (ld r)
// from the LDS LU.
template <typename T, int RMAX>
__device__ __forceinline__ double ctl_x(const CtlLds<T, RMAX>& L, int r, int a, int k) {
  if constexpr (RMAX <= 64) {
    (void)r;
    return L.A[k * RMAX + a];
  } else {
    return L.A[a * r + k];
  }
}

// Fresh column interpolation matrix Bc = X A(I, Jc) (r x nc, row-major, ld ncmax),
// sums over k ascending, then column Jp[k] := e_k.  X is in L.A.  Chunks of
// CH columns: A(I, chunk) staged in L.B, then thread (g, j) forms outputs
// (g + G q, j), q < QM, each a register accumulator over k, so one L.B read
// serves QM products.
template <typename T, int RMAX>
__device__ void ctl_fresh_bc(Node& nd, CtlLds<T, RMAX>& L, double* bc) {
  const int r = nd.r, nc = L.s.nc, ld = nd.ncmax, tid = threadIdx.x;
  const int64_t m = nd.m;
  const T* P = (const T*)nd.panel;
  constexpr int CH = CtlLds<T, RMAX>::CH;
  constexpr int G = kThreads / CH;            // row groups
  constexpr int QM = (RMAX + G - 1) / G;      // outputs per thread
  static_assert(kThreads % CH == 0, "column chunk must divide the block");
  constexpr int GL = (RMAX * CH + kThreads - 1) / kThreads;  // staged elements per thread
  const int j = tid % CH, g = tid / CH;
  for (int c0 = 0; c0 < nc; c0 += CH) {
    const int nb = min(CH, nc - c0);
    // A(I, chunk): this thread's elements e = k CH + jj, all loads issued
    // before the first LDS store (clamped indices; stored only if in range)
    double st[GL];
#pragma unroll
    for (int q = 0; q < GL; ++q) {
      const int e = tid + q * kThreads;
      const int k = min(e / CH, r - 1), jj = min(e % CH, nb - 1);
      st[q] = (double)P[(int64_t)(c0 + jj) * m + L.sI[k]];
    }
#pragma unroll
    for (int q = 0; q < GL; ++q) {
      const int e = tid + q * kThreads;
      if (e < r * CH && e % CH < nb) L.B[e] = st[q];
    }
    __syncthreads();
    if (j < nb) {
      double acc[QM];
#pragma unroll
      for (int q = 0; q < QM; ++q) acc[q] = 0.0;
      for (int k = 0; k < r; ++k) {
        const double b = L.B[k * CH + j];
#pragma unroll
        for (int q = 0; q < QM; ++q) {
          const int a = min(g + G * q, r - 1);
          acc[q] = fma(ctl_x(L, r, a, k), b, acc[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < QM; ++q) {
        const int a = g + G * q;
        if (a < r) bc[(int64_t)a * ld + c0 + j] = acc[q];
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < r * r; idx += kThreads) {
    const int k = idx / r, a = idx % r;
    bc[(int64_t)a * ld + L.sJp[k]] = (a == k) ? 1.0 : 0.0;
  }
  if (bc == L.Bcl) __syncthreads();
  else block_global_sync();
}

// X into L.A: the register LU (r <= 64) already left it there; the LDS LU
// wrote it to nd.X only, from which it is read back after the block has
// published its global stores.
template <typename T, int RMAX>
__device__ void ctl_load_X(Node& nd, CtlLds<T, RMAX>& L) {
  if constexpr (RMAX > 64) {
    const int r = nd.r;
    block_global_sync();
    for (int idx = threadIdx.x; idx < r * r; idx += kThreads) L.A[idx] = nd.X[idx];
    __syncthreads();
  } else {
    (void)nd;
    (void)L;
  }
}

// Elements of the r x nc matrix Bc visited by one thread: flat index
// e = a nc + c (row-major, so the lanes of a wavefront read consecutive
// columns of one row), e = tid + kThreads i, in batches of kColU whose loads
// are issued before any is used.  The (a, c) pair advances by a fixed step;
// past the end, the row is clamped to r - 1 and the element marked invalid.
constexpr int kColU = 8;

struct ColWalk {
  int a, c, sa, sc, nc, r, tot, e;
  __device__ ColWalk(int r_, int nc_, int tid) : nc(nc_), r(r_), tot(r_ * nc_), e(tid) {
    a = tid / nc_;
    c = tid - a * nc_;
    sa = kThreads / nc_;
    sc = kThreads - sa * nc_;
  }
  __device__ bool more() const { return e < tot; }
  // positions of the next batch
  __device__ void batch(int (&ra)[kColU], int (&rc)[kColU], bool (&ok)[kColU]) {
#pragma unroll
    for (int u = 0; u < kColU; ++u) {
      ok[u] = e + u * kThreads < tot;
      ra[u] = min(a, r - 1);
      rc[u] = c;
      c += sc;
      a += sa;
      if (c >= nc) {
        c -= nc;
        ++a;
      }
    }
    e += kColU * kThreads;
  }
};

// The whole COL phase of one node (maxvol on A(I, Jc)^T with I fixed).
// Returns after the phase; L.s.mode is set to the follow-up.  The argmax is
// over |Bc(a, c)| for columns c not in J, ties to the smaller column-major key
// c r + a, so the order in which elements are visited does not matter; each
// swap's rank-one update also forms the next argmax on the values it writes.
template <typename T, int RMAX>
__device__ void ctl_col_phase(Node& nd, CtlLds<T, RMAX>& L, double lim) {
  const int64_t tph = wall_clock64();
  const int r = nd.r, nc = L.s.nc, ld = nd.ncmax, tid = threadIdx.x;
  double* bc = ((int64_t)r * ld <= CtlLds<T, RMAX>::BCCAP) ? L.Bcl : nd.Bc;
  uint8_t* insel = (nc <= CtlLds<T, RMAX>::INSCAP) ? L.insel : nd.insel;
  const int guard_max = 4 * nd.smax + 16;
  auto make = [&](double x, int a, int c) {
    Cand o;
    o.val = fabs(x);
    o.sval = x;
    o.key = (int64_t)c * r + a;
    o.row = a;
    o.pos = c;
    return o;
  };
  // argmax over the columns not in J
  auto fresh = [&]() {
    const int64_t tf = wall_clock64();
    ctl_fresh_bc(nd, L, bc);
    if (tid == 0) nd.tclk[2] += wall_clock64() - tf;
  };
  auto scan = [&]() {
    Cand b = cand_none();
    ColWalk w(r, nc, tid);
    while (w.more()) {
      int ra[kColU], rc[kColU];
      bool ok[kColU];
      w.batch(ra, rc, ok);
      double x[kColU];
      uint8_t f[kColU];
#pragma unroll
      for (int u = 0; u < kColU; ++u) {
        x[u] = bc[(int64_t)ra[u] * ld + rc[u]];
        f[u] = insel[rc[u]];
      }
#pragma unroll
      for (int u = 0; u < kColU; ++u)
        if (ok[u] && !f[u]) cand_take(b, make(x[u], ra[u], rc[u]));
    }
    return block_argmax(b, L.sc);
  };
  ctl_sort_IJ(nd, L, r);
  if (tid == 0) {
    L.s.phase_swaps = 0;
    L.s.since = 0;
  }
  __syncthreads();
  if (nc > r) {
    for (int c = tid; c < nc; c += kThreads) insel[c] = 0;
    if (insel == L.insel) __syncthreads();
    else block_global_sync();
    for (int k = tid; k < r; k += kThreads) insel[L.sJp[k]] = 1;
    if (insel != L.insel) block_global_sync();
    if (!ctl_build(nd, L, true, false)) {
      if (tid == 0) L.s.err = 101;
    } else {
      ctl_load_X(nd, L);
      fresh();
      if (tid == 0) L.s.refreshes++;
      __syncthreads();
      Cand b = cand_none();
      bool have = false;  // b already formed by the last update
      for (int guard = 0;; ++guard) {
        if (guard >= guard_max) {
          if (tid == 0) L.s.err = 102;
          __syncthreads();
          break;
        }
        if (!have) b = scan();
        have = false;
        if (b.row < 0 || b.val <= lim) {
          if (L.s.since == 0) break;
          if (!ctl_build(nd, L, true, false)) {
            if (tid == 0) L.s.err = 103;
            break;
          }
          ctl_load_X(nd, L);
          fresh();
          if (tid == 0) {
            L.s.refreshes++;
            L.s.since = 0;
          }
          __syncthreads();
          continue;
        }
        if (L.s.swaps >= nd.smax) {
          if (tid == 0) L.s.nocap = 1;
          __syncthreads();
          break;
        }
        // swap candidate column c* into slot k*
        const int64_t tsw = wall_clock64();
        const int ks = (int)b.row, cs = b.pos;
        const int cold = L.sJp[ks];  // the column leaving J
        const double p = b.sval;
        double* wv = L.wv;                // w (r)
        double* rowk = (nc <= CtlLds<T, RMAX>::ROWKCAP) ? L.rowk : nd.vec + RMAX;  // old row k*
        for (int a = tid; a < r; a += kThreads) {
          const double x = bc[(int64_t)a * ld + cs];
          wv[a] = (a == ks) ? (p - 1.0) / p : x / p;
        }
        for (int c = tid; c < nc; c += kThreads) rowk[c] = bc[(int64_t)ks * ld + c];
        if (rowk == L.rowk) __syncthreads();
        else block_global_sync();
        // Bc -= w rowk^T, column c* := e_k*; the next argmax on the new values
        // with J' = J - {c_old} + {c*}
        Cand nb = cand_none();
        {
          ColWalk w(r, nc, tid);
          while (w.more()) {
            int ra[kColU], rc[kColU];
            bool ok[kColU];
            w.batch(ra, rc, ok);
            double x[kColU], rk[kColU];
            uint8_t f[kColU];
#pragma unroll
            for (int u = 0; u < kColU; ++u) {
              x[u] = bc[(int64_t)ra[u] * ld + rc[u]];
              rk[u] = rowk[rc[u]];
              f[u] = insel[rc[u]];
            }
#pragma unroll
            for (int u = 0; u < kColU; ++u) {
              double y = fma(-wv[ra[u]], rk[u], x[u]);
              if (rc[u] == cs) y = (ra[u] == ks) ? 1.0 : 0.0;
              if (ok[u]) {
                bc[(int64_t)ra[u] * ld + rc[u]] = y;
                const bool in = rc[u] == cs || (f[u] && rc[u] != cold);
                if (!in) cand_take(nb, make(y, ra[u], rc[u]));
              }
            }
          }
        }
        if (bc == L.Bcl) __syncthreads();
        else block_global_sync();
        b = block_argmax(nb, L.sc);
        have = true;
        if (tid == 0) {
          insel[cold] = 0;
          insel[cs] = 1;
          L.sJp[ks] = cs;
          L.s.swaps++;
          L.s.phase_swaps++;
          L.s.since++;
          nd.tclk[3] += wall_clock64() - tsw;
        }
        if (insel == L.insel) __syncthreads();
        else block_global_sync();
      }
    }
  }
  __syncthreads();
  if (tid == 0) nd.tclk[1] += wall_clock64() - tph;
  if (tid == 0) {
    L.s.phases++;
    if (L.s.err || L.s.nocap || L.s.phase_swaps == 0) {
      L.s.mode = M_FINISH;
    } else {
      L.s.phase++;
      L.s.mode = M_ROW_START;
    }
  }
  __syncthreads();
}

// The COL phase for r <= 64 and r < nc <= 128 with Bc in registers: lane a
// holds row a of Bc, wavefront w the columns c = w + 4 j (j < 32).  Same
// arithmetic as ctl_col_phase, element by element:
//   fresh  Bc(a,c) = sum_k X(a,k) A(I_k, Jc_c), k ascending, columns in J := e_k;
//   argmax over columns not in J, larger |Bc| first, ties to the smaller
//          column-major key c * r + a;
//   swap   p = Bc(ks,cs); v_a = Bc(a,cs)/p (a != ks), v_ks = (p-1)/p;
//          Bc(a,c) = fma(-v_a, Bc(ks,c), Bc(a,c)) for every c; column cs := e_ks.
// A(I, Jc) is staged in L.Bcl row by row, each wavefront's 32 columns
// contiguous (element (k, c) at k * 128 + (c & 3) * 32 + (c >> 2)).
template <typename T, int RMAX>
__device__ void ctl_col_phase_reg(Node& nd, CtlLds<T, RMAX>& L, double lim) {
  static_assert(RMAX <= 64, "register column phase needs r <= 64");
  static_assert(CtlLds<T, RMAX>::BCCAP >= 64 * 128, "A(I, Jc) staging");
  constexpr int NCJ = 32;
  const int64_t tph = wall_clock64();
  const int r = nd.r, nc = L.s.nc, tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t m = nd.m;
  const T* P = (const T*)nd.panel;
  const int guard_max = 4 * nd.smax + 16;
  uint8_t* insel = L.insel;
  int* slot = L.slot;
  double* Ag = L.Bcl;
  double* prow = L.rowk + w * NCJ;  // this wavefront's copy of row ks
  ctl_sort_IJ(nd, L, r);
  if (tid == 0) {
    L.s.phase_swaps = 0;
    L.s.since = 0;
  }
  for (int c = tid; c < nc; c += kThreads) {
    insel[c] = 0;
    slot[c] = -1;
  }
  __syncthreads();
  for (int k = tid; k < r; k += kThreads) {
    insel[L.sJp[k]] = 1;
    slot[L.sJp[k]] = k;
  }
  __syncthreads();
  uint32_t inJ = 0;  // bit j: column w + 4 j is in J (uniform)
#pragma unroll
  for (int j = 0; j < NCJ; ++j) {
    const int c = w + 4 * j;
    if (c < nc && insel[c]) inJ |= 1u << j;
  }
  double bcr[NCJ];
  // fresh Bc from X (L.A, column-major) and A(I, Jc)
  auto fresh = [&]() {
    const int64_t tf = wall_clock64();
    {
      // Every load is issued unconditionally from a valid address (column and
      // k clamped into range; entries for k >= r are not stored), so all 32
      // are in flight together: a tested load compiles to a branch with a
      // wait for its data.  Columns c >= nc are zeroed by a mask the optimiser
      // cannot turn back into a branch.
      const int c = tid & 127;
      const GPtr<const T> Pc = (GPtr<const T>)P + (int64_t)min(c, nc - 1) * m;
      uint32_t cmask = c < nc ? 0xffffffffu : 0u;
      asm("" : "+v"(cmask));
      double v[32];
#pragma unroll
      for (int q = 0; q < 32; ++q) {
        const int k = (tid >> 7) + 2 * q;
        const double x = (double)Pc[L.sI[min(k, r - 1)]];
        const uint64_t bits = (uint64_t)__double_as_longlong(x) & (((uint64_t)cmask << 32) | cmask);
        v[q] = __longlong_as_double((long long)bits);
      }
#pragma unroll
      for (int q = 0; q < 32; ++q) {
        const int k = (tid >> 7) + 2 * q;
        if (k < r) Ag[k * 128 + (c & 3) * NCJ + (c >> 2)] = v[q];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NCJ; ++j) bcr[j] = 0.0;
    const double* Arow = Ag + w * NCJ;
    for (int k = 0; k < r; ++k) {
      const double xa = L.A[k * RMAX + lane];
      double av[NCJ];
#pragma unroll
      for (int j = 0; j < NCJ; ++j) av[j] = Arow[k * 128 + j];
#pragma unroll
      for (int j = 0; j < NCJ; ++j) bcr[j] = fma(xa, av[j], bcr[j]);
    }
#pragma unroll
    for (int j = 0; j < NCJ; ++j)
      if ((inJ >> j) & 1) bcr[j] = (lane == slot[w + 4 * j]) ? 1.0 : 0.0;
    if (tid == 0) nd.tclk[2] += wall_clock64() - tf;
  };
  if (!ctl_build(nd, L, true, false)) {
    if (tid == 0) {
      int code = 108;  // numerically singular cross
      for (int a = 0; a < r; ++a) {  // the cross, for diagnostics
        nd.dbg[a] = (double)L.sI[a];
        nd.dbg[64 + a] = (double)nd.Jc[L.sJp[a]];
      }
      for (int a = 0; a < r; ++a) {
        if (L.sI[a] < 0 || L.sI[a] >= m) code = 132;
        if (L.sJp[a] < 0 || L.sJp[a] >= nc) code = 133;
        for (int b = a + 1; b < r; ++b) {
          if (L.sI[a] == L.sI[b]) code = 130;
          if (L.sJp[a] == L.sJp[b]) code = 131;
        }
      }
      L.s.err = code;
    }
    __syncthreads();
  } else {
    fresh();
    if (tid == 0) L.s.refreshes++;
    __syncthreads();
    for (int guard = 0;; ++guard) {
      const int64_t tsw = wall_clock64();
      if (guard >= guard_max) {
        if (tid == 0) L.s.err = 109;
        __syncthreads();
        break;
      }
      // ---- argmax: per lane over its columns (c ascending), then the wavefront, then the block
      uint64_t bkey = 0;  // bits of |Bc| (monotone for |x| >= 0); 0: none
      int bj = 0;
      double bsv = 0.0;
      if (lane < r) {
#pragma unroll
        for (int j = 0; j < NCJ; ++j) {
          const int c = w + 4 * j;
          if (c < nc && !((inJ >> j) & 1)) {
            const double x = bcr[j];
            const uint64_t u = (x == x) ? (uint64_t)__double_as_longlong(fabs(x)) : 0ull;
            if (u > bkey) {
              bkey = u;
              bj = j;
              bsv = x;
            }
          }
        }
      }
      const uint64_t wbest = wave_max_u64(bkey);
      uint64_t tied = __ballot(bkey == wbest && wbest != 0ull);
      if (wbest != 0ull) {
        int win = (int)__builtin_ctzll(tied);
        if (tied & (tied - 1)) {
          int64_t kbest = INT64_MAX;
          while (tied) {
            const int b = (int)__builtin_ctzll(tied);
            const int64_t kb = (int64_t)(w + 4 * __builtin_amdgcn_readlane(bj, b)) * r + b;
            if (kb < kbest) {
              kbest = kb;
              win = b;
            }
            tied &= tied - 1;
          }
        }
        win = __builtin_amdgcn_readfirstlane(win);
        if (lane == win) {
          Cand o;
          o.val = fabs(bsv);
          o.sval = bsv;
          o.pos = w + 4 * bj;
          o.row = lane;
          o.key = (int64_t)o.pos * r + lane;
          L.sc[w] = o;
        }
      } else if (lane == 0) {
        L.sc[w] = cand_none();
      }
      __syncthreads();
      Cand b = L.sc[0];
#pragma unroll
      for (int q = 1; q < kThreads / 64; ++q) cand_take(b, L.sc[q]);
      __syncthreads();  // L.sc is rewritten by the next argmax
      if (b.row < 0 || b.val <= lim) {
        if (L.s.since == 0) break;
        if (!ctl_build(nd, L, true, false)) {
          if (tid == 0) L.s.err = 110;
          __syncthreads();
          break;
        }
        fresh();
        if (tid == 0) {
          L.s.refreshes++;
          L.s.since = 0;
        }
        __syncthreads();
        continue;
      }
      if (L.s.swaps >= nd.smax) {
        if (tid == 0) L.s.nocap = 1;
        __syncthreads();
        break;
      }
      // ---- swap column cs into slot ks
      const int ks = (int)b.row, cs = b.pos;
      const double p = b.sval;
      if (w == (cs & 3) && lane < r) {
        const double col = reg_pick<NCJ>(bcr, cs >> 2);
        L.wv[lane] = (lane == ks) ? (p - 1.0) / p : col / p;
      }
      if (lane == ks) {
#pragma unroll
        for (int j = 0; j < NCJ; ++j) prow[j] = bcr[j];
      }
      __syncthreads();
      {
        double rk[NCJ];
#pragma unroll
        for (int j = 0; j < NCJ; ++j) rk[j] = prow[j];
        const double va = lane < r ? L.wv[lane] : 0.0;
#pragma unroll
        for (int j = 0; j < NCJ; ++j) {
          const int c = w + 4 * j;
          if (c < nc) bcr[j] = fma(-va, rk[j], bcr[j]);
          if (c == cs) bcr[j] = (lane == ks) ? 1.0 : 0.0;
        }
      }
      const int old = L.sJp[ks];
      if ((old & 3) == w) inJ &= ~(1u << (old >> 2));
      if ((cs & 3) == w) inJ |= 1u << (cs >> 2);
      __syncthreads();  // every wavefront has read L.sJp, prow and L.wv
      if (tid == 0) {
        dbg_log(nd, L.s.swaps, 2.0 + 0.001 * L.s.refreshes, (double)cs, (double)ks, p);
        insel[old] = 0;
        slot[old] = -1;
        insel[cs] = 1;
        slot[cs] = ks;
        L.sJp[ks] = cs;
        L.s.swaps++;
        L.s.phase_swaps++;
        L.s.since++;
        nd.tclk[3] += wall_clock64() - tsw;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if (tid == 0) nd.tclk[1] += wall_clock64() - tph;
  if (tid == 0) {
    L.s.phases++;
    if (L.s.err || L.s.nocap || L.s.phase_swaps == 0) {
      L.s.mode = M_FINISH;
    } else {
      L.s.phase++;
      L.s.mode = M_ROW_START;
    }
  }
  __syncthreads();
}

template <typename T, int RMAX>
__global__ __launch_bounds__(kThreads) void k_ctl(Node* nodes, int32_t* done, int startup, int heavy_ok) {
  Node& nd = nodes[blockIdx.x];
  if (nd.st == ST_DONE) {
    // a node finished by its initialization is counted once, at start-up
    if (startup && threadIdx.x == 0) atomicAdd(done, 1);
    return;
  }
  // the start-up launch only opens swap loops; pass states wait for their pass
  if (startup && nd.st != ST_START_SWAP) return;
  // Steps with an r x r factorization (phase starts, refreshes, column phases,
  // the final volume) run only in launches that admit them (heavy_ok), so
  // that the nodes of a level take them together rather than each holding up
  // a different lock-step iteration; a node that reaches one otherwise waits
  // in ST_DEFER.  The arithmetic and its order are the same either way.
  if (nd.st == ST_DEFER && !heavy_ok) return;
  __shared__ CtlLds<T, RMAX> L;
  const int64_t tctl = wall_clock64();
  const int tid = threadIdx.x;
  const int r = nd.r;
  int64_t m = nd.m;  // a polish node's orientation change swaps it
  const double lim = 1.0 + nd.tau;
  if (tid == 0) {
    CtlShared& s = L.s;
    s.st = nd.st; s.t = nd.t; s.q = nd.q; s.na = nd.na; s.steps = nd.steps; s.nc = nd.nc;
    s.is_short = nd.is_short; s.nocap = nd.nocap; s.err = nd.err; s.phase = nd.phase;
    s.phase_swaps = nd.phase_swaps; s.since = nd.since; s.swaps = nd.swaps; s.phases = nd.phases;
    s.refreshes = nd.refreshes; s.pend_k = nd.pend_k; s.pend_i = nd.pend_i; s.pend_p = nd.pend_p;
    s.vol_m = nd.vol_m; s.vol_e = nd.vol_e;
    s.pend_mode = nd.pend_mode;
    // the pass that just ran: a fresh B empties the swap history; a swap pass
    // added one swap to it, or wrote B out with all of them (the last slot)
    s.lz = nd.lz;
    if (!startup) {
      if (s.st == ST_ROW_FRESH) s.lz = 0;
      else if (s.st == ST_ROW_SWAP) s.lz = (s.lz + 1 == kLz) ? 0 : s.lz + 1;
    }
    s.mode = M_EXIT;
    s.stale = 0;
  }
  for (int k = tid; k < r; k += kThreads) {
    L.sI[k] = nd.I[k];
    L.sJp[k] = nd.Jp[k];
  }
  __syncthreads();
  const int st0 = L.s.st;

  // ---- consume the pass that just ran
  if (st0 == ST_ACA) {
    ctl_reduce(nd, L);
    if (tid == 0) {
      CtlShared& s = L.s;
      const int na_read = s.na;
      int na_new = na_read;
      if (s.t > 0) {
        const int pc = s.pend_k;
        if (pc != na_read - 1) nd.colmap[pc] = nd.colmap[na_read - 1];
        na_new = na_read - 1;
      }
      const Cand& w = s.win;
      if (w.row < 0 || fabs(w.sval) <= nd.theta) {
        s.q = s.t;
        s.mode = M_FINISH_SHORT;
      } else {
        L.sI[s.t] = w.row;
        L.sJp[s.t] = nd.colmap[w.pos];
        s.t++;
        s.q = s.t;
        if (s.t == s.steps) {
          if (s.t == r) {
            s.phase = 0;
            s.mode = M_ROW_START;
          } else {
            s.mode = M_FINISH_SHORT;
          }
        } else {
          s.pend_i = w.row;
          s.pend_k = w.pos;
          s.pend_p = w.sval;
          s.na = na_new;
          s.st = ST_ACA;
          s.mode = M_EXIT;
        }
      }
    }
    __syncthreads();
    if (L.s.mode == M_EXIT) {
      // f_c = R(i*, c) / p in FP64, read from the residual the pass just wrote
      // (FP64 for either input type; the panel itself after the first,
      // read-only, pass)
      const int64_t wr = L.s.pend_i;
      const double p = L.s.pend_p;
      if (L.s.t == 1) {
        const T* R = (const T*)nd.panel;
        for (int c = tid; c < L.s.na; c += kThreads) nd.vec[c] = (double)R[(int64_t)c * m + wr] / p;
      } else {
        const double* R = (const double*)nd.work;
        for (int c = tid; c < L.s.na; c += kThreads) nd.vec[c] = R[(int64_t)c * m + wr] / p;
      }
    }
  } else if (st0 == ST_ROW_FRESH || st0 == ST_ROW_SWAP) {
    ctl_reduce(nd, L);
    if (tid == 0) {
      CtlShared& s = L.s;
      const Cand& w = s.win;
      if (w.row < 0 || w.val <= lim) {
        s.mode = (s.since == 0) ? M_ROW_END : M_REFRESH;
      } else if (s.swaps >= nd.smax) {
        s.nocap = 1;
        s.mode = M_ROW_END;
      } else {
        for (int k = 0; k < r; ++k)
          if (L.sI[k] == w.row) s.err = 121;  // a selected row won: inconsistent pass
        dbg_log(nd, s.swaps, 1.0 + 0.001 * s.refreshes, (double)w.row, (double)w.pos, w.sval);
        s.pend_i = w.row;
        s.pend_k = w.pos;
        s.pend_p = w.sval;
        L.sI[w.pos] = w.row;
        s.swaps++;
        s.phase_swaps++;
        s.since++;
        s.st = ST_ROW_SWAP;
        s.mode = M_SWAPVEC;
      }
    }
    __syncthreads();
    if (L.s.mode == M_SWAPVEC) {
      // v_c = B(i*, c) / p with row i* of the current B: the working matrix
      // plus the pending swaps, replayed in the pass's own operation order
      const double* B = (const double*)nd.work;
      const double* G = (const double*)nd.lzg;
      const int64_t wr = L.s.pend_i;
      const double p = L.s.pend_p;
      const int ks = L.s.pend_k;
      const int S = L.s.lz;
      for (int c = tid; c < r; c += kThreads) {
        double x = B[(int64_t)c * m + wr];
        for (int q = 0; q < S; ++q)
          x = (wr == nd.lzi[q]) ? ((c == nd.lzk[q]) ? 1.0 : 0.0) : fma(-G[(int64_t)q * m + wr], nd.lzv[q * r + c], x);
        nd.lzv[S * r + c] = (c == ks) ? (p - 1.0) / p : x / p;
      }
      if (tid == 0) {
        nd.lzi[S] = wr;
        nd.lzk[S] = ks;
      }
      __syncthreads();
      if (tid == 0) L.s.mode = M_EXIT;
      __syncthreads();
    }
  } else if (st0 == ST_START_SWAP) {
    if (tid == 0) {
      L.s.phase = 0;
      L.s.mode = M_ROW_START;
    }
    __syncthreads();
  } else if (st0 == ST_DEFER) {
    if (tid == 0) L.s.mode = L.s.pend_mode;
    __syncthreads();
  }

  // ---- serial steps until a pass is needed or the node is finished
  for (int guard = 0; guard < 64; ++guard) {
    const int mode = L.s.mode;
    // every wavefront holds this step's mode before thread 0 may overwrite it
    // (a late wavefront would otherwise take the next step's branch and run
    // one barrier out of step with the rest of the block)
    __syncthreads();
    if (mode == M_EXIT) break;
    if (!heavy_ok && (mode == M_ROW_START || mode == M_REFRESH || mode == M_COL || mode == M_FINISH)) {
      if (tid == 0) {
        L.s.pend_mode = mode;
        L.s.st = ST_DEFER;
        L.s.mode = M_EXIT;
      }
      __syncthreads();
      break;
    }
    if (mode == M_REFRESH) {
      // tentative stop after swaps: recompute B fresh for the current orders
      if (!ctl_build(nd, L, true, false)) {
        if (tid == 0) {
          L.s.err = 104;
          L.s.mode = M_ROW_END;
        }
      } else if (tid == 0) {
        L.s.refreshes++;
        L.s.since = 0;
        L.s.st = ST_ROW_FRESH;
        L.s.mode = M_EXIT;
      }
      __syncthreads();
    } else if (mode == M_ROW_START) {
      ctl_sort_IJ(nd, L, r);
      if (tid == 0) {
        L.s.phase_swaps = 0;
        L.s.since = 0;
      }
      __syncthreads();
      if (m == r) {
        if (tid == 0) L.s.mode = M_ROW_END;
      } else if (!ctl_build(nd, L, true, false)) {
        if (tid == 0) {
          L.s.err = 105;
          L.s.mode = M_ROW_END;
        }
      } else if (tid == 0) {
        L.s.refreshes++;
        L.s.st = ST_ROW_FRESH;
        L.s.mode = M_EXIT;
      }
      __syncthreads();
    } else if (mode == M_ROW_END) {
      if (tid == 0) {
        CtlShared& s = L.s;
        s.phases++;
        if (s.err || s.nocap || (s.phase >= 1 && s.phase_swaps == 0)) {
          s.mode = M_FINISH;
        } else {
          s.phase++;
          // a polish node runs its column phases as row phases of A^T (the
          // column phase is the row phase of the transpose, element for element)
          s.mode = (nd.kind == KIND_POLISH) ? M_FLIP : M_COL;
        }
      }
      __syncthreads();
    } else if (mode == M_FLIP) {
      ctl_flip(nd, L, r);
      m = nd.m;
      if (tid == 0) L.s.mode = M_ROW_START;
      __syncthreads();
    } else if (mode == M_COL) {
      if constexpr (RMAX <= 64) {
        if (L.s.nc > r && L.s.nc <= 128)
          ctl_col_phase_reg(nd, L, lim);
        else
          ctl_col_phase(nd, L, lim);
      } else {
        ctl_col_phase(nd, L, lim);
      }
    } else if (mode == M_FINISH) {
      const bool fl = nd.flipped != 0;
      if (fl) {  // back to the A orientation for the volume and the outputs
        ctl_flip(nd, L, r);
        m = nd.m;
      }
      ctl_sort_IJ(nd, L, r);
      if (!L.s.err) {
        if (!ctl_build(nd, L, false, true) && tid == 0) L.s.err = 106;
      }
      __syncthreads();
      if (tid == 0) {
        L.s.st = ST_DONE;
        L.s.mode = M_EXIT;
        atomicAdd(done, 1);
      }
      __syncthreads();
    } else if (mode == M_FINISH_SHORT) {
      ctl_sort_IJ(nd, L, L.s.q);
      if (tid == 0) {
        L.s.is_short = 1;
        L.s.st = ST_DONE;
        L.s.mode = M_EXIT;
        atomicAdd(done, 1);
      }
      __syncthreads();
    } else {
      if (tid == 0) {
        L.s.err = 107;
        L.s.st = ST_DONE;
        L.s.mode = M_EXIT;
        atomicAdd(done, 1);
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int k = tid; k < r; k += kThreads) {
    nd.I[k] = L.sI[k];
    nd.Jp[k] = L.sJp[k];
  }
  if (tid == 0) {
    const CtlShared& s = L.s;
    nd.tclk[5] += wall_clock64() - tctl;
    nd.seq = nd.seq + 1;
    nd.st = s.st; nd.t = s.t; nd.q = s.q; nd.na = s.na; nd.steps = s.steps;
    nd.is_short = s.is_short; nd.nocap = s.nocap; nd.err = s.err; nd.phase = s.phase;
    nd.phase_swaps = s.phase_swaps; nd.since = s.since; nd.swaps = s.swaps; nd.phases = s.phases;
    nd.refreshes = s.refreshes; nd.pend_k = s.pend_k; nd.pend_i = s.pend_i; nd.pend_p = s.pend_p;
    nd.vol_m = s.vol_m; nd.vol_e = s.vol_e;
    nd.lz = s.lz;
    nd.pend_mode = s.pend_mode;
  }
}

// Root -> caller's I, J (ascending original indices, -1 padded).
// Root outputs of every tree: block j writes tree j's (I, J), entries past the
// rank it reached are -1.
struct RootOut {
  int32_t node;  // index of the root in the node table
  int32_t pad;
  int64_t* I;
  int64_t* J;
};

__global__ void k_finalize(const Node* nodes, const RootOut* roots) {
  const RootOut ro = roots[blockIdx.x];
  const Node& nd = nodes[ro.node];
  for (int k = threadIdx.x; k < nd.r; k += blockDim.x) {
    const bool ok = k < nd.q;
    ro.I[k] = ok ? nd.I[k] : -1;
    ro.J[k] = ok ? nd.Jc[nd.Jp[k]] : -1;
  }
}

// Per-node outputs for the host: original indices of I and J.
__global__ void k_export(const Node* nodes, int64_t* I, int64_t* J, int r) {
  const Node& nd = nodes[blockIdx.x];
  for (int k = threadIdx.x; k < r; k += blockDim.x) {
    const bool ok = k < nd.q && nd.st == ST_DONE;
    I[(int64_t)blockIdx.x * r + k] = ok ? nd.I[k] : -1;
    J[(int64_t)blockIdx.x * r + k] = ok ? nd.Jc[nd.Jp[k]] : -1;
  }
}

// ---------------------------------------------------------------- host side
struct LevelPlan {
  int count;
  int first;  // index of the level's first node in the global table
};

struct SelectPlan {
  int r, w;
  int64_t m, n;
  int b;
  std::vector<LevelPlan> levels;
  int total_nodes;
};

static int rmax_bucket(int r) { return r <= 32 ? 32 : (r <= 64 ? 64 : 128); }

template <typename T, int RMAX>
static void launch_ctl(Node* nodes, int count, int32_t* done, int startup, int heavy_ok, hipStream_t s) {
  hipLaunchKernelGGL((k_ctl<T, RMAX>), dim3(count), dim3(kThreads), 0, s, nodes, done, startup, heavy_ok);
}


// Event pair around a pass launch when the measurement counters are on.
static hipEvent_t prof_event(cur_ctx ctx, size_t idx) {
  std::vector<hipEvent_t>& ev = *ctx->prof_ev;
  while (ev.size() <= idx) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ev.push_back(e);
  }
  return ev[idx];
}
// One launch of a row kernel (kind 0: the streaming pass, 1: fresh B) on
// stream s; with the counters on, bracketed by an event pair and given its
// own device byte slot.
template <typename T>
static void row_launch(cur_ctx ctx, int kind, int rb, Node* nodes, int count, int tiles, hipStream_t s,
                       size_t& prof_used) {
  const bool f64 = std::is_same<T, double>::value;
  auto go = [&](unsigned long long* slot) {
    if (kind == 1) fresh_launch(f64, rb, nodes, count, tiles, slot, s);
    else pass_launch(f64, rb, nodes, count, tiles, slot, s);
  };
  const size_t pair = prof_used / 2;
  if (ctx->prof_on < (kind == 1 ? 2 : 1) || pair >= (size_t)kProfSlots) {
    go(nullptr);
    return;
  }
  hipEvent_t e0 = prof_event(ctx, prof_used), e1 = prof_event(ctx, prof_used + 1);
  if (!e0 || !e1) {
    go(nullptr);
    return;
  }
  (void)hipEventRecord(e0, s);
  go(ctx->prof_bytes + 2 * pair);
  (void)hipEventRecord(e1, s);
  if (ctx->prof_kind->size() <= pair) ctx->prof_kind->resize(pair + 1);
  (*ctx->prof_kind)[pair] = kind;
  prof_used += 2;
}

template <typename T>
static void ctl_any(int rb, Node* nodes, int count, int32_t* done, int startup, int heavy_ok, hipStream_t s) {
  if (rb == 32) launch_ctl<T, 32>(nodes, count, done, startup, heavy_ok, s);
  else if (rb == 64) launch_ctl<T, 64>(nodes, count, done, startup, heavy_ok, s);
  else launch_ctl<T, 128>(nodes, count, done, startup, heavy_ok, s);
}

// Streams and events of the node groups, created once per context.
constexpr int kMaxGroups = 4;
cur_status ensure_groups(cur_ctx ctx) {
  if (ctx->groups_ready) return CUR_OK;
  for (int g = 0; g < kMaxGroups; ++g) {
    CUR_HIP_CHECK(hipStreamCreateWithFlags(&ctx->gstream[g], hipStreamNonBlocking));
    CUR_HIP_CHECK(hipEventCreateWithFlags(&ctx->gjoin[g], hipEventDisableTiming));
  }
  CUR_HIP_CHECK(hipEventCreateWithFlags(&ctx->gfork, hipEventDisableTiming));
  ctx->groups_ready = 1;
  return CUR_OK;
}

// Launch-shape autotuner.  The node-group count of a level changes only how
// the level's launches are spread over streams, never a result, so it is
// chosen by measurement: the first calls on a level shape try each candidate
// once (the level's host wall time, which ends with a stream synchronization),
// later calls use the fastest.  The cache lives in the context.
static const int kGroupCand[3] = {1, 2, 3};

static TuneEntry* tune_find(cur_ctx ctx, const int64_t key[6]) {
  for (TuneEntry& e : *ctx->tune)
    if (std::equal(key, key + 6, e.key)) return &e;
  TuneEntry e;
  std::copy(key, key + 6, e.key);
  for (double& v : e.ms) v = -1.0;
  e.tried = 0;
  e.fixed = 0;
  ctx->tune->push_back(e);
  return &ctx->tune->back();
}

// Fastest measured candidate of a fully explored entry.
int tune_best(const TuneEntry& e) {
  int best = 0;
  for (int k = 1; k < 3; ++k)
    if (e.ms[k] < e.ms[best]) best = k;
  return kGroupCand[best];
}

// Group count for a level: `fixed` when the caller set one, else the next
// untried candidate (its index in *cand), else the fastest one measured.
static int tune_pick(cur_ctx ctx, const int64_t key[6], int fixed, int* cand) {
  *cand = -1;
  if (fixed > 0) return fixed;
  TuneEntry* e = tune_find(ctx, key);
  if (e->fixed > 0) return e->fixed;
  if (e->tried < 3) {
    *cand = e->tried;
    return kGroupCand[e->tried];
  }
  return tune_best(*e);
}

static void tune_record(cur_ctx ctx, const int64_t key[6], int cand, std::chrono::steady_clock::time_point t0) {
  if (cand < 0) return;
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  TuneEntry* e = tune_find(ctx, key);
  if (e->tried == cand) {
    e->ms[cand] = ms;
    e->tried++;
  }
}

// Runs pass/ctl iterations on one level until all `count` nodes are done.
// With groups > 1 the level's nodes are split into that many contiguous
// groups, each iterating on a stream of its own with its own done counter
// (d_done[g]) and poll: a node whose controller step is long (an LU rebuild,
// a column phase) then holds back only its own group, and its latency-bound
// controller launch overlaps the other groups' streaming passes.  Groups
// share no node data; all ordering is by stream order within a group.
// Controller launches admit steps with an r x r factorization once every P
// launches (P = 1: every launch), P by the number of nodes sharing the
// launches: >= 32, >= 8, >= 2, 1.  CUR_GATE="a,b,c,d" sets the four periods.
static int gate_period(int nodes) {
  static const std::array<int, 4> per = [] {
    std::array<int, 4> p = {16, 12, 6, 1};
    if (const char* e = std::getenv("CUR_GATE")) {
      int k = 0;
      for (const char* q = e; *q && k < 4; ++k) {
        p[k] = std::max(1, std::atoi(q));
        while (*q && *q != ',') ++q;
        if (*q == ',') ++q;
      }
      for (; k > 0 && k < 4; ++k) p[k] = p[k - 1];  // fewer values: repeat the last
    }
    return p;
  }();
  return nodes >= 32 ? per[0] : nodes >= 8 ? per[1] : nodes >= 2 ? per[2] : per[3];
}

template <typename T>
static cur_status run_level(cur_ctx ctx, int rb, Node* nodes, int count, int tiles, int32_t* d_done,
                            int64_t max_iters, size_t& prof_used, int groups) {
  const int G = std::max(1, std::min(std::min(groups, count), kMaxGroups));
  hipStream_t gs[kMaxGroups];
  hipEvent_t ev[kMaxGroups];
  int off[kMaxGroups + 1];
  bool pending[kMaxGroups], fin[kMaxGroups];
  for (int g = 0; g <= G; ++g) off[g] = (int)((int64_t)count * g / G);
  if (G == 1) {
    gs[0] = ctx->stream;
  } else {
    cur_status st = ensure_groups(ctx);
    if (st != CUR_OK) return st;
    CUR_HIP_CHECK(hipEventRecord(ctx->gfork, ctx->stream));
    for (int g = 0; g < G; ++g) {
      gs[g] = ctx->gstream[g];
      CUR_HIP_CHECK(hipStreamWaitEvent(gs[g], ctx->gfork, 0));
    }
  }
  for (int g = 0; g < G; ++g) {
    CUR_HIP_CHECK(hipEventCreateWithFlags(&ev[g], hipEventDisableTiming));
    pending[g] = fin[g] = false;
  }
  volatile int32_t* h = ctx->host_flag;
  for (int g = 0; g < G; ++g)  // start-up decisions
    ctl_any<T>(rb, nodes + off[g], off[g + 1] - off[g], d_done + g, 1, 1, gs[g]);
  // iterations issued between two polls of the done counters
  static const int K = [] {
    const char* e = std::getenv("CUR_POLL_ITERS");
    return e ? std::max(1, std::min(64, std::atoi(e))) : 4;
  }();
  int64_t it = 0;
  cur_status rc = CUR_OK;
  // A node enters the fresh-B state only in a controller launch that admits
  // factorization steps (a phase start or a refresh builds X), and leaves it
  // at the next controller launch; so the fresh kernel has work only in the
  // iteration after such a launch (the start-up launch is one).
  bool fresh_due[kMaxGroups];
  for (int g = 0; g < G; ++g) fresh_due[g] = true;
  for (;;) {
    for (int g = 0; g < G; ++g) {
      if (fin[g]) continue;
      Node* gn = nodes + off[g];
      const int gc = off[g + 1] - off[g];
      const int P = gate_period(gc);
      for (int j = 0; j < K; ++j) {
        const bool heavy = (it + j) % P == P - 1;
        if (fresh_due[g]) row_launch<T>(ctx, 1, rb, gn, gc, tiles, gs[g], prof_used);
        row_launch<T>(ctx, 0, rb, gn, gc, tiles, gs[g], prof_used);
        ctl_any<T>(rb, gn, gc, d_done + g, 0, heavy ? 1 : 0, gs[g]);
        fresh_due[g] = heavy;
      }
    }
    it += K;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      set_error(std::string("kernel launch: ") + hipGetErrorString(e));
      rc = CUR_ERR_DEVICE;
      break;
    }
    bool all = true;
    for (int g = 0; g < G && rc == CUR_OK; ++g) {
      if (fin[g]) continue;
      if (pending[g]) {
        e = hipEventSynchronize(ev[g]);
        if (e != hipSuccess) {
          set_error(std::string("hipEventSynchronize: ") + hipGetErrorString(e));
          rc = CUR_ERR_DEVICE;
          break;
        }
        if (h[g] >= off[g + 1] - off[g]) {  // -1 (copy not landed) reads as "not done"
          fin[g] = true;
          continue;
        }
      }
      all = false;
      h[g] = -1;
      e = hipMemcpyAsync((void*)(h + g), d_done + g, sizeof(int32_t), hipMemcpyDeviceToHost, gs[g]);
      if (e == hipSuccess) e = hipEventRecord(ev[g], gs[g]);
      if (e != hipSuccess) {
        set_error(std::string("poll: ") + hipGetErrorString(e));
        rc = CUR_ERR_DEVICE;
        break;
      }
      pending[g] = true;
    }
    if (rc != CUR_OK || all) break;
    if (it > max_iters) {
      set_error("selection did not converge within the iteration bound");
      rc = CUR_ERR_INTERNAL;
      break;
    }
  }
  if (G > 1) {
    for (int g = 0; g < G; ++g) {
      (void)hipEventRecord(ctx->gjoin[g], gs[g]);
      (void)hipStreamWaitEvent(ctx->stream, ctx->gjoin[g], 0);
    }
  }
  (void)hipStreamSynchronize(ctx->stream);
  for (int g = 0; g < G; ++g) (void)hipEventDestroy(ev[g]);
  return rc;
}

// Diagnostics (CUR_DEBUG set): unfinished, failed or capped nodes with their
// last swaps, and the controller clocks summed per level.
static void debug_report(cur_ctx ctx, const std::vector<Node>& h, const std::vector<int>& lfirst,
                         const std::vector<int>& lcount) {
  for (size_t l = 0; l < lfirst.size(); ++l)
    for (int k = 0; k < lcount[l]; ++k) {
      const Node& nd = h[lfirst[l] + k];
      if (!(nd.err || nd.st != ST_DONE || nd.nocap)) continue;
      std::fprintf(stderr, "cur: node level %zu index %d kind %d st %d err %d phase %d swaps %d phases %d "
                   "refreshes %d q %d nc %d nocap %d\n", l, k, nd.kind, nd.st, nd.err, nd.phase, nd.swaps,
                   nd.phases, nd.refreshes, nd.q, nd.nc, nd.nocap);
      std::vector<double> ring(4 * kDbgRing);
      if (nd.err == 108 &&
          hipMemcpy(ring.data(), nd.dbg, sizeof(double) * ring.size(), hipMemcpyDeviceToHost) == hipSuccess) {
        std::fprintf(stderr, "  cross I:");
        for (int a = 0; a < nd.r; ++a) std::fprintf(stderr, " %.0f", ring[a]);
        std::fprintf(stderr, "\n  cross J:");
        for (int a = 0; a < nd.r; ++a) std::fprintf(stderr, " %.0f", ring[64 + a]);
        std::fprintf(stderr, "\n");
      } else if (hipMemcpy(ring.data(), nd.dbg, sizeof(double) * ring.size(), hipMemcpyDeviceToHost) == hipSuccess) {
        const int n0 = nd.swaps > kDbgRing ? nd.swaps - kDbgRing : 0;
        for (int q = n0; q < nd.swaps; ++q) {
          const double* e = &ring[4 * (q % kDbgRing)];
          std::fprintf(stderr, "  swap %d kind %.3f index %.0f slot %.0f pivot %.17g\n", q, e[0], e[1], e[2], e[3]);
        }
      }
    }
  const char* lvl = std::getenv("CUR_DEBUG");
  if (!lvl || std::atoi(lvl) < 2) return;  // clocks only at level 2
  int wclk = 100000;  // ticks per ms of wall_clock64 (100 MHz)
  (void)hipDeviceGetAttribute(&wclk, hipDeviceAttributeWallClockRate, ctx->device);  // kHz
  for (size_t l = 0; l < lfirst.size(); ++l) {
    double tsum[8] = {0, 0, 0, 0, 0, 0, 0, 0}, tmax = 0;
    for (int k = 0; k < lcount[l]; ++k) {
      const Node& nd = h[lfirst[l] + k];
      for (int q = 0; q < 8; ++q) tsum[q] += nd.tclk[q];
      tmax = std::max(tmax, (double)nd.tclk[5]);
    }
    std::fprintf(stderr, "cur: level %zu nodes %d ctl ms (sum over nodes): build %.2f (lu %.2f inv %.2f) col %.2f "
                 "colfresh %.2f colswaps %.2f sort %.2f all %.2f; slowest node %.2f\n", l, lcount[l],
                 tsum[0] / wclk, tsum[6] / wclk, tsum[7] / wclk, tsum[1] / wclk, tsum[2] / wclk, tsum[3] / wclk,
                 tsum[4] / wclk, tsum[5] / wclk, tmax / wclk);
  }
}

// One selection tree: a matrix, its options and outputs, and the plan of its
// tree (nodes per level and where they sit in the combined level tables).
template <typename T>
struct TreeJob {
  const T* A;
  int64_t m, n, lda;
  int r;
  cur_opts o;
  int64_t* I;
  int64_t* J;
  cur_info* info;
  bool trans = false;       // select from A^T: m, n are A^T's shape, A and lda the source's
  bool polish = false;      // one more level: the root's cross polished over all n columns
  // a one-node job that polishes a given cross (device arrays of r original
  // indices) over all n columns instead of selecting one
  const int64_t* start_I = nullptr;
  const int64_t* start_J = nullptr;
  int ntiles_alt = 0;       // polish: row tiles of A^T (n rows)
  cur_status status = CUR_OK;
  bool active = true;
  double theta = 0.0;
  int w = 0, b = 0, leafmax = 0, ntiles = 0;
  std::vector<int> count;   // nodes per level of this tree
  std::vector<int> off;     // offset of this tree's nodes in each combined level
  std::vector<int> ncmax;   // candidate capacity per level
};

// Runs the trees of `jobs` (one dtype, one rank bucket) together: level l of
// every tree forms one node table, and each pass / controller launch covers
// all of them.  A single cur_select is the one-tree case.  Per-tree statuses
// go to jobs[j].status; the return value reports device failures only.
template <typename T>
static cur_status select_many(cur_ctx ctx, int rb, std::vector<TreeJob<T>>& jobs, cur_trace* tr) {
  hipStream_t s = ctx->stream;
  const int nj = (int)jobs.size();

  // ---- a0: scans (one launch for every matrix, one synchronization)
  {
    const size_t items_off = (16 * (size_t)nj + 255) & ~size_t(255);
    cur_status ast = ensure_arena(ctx, items_off + sizeof(ScanItem) * (size_t)nj);
    if (ast != CUR_OK) return ast;
    unsigned long long* d = (unsigned long long*)ctx->arena;
    ScanItem* d_items = (ScanItem*)((char*)ctx->arena + items_off);
    std::vector<ScanItem> hitems(nj);
    int64_t maxm = 1;
    for (int j = 0; j < nj; ++j) {
      // (a tree over A^T scans its source in the source's own shape)
      hitems[j] = jobs[j].trans ? ScanItem{jobs[j].A, jobs[j].n, jobs[j].m, jobs[j].lda}
                                : ScanItem{jobs[j].A, jobs[j].m, jobs[j].n, jobs[j].lda};
      maxm = std::max(maxm, jobs[j].m);
    }
    CUR_HIP_CHECK(hipMemsetAsync(d, 0, 16 * (size_t)nj, s));
    CUR_HIP_CHECK(hipMemcpyAsync(d_items, hitems.data(), sizeof(ScanItem) * nj, hipMemcpyHostToDevice, s));
    // ~16k workgroups in all, at most one per row, at most 4096 per matrix
    const int gx = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(4096, 16384 / nj + 1), maxm));
    if (nj > 65535) {
      set_error("too many matrices in one call");
      return CUR_ERR_ARG;
    }
    hipLaunchKernelGGL((k_amax<T>), dim3(gx, nj), dim3(kThreads), 0, s, d_items, d);
    std::vector<unsigned long long> hv(2 * (size_t)nj);
    CUR_HIP_CHECK(hipMemcpyAsync(hv.data(), d, 16 * (size_t)nj, hipMemcpyDeviceToHost, s));
    CUR_HIP_CHECK(hipStreamSynchronize(s));
    for (int j = 0; j < nj; ++j) {
      TreeJob<T>& jb = jobs[j];
      if (hv[2 * j + 1]) {
        jb.status = CUR_ERR_NONFINITE;
        jb.active = false;
        set_error("A holds NaN or Inf");
        continue;
      }
      double amax;
      std::memcpy(&amax, &hv[2 * j], sizeof(double));
      if (amax == 0.0) {
        if (jb.info) {
          std::memset(jb.info, 0, sizeof(*jb.info));
          jb.info->logvol = -HUGE_VAL;
        }
        std::vector<int64_t> neg(jb.r, -1);
        CUR_HIP_CHECK(hipMemcpyAsync(jb.I, neg.data(), jb.r * sizeof(int64_t), hipMemcpyHostToDevice, s));
        CUR_HIP_CHECK(hipMemcpyAsync(jb.J, neg.data(), jb.r * sizeof(int64_t), hipMemcpyHostToDevice, s));
        CUR_HIP_CHECK(hipStreamSynchronize(s));
        jb.status = CUR_ERR_RANK;
        jb.active = false;
        set_error("A is zero");
        continue;
      }
      // max(m,n) 2^-52 ||A||_C for both input types: the ACA pivots are FP64
      // (FP32 input widened exactly), so the rank decisions are the oracle's.
      jb.theta = (double)std::max(jb.m, jb.n) * 0x1p-52 * amax;
    }
  }

  // ---- plan the trees and the combined level tables
  int nlev = 0;
  for (TreeJob<T>& jb : jobs) {
    if (!jb.active) continue;
    jb.w = jb.o.col_block;
    jb.b = (int)std::max<int64_t>(1, jb.n / jb.w);
    jb.count.clear();
    for (int c = jb.b;;) {
      jb.count.push_back(c);
      if (c <= 1) break;
      c = (c + 1) / 2;
    }
    jb.ntiles = (int)((jb.m + kTileRows - 1) / kTileRows);
    jb.ntiles_alt = (jb.polish || jb.start_I) ? (int)((jb.n + kTileRows - 1) / kTileRows) : 0;
    jb.leafmax = 0;
    for (int k = 0; k < jb.b; ++k) {
      const int64_t c0 = (int64_t)k * jb.w, c1 = (k == jb.b - 1) ? jb.n : (int64_t)(k + 1) * jb.w;
      jb.leafmax = std::max<int>(jb.leafmax, (int)(c1 - c0));
    }
    jb.ncmax.assign(jb.count.size(), 2 * jb.r);
    jb.ncmax[0] = jb.leafmax;
    if (jb.polish) {
      jb.count.push_back(1);
      jb.ncmax.push_back((int)jb.n);
    }
    nlev = std::max<int>(nlev, (int)jb.count.size());
  }
  if (nlev == 0) return CUR_OK;  // every tree ended at the scan
  std::vector<int> lcount(nlev, 0), lfirst(nlev, 0);
  for (TreeJob<T>& jb : jobs) {
    if (!jb.active) continue;
    jb.off.assign(jb.count.size(), 0);
    for (size_t l = 0; l < jb.count.size(); ++l) {
      jb.off[l] = lcount[l];
      lcount[l] += jb.count[l];
    }
  }
  int total = 0;
  for (int l = 0; l < nlev; ++l) {
    lfirst[l] = total;
    total += lcount[l];
  }

  // ---- workspace layout
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  // the polish level starts from a cross (no elimination on its candidates):
  // its working matrix holds B only
  auto is_polish = [](const TreeJob<T>& jb, int l) {
    return (jb.polish && l + 1 == (int)jb.count.size()) || jb.start_I != nullptr;
  };
  // a polish node's buffers serve both orientations: B and the swap history
  // hold max(m, n) rows, the tile winners max of both tile counts, and A^T is
  // the source itself when its rows are packed (lda == n), else a copy
  auto rows_of = [&](const TreeJob<T>& jb, int l) { return is_polish(jb, l) ? std::max(jb.m, jb.n) : jb.m; };
  auto tiles_of = [&](const TreeJob<T>& jb, int l) {
    return is_polish(jb, l) ? std::max(jb.ntiles, jb.ntiles_alt) : jb.ntiles;
  };
  auto alt_copy = [&](const TreeJob<T>& jb, int l) { return is_polish(jb, l) && jb.lda != jb.n; };
  auto node_bytes = [&](const TreeJob<T>& jb, int l) {
    const int nc = jb.ncmax[l], r = jb.r;
    const int wd = is_polish(jb, l) ? r : std::max(nc, r);
    const int64_t m = jb.m, mr = rows_of(jb, l);
    size_t per = 0;
    per += al(sizeof(T) * m * nc);                // panel
    if (alt_copy(jb, l)) per += al(sizeof(T) * jb.n * m);  // A^T for a polish node
    per += al(sizeof(double) * mr * wd);          // work: ACA residual, then B (FP64)
    per += al(sizeof(double) * r * r);            // X
    per += al(sizeof(double) * r * nc);           // Bc
    per += al(sizeof(double) * (wd + 128 + nc));  // vec (w | rowk)
    per += al(sizeof(Partial) * tiles_of(jb, l));
    per += al(sizeof(int64_t) * nc);              // Jc
    per += al(sizeof(int32_t) * nc) * 2;          // colmap, srcpos
    per += al(nc);                                // insel
    per += al(sizeof(int64_t) * r) + al(sizeof(int32_t) * r);
    per += al(sizeof(double) * 4 * kDbgRing);
    per += al(sizeof(double) * mr * kLz);         // swap history: columns g_s
    per += al(sizeof(double) * kLz * r);          // swap history: factors v_s
    return per;
  };
  size_t bytes = 4096;  // done counters (16 per level)
  const bool propose = nj == 1 && jobs[0].active && jobs[0].o.propose == 1;
  if (propose) bytes += propose_scratch(jobs[0].m, jobs[0].n, jobs[0].r, jobs[0].b) + 256;
  bytes += al(sizeof(Node) * total);
  bytes += al(sizeof(RootOut) * nj);
  for (const TreeJob<T>& jb : jobs)
    if (jb.active)
      for (size_t l = 0; l < jb.count.size(); ++l) bytes += node_bytes(jb, (int)l) * jb.count[l];
  const int rtr = tr ? jobs[0].r : 0;
  if (tr) bytes += al(sizeof(int64_t) * 2 * (size_t)total * rtr);  // export buffers
  if (16 * nlev * (int)sizeof(int32_t) > 4096) {
    set_error("tree too deep");
    return CUR_ERR_INTERNAL;
  }
  cur_status st = ensure_arena(ctx, bytes);
  if (st != CUR_OK) return st;
  Arena ar{(char*)ctx->arena, ctx->arena_bytes, 0};
  int32_t* d_done = (int32_t*)ar.take(4096);
  Node* d_nodes = (Node*)ar.take(sizeof(Node) * total);
  RootOut* d_roots = (RootOut*)ar.take(sizeof(RootOut) * nj);
  std::vector<Node> h(total);
  std::memset(h.data(), 0, sizeof(Node) * total);
  int maxm = 0, rmax = 0, leafmax = 0, maxtiles = 0;
  int64_t iter_bound = 0;
  std::vector<RootOut> roots;
  struct AltCopy {
    void* dst;
    const T* src;
    int64_t n, m, lda;
  };
  std::vector<AltCopy> alt_copies;  // A^T panels of polish nodes whose source rows are padded
  for (TreeJob<T>& jb : jobs) {
    if (!jb.active) continue;
    const int r = jb.r;
    maxm = std::max<int>(maxm, (int)std::min<int64_t>(jb.m, INT32_MAX));
    rmax = std::max(rmax, r);
    leafmax = std::max(leafmax, jb.leafmax);
    maxtiles = std::max(maxtiles, tiles_of(jb, 0));
    iter_bound = std::max<int64_t>(iter_bound, 16 * (int64_t)(r + 4) + 8 * (int64_t)jb.o.max_swaps + 4096);
    for (size_t l = 0; l < jb.count.size(); ++l) {
      const int nc = jb.ncmax[l];
      const int wd = is_polish(jb, (int)l) ? r : std::max(nc, r);
      for (int k = 0; k < jb.count[l]; ++k) {
        Node& nd = h[lfirst[l] + jb.off[l] + k];
        nd.m = jb.m;
        nd.r = r;
        nd.ncmax = nc;
        nd.ntiles = jb.ntiles;
        nd.smax = jb.o.max_swaps;
        nd.tau = jb.o.tau;
        nd.theta = jb.theta;
        nd.panel = ar.take(sizeof(T) * jb.m * nc);
        nd.work = ar.take(sizeof(double) * rows_of(jb, (int)l) * wd);
        nd.X = (double*)ar.take(sizeof(double) * r * r);
        nd.Bc = (double*)ar.take(sizeof(double) * r * nc);
        nd.vec = (double*)ar.take(sizeof(double) * (wd + 128 + nc));
        nd.part = (Partial*)ar.take(sizeof(Partial) * tiles_of(jb, (int)l));
        if (is_polish(jb, (int)l)) {
          if (jb.trans) {
            set_error("a polish over a transposed source");
            return CUR_ERR_INTERNAL;
          }
          if (alt_copy(jb, (int)l)) {
            nd.panel_alt = ar.take(sizeof(T) * jb.n * jb.m);
            if (!nd.panel_alt) {
              set_error("workspace layout overflow");
              return CUR_ERR_INTERNAL;
            }
            alt_copies.push_back({nd.panel_alt, jb.A, jb.n, jb.m, jb.lda});
          } else {
            nd.panel_alt = const_cast<T*>(jb.A);
          }
          nd.m_alt = jb.n;
          nd.ntiles_alt = jb.ntiles_alt;
          nd.flipped = 0;
        }
        nd.Jc = (int64_t*)ar.take(sizeof(int64_t) * nc);
        nd.colmap = (int32_t*)ar.take(sizeof(int32_t) * nc);
        nd.srcpos = (int32_t*)ar.take(sizeof(int32_t) * nc);
        nd.insel = (uint8_t*)ar.take(nc);
        nd.I = (int64_t*)ar.take(sizeof(int64_t) * r);
        nd.Jp = (int32_t*)ar.take(sizeof(int32_t) * r);
        nd.dbg = (double*)ar.take(sizeof(double) * 4 * kDbgRing);
        nd.lzg = ar.take(sizeof(double) * rows_of(jb, (int)l) * kLz);
        nd.lzv = (double*)ar.take(sizeof(double) * kLz * r);
        if (!nd.panel || !nd.work || !nd.insel || !nd.Jp || !nd.dbg || !nd.lzv) {
          set_error("workspace layout overflow");
          return CUR_ERR_INTERNAL;
        }
        if (l == 0) {
          const int64_t c0 = (int64_t)k * jb.w, c1 = (k == jb.b - 1) ? jb.n : (int64_t)(k + 1) * jb.w;
          nd.kind = KIND_LEAF;
          nd.child0 = nd.child1 = -1;
          nd.nc = (int)(c1 - c0);
          nd.st = ST_ACA;
          nd.t = 0;
          nd.na = nd.nc;
          nd.steps = (int)std::min<int64_t>(std::min<int64_t>(r, nd.nc), jb.m);
          nd.src = jb.A;
          nd.lda = jb.lda;
          nd.trans = jb.trans ? 1 : 0;
          nd.col0 = c0;
          if (jb.start_I) {  // the given cross, loaded by k_start_cross
            nd.kind = KIND_POLISH;
            nd.st = ST_START_SWAP;
            nd.t = nd.q = r;
          }
        } else if (is_polish(jb, (int)l)) {
          nd.kind = KIND_POLISH;
          nd.child0 = jb.off[l - 1];
          nd.child1 = -1;
          nd.nc = (int)jb.n;
          nd.src = jb.A;
          nd.lda = jb.lda;
          nd.trans = jb.trans ? 1 : 0;
          nd.col0 = 0;
          nd.st = ST_DONE;
        } else {
          const int pc = jb.count[l - 1], po = jb.off[l - 1];
          if (2 * k + 1 < pc) {
            nd.kind = KIND_MERGE;
            nd.child0 = po + 2 * k;
            nd.child1 = po + 2 * k + 1;
          } else {
            nd.kind = KIND_PROMOTED;
            nd.child0 = po + 2 * k;
            nd.child1 = -1;
            const Node& c = h[lfirst[l - 1] + po + 2 * k];
            nd.panel = c.panel;
            nd.Jc = c.Jc;
            nd.ncmax = c.ncmax;
          }
          nd.st = ST_DONE;
        }
      }
    }
    const int lt = (int)jb.count.size() - 1;
    roots.push_back({lfirst[lt] + jb.off[lt], 0, jb.I, jb.J});
  }
  int64_t* d_expI = tr ? (int64_t*)ar.take(sizeof(int64_t) * (size_t)total * rtr) : nullptr;
  int64_t* d_expJ = tr ? (int64_t*)ar.take(sizeof(int64_t) * (size_t)total * rtr) : nullptr;
  CUR_HIP_CHECK(hipMemcpyAsync(d_nodes, h.data(), sizeof(Node) * total, hipMemcpyHostToDevice, s));
  for (const AltCopy& c : alt_copies)  // A^T column-major (ld n) = the rows of A, packed
    CUR_HIP_CHECK(hipMemcpy2DAsync(c.dst, sizeof(T) * c.n, c.src, sizeof(T) * c.lda, sizeof(T) * c.n, c.m,
                                   hipMemcpyDeviceToDevice, s));
  CUR_HIP_CHECK(hipMemcpyAsync(d_roots, roots.data(), sizeof(RootOut) * roots.size(), hipMemcpyHostToDevice, s));
  CUR_HIP_CHECK(hipMemsetAsync(d_done, 0, 4096, s));
  if (ctx->prof_on) CUR_HIP_CHECK(hipMemsetAsync(ctx->prof_bytes, 0, sizeof(unsigned long long) * 2 * kProfSlots, s));

  int fixed_groups = 0;
  for (const TreeJob<T>& jb : jobs)
    if (jb.active) {
      fixed_groups = jb.o.groups;
      break;
    }
  const int f64 = std::is_same<T, double>::value ? 1 : 0;

  // ---- level 0: every leaf of every tree
  size_t prof_used = 0;
  {
    const int b = lcount[0];
    hipLaunchKernelGGL(k_leaf_init, dim3(b), dim3(kThreads), 0, s, d_nodes);
    for (const TreeJob<T>& jb : jobs)
      if (jb.active && jb.start_I)
        hipLaunchKernelGGL(k_start_cross, dim3(1), dim3(kThreads), 0, s, d_nodes + lfirst[0] + jb.off[0], jb.start_I,
                           jb.start_J);
    hipLaunchKernelGGL((k_panel_from_A<T>), dim3((maxm + kTR - 1) / kTR, (leafmax + 63) / 64, b), dim3(kThreads),
                       0, s, d_nodes);
    if (propose) {  // learned candidates: the restricted start of every leaf that admits one
      const TreeJob<T>& jb = jobs[0];
      char* scratch = (char*)ar.take(propose_scratch(jb.m, jb.n, jb.r, jb.b));
      if (!scratch) {
        set_error("workspace layout overflow");
        return CUR_ERR_INTERNAL;
      }
      cur_status prc = propose_leaves<T>(ctx, jb.A, jb.m, jb.n, jb.lda, jb.r, jb.w, jb.b, jb.o.mlp, jb.o.seed, d_nodes,
                                         scratch);
      if (prc != CUR_OK) return prc;
    }
    const int64_t key[6] = {f64, rb, b, maxtiles, maxm, 1};
    int cand = -1;
    const int groups = tune_pick(ctx, key, fixed_groups, &cand);
    const auto t0 = std::chrono::steady_clock::now();
    cur_status rc = run_level<T>(ctx, rb, d_nodes, b, maxtiles, d_done + 0, iter_bound, prof_used, groups);
    if (rc == CUR_OK) tune_record(ctx, key, cand, t0);
    if (rc != CUR_OK) return rc;
  }

  // ---- merges
  for (int l = 1; l < nlev; ++l) {
    Node* cur = d_nodes + lfirst[l];
    Node* prev = d_nodes + lfirst[l - 1];
    const int cnt = lcount[l];
    int lm = 0, lt = 0;
    for (const TreeJob<T>& jb : jobs)
      if (jb.active && (int)jb.count.size() > l) {
        lm = std::max<int>(lm, (int)std::min<int64_t>(jb.m, INT32_MAX));
        lt = std::max(lt, tiles_of(jb, l));
      }
    int32_t* dd = d_done + 16 * l;
    hipLaunchKernelGGL(k_merge_init, dim3(cnt), dim3(kThreads), 0, s, cur, prev);
    const int gx = (int)std::min<int64_t>((lm + kThreads - 1) / kThreads, 64);
    hipLaunchKernelGGL((k_panel_build<T>), dim3(gx, 2 * rmax, cnt), dim3(kThreads), 0, s, cur, prev);
    int64_t polish_n = 0;  // a polish node's panel: every column of its matrix
    for (const TreeJob<T>& jb : jobs)
      if (jb.active && jb.polish && (int)jb.count.size() == l + 1) polish_n = std::max(polish_n, jb.n);
    if (polish_n > 0)
      hipLaunchKernelGGL((k_panel_from_A<T>), dim3((lm + kTR - 1) / kTR, (unsigned)((polish_n + 63) / 64), cnt),
                         dim3(kThreads), 0, s, cur);
    const int64_t key[6] = {f64, rb, cnt, lt, lm, 0};
    int cand = -1;
    const int groups = tune_pick(ctx, key, fixed_groups, &cand);
    const auto t0 = std::chrono::steady_clock::now();
    cur_status rc = run_level<T>(ctx, rb, cur, cnt, lt, dd, iter_bound, prof_used, groups);
    if (rc == CUR_OK) tune_record(ctx, key, cand, t0);
    if (rc != CUR_OK) return rc;
  }

  // ---- outputs
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)roots.size()), dim3(kThreads), 0, s, d_nodes, d_roots);
  CUR_HIP_CHECK(hipMemcpyAsync(h.data(), d_nodes, sizeof(Node) * total, hipMemcpyDeviceToHost, s));
  std::vector<int64_t> eI, eJ;
  if (tr) {
    hipLaunchKernelGGL(k_export, dim3(total), dim3(kThreads), 0, s, d_nodes, d_expI, d_expJ, rtr);
    eI.resize((size_t)total * rtr);
    eJ.resize((size_t)total * rtr);
    CUR_HIP_CHECK(hipMemcpyAsync(eI.data(), d_expI, sizeof(int64_t) * eI.size(), hipMemcpyDeviceToHost, s));
    CUR_HIP_CHECK(hipMemcpyAsync(eJ.data(), d_expJ, sizeof(int64_t) * eJ.size(), hipMemcpyDeviceToHost, s));
  }
  CUR_HIP_CHECK(hipStreamSynchronize(s));
  if (ctx->prof_on && prof_used >= 2) {
    const size_t pairs = prof_used / 2;
    std::vector<unsigned long long> hb(2 * pairs);
    CUR_HIP_CHECK(hipMemcpy(hb.data(), ctx->prof_bytes, sizeof(unsigned long long) * 2 * pairs, hipMemcpyDeviceToHost));
    std::vector<hipEvent_t>& ev = *ctx->prof_ev;
    for (size_t k = 0; k < pairs; ++k) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]) != hipSuccess) continue;
      cur_profile& p = ctx->prof;
      const unsigned long long b = hb[2 * k], bm = hb[2 * k + 1];
      if ((*ctx->prof_kind)[k] == 1) {
        p.fresh_launches += 1;
        p.fresh_busy += b > 0;
        p.fresh_seconds += 1e-3 * ms;
        if (b > 0) p.fresh_busy_seconds += 1e-3 * ms;
        p.fresh_bytes += (double)b;
        p.fresh_bytes_inplace += (double)bm;
      } else {
        p.launches += 1;
        p.busy += b > 0;
        p.seconds += 1e-3 * ms;
        if (b > 0) p.busy_seconds += 1e-3 * ms;
        p.bytes += (double)b;
        p.bytes_inplace += (double)bm;
      }
    }
  }
  if (std::getenv("CUR_DEBUG")) debug_report(ctx, h, lfirst, lcount);
  for (int k = 0; k < total; ++k)
    if (h[k].st != ST_DONE) {
      set_error("a tree node was left unfinished");
      return CUR_ERR_INTERNAL;
    }

  // ---- per-tree results
  auto polish_idle = [&](const TreeJob<T>& jb) {
    if (!jb.polish) return false;
    const size_t l = jb.count.size() - 2;  // the tree's root, the polish node's start
    const Node& c = h[lfirst[l] + jb.off[l]];
    return c.is_short != 0 || c.err != 0;
  };
  for (TreeJob<T>& jb : jobs) {
    if (!jb.active) continue;
    auto node = [&](size_t l, int k) -> const Node& { return h[lfirst[l] + jb.off[l] + k]; };
    // a polish level over a rank-short or failed root did nothing: no node,
    // no counters, no trace record
    const bool pol_idle = polish_idle(jb);
    cur_status result = CUR_OK;
    int32_t nodes = 0, phases = 0, refreshes = 0;
    int64_t swaps = 0;
    bool nocap = false;
    std::string where;
    for (size_t l = 0; l < jb.count.size(); ++l)
      for (int k = 0; k < jb.count[l]; ++k) {
        const Node& nd = node(l, k);
        if (nd.err && result == CUR_OK) {
          result = CUR_ERR_INTERNAL;
          where = " (level " + std::to_string(l) + " node " + std::to_string(k) + " code " + std::to_string(nd.err) +
                  " phase " + std::to_string(nd.phase) + " swaps " + std::to_string(nd.swaps) + ")";
        }
        if (nd.kind == KIND_PROMOTED || (pol_idle && nd.kind == KIND_POLISH)) continue;
        nodes++;
        phases += nd.phases;
        refreshes += nd.refreshes;
        swaps += nd.swaps;
        nocap |= nd.nocap != 0;
      }
    const Node& root = node(jb.count.size() - 1, 0);
    if (result == CUR_OK) {
      if (root.is_short) {
        result = CUR_ERR_RANK;
        set_error("rank-short: fewer than r pivots above the threshold");
      } else if (nocap) {
        result = CUR_WARN_NOCONV;
      }
    } else {
      set_error("singular cross met inside the swap loop" + where);
    }
    if (jb.info) {
      jb.info->rank = root.q;
      jb.info->nodes = nodes;
      jb.info->phases = phases;
      jb.info->refreshes = refreshes;
      jb.info->swaps = swaps;
      jb.info->logvol = root.is_short ? -HUGE_VAL : std::log(root.vol_m) + root.vol_e * 0.69314718055994530942;
    }
    jb.status = result;
  }
  if (tr && jobs[0].active) {
    const TreeJob<T>& jb = jobs[0];
    const int cap = tr->capacity;
    const bool pol_idle = polish_idle(jb);
    int slot = 0;
    for (size_t l = 0; l < jb.count.size(); ++l)
      for (int k = 0; k < jb.count[l]; ++k, ++slot) {
        const size_t gi = lfirst[l] + jb.off[l] + k;
        const Node& nd = h[gi];
        if (pol_idle && nd.kind == KIND_POLISH) {
          --slot;
          continue;
        }
        if (slot >= cap) continue;
        int64_t* mt = tr->meta + (size_t)slot * kMetaFields;
        const bool pr = nd.kind == KIND_PROMOTED;
        mt[0] = (int64_t)l;
        mt[1] = k;
        mt[2] = nd.q;
        mt[3] = nd.is_short;
        mt[4] = pr ? 1 : 0;
        mt[5] = pr ? 0 : nd.nocap;
        mt[6] = pr ? 0 : nd.swaps;
        mt[7] = pr ? 0 : nd.phases;
        mt[8] = pr ? 0 : nd.refreshes;
        mt[9] = nd.is_short ? 0 : nd.vol_e;
        tr->vol_mant[slot] = nd.is_short ? 0.0 : nd.vol_m;
        for (int j = 0; j < rtr; ++j) {
          tr->I[(size_t)slot * rtr + j] = eI[gi * rtr + j];
          tr->J[(size_t)slot * rtr + j] = eJ[gi * rtr + j];
        }
      }
    tr->count = slot;
  }
  return CUR_OK;
}

template <typename T>
static cur_status select_one(cur_ctx ctx, const T* A, int64_t m, int64_t n, int64_t lda, int r, const cur_opts& o,
                             int64_t* I, int64_t* J, cur_info* info) {
  std::vector<TreeJob<T>> jobs(1);
  TreeJob<T>& jb = jobs[0];
  jb.A = A;
  jb.m = m;
  jb.n = n;
  jb.lda = lda;
  jb.r = r;
  jb.o = o;
  jb.I = I;
  jb.J = J;
  jb.info = info;
  jb.polish = o.polish != 0;
  cur_status rc = select_many<T>(ctx, rmax_bucket(r), jobs, o.trace);
  if (rc != CUR_OK) return rc;
  return jobs[0].status;
}

cur_status select_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n,
                           int64_t lda, int r, const cur_opts& o, int64_t* I, int64_t* J,
                           cur_info* info) {
  if (dtype == CUR_F64)
    return select_one<double>(ctx, (const double*)A, m, n, lda, r, o, I, J, info);
  return select_one<float>(ctx, (const float*)A, m, n, lda, r, o, I, J, info);
}

// Alg. 2 with a row count r and a column count c: J from the column-block
// tree on A with rank c, I from the same tree on A^T with rank r (the row
// blocks of A); each tree's other index set goes to `discard` (device,
// max(r, c) entries per tree).  Trees of one rank bucket share one engine
// run (their levels advance together), otherwise they run one after the
// other.  Status: a rank shortfall of either, then a spent swap budget.
template <typename T>
static cur_status select_rect_impl(cur_ctx ctx, const T* A, int64_t m, int64_t n, int64_t lda, int r, int c,
                                   const cur_opts& o, int64_t* I, int64_t* J, int64_t* discard, cur_info* info) {
  std::vector<TreeJob<T>> jobs(2);
  cur_info inf[2];
  for (int k = 0; k < 2; ++k) {
    TreeJob<T>& jb = jobs[k];
    const bool rows = k == 1;
    jb.A = A;
    jb.trans = rows;
    jb.m = rows ? n : m;
    jb.n = rows ? m : n;
    jb.lda = lda;
    jb.r = rows ? r : c;
    jb.o = o;
    jb.o.trace = nullptr;
    jb.I = discard + (int64_t)k * std::max(r, c);
    jb.J = rows ? I : J;
    jb.info = &inf[k];
  }
  cur_status rc = CUR_OK;
  if (rmax_bucket(r) == rmax_bucket(c)) {
    rc = select_many<T>(ctx, rmax_bucket(r), jobs, nullptr);
  } else {
    for (int k = 0; k < 2 && rc == CUR_OK; ++k) {
      std::vector<TreeJob<T>> one(1, jobs[k]);
      rc = select_many<T>(ctx, rmax_bucket(one[0].r), one, nullptr);
      jobs[k].status = one[0].status;
    }
  }
  if (rc != CUR_OK) return rc;
  if (info) {
    *info = inf[0];
    info->rank = std::min(inf[0].rank, inf[1].rank);
    info->swaps += inf[1].swaps;
    info->phases += inf[1].phases;
    info->refreshes += inf[1].refreshes;
    info->nodes += inf[1].nodes;
    info->logvol = std::nan("");  // no single square cross
  }
  auto worse = [](cur_status a, cur_status b) {
    for (cur_status s : {CUR_ERR_RANK, CUR_WARN_NOCONV})
      if (a == s || b == s) return s;
    return a != CUR_OK ? a : b;
  };
  cur_status res = worse(jobs[0].status, jobs[1].status);
  // r == c: the swap loop once more on the cross (I, J) of the two trees,
  // every column a candidate; skipped when either tree fell short or failed
  if (o.polish && r == c && (res == CUR_OK || res == CUR_WARN_NOCONV)) {
    std::vector<TreeJob<T>> pj(1);
    TreeJob<T>& jb = pj[0];
    cur_info pinf{};
    jb.A = A;
    jb.m = m;
    jb.n = n;
    jb.lda = lda;
    jb.r = r;
    jb.o = o;
    jb.o.trace = nullptr;
    jb.o.col_block = (int32_t)n;  // one node over every column
    jb.I = I;
    jb.J = J;
    jb.info = &pinf;
    jb.start_I = I;
    jb.start_J = J;
    rc = select_many<T>(ctx, rmax_bucket(r), pj, nullptr);
    if (rc != CUR_OK) return rc;
    if (info) {
      info->rank = pinf.rank;
      info->swaps += pinf.swaps;
      info->phases += pinf.phases;
      info->refreshes += pinf.refreshes;
      info->nodes += pinf.nodes;
      info->logvol = pinf.logvol;
    }
    res = worse(res, pj[0].status);
  }
  return res;
}

cur_status select_rect_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n, int64_t lda,
                                int r, int c, const cur_opts& o, int64_t* I, int64_t* J, int64_t* discard,
                                cur_info* info) {
  if (dtype == CUR_F64)
    return select_rect_impl<double>(ctx, (const double*)A, m, n, lda, r, c, o, I, J, discard, info);
  return select_rect_impl<float>(ctx, (const float*)A, m, n, lda, r, c, o, I, J, discard, info);
}

// Items of one dtype and one rank bucket run as one set of trees.
template <typename T>
static cur_status select_group(cur_ctx ctx, int rb, const std::vector<int>& idx, const cur_item* items,
                               const std::vector<cur_opts>& opts, cur_status* per_item) {
  std::vector<TreeJob<T>> jobs(idx.size());
  for (size_t q = 0; q < idx.size(); ++q) {
    const cur_item& it = items[idx[q]];
    TreeJob<T>& jb = jobs[q];
    jb.A = (const T*)it.A;
    jb.m = it.m;
    jb.n = it.n;
    jb.lda = it.lda;
    jb.r = it.r;
    jb.o = opts[idx[q]];
    jb.I = it.I;
    jb.J = it.J;
    jb.info = nullptr;
    jb.polish = jb.o.polish != 0;
  }
  cur_status rc = select_many<T>(ctx, rb, jobs, nullptr);
  for (size_t q = 0; q < idx.size(); ++q) per_item[idx[q]] = rc != CUR_OK ? rc : jobs[q].status;
  return rc;
}

cur_status select_batched_dispatch(cur_ctx ctx, int32_t count, const cur_item* items, const std::vector<cur_opts>& opts,
                                   cur_status* per_item) {
  for (int f64 = 1; f64 >= 0; --f64)
    for (int rb : {32, 64, 128}) {
      std::vector<int> idx;
      for (int32_t i = 0; i < count; ++i)
        if ((items[i].dtype == CUR_F64) == (f64 == 1) && rmax_bucket(items[i].r) == rb) idx.push_back(i);
      if (idx.empty()) continue;
      cur_status rc = f64 ? select_group<double>(ctx, rb, idx, items, opts, per_item)
                          : select_group<float>(ctx, rb, idx, items, opts, per_item);
      if (rc != CUR_OK) return rc;
    }
  return CUR_OK;
}

}  // namespace cur
