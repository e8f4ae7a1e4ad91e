// The row pass of the selection: one launch covers every active node of a
// tree level, grid (row tiles x nodes).  Per node it is the bandwidth-bound
// sweep over the m x (active columns) working matrix -- an ACA rank-1 update
// (Alg. 1), a fresh B = A(:,J) A(I,J)^-1, or a row swap (Sherman-Morrison
// update) -- fused with the per-tile argmax that the next decision needs.
// Column-major panels with leading dimension m: a wavefront reads and writes
// 64 consecutive rows of one column.
#include <hip/hip_runtime.h>

#include <cmath>

#include "cur_device.hpp"
#include "cur_internal.hpp"

namespace cur {

constexpr int kPassWaves = 6;  // wavefronts per SIMD the pass is compiled for

// Best candidate of one row scanned in ascending column order (key row * r + c):
// the first strictly larger |x| wins, NaN never does.  Compares the bit
// pattern of |x|, which orders like the value for |x| >= 0.
struct RowBest {
  uint64_t bits = 0;
  double x = 0.0;
  int c = -1;
  __device__ __forceinline__ void take(double v, int col) {
    const uint64_t u = (uint64_t)__double_as_longlong(v) & 0x7fffffffffffffffull;
    if (v == v && (c < 0 || u > bits)) {
      bits = u;
      x = v;
      c = col;
    }
  }
};

// Tile epilogue of both row kernels: block argmax, the tile winner to the
// node's partial array, and (when profiling) the node's algorithmic bytes,
// added once per node by its first tile.
__device__ __forceinline__ void pass_finish(Node& nd, int tile, Cand best, Cand* sc, unsigned long long* prof,
                                            int64_t node_bytes) {
  best = block_argmax(best, sc);
  if (threadIdx.x == 0) {
    if (prof && tile == 0) atomicAdd(prof, (unsigned long long)node_bytes);
    Partial p;
    p.val = best.val;
    p.sval = best.sval;
    p.key = best.key;
    p.row = best.row;
    p.pos = best.pos;
    p.seq = nd.seq;
    nd.part[tile] = p;
  }
}

// ACA step, fresh B, or row swap over one tile of kTileRows rows, fused with
// the tile's argmax; the tile winner goes to the node's partial array.
template <typename T, int RMAX>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kPassWaves)))
void k_pass(Node* nodes, unsigned long long* prof) {
  Node& nd = nodes[blockIdx.y];
  const int st = nd.st;
  if (st != ST_ACA && st != ST_ROW_SWAP) return;
  const int tile = blockIdx.x;
  if (tile >= nd.ntiles) return;
  const int64_t m = nd.m;
  const int r = nd.r;
  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)tile * kTileRows;
  const int64_t row = row0 + tid;
  const bool valid = row < m;
  T* W = (T*)nd.work;
  const T* P = (const T*)nd.panel;

  __shared__ Cand sc[kThreads / 64];

  Cand best = cand_none();
  // Columns per register round: every load of a round is issued before the
  // round's first store (the stores go to the array the loads read, which the
  // compiler cannot reorder across).  64 bytes per lane per round keeps the
  // register count low enough for kPassWaves wavefronts per SIMD: a launch is
  // thousands of short workgroups, each a chain of dependent latencies (node
  // fields, data, block argmax), so residency, not per-wavefront depth, sets
  // the pass time.
  constexpr int NR = 64 / (int)sizeof(T);

  if (st == ST_ACA) {
    const int t = nd.t, na = nd.na, nc = nd.nc;
    const int32_t* cmap = nd.colmap;
    const T* src = (t <= 1) ? P : W;
    if (t == 0) {
      if (valid)
        for (int c0 = 0; c0 < na; c0 += NR) {
          T xs[NR];
#pragma unroll
          for (int u = 0; u < NR; ++u) xs[u] = (c0 + u < na) ? src[(int64_t)(c0 + u) * m + row] : (T)0;
#pragma unroll
          for (int u = 0; u < NR; ++u) {
            const int c = c0 + u;
            if (c >= na) break;
            Cand o;
            o.val = fabs((double)xs[u]);
            o.sval = (double)xs[u];
            o.key = row * nc + cmap[c];
            o.row = row;
            o.pos = c;
            cand_take(best, o);
          }
        }
    } else {
      // R <- R - R(:, pc) f^T with row pi zeroed; the last active column moves
      // into the freed slot pc.  A later round only reads columns past the
      // earlier ones and writes those columns or pc, which was read already.
      const int pc = nd.pend_k;
      const int64_t pi = nd.pend_i;
      const double* f = nd.vec;
      if (valid) {
        const T g = src[(int64_t)pc * m + row];
        for (int c0 = 0; c0 < na; c0 += NR) {
          T xs[NR];
#pragma unroll
          for (int u = 0; u < NR; ++u) xs[u] = (c0 + u < na) ? src[(int64_t)(c0 + u) * m + row] : (T)0;
#pragma unroll
          for (int u = 0; u < NR; ++u) {
            const int c = c0 + u;
            if (c >= na) break;
            if (c == pc) continue;
            T x = fma_t<T>(-g, (T)f[c], xs[u]);
            if (row == pi) x = (T)0;
            const int np = (c == na - 1) ? pc : c;
            W[(int64_t)np * m + row] = x;
            Cand o;
            o.val = fabs((double)x);
            o.sval = (double)x;
            o.key = row * nc + cmap[c];
            o.row = row;
            o.pos = np;
            cand_take(best, o);
          }
        }
      }
    }
  } else {
    // No mask of the selected rows here: a selected row is exactly e_k, the
    // update keeps it so (its entry in column ks is 0, and fma(-0, v, x) = x),
    // and |e_k| <= 1 < 1 + tau, so such a row can win a tile only when no
    // row swap is due, where the winner's identity is not used.
    RowBest rb;
    {
      // B <- B - B(:, ks) v^T, row is set to e_ks^T
      const int ks = nd.pend_k;
      const int64_t is = nd.pend_i;
      const double* v = nd.vec;
      if (valid) {
        const T g = W[(int64_t)ks * m + row];
        for (int c0 = 0; c0 < r; c0 += NR) {
          T bs[NR];
#pragma unroll
          for (int u = 0; u < NR; ++u) bs[u] = (c0 + u < r) ? W[(int64_t)(c0 + u) * m + row] : (T)0;
#pragma unroll
          for (int u = 0; u < NR; ++u) {
            const int c = c0 + u;
            if (c >= r) break;
            T b = fma_t<T>(-g, (T)v[c], bs[u]);
            if (row == is) b = (c == ks) ? (T)1 : (T)0;
            W[(int64_t)c * m + row] = b;
            rb.take((double)b, c);
          }
        }
      }
    }
    if (rb.c >= 0) {
      best.val = fabs(rb.x);
      best.sval = rb.x;
      best.key = row * r + rb.c;
      best.row = row;
      best.pos = rb.c;
    }
  }

  int64_t cols;  // algorithmic columns: working columns read + columns written
  if (st == ST_ACA) cols = (nd.t == 0) ? nd.na : 2 * nd.na - 1;
  else cols = 2 * (int64_t)r;
  pass_finish(nd, tile, best, sc, prof, m * cols * (int64_t)sizeof(T));
}

// Fresh B = A(:, J) X over one tile of kTileRows rows (X = A(I, J)^-1, r x r
// row-major), rows I set to unit rows, fused with the tile's argmax over the
// other rows.  Every output is the FP64 sum over k ascending of
// A(row, Jp_k) X(k, c).  X is staged in LDS CB columns at a time (broadcast
// reads); A(row, Jp_k) is read 8 columns at a time per chunk, from L2 after
// the first chunk.  Its own kernel: the product wants registers that would
// cost the streaming pass its residency.
template <typename T, int RMAX>
__global__ __launch_bounds__(kThreads) void k_fresh(Node* nodes, unsigned long long* prof) {
  Node& nd = nodes[blockIdx.y];
  if (nd.st != ST_ROW_FRESH) return;
  const int tile = blockIdx.x;
  if (tile >= nd.ntiles) return;
  const int64_t m = nd.m;
  const int r = nd.r;
  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)tile * kTileRows;
  const int64_t row = row0 + tid;
  const bool valid = row < m;
  T* W = (T*)nd.work;
  const T* P = (const T*)nd.panel;

  constexpr int CB = 16;  // columns of X staged per chunk
  __shared__ double sX[RMAX * CB];
  __shared__ int sJp[RMAX];
  __shared__ int sslot[kTileRows];
  __shared__ Cand sc[kThreads / 64];
  sslot[tid] = -1;
  __syncthreads();
  for (int k = tid; k < r; k += kThreads) {
    const int64_t i = nd.I[k];
    if (i >= row0 && i < row0 + kTileRows) sslot[i - row0] = k;
    sJp[k] = nd.Jp[k];
  }
  __syncthreads();
  const int slot = sslot[tid];
  RowBest rb;
  for (int c0 = 0; c0 < r; c0 += CB) {
    const int nb = min(CB, r - c0);
    __syncthreads();
    for (int idx = tid; idx < r * CB; idx += kThreads) {
      const int k = idx / CB, j = idx % CB;
      sX[idx] = (j < nb) ? nd.X[(int64_t)k * r + c0 + j] : 0.0;
    }
    __syncthreads();
    if (valid) {
      double acc[CB];
#pragma unroll
      for (int j = 0; j < CB; ++j) acc[j] = 0.0;
      constexpr int U = 8;
      for (int k0 = 0; k0 < r; k0 += U) {
        double pk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) pk[u] = (k0 + u < r) ? (double)P[(int64_t)sJp[k0 + u] * m + row] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (k0 + u < r) {
#pragma unroll
            for (int j = 0; j < CB; ++j) acc[j] = fma(pk[u], sX[(k0 + u) * CB + j], acc[j]);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        if (j < nb) {
          const int c = c0 + j;
          T b = (T)acc[j];
          if (slot >= 0) b = (c == slot) ? (T)1 : (T)0;
          W[(int64_t)c * m + row] = b;
          if (slot < 0) rb.take((double)b, c);
        }
      }
    }
  }
  Cand best = cand_none();
  if (rb.c >= 0) {
    best.val = fabs(rb.x);
    best.sval = rb.x;
    best.key = row * r + rb.c;
    best.row = row;
    best.pos = rb.c;
  }
  pass_finish(nd, tile, best, sc, prof, m * 2 * (int64_t)r * (int64_t)sizeof(T));
}

template <typename T, int RMAX>
static void launch_fresh_t(Node* nodes, int count, int tiles, unsigned long long* prof, hipStream_t s) {
  hipLaunchKernelGGL((k_fresh<T, RMAX>), dim3(tiles, count), dim3(kThreads), 0, s, nodes, prof);
}

template <typename T, int RMAX>
static void launch_pass_t(Node* nodes, int count, int tiles, unsigned long long* prof, hipStream_t s) {
  hipLaunchKernelGGL((k_pass<T, RMAX>), dim3(tiles, count), dim3(kThreads), 0, s, nodes, prof);
}

// The fresh kernel touches only nodes in the fresh state and the pass kernel
// only the others, so within an iteration the two are independent.
void fresh_launch(bool f64, int rb, Node* nodes, int count, int tiles, unsigned long long* prof, hipStream_t s) {
  if (f64) {
    if (rb == 32) launch_fresh_t<double, 32>(nodes, count, tiles, prof, s);
    else if (rb == 64) launch_fresh_t<double, 64>(nodes, count, tiles, prof, s);
    else launch_fresh_t<double, 128>(nodes, count, tiles, prof, s);
  } else {
    if (rb == 32) launch_fresh_t<float, 32>(nodes, count, tiles, prof, s);
    else if (rb == 64) launch_fresh_t<float, 64>(nodes, count, tiles, prof, s);
    else launch_fresh_t<float, 128>(nodes, count, tiles, prof, s);
  }
}

void pass_launch(bool f64, int rb, Node* nodes, int count, int tiles, unsigned long long* prof, hipStream_t s) {
  if (f64) {
    if (rb == 32) launch_pass_t<double, 32>(nodes, count, tiles, prof, s);
    else if (rb == 64) launch_pass_t<double, 64>(nodes, count, tiles, prof, s);
    else launch_pass_t<double, 128>(nodes, count, tiles, prof, s);
  } else {
    if (rb == 32) launch_pass_t<float, 32>(nodes, count, tiles, prof, s);
    else if (rb == 64) launch_pass_t<float, 64>(nodes, count, tiles, prof, s);
    else launch_pass_t<float, 128>(nodes, count, tiles, prof, s);
  }
}

}  // namespace cur
