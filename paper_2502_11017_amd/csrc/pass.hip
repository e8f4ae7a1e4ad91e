// The row pass of the selection: one launch covers every active node of a
// tree level, grid (row tiles x nodes).  Per node it is the bandwidth-bound
// sweep over the m x (active columns) working matrix -- an ACA rank-1 update
// (Alg. 1), a fresh B = A(:,J) A(I,J)^-1, or a row swap (Sherman-Morrison
// update) -- fused with the per-tile argmax that the next decision needs.
// Column-major panels with leading dimension m: a wavefront reads and writes
// 64 consecutive rows of one column.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "cur_device.hpp"
#include "cur_internal.hpp"

namespace cur {

constexpr int kPassWaves = 6;  // wavefronts per SIMD the pass is compiled for

// |x| as an unsigned integer of the element's width: for |x| >= 0 the bit
// pattern orders like the value, so a lane compares candidates with one
// integer compare in the input type (no conversion to FP64 per element).
template <typename T>
struct AbsBits;
template <>
struct AbsBits<double> {
  using U = uint64_t;
  static __device__ __forceinline__ U of(double x) {
    return (U)__double_as_longlong(x) & 0x7fffffffffffffffull;
  }
};
template <>
struct AbsBits<float> {
  using U = uint32_t;
  static __device__ __forceinline__ U of(float x) { return (U)__float_as_uint(x) & 0x7fffffffu; }
};

// Best candidate of one row scanned in ascending column order (key row * r + c):
// the first strictly larger |x| wins, NaN never does.
template <typename T>
struct RowBest {
  typename AbsBits<T>::U bits = 0;
  T x = (T)0;
  int c = -1;
  __device__ __forceinline__ void take(T v, int col) {
    const typename AbsBits<T>::U u = AbsBits<T>::of(v);
    if (v == v && (c < 0 || u > bits)) {
      bits = u;
      x = v;
      c = col;
    }
  }
  // the row's candidate in the tile-argmax order
  __device__ __forceinline__ void to_cand(Cand& best, int64_t row, int r) const {
    if (c >= 0) {
      best.val = fabs((double)x);
      best.sval = (double)x;
      best.key = row * r + c;
      best.row = row;
      best.pos = c;
    }
  }
};

// Best candidate of one row in an ACA step: larger |x| first, ties to the
// smaller original column id (the key row * nc + id), NaN never.  Same order
// as the tile argmax restricted to one row.
template <typename T>
struct AcaBest {
  typename AbsBits<T>::U bits = 0;
  T x = (T)0;
  int id = 0x7fffffff;
  int pos = -1;
  __device__ __forceinline__ void take(T v, int cid, int p) {
    const typename AbsBits<T>::U u = AbsBits<T>::of(v);
    if (v == v && (pos < 0 || u > bits || (u == bits && cid < id))) {
      bits = u;
      x = v;
      id = cid;
      pos = p;
    }
  }
  __device__ __forceinline__ void to_cand(Cand& best, int64_t row, int nc) const {
    if (pos >= 0) {
      best.val = fabs((double)x);
      best.sval = (double)x;
      best.key = row * nc + id;
      best.row = row;
      best.pos = pos;
    }
  }
};

// Element at byte offset `off` of a column whose base is wavefront-uniform:
// a scalar base plus one 32-bit offset register per lane, shared by every
// load and store of the row (the selection checks m * sizeof(T) < 2^32).
template <typename T>
__device__ __forceinline__ T col_ld(GPtr<const T> col, uint32_t off) {
  return *(GPtr<const T>)((__attribute__((address_space(1))) const char*)col + off);
}
template <typename T>
__device__ __forceinline__ void col_st(GPtr<T> col, uint32_t off, T v) {
  *(GPtr<T>)((__attribute__((address_space(1))) char*)col + off) = v;
}

// Per-column values of a pass (up to 256 columns) held one per lane: column
// c in lane c & 63 of register c >> 6, read back with readlane.  Loaded once
// per workgroup with coalesced loads, they cost no memory access between a
// round's loads and its stores.
constexpr int kLaneCols = 256;
template <typename V>
__device__ __forceinline__ void lane_load(V (&reg)[4], const V* src_generic, int n) {
  const int lane = threadIdx.x & 63;
  const GPtr<const V> src = (GPtr<const V>)src_generic;
#pragma unroll
  for (int q = 0; q < 4; ++q) {  // n >= 1: clamped loads, then a select (no branch per load)
    const int c = lane + 64 * q;
    const V v = src[min(c, n - 1)];
    reg[q] = c < n ? v : (V)0;
  }
}
// reg[q] for a wavefront-uniform q < 4, as a select tree (stays in registers)
template <typename V>
__device__ __forceinline__ V lane_reg(const V (&reg)[4], int q) {
  const V lo = (q & 1) ? reg[1] : reg[0];
  const V hi = (q & 1) ? reg[3] : reg[2];
  return (q & 2) ? hi : lo;
}
__device__ __forceinline__ double lane_read(double v, int l) { return readlane_f64(v, l); }
__device__ __forceinline__ float lane_read(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ int lane_read(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// Tile epilogue of both row kernels: block argmax, the tile winner to the
// node's partial array, and (when profiling) the node's bytes, added once per
// node by its first tile to the launch's two slots: prof[0] the bytes this
// implementation must move, prof[1] those of the plain in-place algorithm
// (an elimination step or a row swap reads and writes the whole active
// working matrix; a fresh B reads A(:, J) and writes B).
__device__ __forceinline__ void pass_finish(Node& nd, int tile, Cand best, Cand* sc, unsigned long long* prof,
                                            int64_t node_bytes, int64_t model_bytes) {
  best = block_argmax(best, sc);
  if (threadIdx.x == 0) {
    if (prof && tile == 0) {
      atomicAdd(prof, (unsigned long long)node_bytes);
      atomicAdd(prof + 1, (unsigned long long)model_bytes);
    }
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

// ACA step or row swap over one tile of kTileRows rows, fused with the
// tile's argmax; the tile winner goes to the node's partial array.
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
  const GPtr<T> W = (GPtr<T>)nd.work;
  const GPtr<const T> P = (GPtr<const T>)nd.panel;
  // element (row, c) of a column-major working matrix: the column's base
  // (wavefront-uniform) plus the row's byte offset.  Rows past m load row
  // m - 1 and store nothing: the rounds run with every lane active, because
  // the per-column values below are read across lanes (readlane), which needs
  // them computed in all lanes.
  const uint32_t ro = (uint32_t)(valid ? row : m - 1) * (uint32_t)sizeof(T);

  __shared__ Cand sc[kThreads / 64];

  Cand best = cand_none();
  // Columns per register round: every load of a round is issued before the
  // round's first store (the stores go to the array the loads read, which the
  // compiler cannot reorder across).  16 columns per round keeps the
  // register count low enough for kPassWaves wavefronts per SIMD: a launch is
  // thousands of short workgroups, each a chain of dependent latencies (node
  // fields, data, block argmax), so residency, not per-wavefront depth, sets
  // the pass time.  A round never crosses a multiple of 64 columns, so its
  // per-column values sit in one lane register.
  constexpr int NR = 16;
  static_assert(64 % NR == 0, "rounds must not straddle lane registers");
  using BT = std::integral_constant<bool, true>;
  using BF = std::integral_constant<bool, false>;

  if (st == ST_ACA) {
    // The ACA residual is FP64 for either input type (FP32 input widens
    // exactly), so the pivots, and with them the rank decisions, are those of
    // FP64 elimination on the input, as in the FP64 path.
    const int t = nd.t, na = nd.na, nc = nd.nc;
    const int32_t* cmap = nd.colmap;
    const double* f = nd.vec;
    const GPtr<double> WA = (GPtr<double>)nd.work;
    const uint32_t rowc = (uint32_t)(valid ? row : m - 1);
    const uint32_t ro8 = rowc * 8u;  // byte offset of the row in an FP64 column
    const bool in_lanes = na <= kLaneCols;
    int idr[4];
    double fr[4];
    if (in_lanes) {
      lane_load(idr, cmap, na);
      if (t > 0) lane_load(fr, f, na);
    }
    AcaBest<double> ab;
    if (t == 0) {
      // first step: the argmax of the panel itself
      auto rounds = [&](auto lanes) {
        for (int c0 = 0; c0 < na; c0 += NR) {
          T xs[NR];
#pragma unroll
          for (int u = 0; u < NR; ++u) {
            const int cc = min(c0 + u, na - 1);  // in range; extra lanes of the round are ignored
            xs[u] = col_ld<T>(P + (int64_t)cc * m, ro);
          }
          int idq = 0;
          if constexpr (decltype(lanes)::value) idq = lane_reg(idr, c0 >> 6);
#pragma unroll
          for (int u = 0; u < NR; ++u) {
            const int c = c0 + u;
            if (c < na) {
              int idu;
              if constexpr (decltype(lanes)::value) idu = lane_read(idq, c & 63);
              else idu = cmap[c];
              if (valid) ab.take((double)xs[u], idu, c);
            }
          }
        }
      };
      if (in_lanes) rounds(BT());
      else rounds(BF());
    } else {
      // R <- R - R(:, pc) f^T with row pi zeroed; the last active column moves
      // into the freed slot pc.  A later round only reads columns past the
      // earlier ones and writes those columns or pc, which was read already.
      // The residual is read from the panel (input type) at t = 1, from the
      // FP64 working matrix after that.
      const int pc = nd.pend_k;
      const int64_t pi = nd.pend_i;
      auto rounds = [&](auto src, uint32_t rs, auto lanes) {
        using E = std::remove_cv_t<std::remove_pointer_t<decltype(src)>>;
        const GPtr<const E> S = (GPtr<const E>)src;
        const double g = (double)col_ld<E>(S + (int64_t)pc * m, rs);
        for (int c0 = 0; c0 < na; c0 += NR) {
          E xs[NR];
#pragma unroll
          for (int u = 0; u < NR; ++u) {
            const int cc = min(c0 + u, na - 1);
            xs[u] = col_ld<E>(S + (int64_t)cc * m, rs);
          }
          double fq = 0.0;
          int idq = 0;
          if constexpr (decltype(lanes)::value) {
            fq = lane_reg(fr, c0 >> 6);
            idq = lane_reg(idr, c0 >> 6);
          }
#pragma unroll
          for (int u = 0; u < NR; ++u) {
            const int c = c0 + u;
            if (c < na && c != pc) {
              // more than kLaneCols columns (a leaf block wider than 256): the
              // coefficients are read here, after the previous stores (slower)
              double fcu;
              int idu;
              if constexpr (decltype(lanes)::value) {
                fcu = lane_read(fq, c & 63);
                idu = lane_read(idq, c & 63);
              } else {
                fcu = f[c];
                idu = cmap[c];
              }
              double x = fma(-g, fcu, (double)xs[u]);
              if (row == pi) x = 0.0;
              const int np = (c == na - 1) ? pc : c;
              if (valid) {
                col_st<double>(WA + (int64_t)np * m, ro8, x);
                ab.take(x, idu, np);
              }
            }
          }
        }
      };
      const T* Pg = (const T*)nd.panel;
      const double* Wg = (const double*)nd.work;
      if (t == 1) {
        if (in_lanes) rounds(Pg, ro, BT());
        else rounds(Pg, ro, BF());
      } else {
        if (in_lanes) rounds(Wg, ro8, BT());
        else rounds(Wg, ro8, BF());
      }
    }
    ab.to_cand(best, row, nc);
  } else {
    // B <- B - B(:, ks) v^T, row is set to e_ks^T.  The working matrix holds
    // B before the S = nd.lz pending swaps of the history; every element is
    // rebuilt by replaying them (g_q = the row's entry of B(:, k_q) before
    // swap q, kept per swap) and then this swap, each step the in-place
    // update's own operation, so the values equal those of updating B in
    // place.  This swap's g goes to the history; the pass that fills the
    // last slot writes B out instead.  No mask of the selected rows here: a
    // selected row is exactly e_k, the update keeps it so (its entry in
    // column ks is 0, and fma(-0, v, x) = x), and |e_k| <= 1 < 1 + tau, so
    // such a row can win a tile only when no row swap is due, where the
    // winner's identity is not used.
    const int ks = nd.pend_k;
    const int64_t is = nd.pend_i;
    const int S = nd.lz;
    const bool wout = S == kLz - 1;
    // v_q(c), q <= S: for r <= 64 one register per slot, column c in lane c
    // (read back with readlane: no staging barrier), else staged in LDS
    constexpr bool kVL = RMAX <= 64;
    __shared__ double sv[kVL ? 1 : kLz * RMAX];  // v_q(c) at q * r + c
    double vl[kLz];
    if constexpr (kVL) {
      const int lane = threadIdx.x & 63;
#pragma unroll
      for (int q = 0; q < kLz; ++q) vl[q] = (q <= S) ? nd.lzv[q * r + min(lane, r - 1)] : 0.0;
    } else {
      for (int idx = tid; idx < (S + 1) * r; idx += kThreads) sv[idx] = nd.lzv[idx];
    }
    auto vval = [&](int q, int c) -> double {
      if constexpr (kVL) return lane_read(vl[q], c);
      else return sv[q * r + c];
    };
    const GPtr<double> G = (GPtr<double>)nd.lzg;
    const GPtr<double> WB = (GPtr<double>)nd.work;
    const uint32_t ro8 = (uint32_t)(valid ? row : m - 1) * 8u;
    double gq[kLz - 1];
    int64_t iq[kLz - 1];
    int kq[kLz - 1];
#pragma unroll
    for (int q = 0; q < kLz - 1; ++q) {
      gq[q] = (q < S) ? col_ld<double>(G + (int64_t)q * m, ro8) : 0.0;
      iq[q] = nd.lzi[q];
      kq[q] = nd.lzk[q];
    }
    if constexpr (!kVL) __syncthreads();
    // the pending swaps applied to one element (row, c) of the working matrix
    auto replay = [&](double x, int c) {
#pragma unroll
      for (int q = 0; q < kLz - 1; ++q)
        if (q < S) x = (row == iq[q]) ? ((c == kq[q]) ? 1.0 : 0.0) : fma(-gq[q], vval(q, c), x);
      return x;
    };
    const double g = replay(col_ld<double>(WB + (int64_t)ks * m, ro8), ks);
    if (!wout && valid) col_st<double>(G + (int64_t)S * m, ro8, g);
    RowBest<double> rb;
    {
      // all rounds unrolled (r <= RMAX): no loop header at which the compiler
      // would wait for every outstanding load
#pragma unroll
      for (int q = 0; q < (RMAX + NR - 1) / NR; ++q) {
        const int c0 = q * NR;
        if (c0 >= r) break;
        double bs[NR];
#pragma unroll
        for (int u = 0; u < NR; ++u) {
          const int cc = min(c0 + u, r - 1);  // in range; extra lanes of the round are ignored
          bs[u] = col_ld<double>(WB + (int64_t)cc * m, ro8);
        }
#pragma unroll
        for (int u = 0; u < NR; ++u) {
          const int c = c0 + u;
          if (c < r) {
            double b = fma(-g, vval(S, c), replay(bs[u], c));
            if (row == is) b = (c == ks) ? 1.0 : 0.0;
            if (valid) {
              if (wout) col_st<double>(WB + (int64_t)c * m, ro8, b);
              rb.take(b, c);
            }
          }
        }
      }
    }
    rb.to_cand(best, row, r);
  }

  // algorithmic bytes: every working and history column read, every column
  // written (the panel in the input type, everything else FP64)
  // The in-place model counts an elimination step at t pivots as a read and a
  // write of the nc - t active columns, a row swap as a read and a write of
  // the m x r matrix B, in the input's element size.
  int64_t bytes, model;
  if (st == ST_ACA) {
    const int64_t na = nd.na, es = (nd.t <= 1) ? (int64_t)sizeof(T) : 8;
    bytes = (nd.t == 0) ? na * es : na * es + (na - 1) * 8;
    model = 2 * (int64_t)(nd.nc - nd.t) * (int64_t)sizeof(T);
  } else {
    bytes = ((int64_t)r + nd.lz + ((nd.lz == kLz - 1) ? r : 1)) * 8;
    model = 2 * (int64_t)r * (int64_t)sizeof(T);
  }
  pass_finish(nd, tile, best, sc, prof, m * bytes, m * model);
}

// Fresh B = A(:, J) X over one tile of kTileRows rows (X = A(I, J)^-1, r x r
// row-major), rows I set to unit rows, fused with the tile's argmax over the
// other rows.  Every output is the FP64 sum over k ascending of
// A(row, Jp_k) X(k, c).  X is staged in LDS CB columns at a time (broadcast
// reads): for r <= 64 all of it, so each A(row, Jp_k) is loaded once, U of
// them in flight, and each thread accumulates its whole row of B in
// registers; for larger r 16 columns at a time, A(row, Jp_k) re-read per
// chunk from L2.  Its own kernel: the product wants registers that would
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
  // global-address-space views: the A loads and B stores are global_*
  // instructions, whose completion counts apart from LDS (generic pointers
  // give flat ones, which also count as LDS operations, so each LDS read of an
  // index would wait for the previous loads of A)
  const GPtr<double> W = (GPtr<double>)nd.work;
  const GPtr<const T> P = (GPtr<const T>)nd.panel;

  constexpr int CB = RMAX <= 64 ? RMAX : 16;  // columns of X staged per chunk
  constexpr int U = RMAX <= 64 ? 16 : 8;      // loads of A(row, Jp_k) in flight
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
  RowBest<double> rb;
  // X chunk: all of a thread's entries are requested before the first is
  // stored (clamped indices, no tests: entries k >= r are never read, and
  // columns j >= nb only feed accumulators that are not stored)
  constexpr int XPER = RMAX * CB / kThreads;
  static_assert(RMAX * CB % kThreads == 0, "X staging");
  const GPtr<const double> Xg = (GPtr<const double>)nd.X;
  for (int c0 = 0; c0 < r; c0 += CB) {
    const int nb = min(CB, r - c0);
    double xv[XPER];
#pragma unroll
    for (int q = 0; q < XPER; ++q) {
      const int idx = tid + q * kThreads, k = idx / CB, j = idx % CB;
      xv[q] = Xg[(int64_t)min(k, r - 1) * r + c0 + min(j, nb - 1)];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < XPER; ++q) sX[tid + q * kThreads] = xv[q];
    __syncthreads();
    if (valid) {
      double acc[CB];
#pragma unroll
      for (int j = 0; j < CB; ++j) acc[j] = 0.0;
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
          double b = acc[j];
          if (slot >= 0) b = (c == slot) ? 1.0 : 0.0;
          W[(int64_t)c * m + row] = b;
          if (slot < 0) rb.take(b, c);
        }
      }
    }
  }
  Cand best = cand_none();
  rb.to_cand(best, row, r);
  pass_finish(nd, tile, best, sc, prof, m * (int64_t)r * ((int64_t)sizeof(T) + 8), 2 * m * (int64_t)r * (int64_t)sizeof(T));
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
