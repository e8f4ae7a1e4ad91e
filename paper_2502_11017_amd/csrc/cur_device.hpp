// Device-side building blocks shared by the selection and assembly kernels.
// All arithmetic that feeds a selection decision is written as explicit fma()
// in a fixed order, and the library is built with -ffp-contract=off, so the
// FP64 results are reproducible bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cur_internal.hpp"

namespace cur {

// ---------------------------------------------------------------- argmax candidates
// Total order of candidates: larger |x| first, then the smaller scan key.  Every
// scan of the method (ACA, row swaps, column swaps, LU pivots) is "first strictly
// larger value in ascending scan order", which is exactly this order with the
// scan position as key.
struct Cand {
  double val;   // |x| (< 0: no candidate)
  double sval;  // x
  int64_t key;
  int64_t row;
  int32_t pos;
};

__device__ __forceinline__ Cand cand_none() {
  Cand c;
  c.val = -1.0;
  c.sval = 0.0;
  c.key = INT64_MAX;
  c.row = -1;
  c.pos = -1;
  return c;
}

__device__ __forceinline__ bool cand_better(double va, int64_t ka, double vb, int64_t kb) {
  return va > vb || (va == vb && ka < kb);
}

__device__ __forceinline__ void cand_take(Cand& b, const Cand& o) {
  if (cand_better(o.val, o.key, b.val, b.key)) b = o;
}

__device__ __forceinline__ Cand cand_shfl_xor(const Cand& c, int mask) {
  Cand o;
  o.val = __shfl_xor(c.val, mask, 64);
  o.sval = __shfl_xor(c.sval, mask, 64);
  o.key = __shfl_xor(c.key, mask, 64);
  o.row = __shfl_xor(c.row, mask, 64);
  o.pos = __shfl_xor(c.pos, mask, 64);
  return o;
}

__device__ __forceinline__ Cand wave_argmax(Cand c) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) cand_take(c, cand_shfl_xor(c, s));
  return c;
}

// Block-wide argmax; every thread returns the winner.  `sc` needs
// kThreads / 64 entries of LDS.  Contains __syncthreads().
__device__ __forceinline__ Cand block_argmax(Cand c, Cand* sc) {
  c = wave_argmax(c);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sc[wid] = c;
  __syncthreads();
  Cand b = sc[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) cand_take(b, sc[w]);
  __syncthreads();
  return b;
}

// Make the block's global-memory stores visible to every thread of the block.
// A workgroup barrier orders LDS but not the global stores of other
// wavefronts, so each thread first completes and publishes its own stores
// (agent-scope fence: waits for them and drops stale vector-L1 lines), then
// the block synchronizes.  Used only where one wavefront reads global data
// that another wavefront of the same block wrote in the same launch.
__device__ __forceinline__ void block_global_sync() {
  __threadfence();
  __syncthreads();
}

// ---------------------------------------------------------------- small dense kernels
// LU with partial pivoting of the r x r row-major G held in LDS, in place and
// without moving rows: rowmap[p] is the LDS row that holds position p (rows
// stay where they were loaded, so rowmap[p] is also the original row of
// position p).  The arithmetic is exactly that of swapping rows: pivot of
// column k = largest |G(p,k)| over positions p >= k, ties to the smallest p;
// multiplier l = G(p,k) / G(k,k) stored in place; G(p,c) = fma(-l, G(k,c), G(p,c)).
// Every LDS location is written in a phase in which no other thread reads it
// (phases separated by block barriers).  lk: r doubles of LDS; spiv: one int.
// Returns false (uniformly) if G is singular.
__device__ bool block_gepp(double* G, int r, int* rowmap, double* lk, int* spiv) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nt = blockDim.x;
  for (int i = tid; i < r; i += nt) rowmap[i] = i;
  __syncthreads();
  for (int k = 0; k < r; ++k) {
    // phase A: pivot search (wavefront 0); the winner is published after the
    // cross-lane reduction, which every lane's load feeds.
    if (wave == 0) {
      double best = -1.0;
      int arg = r;
      for (int p = k + lane; p < r; p += 64) {
        const double v = fabs(G[rowmap[p] * r + k]);
        if (v > best) { best = v; arg = p; }
      }
#pragma unroll
      for (int s = 32; s >= 1; s >>= 1) {
        const double ob = __shfl_xor(best, s, 64);
        const int oa = __shfl_xor(arg, s, 64);
        if (ob > best || (ob == best && oa < arg)) { best = ob; arg = oa; }
      }
      if (lane == 0) {
        if (best == 0.0) {
          *spiv = -1;
        } else {
          *spiv = arg;
          const int t = rowmap[k];
          rowmap[k] = rowmap[arg];
          rowmap[arg] = t;
        }
      }
    }
    __syncthreads();
    if (*spiv < 0) return false;
    const int pr = rowmap[k];
    const double d = G[pr * r + k];
    // phase B: multipliers of the rows below the pivot position
    for (int p = k + 1 + tid; p < r; p += nt) lk[p] = G[rowmap[p] * r + k] / d;
    __syncthreads();
    // phase C: trailing update; column k receives the multipliers
    const int cols = r - k, rows = r - k - 1;
    for (int idx = tid; idx < rows * cols; idx += nt) {
      const int p = k + 1 + idx / cols, c = k + idx % cols;
      const int ph = rowmap[p];
      if (c == k)
        G[ph * r + k] = lk[p];
      else
        G[ph * r + c] = fma(-lk[p], G[pr * r + c], G[ph * r + c]);
    }
    __syncthreads();
  }
  return true;
}

// X = G^{-1} (row-major r x r, written to Xg: global or LDS) from the factors
// of block_gepp, column chunk by column chunk in the LDS buffer Y (r x ch):
// forward substitution L y = P e_j with the sum over k ascending, then back
// substitution U x = y with the sum over k descending and x_k = s / U(k,k).
// Each element receives its updates in exactly that order.
__device__ void block_lu_inverse(const double* LU, const int* rowmap, int r, double* Y, int ch,
                                 double* Xg) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int j0 = 0; j0 < r; j0 += ch) {
    const int nch = min(ch, r - j0);
    for (int idx = tid; idx < r * nch; idx += nt) {
      const int i = idx / nch, jj = idx % nch;
      Y[i * ch + jj] = (rowmap[i] == j0 + jj) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < r - 1; ++k) {
      const int rows = r - k - 1;
      for (int idx = tid; idx < rows * nch; idx += nt) {
        const int i = k + 1 + idx / nch, jj = idx % nch;
        Y[i * ch + jj] = fma(-LU[rowmap[i] * r + k], Y[k * ch + jj], Y[i * ch + jj]);
      }
      __syncthreads();
    }
    for (int k = r - 1; k >= 0; --k) {
      const double ukk = LU[rowmap[k] * r + k];
      // x_k is final once every U(k, k') (k' > k) term has been applied.
      for (int idx = tid; idx < (k + 1) * nch; idx += nt) {
        const int i = idx / nch, jj = idx % nch;
        const double xk = Y[k * ch + jj] / ukk;
        if (i == k)
          Xg[(int64_t)k * r + j0 + jj] = xk;
        else
          Y[i * ch + jj] = fma(-LU[rowmap[i] * r + k], xk, Y[i * ch + jj]);
      }
      __syncthreads();
    }
  }
}

// The same inverse with one thread per column j and the column held in
// registers (r <= RMAX <= 64): forward substitution y_i = [rowmap[i] == j] -
// sum_{k<i} L(i,k) y_k (k ascending), then back substitution
// x_i = (y_i - sum_{k>i} U(i,k) x_k) / U(i,i) with k descending from r-1 --
// the per-element operation order of block_lu_inverse, without barriers.
// LUp: LDS scratch of RMAX*RMAX doubles (position-ordered copy of the factors).
template <int RMAX>
__device__ void block_lu_inverse_reg(const double* LU, const int* rowmap, int r, double* LUp,
                                     double* Xg, double* Xl = nullptr) {
  const int tid = threadIdx.x;
  for (int idx = tid; idx < r * r; idx += blockDim.x) {
    const int i = idx / r, k = idx % r;
    LUp[i * RMAX + k] = LU[rowmap[i] * r + k];
  }
  __syncthreads();
  const int j = tid;
  if (j < r) {
    double y[RMAX];
#pragma unroll
    for (int i = 0; i < RMAX; ++i) {
      if (i < r) {
        double s = (rowmap[i] == j) ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < i; ++k) s = fma(-LUp[i * RMAX + k], y[k], s);
        y[i] = s;
      }
    }
#pragma unroll
    for (int i = RMAX - 1; i >= 0; --i) {
      if (i < r) {
        double s = y[i];
#pragma unroll
        for (int k = RMAX - 1; k > i; --k)
          if (k < r) s = fma(-LUp[i * RMAX + k], y[k], s);
        y[i] = s / LUp[i * RMAX + i];
      }
    }
#pragma unroll
    for (int i = 0; i < RMAX; ++i)
      if (i < r) {
        Xg[(int64_t)i * r + j] = y[i];
        if (Xl) Xl[i * r + j] = y[i];
      }
  }
  __syncthreads();
}

// |det| = prod |U(k,k)| as mant * 2^expo, mant in [0.5,1): frexp split of each
// factor, one rounded product per step, exact renormalisation.  Thread 0 only.
__device__ void lu_volume(const double* LU, const int* rowmap, int r, double* mant, int* expo) {
  double mt = 1.0;
  int e = 0;
  for (int k = 0; k < r; ++k) {
    int eu, em;
    double u = frexp(fabs(LU[rowmap[k] * r + k]), &eu);
    mt = frexp(mt * u, &em);
    e += eu + em;
  }
  *mant = mt;
  *expo = e;
}

// Ascending sort of n <= blockDim.x distinct values by rank counting; the
// values are read from and written back to `v` (global or LDS); `tmp` is an
// LDS scratch of n entries.
template <typename V>
__device__ void block_sort(V* v, int n, V* tmp) {
  const int tid = threadIdx.x;
  V mine = 0;
  int rank = 0;
  if (tid < n) {
    mine = v[tid];
    for (int j = 0; j < n; ++j) {
      V o = v[j];
      rank += (o < mine) || (o == mine && j < tid);
    }
  }
  __syncthreads();
  if (tid < n) tmp[rank] = mine;
  __syncthreads();
  if (tid < n) v[tid] = tmp[tid];
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c);
template <>
__device__ __forceinline__ double fma_t<double>(double a, double b, double c) { return fma(a, b, c); }
template <>
__device__ __forceinline__ float fma_t<float>(float a, float b, float c) { return fmaf(a, b, c); }

}  // namespace cur
