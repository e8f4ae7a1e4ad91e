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
// LU with partial pivoting of the r x r row-major G held in LDS, in place,
// rows physically swapped as in the textbook algorithm: pivot of column k =
// largest |G(p,k)| over p >= k, ties to the smallest p; multiplier
// l = G(p,k) / G(k,k) stored in place; G(p,c) = fma(-l, G(k,c), G(p,c)).
// perm[k] receives the original row now at position k.  Three phases per
// step, separated by block barriers, so that no LDS location is written while
// another thread reads it:
//   A  wavefront 0 finds the pivot;
//   B  rows k and piv exchange every column except k, and the multipliers are
//      formed from the unswapped column k (the swapped row p reads row piv);
//   C  trailing update of rows p > k, column k receives the multipliers and
//      the pivot.
// Threads map to (column = lane-group, row = wave + 4*i): no divisions.
// lk: r doubles of LDS; spiv: one int.  Returns false (uniformly) if singular.
__device__ bool block_gepp(double* G, int r, int* perm, double* lk, int* spiv) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  for (int i = tid; i < r; i += blockDim.x) perm[i] = i;
  __syncthreads();
  for (int k = 0; k < r; ++k) {
    if (wave == 0) {
      double best = -1.0;
      int arg = r;
      for (int p = k + lane; p < r; p += 64) {
        const double v = fabs(G[p * r + k]);
        if (v > best) { best = v; arg = p; }
      }
#pragma unroll
      for (int s = 32; s >= 1; s >>= 1) {
        const double ob = __shfl_xor(best, s, 64);
        const int oa = __shfl_xor(arg, s, 64);
        if (ob > best || (ob == best && oa < arg)) { best = ob; arg = oa; }
      }
      if (lane == 0) *spiv = (best > 0.0) ? arg : -1;  // zero or non-finite column: singular
    }
    __syncthreads();
    const int piv = *spiv;
    if (piv < 0) return false;
    const double d = G[piv * r + k];  // the pivot (row piv, before the exchange)
    // phase B
    if (piv != k)
      for (int c = tid; c < r; c += blockDim.x)
        if (c != k) {
          const double t = G[k * r + c];
          G[k * r + c] = G[piv * r + c];
          G[piv * r + c] = t;
        }
    for (int p = k + 1 + tid; p < r; p += blockDim.x) {
      const int src = (p == piv) ? k : p;  // after the exchange row p holds old row src
      lk[p] = G[src * r + k] / d;
    }
    if (tid == 0 && piv != k) {
      const int t = perm[k];
      perm[k] = perm[piv];
      perm[piv] = t;
    }
    __syncthreads();
    // phase C
    for (int c = k + lane; c < r; c += 64) {
      if (c == k) {
        if (wave == 0) G[k * r + k] = d;
        for (int p = k + 1 + wave; p < r; p += nw) G[p * r + k] = lk[p];
      } else {
        const double gk = G[k * r + c];
        for (int p = k + 1 + wave; p < r; p += nw) G[p * r + c] = fma(-lk[p], gk, G[p * r + c]);
      }
    }
    __syncthreads();
  }
  return true;
}

// X = G^{-1} (row-major r x r, written to Xg: global or LDS) from the factors
// of block_gepp, CH columns at a time in the LDS buffer Y (r x CH): forward
// substitution L y = P e_j with the sum over k ascending, then back
// substitution U x = y with the sum over k descending and x_k = s / U(k,k).
// Each element receives its updates in exactly that order.  Thread t owns
// column t % CH of the chunk and the rows congruent to t / CH; one barrier per
// elimination step.  CH is a power of two dividing the block size.
template <int CH>
__device__ void block_lu_inverse(const double* LU, const int* perm, int r, double* Y, double* Xg) {
  static_assert((CH & (CH - 1)) == 0 && kThreads % CH == 0, "chunk width");
  const int tid = threadIdx.x, jj = tid & (CH - 1), g = tid / CH;
  constexpr int NG = kThreads / CH;
  for (int j0 = 0; j0 < r; j0 += CH) {
    const bool act = j0 + jj < r;
    if (act)
      for (int i = g; i < r; i += NG) Y[i * CH + jj] = (perm[i] == j0 + jj) ? 1.0 : 0.0;
    __syncthreads();
    for (int k = 0; k < r - 1; ++k) {
      if (act) {
        const double yk = Y[k * CH + jj];
        for (int i = k + 1 + g; i < r; i += NG) Y[i * CH + jj] = fma(-LU[i * r + k], yk, Y[i * CH + jj]);
      }
      __syncthreads();
    }
    for (int k = r - 1; k >= 0; --k) {
      // x_k is final once every U(k, k') (k' > k) term has been applied.
      if (act) {
        const double xk = Y[k * CH + jj] / LU[k * r + k];
        if (g == 0) Xg[(int64_t)k * r + j0 + jj] = xk;
        for (int i = g; i < k; i += NG) Y[i * CH + jj] = fma(-LU[i * r + k], xk, Y[i * CH + jj]);
      }
      __syncthreads();
    }
  }
}

// |det| = prod |U(k,k)| as mant * 2^expo, mant in [0.5,1): frexp split of each
// factor, one rounded product per step, exact renormalisation.  Thread 0 only.
__device__ void lu_volume(const double* LU, int r, double* mant, int* expo) {
  double mt = 1.0;
  int e = 0;
  for (int k = 0; k < r; ++k) {
    int eu, em;
    double u = frexp(fabs(LU[k * r + k]), &eu);
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
