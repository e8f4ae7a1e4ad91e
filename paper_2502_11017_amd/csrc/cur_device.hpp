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

// ---------------------------------------------------------------- small dense kernels
// LU with partial pivoting of the r x r row-major G held in LDS, in place.
// Pivot of column k: largest |G(a,k)| over a >= k, ties to the smallest a.
// perm[k] receives the original row now at position k.  lk: r doubles of LDS;
// spiv: one int of LDS.  Returns false (uniformly) if G is singular.
__device__ bool block_gepp(double* G, int r, int* perm, double* lk, int* spiv) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < r; i += nt) perm[i] = i;
  __syncthreads();
  for (int k = 0; k < r; ++k) {
    if (tid < 64) {
      double best = -1.0;
      int arg = r;
      for (int a = k + tid; a < r; a += 64) {
        double v = fabs(G[a * r + k]);
        if (v > best) { best = v; arg = a; }
      }
#pragma unroll
      for (int s = 32; s >= 1; s >>= 1) {
        double ob = __shfl_xor(best, s, 64);
        int oa = __shfl_xor(arg, s, 64);
        if (ob > best || (ob == best && oa < arg)) { best = ob; arg = oa; }
      }
      if (tid == 0) *spiv = (best == 0.0) ? -1 : arg;
    }
    __syncthreads();
    const int piv = *spiv;
    if (piv < 0) return false;
    if (piv != k) {
      for (int c = tid; c < r; c += nt) {
        double t = G[k * r + c];
        G[k * r + c] = G[piv * r + c];
        G[piv * r + c] = t;
      }
      if (tid == 0) {
        int t = perm[k];
        perm[k] = perm[piv];
        perm[piv] = t;
      }
    }
    __syncthreads();
    const double d = G[k * r + k];
    for (int a = k + 1 + tid; a < r; a += nt) lk[a] = G[a * r + k] / d;
    __syncthreads();
    const int cols = r - k, rows = r - k - 1;
    for (int idx = tid; idx < rows * cols; idx += nt) {
      const int a = k + 1 + idx / cols, c = k + idx % cols;
      if (c == k)
        G[a * r + k] = lk[a];
      else
        G[a * r + c] = fma(-lk[a], G[k * r + c], G[a * r + c]);
    }
    __syncthreads();
  }
  return true;
}

// X = G^{-1} (row-major r x r, written to global Xg) from the factors of
// block_gepp, column chunk by column chunk in the LDS buffer Y (r x ch):
// forward substitution L y = P e_j with the sum over k ascending, then back
// substitution U x = y with the sum over k descending and x_k = s / U(k,k).
// Each element receives its updates in exactly that order.
__device__ void block_lu_inverse(const double* LU, const int* perm, int r, double* Y, int ch,
                                 double* Xg) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int j0 = 0; j0 < r; j0 += ch) {
    const int nch = min(ch, r - j0);
    for (int idx = tid; idx < r * nch; idx += nt) {
      const int i = idx / nch, jj = idx % nch;
      Y[i * ch + jj] = (perm[i] == j0 + jj) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < r - 1; ++k) {
      const int rows = r - k - 1;
      for (int idx = tid; idx < rows * nch; idx += nt) {
        const int i = k + 1 + idx / nch, jj = idx % nch;
        Y[i * ch + jj] = fma(-LU[i * r + k], Y[k * ch + jj], Y[i * ch + jj]);
      }
      __syncthreads();
    }
    for (int k = r - 1; k >= 0; --k) {
      const double ukk = LU[k * r + k];
      // x_k is final once every U(k, k') (k' > k) term has been applied.
      for (int idx = tid; idx < (k + 1) * nch; idx += nt) {
        const int i = idx / nch, jj = idx % nch;
        const double xk = Y[k * ch + jj] / ukk;
        if (i == k)
          Xg[(int64_t)k * r + j0 + jj] = xk;
        else
          Y[i * ch + jj] = fma(-LU[i * r + k], xk, Y[i * ch + jj]);
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
