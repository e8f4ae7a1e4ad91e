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

// Global-address-space view of a device pointer: loads and stores through it
// become global_* instructions, whose completion counts apart from LDS and
// scalar loads, so a wait for one does not drain the other (a generic pointer
// gives flat instructions, which count as both).
template <typename T>
using GPtr = __attribute__((address_space(1))) T*;

// Maximum that keeps a NaN: once either operand is NaN the result is NaN
// (fmax would drop it), so a non-finite residual entry reaches the caller.
__device__ __forceinline__ double nan_max(double a, double b) { return (b > a || b != b) ? b : a; }

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

// ---------------------------------------------------------------- register LU (r <= 64)
// LU with partial pivoting and G^{-1} for r <= RMAX <= 64, held in registers:
// lane p owns row p of G (physical order, never moved).  Columns come in
// blocks of 8 dealt round-robin to the 4 wavefronts: column c is in
// wavefront (c / 8) & 3 at local index lu_j(c).  Row exchanges are tracked as
// positions instead of data moves.  Every value that reaches U, X or the
// volume is computed with the operands and in the order of block_gepp
// followed by block_lu_inverse, so the results are identical bit for bit:
//   * the pivot of step k is the largest |G(p,k)| over unpivoted rows, ties to
//     the smallest position; multipliers l_p = G(p,k) / d;
//   * G(p,c) = fma(-l_p, G(P,c), G(p,c)) on unpivoted rows p, steps in
//     ascending order for every element;
//   * the forward substitution L y = P e_c rides along as an augmented right
//     side Y (starting from the identity in physical order), updated with the
//     same multipliers: row p receives fma(-L(i,k), y_k, .) for k ascending;
//   * the back substitution runs per wavefront over its own columns of Y,
//     positions descending, x_k = s / U(k,k).
// With Y carried along, the multipliers are dead once their step is done (the
// back substitution reads U only), so a step updates every column of the
// unpivoted rows without testing c > k: the L part is left as scratch.  In Y,
// row P is exactly +0 in every column c whose row c is not yet pivoted, and an
// fma with a +0 product leaves a target that is never -0 unchanged.
// Blocked schedule: the wavefront owning the 8 columns of panel b factors
// them alone (pivot search, multipliers, updates inside the panel; the pivot
// row's values come from its own lanes by readlane) and publishes the 8
// steps' multipliers and pivots through LDS; after one block barrier every
// wavefront replays those steps on its other columns.  Each element still
// receives its updates one step at a time in ascending order, so the
// arithmetic is that of the unblocked elimination; a barrier is paid per 8
// steps instead of per step.
struct LuScratch {
  double pl[3][8][64];  // multipliers of a panel's steps (three panels in flight)
  int pinfo[3][8];      // per step: pivot row | position << 8 | singular << 16
  double diag[64];      // U(k,k) in step order
  int perm[64];         // physical row at position k
  double xb[4][16];     // per-wavefront staging of one row of X
};
template <int RMAX>
struct LuRegs {
  static_assert(RMAX == 32 || RMAX == 64, "register LU covers r <= 64");
  static constexpr int NJ = RMAX / 4;
  double g[NJ];  // G / LU, this wavefront's columns of row `lane`
  double y[NJ];  // augmented right side, same columns
  int pos;       // position of this lane's row
};

// Column of local index j in wavefront w (8-column blocks dealt round-robin).
__device__ __forceinline__ int lu_col(int w, int j) { return ((((j >> 3) << 2) + w) << 3) + (j & 7); }

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, 0xF, 0xF, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, true);
  return ((uint64_t)hi << 32) | lo;
}

// Largest 64-bit unsigned value over the wavefront, returned uniformly: DPP
// exchanges inside each 16-lane row (quad xor 1, quad xor 2, half-row mirror,
// row mirror), then the four row results are combined.
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  v = max(v, dpp_u64<0xB1>(v));
  v = max(v, dpp_u64<0x4E>(v));
  v = max(v, dpp_u64<0x141>(v));
  v = max(v, dpp_u64<0x140>(v));
  return max(max(readlane_u64(v, 0), readlane_u64(v, 16)), max(readlane_u64(v, 32), readlane_u64(v, 48)));
}

// Largest 32-bit unsigned value over the wavefront, returned uniformly (same
// exchanges as wave_max_u64 on one word).
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, true));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, true));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, true));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, true));
  const uint32_t a = max((uint32_t)__builtin_amdgcn_readlane((int)v, 0), (uint32_t)__builtin_amdgcn_readlane((int)v, 16));
  const uint32_t b = max((uint32_t)__builtin_amdgcn_readlane((int)v, 32), (uint32_t)__builtin_amdgcn_readlane((int)v, 48));
  return max(a, b);
}

// The same maximum for 64-bit values as two 32-bit passes: the high words,
// then the low words of the lanes whose high word is the maximum.
__device__ __forceinline__ uint64_t wave_max_u64_split(uint64_t v) {
  const uint32_t hi = (uint32_t)(v >> 32);
  const uint32_t mh = wave_max_u32(hi);
  const uint32_t ml = wave_max_u32(hi == mh ? (uint32_t)v : 0u);
  return ((uint64_t)mh << 32) | ml;
}

// Order the LDS accesses of one wavefront's lanes around a hand-off.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// a[j] for a wavefront-uniform j < NJ (a power of two): a tree of selects on
// the bits of j, which keeps the array in registers.
template <int NJ>
__device__ __forceinline__ double reg_pick(const double (&a)[NJ], int j) {
  double t[NJ];
#pragma unroll
  for (int q = 0; q < NJ; ++q) t[q] = a[q];
#pragma unroll
  for (int h = NJ / 2, b = 0; h >= 1; h >>= 1, ++b) {
    const bool hi = (j >> b) & 1;
#pragma unroll
    for (int q = 0; q < h; ++q) t[q] = hi ? t[2 * q + 1] : t[2 * q];
  }
  return t[0];
}

// Factorization and forward substitution.  ldg(p, c) returns G(p, c) (called
// with p, c < r only; a loader through global-address-space pointers keeps
// the loads apart from the LDS wait counts).  U is
// left in R.g and, column-major (element (p, c) at c * RMAX + p, physical
// rows; entries left of a row's pivot are scratch), in LUl; S.diag / S.perm
// hold U(k,k) and the row order.  Returns false (uniformly) on a zero pivot.
// Ends with a block barrier.
template <int RMAX, class LoadG>
__device__ __forceinline__ bool lu_fwd_reg(LoadG ldg, int r, LuRegs<RMAX>& R, double* LUl, LuScratch& S) {
  constexpr int NJ = LuRegs<RMAX>::NJ;
  constexpr int NB = NJ / 8;  // column blocks per wavefront
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool live = lane < r;
  // G's entries: every load is issued unconditionally from a valid address
  // (row and column clamped into range), lanes past r are zeroed by a mask
  // the optimiser cannot turn back into a branch (a lane-divergent tested
  // load compiles to a branch with a wait for its data), columns past r by
  // a wavefront-uniform select.
  uint32_t lmask = live ? 0xffffffffu : 0u;
  asm("" : "+v"(lmask));
  const uint64_t lm64 = ((uint64_t)lmask << 32) | lmask;
  const int pl = min(lane, r - 1);
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int c = lu_col(w, j);
    const double x = ldg(pl, min(c, r - 1));
    const double xm = __longlong_as_double((long long)((uint64_t)__double_as_longlong(x) & lm64));
    R.g[j] = c < r ? xm : 0.0;
    R.y[j] = (lane == c) ? 1.0 : 0.0;
  }
  R.pos = lane;
  bool done = !live;
  const int npanels = (r + 7) >> 3;
  // One step of a published panel on column set `cols` of this wavefront:
  // 0 all G columns except local block `skip`, plus Y; 1 only local block
  // `only` of G.  The published multiplier is 0 for the pivot row and the rows
  // pivoted before, and fma(-0, u, g) is g (up to the sign of a zero g, which
  // no comparison, pivot or result value sees), so no select is needed.
  auto replay = [&](int pb, int which, int blk) {
    const int pbuf = pb % 3;
    const int pns = min(8, r - (pb << 3));
#pragma unroll
    for (int st = 0; st < 8; ++st) {
      if (st >= pns) break;
      const int P = __builtin_amdgcn_readfirstlane(S.pinfo[pbuf][st]) & 0xff;
      const double l = S.pl[pbuf][st][lane];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        if (which == 0 && (j >> 3) == blk) continue;
        if (which == 1 && (j >> 3) != blk) continue;
        R.g[j] = fma(-l, readlane_f64(R.g[j], P), R.g[j]);
      }
      if (which == 0) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) R.y[j] = fma(-l, readlane_f64(R.y[j], P), R.y[j]);
      }
    }
  };
  // Schedule per panel b (owner b & 3):
  //   owner:       factors b (its block lb = b >> 2 is up to date), publishes;
  //   barrier;
  //   every wave:  takes the position bookkeeping of b's steps (the owner did);
  //   next owner:  replays b on its block of panel b + 1 only (the critical
  //                path), and owes b on everything else;
  //   the others:  pay what they owe (the previous panel, on all but the block
  //                they factored), then replay b on all their columns (the
  //                owner: all but its panel).
  // Every element still receives the steps in ascending order.
  int owe = -1, owe_skip = -1;
  for (int b = 0; b < npanels; ++b) {
    const int buf = b % 3;
    const int k0 = b << 3;
    const int ns = min(8, r - k0);
    const int owner = b & 3, lbo = b >> 2;  // owning wavefront, its local block
    if (w == owner) {
#pragma unroll
      for (int lb = 0; lb < NB; ++lb) {
        if (lb != lbo) continue;
        int pinf[8];
        double dg[8];
#pragma unroll
        for (int st = 0; st < 8; ++st) {
          pinf[st] = 1 << 16;
          dg[st] = 0.0;
        }
#pragma unroll
        for (int st = 0; st < 8; ++st) {
          if (st >= ns) break;
          const int k = k0 + st;
          const double v = R.g[lb * 8 + st];
          // pivot: largest |v| over unpivoted rows (bit pattern of |v| orders
          // like the value; NaN is no candidate), ties to the smallest position
          const uint64_t key = (!done && v == v) ? (uint64_t)__double_as_longlong(fabs(v)) : 0ull;
          const uint64_t best = wave_max_u64_split(key);
          uint64_t tied = __ballot(key == best);
          int P = (int)__builtin_ctzll(tied);
          if (tied & (tied - 1)) {
            int bp = 0x7fffffff;
            while (tied) {
              const int q = (int)__builtin_ctzll(tied);
              const int pq = __builtin_amdgcn_readlane(R.pos, q);
              if (pq < bp) {
                bp = pq;
                P = q;
              }
              tied &= tied - 1;
            }
          }
          P = __builtin_amdgcn_readfirstlane(P);
          const int pp = __builtin_amdgcn_readlane(R.pos, P);
          const double d = readlane_f64(v, P);
          const bool bad = best == 0ull;
          const bool upd = !done && lane != P && !bad;
          const double l = upd ? v / d : 0.0;
          S.pl[buf][st][lane] = l;
          pinf[st] = P | (pp << 8) | ((bad ? 1 : 0) << 16);
          dg[st] = d;
          if (bad) break;
          // the rest of the panel (columns k+1 .. of this block)
#pragma unroll
          for (int t = st + 1; t < 8; ++t) R.g[lb * 8 + t] = fma(-l, readlane_f64(R.g[lb * 8 + t], P), R.g[lb * 8 + t]);
          if (lane == P) {
            done = true;
            R.pos = k;
          } else if (!done && R.pos == k) {
            R.pos = pp;
          }
        }
        if (lane == 0) {
#pragma unroll
          for (int st = 0; st < 8; ++st) {
            if (st >= ns) break;
            S.pinfo[buf][st] = pinf[st];
            S.diag[k0 + st] = dg[st];
            S.perm[k0 + st] = pinf[st] & 0xff;
          }
        }
      }
    }
    __syncthreads();
    const bool mine = w == owner;
#pragma unroll
    for (int st = 0; st < 8; ++st) {
      if (st >= ns) break;
      const int info = __builtin_amdgcn_readfirstlane(S.pinfo[buf][st]);
      if (info >> 16) return false;
      if (!mine) {  // the owner's lanes already took this step's bookkeeping
        const int P = info & 0xff, pp = (info >> 8) & 0xff;
        if (lane == P) {
          done = true;
          R.pos = k0 + st;
        } else if (!done && R.pos == k0 + st) {
          R.pos = pp;
        }
      }
    }
    const bool next_owner = b + 1 < npanels && w == ((b + 1) & 3);
    if (next_owner) {
      replay(b, 1, (b + 1) >> 2);
      owe = b;
      owe_skip = (b + 1) >> 2;
    } else {
      if (owe >= 0) {
        replay(owe, 0, owe_skip);
        owe = -1;
      }
      replay(b, 0, mine ? lbo : -1);
    }
  }
  if (live) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int c = lu_col(w, j);
      if (c < r) LUl[c * RMAX + lane] = R.g[j];
    }
  }
  __syncthreads();
  return true;
}

// Back substitution after lu_fwd_reg: X = G^{-1}, written row-major r x r to
// Xg and column-major (element (k, c) at c * RMAX + k) to Xl; either may be
// null.  Each wavefront works on its own columns
// without block barriers; the row being divided is staged through S.xb.
// Ends with a block barrier.
template <int RMAX>
__device__ __forceinline__ void lu_back_reg(int r, LuRegs<RMAX>& R, const double* LUl, LuScratch& S, double* Xg,
                                            double* Xl) {
  constexpr int NJ = LuRegs<RMAX>::NJ;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int permv = lane < r ? S.perm[lane] : 0;
  const double diagv = lane < r ? S.diag[lane] : 1.0;
  double* xb = S.xb[w];
  const int cl = lu_col(w, lane);  // the column this lane divides (lanes < NJ)
  double u = lane < r ? LUl[(r - 1) * RMAX + lane] : 0.0;  // U(pos, k) of this lane's row
  for (int k = r - 1; k >= 0; --k) {
    const int Pk = __builtin_amdgcn_readlane(permv, k);
    const double dk = readlane_f64(diagv, k);
    const double un = (k > 0 && lane < r) ? LUl[(k - 1) * RMAX + lane] : 0.0;
    if (lane == Pk) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) xb[j] = R.y[j];
    }
    wave_lds_sync();
    if (lane < NJ) {
      const double x = xb[lane] / dk;
      xb[lane] = x;
      if (cl < r) {
        if (Xg) Xg[(int64_t)k * r + cl] = x;
        if (Xl) Xl[cl * RMAX + k] = x;
      }
    }
    wave_lds_sync();
    double xk[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) xk[j] = xb[j];
    if (R.pos < k) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) R.y[j] = fma(-u, xk[j], R.y[j]);
    }
    wave_lds_sync();
    u = un;
  }
  __syncthreads();
}

// |det| = prod |U(k,k)| as mant * 2^expo, mant in [0.5,1): frexp split of each
// factor, one rounded product per step, exact renormalisation.  U(k,k) is
// diag[k * stride].  Thread 0 only.
__device__ void lu_volume(const double* diag, int stride, int r, double* mant, int* expo) {
  double mt = 1.0;
  int e = 0;
  for (int k = 0; k < r; ++k) {
    int eu, em;
    double u = frexp(fabs(diag[k * stride]), &eu);
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
