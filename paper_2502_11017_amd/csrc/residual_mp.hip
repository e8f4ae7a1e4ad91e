// Reduced-precision residual of the CUR form for FP32 input: E = A - P with
// P = Bm R and Bm = C U, both products on MFMA with FP32 accumulation, the
// difference, maximum and sums in FP64.
//
//   BF16x3: x = hi + lo with hi = bf16(x), lo = bf16(x - hi); a product is
//           hi_a hi_b + hi_a lo_b + lo_a hi_b (the lo_a lo_b term, ~2^-16
//           relative, is dropped), v_mfma_f32_16x16x32_bf16.  U is split the
//           same way (its lo part keeps the product compensated to ~2^-16).
//   FP8:    OCP e4m3 with one scale per operand tile of 16 strips (rows of C
//           or Bm, columns of U or R) over all k, s = max|tile| / 448; two
//           terms q1 = e4m3(x/s), q2 = e4m3(16 (x/s - q1)); a product is
//           q1 q1 + (q1 q2 + q2 q1) / 16, v_mfma_f32_16x16x32_fp8_fp8.
//
// Steps: the column operands (U and R) are split by k_split_cols; k_cu_lowp
// forms Bm = C U from C's rows (split as they are staged) and writes Bm
// directly in the split form the tile kernel reads; k_resid_mp forms P tile by
// tile and reduces E.  Bm never exists in FP64 or FP32 in memory.
//
// Operand layouts (r padded to rp, a multiple of 32, with zeros): a row
// operand is row-major strips x rp (C, Bm), a column operand is stored
// transposed, strips x rp (U, R), so that a lane's eight consecutive k values
// are one 16-byte (bf16) or 8-byte (fp8) load.  MFMA lanes: lane l supplies
// X[l & 15][8 (l >> 4) + e] of the first operand and Y[8 (l >> 4) + e][l & 15]
// of the second, e < 8, and holds D[4 (l >> 4) + v][l & 15].  Both kernels
// compute the transposed product (first operand: the column strips), so a
// lane's four results are four consecutive columns of one row: Bm is written
// and A is read four elements at a time.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>
#include <utility>

#include "cur_device.hpp"
#include "cur_internal.hpp"

namespace cur {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// Plain vector types for the 16-byte staging copies (a HIP uint4/float4 is a
// struct, whose copies go through memory and put the stage in scratch).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kMT = 128;  // tile of E per block (rows and columns)
constexpr int kMK = 32;   // k values per staged chunk
constexpr int kST = 16;   // strips per FP8 scale tile
// The two product kernels run 8 wavefronts per block, each on 64 rows x 32
// columns (4 x 2 blocks of 16 x 16): ~128 VGPRs, so two blocks (four
// wavefronts per SIMD) fit a CU and hide each other's memory latency.
constexpr int kMpThreads = 512;
constexpr int kNA = 2;  // 16-column blocks per wavefront (first operand)
constexpr int kNB = 4;  // 16-row blocks per wavefront (second operand)

__device__ __forceinline__ uint8_t to_e4m3(float x) {
  return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false) & 0xff);
}
__device__ __forceinline__ float from_e4m3(uint8_t q) { return __builtin_amdgcn_cvt_f32_fp8((int)q, 0); }
__device__ __forceinline__ float fp8_scale(float amax) { return amax > 0.0f ? amax / 448.0f : 1.0f; }

// ---------------------------------------------------------------- column operands
// X (r x n, leading dimension ldx, element V) -> transposed hi/lo bf16, n x rp.
template <typename V>
__global__ __launch_bounds__(kThreads) void k_split_cols_bf16(const V* __restrict__ X, int r, int64_t n, int64_t ldx,
                                                              int rp, __bf16* __restrict__ h, __bf16* __restrict__ l) {
  const int64_t total = n * rp;
  for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * kThreads) {
    const int64_t j = idx / rp;
    const int k = (int)(idx - j * rp);
    const double x = k < r ? (double)X[(int64_t)k * ldx + j] : 0.0;
    const __bf16 hi = (__bf16)(float)x;
    h[idx] = hi;
    l[idx] = (__bf16)(float)(x - (double)(float)hi);
  }
}

// X (r x n, ld ldx) -> transposed two-term e4m3, n x rp, one scale per tile of
// kST columns (all k).  One wavefront per tile.
template <typename V>
__global__ __launch_bounds__(kThreads) void k_split_cols_fp8(const V* __restrict__ X, int r, int64_t n, int64_t ldx,
                                                             int rp, uint8_t* __restrict__ q1, uint8_t* __restrict__ q2,
                                                             float* __restrict__ s) {
  const int lane = threadIdx.x & 63;
  const int64_t tiles = (n + kST - 1) / kST;
  const int64_t waves = (int64_t)gridDim.x * (kThreads / 64);
  for (int64_t t = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); t < tiles; t += waves) {
    const int64_t j0 = t * kST;
    const int cnt = kST * rp;  // (column, k) pairs of the tile, column-major in k
    float amax = 0.0f;
    for (int idx = lane; idx < cnt; idx += 64) {
      const int64_t j = j0 + idx / rp;
      const int k = idx % rp;
      if (j < n && k < r) amax = fmaxf(amax, fabsf((float)X[(int64_t)k * ldx + j]));
    }
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) amax = fmaxf(amax, __shfl_xor(amax, sh, 64));
    const float sc = fp8_scale(amax);
    const double inv = 1.0 / (double)sc;
    for (int idx = lane; idx < cnt; idx += 64) {
      const int64_t j = j0 + idx / rp;
      const int k = idx % rp;
      if (j >= n) continue;
      const float v = k < r ? (float)((double)X[(int64_t)k * ldx + j] * inv) : 0.0f;
      const uint8_t a = to_e4m3(v);
      q1[j * rp + k] = a;
      q2[j * rp + k] = to_e4m3(16.0f * (v - from_e4m3(a)));
    }
    if (lane == 0) s[t] = sc;
  }
}

// ---------------------------------------------------------------- shared MFMA machinery
template <int PREC>
struct MpOps {
  static constexpr int ES = PREC == CUR_PREC_BF16X3 ? 2 : 1;  // bytes per element
  static constexpr int ROWB = kMK * ES + 16;                  // bytes per staged strip (padded)
};

template <int PREC>
struct MpLds {
  static constexpr int ROWB = MpOps<PREC>::ROWB;
  alignas(16) uint8_t x[2][kMT * ROWB];  // two terms of the first operand (column strips)
  alignas(16) uint8_t y[2][kMT * ROWB];  // two terms of the second operand (row strips)
  double red[3][kMpThreads / 64];
  float tmax[kMT / (16 * kNA)][kMT / kST];  // k_cu_lowp: FP8 tile maxima of Bm, per column range
};

// One staged chunk's products for a wavefront's kNA x kNB blocks: first-operand
// strips xs0 + 16 a + (l & 15), second-operand strips ys0 + 16 b + (l & 15).
template <int PREC>
__device__ __forceinline__ void mp_chunk(const MpLds<PREC>& L, int kc, int xs0, int ys0, int lr, int lk,
                                         f32x4 (&acc)[kNA][kNB], f32x4 (&acc2)[kNA][kNB]) {
  constexpr int ES = MpOps<PREC>::ES, ROWB = MpOps<PREC>::ROWB;
  for (int k = 0; k < kc; k += 32) {
    const int off = (k + 8 * lk) * ES;
    if constexpr (PREC == CUR_PREC_BF16X3) {
      bf16x8 xh[kNA], xl[kNA];
#pragma unroll
      for (int a = 0; a < kNA; ++a) {
        xh[a] = *(const bf16x8*)(L.x[0] + (xs0 + 16 * a + lr) * ROWB + off);
        xl[a] = *(const bf16x8*)(L.x[1] + (xs0 + 16 * a + lr) * ROWB + off);
      }
#pragma unroll
      for (int b = 0; b < kNB; ++b) {  // one second-operand fragment live at a time
        const bf16x8 yh = *(const bf16x8*)(L.y[0] + (ys0 + 16 * b + lr) * ROWB + off);
        const bf16x8 yl = *(const bf16x8*)(L.y[1] + (ys0 + 16 * b + lr) * ROWB + off);
#pragma unroll
        for (int a = 0; a < kNA; ++a) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl[a], yh, acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[a], yl, acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[a], yh, acc[a][b], 0, 0, 0);
        }
      }
    } else {
      long x1[kNA], x2[kNA];
#pragma unroll
      for (int a = 0; a < kNA; ++a) {
        x1[a] = *(const long*)(L.x[0] + (xs0 + 16 * a + lr) * ROWB + off);
        x2[a] = *(const long*)(L.x[1] + (xs0 + 16 * a + lr) * ROWB + off);
      }
#pragma unroll
      for (int b = 0; b < kNB; ++b) {
        const long y1 = *(const long*)(L.y[0] + (ys0 + 16 * b + lr) * ROWB + off);
        const long y2 = *(const long*)(L.y[1] + (ys0 + 16 * b + lr) * ROWB + off);
#pragma unroll
        for (int a = 0; a < kNA; ++a) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(x1[a], y1, acc[a][b], 0, 0, 0);
          acc2[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(x1[a], y2, acc2[a][b], 0, 0, 0);
          acc2[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(x2[a], y1, acc2[a][b], 0, 0, 0);
        }
      }
    }
  }
}

// Staging of kMT strips (from strip g0, g0 + s < lim) of the two terms of a
// split operand, k values k0 .. k0 + kMK: mp_load brings them into registers
// (issued a chunk ahead, so their latency overlaps the current chunk's
// products), mp_store writes them to an LDS operand slot pair.
template <int PREC>
struct MpStage {
  static constexpr int PIECES = kMK * MpOps<PREC>::ES / 16;  // 16-byte pieces per strip
  static constexpr int PER = 2 * kMT * PIECES / kMpThreads;
  u32x4 v[PER];
};

// Strips at or past lim: MODE 0 loads zeros, MODE 1 assumes there are none (no
// test at all), MODE 2 loads strip lim - 1 again.  A tested load compiles to a
// branch with a wait for its data, so modes 1 and 2 keep all loads in flight.
// The pieces are expanded by a parameter pack rather than a loop: a loop of
// plain copies is turned into a memcpy, which puts the stage in scratch memory.
template <int PREC, int MODE>
__device__ __forceinline__ void mp_load_piece(MpStage<PREC>& st, int q, const uint8_t* t1, const uint8_t* t2,
                                              int64_t g0, int64_t lim, int rp, int k0) {
  constexpr int ES = MpOps<PREC>::ES, PIECES = MpStage<PREC>::PIECES;
  const int idx = threadIdx.x + q * kMpThreads;
  const int term = idx / (kMT * PIECES), rem = idx % (kMT * PIECES);
  const int strip = rem / PIECES, piece = rem % PIECES;
  const int64_t g = MODE == 2 ? min(g0 + strip, lim - 1) : g0 + strip;
  const int kk = k0 + piece * (16 / ES);  // < rp: k0 < rp and both are multiples of kMK
  const uint8_t* src = term ? t2 : t1;
  if (MODE == 0) st.v[q] = g < lim ? *(const u32x4*)(src + (g * rp + kk) * ES) : u32x4{0u, 0u, 0u, 0u};
  else st.v[q] = *(const u32x4*)(src + (g * rp + kk) * ES);
}

template <int PREC, int MODE, int... Q>
__device__ __forceinline__ void mp_load_pieces(MpStage<PREC>& st, const uint8_t* t1, const uint8_t* t2, int64_t g0,
                                               int64_t lim, int rp, int k0, std::integer_sequence<int, Q...>) {
  (mp_load_piece<PREC, MODE>(st, Q, t1, t2, g0, lim, rp, k0), ...);
}

template <int PREC, int MODE = 0>
__device__ __forceinline__ void mp_load(MpStage<PREC>& st, const uint8_t* t1, const uint8_t* t2, int64_t g0,
                                        int64_t lim, int rp, int k0) {
  mp_load_pieces<PREC, MODE>(st, t1, t2, g0, lim, rp, k0, std::make_integer_sequence<int, MpStage<PREC>::PER>());
}

template <int PREC, int... Q>
__device__ __forceinline__ void mp_store_pieces(const MpStage<PREC>& st, uint8_t* d1, uint8_t* d2,
                                                std::integer_sequence<int, Q...>) {
  constexpr int ROWB = MpOps<PREC>::ROWB, PIECES = MpStage<PREC>::PIECES;
  auto one = [&](int q) {
    const int idx = threadIdx.x + q * kMpThreads;
    const int term = idx / (kMT * PIECES), rem = idx % (kMT * PIECES);
    const int strip = rem / PIECES, piece = rem % PIECES;
    *(u32x4*)((term ? d2 : d1) + strip * ROWB + piece * 16) = st.v[q];
  };
  (one(Q), ...);
}

template <int PREC>
__device__ __forceinline__ void mp_store(const MpStage<PREC>& st, uint8_t* d1, uint8_t* d2) {
  mp_store_pieces<PREC>(st, d1, d2, std::make_integer_sequence<int, MpStage<PREC>::PER>());
}

// ---------------------------------------------------------------- Bm = C U
// One block per kMT rows of C (r <= 128, so all of Bm's rp columns).  C's rows
// are split as they are staged (FP8: with the scale of their 16-row tile,
// from a prologue over the block's rows); U's split columns are staged from
// the column-operand form.  Wavefront w computes Bm rows [64 (w & 1), +64) x
// columns [32 (w >> 1), +32) of the block as the transposed product (first
// operand: U's column strips).  Output: Bm split in the row-operand form
// (m x rp per term) and, for FP8, one scale per 16-row tile of Bm.
// FULL = true: the block's kMT rows lie inside C and r = rp, so C's loads and
// Bm's row stores need no bounds test, and U's strips past r (columns of Bm
// past rp, never stored) repeat strip r - 1 instead of being zeroed: a repeat
// of a column that is already there leaves the FP8 tile maxima unchanged.
// Block b0 + blockIdx.x covers rows from kMT (b0 + blockIdx.x).
template <int PREC, bool FULL>
__global__ __launch_bounds__(kMpThreads, 2) void k_cu_lowp(const float* __restrict__ C, int64_t m, int r, int rp,
                                                           const void* __restrict__ u1v, const void* __restrict__ u2v,
                                                           const float* __restrict__ us, void* __restrict__ o1v,
                                                           void* __restrict__ o2v, float* __restrict__ os, int b0) {
  using L_t = MpLds<PREC>;
  constexpr int ROWB = MpOps<PREC>::ROWB;
  __shared__ L_t L;
  __shared__ float cs[kMT / kST];  // FP8: scales of the block's 16-row tiles of C
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t rb0 = (int64_t)(b0 + blockIdx.x) * kMT;
  const int wi = (w & 1) * 64, wj = (w >> 1) * 32;  // rows of Bm, columns of Bm
  if constexpr (PREC == CUR_PREC_FP8) {
    // row tile w of C: contiguous 16 r floats (C is m x r, leading dimension r)
    const int64_t i0 = rb0 + w * kST;
    const int64_t cnt = (int64_t)max<int64_t>(0, min<int64_t>(kST, m - i0)) * r;
    float amax = 0.0f;
    for (int64_t idx = lane; idx < cnt; idx += 64) amax = fmaxf(amax, fabsf(C[i0 * r + idx]));
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) amax = fmaxf(amax, __shfl_xor(amax, sh, 64));
    if (lane == 0) cs[w] = fp8_scale(amax);
    __syncthreads();
  }
  f32x4 acc[kNA][kNB], acc2[kNA][kNB];
#pragma unroll
  for (int a = 0; a < kNA; ++a)
#pragma unroll
    for (int b = 0; b < kNB; ++b) {
      acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
      acc2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  // C chunk: thread t converts row t >> 2, k values 8 (t & 3) .. + 8; the next
  // chunk's C values and U pieces are loaded before this chunk's products
  const int crow = tid >> 2, ck = 8 * (tid & 3);
  const int64_t gi = rb0 + crow;
  float cv[8];
  MpStage<PREC> us_st;
  auto load_c = [&](int k0) {
    if (FULL) {  // two 16-byte loads (C's rows start 16-byte aligned: r = rp, a multiple of 32)
      const f32x4 c0v = *(const f32x4*)(C + gi * r + k0 + ck), c1v = *(const f32x4*)(C + gi * r + k0 + ck + 4);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        cv[q] = c0v[q];
        cv[4 + q] = c1v[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = k0 + ck + q;
        cv[q] = (gi < m && k < r) ? C[gi * r + k] : 0.0f;
      }
    }
    mp_load<PREC, FULL ? 2 : 0>(us_st, (const uint8_t*)u1v, (const uint8_t*)u2v, 0, r, rp, k0);  // U's r column strips
  };
  load_c(0);
  for (int k0 = 0; k0 < rp; k0 += kMK) {
    __syncthreads();  // the previous chunk's fragments have been read
    mp_store<PREC>(us_st, L.x[0], L.x[1]);
    if constexpr (PREC == CUR_PREC_BF16X3) {
      __bf16 hv[8], lv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        hv[q] = (__bf16)cv[q];
        lv[q] = (__bf16)(cv[q] - (float)hv[q]);
      }
      *(uint4*)(L.y[0] + crow * ROWB + 2 * ck) = *(const uint4*)hv;
      *(uint4*)(L.y[1] + crow * ROWB + 2 * ck) = *(const uint4*)lv;
    } else {
      const float inv = 1.0f / cs[crow / kST];
      uint8_t q1v[8], q2v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float v = cv[q] * inv;
        q1v[q] = to_e4m3(v);
        q2v[q] = to_e4m3(16.0f * (v - from_e4m3(q1v[q])));
      }
      *(uint2*)(L.y[0] + crow * ROWB + ck) = *(const uint2*)q1v;
      *(uint2*)(L.y[1] + crow * ROWB + ck) = *(const uint2*)q2v;
    }
    __syncthreads();
    if (k0 + kMK < rp) load_c(k0 + kMK);
    mp_chunk<PREC>(L, min(kMK, rp - k0), wj, wi, lr, lk, acc, acc2);
  }
  // Bm(i, j) of block (a, b): i = wi + 16 b + (l & 15), j = wj + 16 a + 4 (l >> 4) + v
  float bm[kNA][kNB][4];
#pragma unroll
  for (int a = 0; a < kNA; ++a)
#pragma unroll
    for (int b = 0; b < kNB; ++b) {
      // (column tiles past r hold zeros and have no scale of their own)
      const float sc = (PREC == CUR_PREC_FP8) ? (wj + 16 * a < r ? us[(wj + 16 * a) / kST] : 0.0f) *
                                                    cs[(wi + 16 * b) / kST]
                                              : 1.0f;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float p = acc[a][b][v];
        if constexpr (PREC == CUR_PREC_FP8) p = sc * (p + 0.0625f * acc2[a][b][v]);
        bm[a][b][v] = p;
      }
    }
  if constexpr (PREC == CUR_PREC_BF16X3) {
#pragma unroll
    for (int b = 0; b < kNB; ++b) {
      const int64_t gi2 = rb0 + wi + 16 * b + lr;
      if (!FULL && gi2 >= m) continue;
#pragma unroll
      for (int a = 0; a < kNA; ++a) {
        const int j = wj + 16 * a + 4 * lk;
        if (j >= rp) continue;
        __bf16 hv[4], lv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          hv[v] = (__bf16)bm[a][b][v];
          lv[v] = (__bf16)(bm[a][b][v] - (float)hv[v]);
        }
        *(uint2*)((__bf16*)o1v + gi2 * rp + j) = *(const uint2*)hv;
        *(uint2*)((__bf16*)o2v + gi2 * rp + j) = *(const uint2*)lv;
      }
    }
  } else {
    // scale of each 16-row tile of Bm: the maximum over the tile's rows (lanes
    // l & 15) and all rp columns (the four wavefronts that share these rows,
    // through LDS)
#pragma unroll
    for (int b = 0; b < kNB; ++b) {
      float mx = 0.0f;
#pragma unroll
      for (int a = 0; a < kNA; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) mx = fmaxf(mx, fabsf(bm[a][b][v]));
#pragma unroll
      for (int sh = 32; sh >= 1; sh >>= 1) mx = fmaxf(mx, __shfl_xor(mx, sh, 64));
      if (lane == 0) L.tmax[w >> 1][(wi + 16 * b) / kST] = mx;
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < kNB; ++b) {
      const int tt = (wi + 16 * b) / kST;
      float mx = L.tmax[0][tt];
#pragma unroll
      for (int q = 1; q < kMT / (16 * kNA); ++q) mx = fmaxf(mx, L.tmax[q][tt]);
      const float sc = fp8_scale(mx);
      const float inv = 1.0f / sc;
      const int64_t gi2 = rb0 + wi + 16 * b + lr;
      if (w >> 1 == 0 && lane == 0 && rb0 + wi + 16 * b < m) os[(rb0 + wi + 16 * b) / kST] = sc;
      if (!FULL && gi2 >= m) continue;
#pragma unroll
      for (int a = 0; a < kNA; ++a) {
        const int j = wj + 16 * a + 4 * lk;
        if (j >= rp) continue;
        uint8_t q1v[4], q2v[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float x = bm[a][b][v] * inv;
          q1v[v] = to_e4m3(x);
          q2v[v] = to_e4m3(16.0f * (x - from_e4m3(q1v[v])));
        }
        *(uint32_t*)((uint8_t*)o1v + gi2 * rp + j) = *(const uint32_t*)q1v;
        *(uint32_t*)((uint8_t*)o2v + gi2 * rp + j) = *(const uint32_t*)q2v;
      }
    }
  }
}

// ---------------------------------------------------------------- the tile kernel
// The chip hands workgroups to its 8 XCDs in turn (linear id mod 8), each XCD
// with its own L2.  Taken in grid order, the few column tiles of a tall
// matrix's row strip (consecutive ids) land on different XCDs and each of them
// fetches the strip's row operand (at 2^20 x 1024, r = 128, BF16x3: 8.7 GB
// fetched per call instead of 4.8).  xcd_tile maps linear id L of a grid of
// `total` tiles to tile T such that XCD x takes one contiguous range of tiles,
// in order: [x base + min(x, rem), ...) with base = total / 8, rem = total % 8
// (a bijection on [0, total)).
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_tile(int64_t L, int64_t total) {
  const int64_t x = L % kXcds, local = L / kXcds, base = total / kXcds, rem = total % kXcds;
  return x * base + min(x, rem) + local;
}

// One 128 x 128 tile of E per block; wavefront w computes rows [64 (w & 1),
// +64) x columns [32 (w >> 1), +32) as the transposed product P^T = R^T Bm^T
// (first operand: R's column strips), so a lane's four results are four
// consecutive columns of one row and its part of the tile of A is one 16-byte
// load per 16 x 16 block (VEC4: A's rows 16-byte aligned and n a multiple of
// 4; four scalar loads otherwise).  The tile of A is requested before the
// products, so its latency overlaps them; the next chunk of both operands is
// loaded before the current chunk's products.  Operands staged in LDS kMK
// values of k at a time (~41 KB BF16, ~25 KB FP8), two blocks per CU.
// part[3*block] = {max|E|, sum E^2, sum A^2}.
// EDGE = false is the instance for tiles wholly inside the matrix (operand
// loads without bounds tests, no range checks in the epilogue); EDGE = true
// runs over the ragged right and bottom strips.  Tiles are taken in the
// XCD-contiguous order of xcd_tile; tile (tx0 + tile % gx, ty0 + tile / gx)
// writes part[3 (ty gxall + tx)].
template <int PREC, bool VEC4, bool EDGE>
__global__ __launch_bounds__(kMpThreads, 2) __attribute__((amdgpu_waves_per_eu(4))) void k_resid_mp(const float* __restrict__ A, int64_t m, int64_t n,
                                                            int64_t lda, int rp, const void* __restrict__ a1v,
                                                            const void* __restrict__ a2v, const float* __restrict__ as,
                                                            const void* __restrict__ b1v, const void* __restrict__ b2v,
                                                            const float* __restrict__ bs, double* part, int tx0,
                                                            int ty0, int gxall) {
  using L_t = MpLds<PREC>;
  __shared__ L_t L;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t tile = xcd_tile((int64_t)blockIdx.y * gridDim.x + blockIdx.x, (int64_t)gridDim.x * gridDim.y);
  const int tx = tx0 + (int)(tile % gridDim.x), ty = ty0 + (int)(tile / gridDim.x);
  const int64_t rb0 = (int64_t)ty * kMT, cb0 = (int64_t)tx * kMT;
  const int wi = (w & 1) * 64, wj = (w >> 1) * 32;  // rows, columns of the tile
  f32x4 acc[kNA][kNB], acc2[kNA][kNB];
#pragma unroll
  for (int a = 0; a < kNA; ++a)
#pragma unroll
    for (int b = 0; b < kNB; ++b) {
      acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
      acc2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  // A(i, j) of block (a, b): i = rb0 + wi + 16 b + (l & 15),
  // j = cb0 + wj + 16 a + 4 (l >> 4) + v.  Rows past m and columns past n read
  // a clamped in-range element and are skipped in the epilogue; every load is
  // unconditional, so all of them are in flight before the first wait (VEC4:
  // the column clamped to n - 4, a multiple of 4).
  float4 av[kNA][kNB];
  auto load_a = [&](int b) {
    const int64_t i = min(rb0 + wi + 16 * b + lr, m - 1);
    const float* rowp = A + i * lda;
#pragma unroll
    for (int a = 0; a < kNA; ++a) {
      const int64_t j = cb0 + wj + 16 * a + 4 * lk;
      if constexpr (VEC4) {
        av[a][b] = *(const float4*)(rowp + min(j, n - 4));
      } else {
        av[a][b] = make_float4(rowp[min(j, n - 1)], rowp[min(j + 1, n - 1)], rowp[min(j + 2, n - 1)],
                               rowp[min(j + 3, n - 1)]);
      }
    }
  };
  constexpr int PF = PREC == CUR_PREC_FP8 ? 1 : 2;  // A row groups requested before the products
#pragma unroll
  for (int b = 0; b < PF; ++b) load_a(b);
  MpStage<PREC> sx, sy;  // the next chunk of both operands, loaded a chunk ahead
  mp_load<PREC, EDGE ? 0 : 1>(sx, (const uint8_t*)b1v, (const uint8_t*)b2v, cb0, n, rp, 0);
  mp_load<PREC, EDGE ? 0 : 1>(sy, (const uint8_t*)a1v, (const uint8_t*)a2v, rb0, m, rp, 0);
  for (int k0 = 0; k0 < rp; k0 += kMK) {
    __syncthreads();  // the previous chunk's fragments have been read
    mp_store<PREC>(sx, L.x[0], L.x[1]);
    mp_store<PREC>(sy, L.y[0], L.y[1]);
    __syncthreads();
    if (k0 + kMK < rp) {
      mp_load<PREC, EDGE ? 0 : 1>(sx, (const uint8_t*)b1v, (const uint8_t*)b2v, cb0, n, rp, k0 + kMK);
      mp_load<PREC, EDGE ? 0 : 1>(sy, (const uint8_t*)a1v, (const uint8_t*)a2v, rb0, m, rp, k0 + kMK);
    }
    mp_chunk<PREC>(L, min(kMK, rp - k0), wj, wi, lr, lk, acc, acc2);
  }
#pragma unroll
  for (int b = PF; b < kNB; ++b) load_a(b);
  double emax = 0.0, esq = 0.0, asq = 0.0;
#pragma unroll
  for (int b = 0; b < kNB; ++b) {
    const int64_t i = rb0 + wi + 16 * b + lr;
    if (EDGE && i >= m) continue;
#pragma unroll
    for (int a = 0; a < kNA; ++a) {
      if (EDGE && cb0 + wj + 16 * a >= n) continue;
      const float sc = (PREC == CUR_PREC_FP8) ? as[(rb0 + wi + 16 * b) / kST] * bs[(cb0 + wj + 16 * a) / kST] : 1.0f;
      const float avs[4] = {av[a][b].x, av[a][b].y, av[a][b].z, av[a][b].w};
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t j = cb0 + wj + 16 * a + 4 * lk + v;
        if (EDGE && j >= n) continue;
        float p = acc[a][b][v];
        if constexpr (PREC == CUR_PREC_FP8) p = sc * (p + 0.0625f * acc2[a][b][v]);
        const double x = (double)avs[v];
        const double e = x - (double)p;
        emax = nan_max(emax, fabs(e));
        esq = fma(e, e, esq);
        asq = fma(x, x, asq);
      }
    }
  }
#pragma unroll
  for (int sh = 32; sh >= 1; sh >>= 1) {
    emax = nan_max(emax, __shfl_xor(emax, sh, 64));
    esq += __shfl_xor(esq, sh, 64);
    asq += __shfl_xor(asq, sh, 64);
  }
  if (lane == 0) {
    L.red[0][w] = emax;
    L.red[1][w] = esq;
    L.red[2][w] = asq;
  }
  __syncthreads();
  if (tid == 0) {
    for (int q = 1; q < kMpThreads / 64; ++q) {
      emax = nan_max(emax, L.red[0][q]);
      esq += L.red[1][q];
      asq += L.red[2][q];
    }
    const int64_t bid = (int64_t)ty * gxall + tx;
    part[3 * bid + 0] = emax;
    part[3 * bid + 1] = esq;
    part[3 * bid + 2] = asq;
  }
}

// ---------------------------------------------------------------- host side
// Scratch: [Bm terms (m x rp each) | R terms (n x rp) | U terms (rp x rp) |
// FP8 scales of Bm, R, U tiles].
static size_t mp_layout(int64_t m, int64_t n, int r, int prec, size_t off[10]) {
  const int rp = (r + 31) / 32 * 32;
  const size_t es = prec == CUR_PREC_BF16X3 ? 2 : 1;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t sizes[9] = {es * (size_t)m * rp, es * (size_t)m * rp, es * (size_t)n * rp, es * (size_t)n * rp,
                           es * (size_t)rp * rp, es * (size_t)rp * rp,
                           sizeof(float) * (size_t)((m + kST - 1) / kST), sizeof(float) * (size_t)((n + kST - 1) / kST),
                           sizeof(float) * (size_t)((rp + kST - 1) / kST)};
  size_t o = 0;
  for (int k = 0; k < 9; ++k) {
    off[k] = o;
    o += al(sizes[k]);
  }
  off[9] = o;
  return o;
}

size_t residual_mp_scratch(int64_t m, int64_t n, int r, int prec) {
  size_t off[10];
  return mp_layout(m, n, r, prec, off) + 256;
}

int64_t residual_mp_tiles(int64_t m, int64_t n) { return ((n + kMT - 1) / kMT) * ((m + kMT - 1) / kMT); }

cur_status residual_mp_launch(cur_ctx ctx, const float* A, int64_t m, int64_t n, int64_t lda, int r, const float* C,
                              const double* U, const float* R, int prec, char* scratch, size_t scratch_bytes,
                              double* part, int64_t* nb) {
  hipStream_t s = ctx->stream;
  const int rp = (r + 31) / 32 * 32;
  size_t off[10];
  if (mp_layout(m, n, r, prec, off) > scratch_bytes) {
    set_error("internal: residual scratch too small");
    return CUR_ERR_INTERNAL;
  }
  void* a1 = scratch + off[0];
  void* a2 = scratch + off[1];
  void* b1 = scratch + off[2];
  void* b2 = scratch + off[3];
  void* u1 = scratch + off[4];
  void* u2 = scratch + off[5];
  float* as = (float*)(scratch + off[6]);
  float* bs = (float*)(scratch + off[7]);
  float* us = (float*)(scratch + off[8]);
  const int64_t gx = (n + kMT - 1) / kMT, gy = (m + kMT - 1) / kMT;
  if (gy > 65535) {
    set_error("matrix too tall for the residual grid");
    return CUR_ERR_ARG;
  }
  auto grid = [](int64_t work) { return (int)std::max<int64_t>(1, std::min<int64_t>((work + kThreads - 1) / kThreads, 65536)); };
  auto wgrid = [](int64_t tiles) { return (int)std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, 65536)); };
  const bool vec4 = lda % 4 == 0 && n % 4 == 0 && ((uintptr_t)A % 16) == 0;
  // interior tiles without bounds tests, then the ragged right strip (corner
  // included) and bottom strip with them
  const int nf = (int)(n / kMT), mf = (int)(m / kMT);
  auto tile_kernel = [&](auto prec_c) {
    constexpr int P = decltype(prec_c)::value;
    auto launch = [&](auto vec_c) {
      constexpr bool V = decltype(vec_c)::value;
      if (nf > 0 && mf > 0)
        hipLaunchKernelGGL((k_resid_mp<P, V, false>), dim3((unsigned)nf, (unsigned)mf), dim3(kMpThreads), 0, s, A, m,
                           n, lda, rp, a1, a2, as, b1, b2, bs, part, 0, 0, (int)gx);
      if (n % kMT)
        hipLaunchKernelGGL((k_resid_mp<P, V, true>), dim3(1u, (unsigned)gy), dim3(kMpThreads), 0, s, A, m, n, lda, rp,
                           a1, a2, as, b1, b2, bs, part, nf, 0, (int)gx);
      if (m % kMT && nf > 0)
        hipLaunchKernelGGL((k_resid_mp<P, V, true>), dim3((unsigned)nf, 1u), dim3(kMpThreads), 0, s, A, m, n, lda, rp,
                           a1, a2, as, b1, b2, bs, part, 0, mf, (int)gx);
    };
    if (vec4) launch(std::true_type());
    else launch(std::false_type());
  };
  // Bm = C U: full row blocks without bounds tests when r is a multiple of kMK
  auto cu_kernel = [&](auto prec_c) {
    constexpr int P = decltype(prec_c)::value;
    const int full = r == rp ? mf : 0;
    if (full > 0)
      hipLaunchKernelGGL((k_cu_lowp<P, true>), dim3((unsigned)full), dim3(kMpThreads), 0, s, C, m, r, rp, u1, u2, us,
                         a1, a2, as, 0);
    if (gy > full)
      hipLaunchKernelGGL((k_cu_lowp<P, false>), dim3((unsigned)(gy - full)), dim3(kMpThreads), 0, s, C, m, r, rp, u1,
                         u2, us, a1, a2, as, full);
  };
  if (prec == CUR_PREC_BF16X3) {
    hipLaunchKernelGGL((k_split_cols_bf16<float>), dim3(grid(n * rp)), dim3(kThreads), 0, s, R, r, n, n, rp,
                       (__bf16*)b1, (__bf16*)b2);
    hipLaunchKernelGGL((k_split_cols_bf16<double>), dim3(grid((int64_t)rp * rp)), dim3(kThreads), 0, s, U, r,
                       (int64_t)r, (int64_t)r, rp, (__bf16*)u1, (__bf16*)u2);
    cu_kernel(std::integral_constant<int, CUR_PREC_BF16X3>());
    tile_kernel(std::integral_constant<int, CUR_PREC_BF16X3>());
  } else {
    hipLaunchKernelGGL((k_split_cols_fp8<float>), dim3(wgrid((n + kST - 1) / kST)), dim3(kThreads), 0, s, R, r, n, n,
                       rp, (uint8_t*)b1, (uint8_t*)b2, bs);
    hipLaunchKernelGGL((k_split_cols_fp8<double>), dim3(wgrid((rp + kST - 1) / kST)), dim3(kThreads), 0, s, U, r,
                       (int64_t)r, (int64_t)r, rp, (uint8_t*)u1, (uint8_t*)u2, us);
    cu_kernel(std::integral_constant<int, CUR_PREC_FP8>());
    tile_kernel(std::integral_constant<int, CUR_PREC_FP8>());
  }
  CUR_HIP_CHECK(hipGetLastError());
  *nb = gx * gy;
  return CUR_OK;
}

}  // namespace cur
