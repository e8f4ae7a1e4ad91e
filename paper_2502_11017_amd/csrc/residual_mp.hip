// Reduced-precision residual of the CUR form for FP32 input: E = A - P with
// P = Bm R, Bm = C U (FP64, as in the native path), the m x n x r product on
// MFMA with FP32 accumulation and the difference, maximum and sums in FP64.
//
//   BF16x3: x = hi + lo with hi = bf16(x), lo = bf16(x - hi); the product is
//           hi_a hi_b + hi_a lo_b + lo_a hi_b (the lo_a lo_b term, ~2^-16
//           relative, is dropped), v_mfma_f32_16x16x32_bf16.
//   FP8:    OCP e4m3 with one scale per row of Bm and per column of R,
//           s = max|strip| / 448; two terms q1 = e4m3(x/s),
//           q2 = e4m3(16 (x/s - q1)), product q1 q1 + (q1 q2 + q2 q1) / 16,
//           v_mfma_f32_16x16x32_fp8_fp8.
//
// Operand layouts (r padded to rp, a multiple of 32, with zeros): the split
// Bm is row-major m x rp, the split R is stored transposed, n x rp, so that a
// lane's eight consecutive k values are one 16-byte (bf16) or 8-byte (fp8)
// load.  MFMA lanes: lane l supplies A[l & 15][8 (l >> 4) + e] and
// B[8 (l >> 4) + e][l & 15], e < 8, and holds D[4 (l >> 4) + v][l & 15].
#include <hip/hip_runtime.h>

#include <cmath>

#include "cur_device.hpp"
#include "cur_internal.hpp"

namespace cur {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMT = 128;  // tile of E per block (rows and columns)

// ---------------------------------------------------------------- splits
// Bm (m x r FP64, row-major) -> hi/lo bf16, m x rp.
__global__ __launch_bounds__(kThreads) void k_split_rows_bf16(const double* __restrict__ Bm, int64_t m, int r,
                                                              int rp, __bf16* __restrict__ h,
                                                              __bf16* __restrict__ l) {
  const int64_t total = m * rp;
  for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * kThreads) {
    const int64_t i = idx / rp;
    const int k = (int)(idx - i * rp);
    const double x = k < r ? Bm[i * r + k] : 0.0;
    const __bf16 hi = (__bf16)(float)x;
    h[idx] = hi;
    l[idx] = (__bf16)(float)(x - (double)(float)hi);
  }
}

// R (r x n, ld n) -> transposed hi/lo bf16, n x rp.
__global__ __launch_bounds__(kThreads) void k_split_cols_bf16(const float* __restrict__ R, int r, int64_t n, int rp,
                                                              __bf16* __restrict__ h, __bf16* __restrict__ l) {
  const int64_t total = n * rp;
  for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * kThreads) {
    const int64_t j = idx / rp;
    const int k = (int)(idx - j * rp);
    const float x = k < r ? R[(int64_t)k * n + j] : 0.0f;
    const __bf16 hi = (__bf16)x;
    h[idx] = hi;
    l[idx] = (__bf16)(x - (float)hi);
  }
}

__device__ __forceinline__ uint8_t to_e4m3(float x) {
  return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false) & 0xff);
}
__device__ __forceinline__ float from_e4m3(uint8_t q) { return __builtin_amdgcn_cvt_f32_fp8((int)q, 0); }

// One strip of length r <= 128 (values x[k * stride]) -> scale s and two e4m3
// terms (q1, q2 at q[k], k < rp; zero padding).  One wavefront per strip:
// lane l handles k = l and k = l + 64.
template <typename V>
__device__ void split_strip_fp8(const V* x, int64_t stride, int r, int rp, uint8_t* q1, uint8_t* q2, float* s) {
  const int lane = threadIdx.x & 63;
  double v0 = lane < r ? (double)x[lane * stride] : 0.0;
  double v1 = lane + 64 < r ? (double)x[(lane + 64) * stride] : 0.0;
  double amax = fmax(fabs(v0), fabs(v1));
#pragma unroll
  for (int sh = 32; sh >= 1; sh >>= 1) amax = fmax(amax, __shfl_xor(amax, sh, 64));
  const float sc = amax > 0.0 ? (float)(amax / 448.0) : 1.0f;
  const double inv = 1.0 / (double)sc;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int k = lane + 64 * h;
    if (k >= rp) break;
    const float v = (float)((h ? v1 : v0) * inv);
    const uint8_t a = to_e4m3(v);
    q1[k] = a;
    q2[k] = to_e4m3(16.0f * (v - from_e4m3(a)));
  }
  if (lane == 0) *s = sc;
}

__global__ __launch_bounds__(kThreads) void k_split_rows_fp8(const double* __restrict__ Bm, int64_t m, int r, int rp,
                                                             uint8_t* q1, uint8_t* q2, float* s) {
  const int64_t waves = (int64_t)gridDim.x * (kThreads / 64);
  for (int64_t i = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); i < m; i += waves)
    split_strip_fp8<double>(Bm + i * r, 1, r, rp, q1 + i * rp, q2 + i * rp, s + i);
}

__global__ __launch_bounds__(kThreads) void k_split_cols_fp8(const float* __restrict__ R, int r, int64_t n, int rp,
                                                             uint8_t* q1, uint8_t* q2, float* s) {
  const int64_t waves = (int64_t)gridDim.x * (kThreads / 64);
  for (int64_t j = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); j < n; j += waves)
    split_strip_fp8<float>(R + j, n, r, rp, q1 + j * rp, q2 + j * rp, s + j);
}

// ---------------------------------------------------------------- the tile kernel
// Wavefront w computes the 64 x 64 quadrant (w >> 1, w & 1) of the block's
// 128 x 128 tile as 4 x 4 MFMA blocks of 16 x 16.  The block's rows of the
// split Bm and columns of the split R are staged in LDS, KC values of k at a
// time (each row padded by 16 bytes); fragments are 16-byte (bf16) or 8-byte
// (fp8) LDS reads.  ~70 KB of LDS, two blocks per CU, so one block's MFMAs
// cover the other's staging and epilogue.  Rows or columns beyond m, n are
// zero operands and are skipped in the epilogue.
// part[3*block] = {max|E|, sum E^2, sum A^2}.
constexpr int kMK = 32;  // k values per staged chunk

template <int PREC>
struct MpLds {
  static constexpr int ES = PREC == CUR_PREC_BF16X3 ? 2 : 1;  // bytes per element
  static constexpr int ROWB = kMK * ES + 16;                  // bytes per staged row (padded)
  alignas(16) uint8_t a[2][kMT * ROWB];                       // two terms of the row operand
  alignas(16) uint8_t b[2][kMT * ROWB];                       // two terms of the column operand
  double red[3][kThreads / 64];
};

template <int PREC>
__global__ __launch_bounds__(kThreads, 2) void k_resid_mp(const float* __restrict__ A, int64_t m, int64_t n,
                                                          int64_t lda, int rp, const void* __restrict__ a1v,
                                                          const void* __restrict__ a2v, const float* __restrict__ as,
                                                          const void* __restrict__ b1v, const void* __restrict__ b2v,
                                                          const float* __restrict__ bs, double* part) {
  using L_t = MpLds<PREC>;
  constexpr int ES = L_t::ES, ROWB = L_t::ROWB;
  __shared__ L_t L;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t rb0 = (int64_t)blockIdx.y * kMT, cb0 = (int64_t)blockIdx.x * kMT;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  const uint8_t* src[4] = {(const uint8_t*)a1v, (const uint8_t*)a2v, (const uint8_t*)b1v, (const uint8_t*)b2v};
  f32x4 acc[4][4], acc2[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      acc2[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  // The tile of A (the only operand streamed from HBM) is requested first,
  // so its latency overlaps the products; rows/columns past the matrix load
  // a clamped in-range element and are skipped in the epilogue.  The FP8
  // form holds a second accumulator set, so it requests the first PF of its
  // four 16-row groups here and the rest at the start of the epilogue.
  constexpr int PF = PREC == CUR_PREC_FP8 ? 2 : 4;
  float av[4][4][4];
  auto load_a = [&](int i) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = min(rb0 + wr + 16 * i + 4 * lk + v, m - 1);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t col = min(cb0 + wc + 16 * j + lr, n - 1);
        av[i][v][j] = A[row * lda + col];
      }
    }
  };
#pragma unroll
  for (int i = 0; i < PF; ++i) load_a(i);
  for (int k0 = 0; k0 < rp; k0 += kMK) {
    // stage: 4 operand terms x 128 strips x (kMK * ES) bytes as 16-byte pieces
    constexpr int PIECES = kMK * ES / 16;  // per strip
    constexpr int TOTAL = 4 * kMT * PIECES;
    constexpr int PER = TOTAL / kThreads;
    uint4 v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * kThreads;
      const int term = idx / (kMT * PIECES), rem = idx % (kMT * PIECES);
      const int strip = rem / PIECES, piece = rem % PIECES;
      const int64_t lim = term < 2 ? m : n;
      const int64_t g = (term < 2 ? rb0 : cb0) + strip;
      const int kk = k0 + piece * (16 / ES);
      v[q] = (g < lim && kk < rp) ? *(const uint4*)(src[term] + (g * rp + kk) * ES) : make_uint4(0, 0, 0, 0);
    }
    __syncthreads();  // the previous chunk's fragments have been read
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = tid + q * kThreads;
      const int term = idx / (kMT * PIECES), rem = idx % (kMT * PIECES);
      const int strip = rem / PIECES, piece = rem % PIECES;
      uint8_t* dst = (term < 2 ? L.a[term] : L.b[term - 2]) + strip * ROWB + piece * 16;
      *(uint4*)dst = v[q];
    }
    __syncthreads();
    const int kc = min(kMK, rp - k0);
    for (int k = 0; k < kc; k += 32) {
      const int off = (k + 8 * lk) * ES;
      if constexpr (PREC == CUR_PREC_BF16X3) {
        bf16x8 xh[4], xl[4], yh[4], yl[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          xh[i] = *(const bf16x8*)(L.a[0] + (wr + 16 * i + lr) * ROWB + off);
          xl[i] = *(const bf16x8*)(L.a[1] + (wr + 16 * i + lr) * ROWB + off);
          yh[i] = *(const bf16x8*)(L.b[0] + (wc + 16 * i + lr) * ROWB + off);
          yl[i] = *(const bf16x8*)(L.b[1] + (wc + 16 * i + lr) * ROWB + off);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl[i], yh[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[i], yl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[i], yh[j], acc[i][j], 0, 0, 0);
          }
      } else {
        long x1[4], x2[4], y1[4], y2[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          x1[i] = *(const long*)(L.a[0] + (wr + 16 * i + lr) * ROWB + off);
          x2[i] = *(const long*)(L.a[1] + (wr + 16 * i + lr) * ROWB + off);
          y1[i] = *(const long*)(L.b[0] + (wc + 16 * i + lr) * ROWB + off);
          y2[i] = *(const long*)(L.b[1] + (wc + 16 * i + lr) * ROWB + off);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(x1[i], y1[j], acc[i][j], 0, 0, 0);
            acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(x1[i], y2[j], acc2[i][j], 0, 0, 0);
            acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(x2[i], y1[j], acc2[i][j], 0, 0, 0);
          }
      }
    }
  }
#pragma unroll
  for (int i = PF; i < 4; ++i) load_a(i);
  double emax = 0.0, esq = 0.0, asq = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = rb0 + wr + 16 * i + 4 * lk + v;
      if (row >= m) continue;
      const float sa = (PREC == CUR_PREC_FP8) ? as[row] : 1.0f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t col = cb0 + wc + 16 * j + lr;
        if (col >= n) continue;
        float p = acc[i][j][v];
        if constexpr (PREC == CUR_PREC_FP8) p = sa * bs[col] * (p + 0.0625f * acc2[i][j][v]);
        const double a = (double)av[i][v][j];
        const double e = a - (double)p;
        emax = nan_max(emax, fabs(e));
        esq = fma(e, e, esq);
        asq = fma(a, a, asq);
      }
    }
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
    emax = nan_max(emax, __shfl_xor(emax, s, 64));
    esq += __shfl_xor(esq, s, 64);
    asq += __shfl_xor(asq, s, 64);
  }
  if (lane == 0) {
    L.red[0][w] = emax;
    L.red[1][w] = esq;
    L.red[2][w] = asq;
  }
  __syncthreads();
  if (tid == 0) {
    for (int q = 1; q < kThreads / 64; ++q) {
      emax = nan_max(emax, L.red[0][q]);
      esq += L.red[1][q];
      asq += L.red[2][q];
    }
    const int64_t bid = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    part[3 * bid + 0] = emax;
    part[3 * bid + 1] = esq;
    part[3 * bid + 2] = asq;
  }
}

// ---------------------------------------------------------------- host side
// Arena: [Bm FP64 m x r | A-operand terms | B-operand terms | scales | partials].
// Bm has been formed (FP64) at `Bm` by the caller; `part` receives the tile
// partials, whose count is returned through *nb.
cur_status residual_mp_launch(cur_ctx ctx, const float* A, int64_t m, int64_t n, int64_t lda, int r,
                              const double* Bm, const float* R, int prec, char* scratch, size_t scratch_bytes,
                              double* part, int64_t* nb) {
  hipStream_t s = ctx->stream;
  const int rp = (r + 31) / 32 * 32;
  const size_t esz = prec == CUR_PREC_BF16X3 ? 2 : 1;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t sa1 = al(esz * (size_t)m * rp), sb1 = al(esz * (size_t)n * rp);
  const size_t need = 2 * sa1 + 2 * sb1 + al(sizeof(float) * m) + al(sizeof(float) * n);
  if (need > scratch_bytes) {
    set_error("internal: residual scratch too small");
    return CUR_ERR_INTERNAL;
  }
  char* a1 = scratch;
  char* a2 = a1 + sa1;
  char* b1 = a2 + sa1;
  char* b2 = b1 + sb1;
  float* as = (float*)(b2 + sb1);
  float* bs = (float*)((char*)as + al(sizeof(float) * m));
  const int64_t gx = (n + kMT - 1) / kMT, gy = (m + kMT - 1) / kMT;
  if (gy > 65535) {
    set_error("matrix too tall for the residual grid");
    return CUR_ERR_ARG;
  }
  auto grid = [](int64_t work) { return (int)std::max<int64_t>(1, std::min<int64_t>((work + kThreads - 1) / kThreads, 65536)); };
  if (prec == CUR_PREC_BF16X3) {
    hipLaunchKernelGGL(k_split_rows_bf16, dim3(grid(m * rp)), dim3(kThreads), 0, s, Bm, m, r, rp, (__bf16*)a1,
                       (__bf16*)a2);
    hipLaunchKernelGGL(k_split_cols_bf16, dim3(grid(n * rp)), dim3(kThreads), 0, s, R, r, n, rp, (__bf16*)b1,
                       (__bf16*)b2);
    hipLaunchKernelGGL((k_resid_mp<CUR_PREC_BF16X3>), dim3((unsigned)gx, (unsigned)gy), dim3(kThreads), 0, s, A, m,
                       n, lda, rp, a1, a2, as, b1, b2, bs, part);
  } else {
    hipLaunchKernelGGL(k_split_rows_fp8, dim3(grid(64 * m)), dim3(kThreads), 0, s, Bm, m, r, rp, (uint8_t*)a1,
                       (uint8_t*)a2, as);
    hipLaunchKernelGGL(k_split_cols_fp8, dim3(grid(64 * n)), dim3(kThreads), 0, s, R, r, n, rp, (uint8_t*)b1,
                       (uint8_t*)b2, bs);
    hipLaunchKernelGGL((k_resid_mp<CUR_PREC_FP8>), dim3((unsigned)gx, (unsigned)gy), dim3(kThreads), 0, s, A, m, n,
                       lda, rp, a1, a2, as, b1, b2, bs, part);
  }
  CUR_HIP_CHECK(hipGetLastError());
  *nb = gx * gy;
  return CUR_OK;
}

size_t residual_mp_scratch(int64_t m, int64_t n, int r, int prec) {
  const int rp = (r + 31) / 32 * 32;
  const size_t esz = prec == CUR_PREC_BF16X3 ? 2 : 1;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  return 2 * al(esz * (size_t)m * rp) + 2 * al(esz * (size_t)n * rp) + al(sizeof(float) * m) +
         al(sizeof(float) * n) + 256;
}

int64_t residual_mp_tiles(int64_t m, int64_t n) { return ((n + kMT - 1) / kMT) * ((m + kMT - 1) / kMT); }

}  // namespace cur
