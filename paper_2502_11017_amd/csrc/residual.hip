// Residual of the CUR form (Thm 1 Chebyshev norm, Sec. 3.1 Frobenius error):
// E = A - (C U) R, reduced on the fly (E is never stored).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <type_traits>
#include <vector>

#include "cur_device.hpp"
#include "cur_internal.hpp"

namespace cur {

// One 128 x 128 tile of E per block on FP64 MFMA (v_mfma_f64_16x16x4f64).
// Wavefront w computes the 64 x 64 quadrant (w >> 1, w & 1) as 4 x 4 blocks of
// 16 x 16 (row group i, column group j).  Operand lanes: lane l supplies
// Bm[row 16i + (l & 15)][k + (l >> 4)] and R[k + (l >> 4)][col 16j + (l & 15)];
// the accumulator holds D[4v + (l >> 4)][l & 15] in element v.
// The block's rows of Bm and columns of R are staged in LDS, kKC values of k at
// a time, with coalesced loads (consecutive lanes read consecutive elements of
// a row; rows padded by one double, so that the fragment reads are free of
// bank conflicts).  k indices past the chunk are clamped to its last one when
// loading and the staged entries [kc, kc rounded up to 4) are zeroed, so the
// last MFMA step of a ragged chunk adds zeros.  The epilogue requests the A
// values of row group i + 1 before reducing group i.
// EDGE = false is the instance for tiles that lie wholly inside the matrix: no
// load carries a bounds test, which lets all of them issue back to back (a
// guarded load compiles to a branch with a wait for its data).  EDGE = true
// guards rows and columns (out-of-range entries are zero operands and zero A,
// so they contribute E = 0) and runs only over the ragged right and bottom
// strips.  Tile (tx0 + blockIdx.x, ty0 + blockIdx.y) writes
// part[3 (ty gx + tx)] = {max|E|, sum E^2, sum A^2} of the tile.
// The LDS footprint (~67 KB) allows two blocks per CU.
constexpr int kRT = 128, kKC = 32;
typedef double f64x4 __attribute__((ext_vector_type(4)));

struct ResidLds {
  double B[kRT][kKC + 1];   // Bm rows of the block, k chunk
  double R[kKC][kRT + 1];   // R columns of the block, k chunk
  double red[3][kThreads / 64];
};

template <typename T, bool EDGE>
__global__ __launch_bounds__(kThreads, 2) void k_resid_mfma(const T* __restrict__ A, int64_t m, int64_t n,
                                                         int64_t lda, int r, const double* __restrict__ Bm,
                                                         const T* __restrict__ R, double* part, int tx0, int ty0,
                                                         int gxall) {
  __shared__ ResidLds L;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int tx = tx0 + blockIdx.x, ty = ty0 + blockIdx.y;
  const int64_t r0 = (int64_t)ty * kRT, c0 = (int64_t)tx * kRT;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;  // quadrant inside the block
  f64x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  // staging: element q of thread t is Bm[r0 + 8 q + (t >> 5)][k0 + (t & 31)] and
  // R[k0 + 2 q + (t >> 7)][c0 + (t & 127)]
  const int64_t brow = r0 + (tid >> 5), rcol = c0 + (tid & 127);
  const double* bp = Bm + brow * r;
  const T* rp = R + rcol;
  for (int k0 = 0; k0 < r; k0 += kKC) {
    const int kc = min(kKC, r - k0);
    double vb[16];
    T vr[16];
    const int bk = k0 + min(tid & 31, kc - 1);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if (EDGE) vb[q] = brow + 8 * q < m ? bp[(int64_t)8 * q * r + bk] : 0.0;
      else vb[q] = bp[(int64_t)8 * q * r + bk];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int64_t off = (int64_t)(k0 + min(2 * q + (tid >> 7), kc - 1)) * n;
      if (EDGE) vr[q] = rcol < n ? rp[off] : (T)0;
      else vr[q] = rp[off];
    }
    __syncthreads();  // the previous chunk's fragments have been read
#pragma unroll
    for (int q = 0; q < 16; ++q) L.B[8 * q + (tid >> 5)][tid & 31] = vb[q];
#pragma unroll
    for (int q = 0; q < 16; ++q) L.R[2 * q + (tid >> 7)][tid & 127] = (double)vr[q];
    __syncthreads();
    if (kc & 3) {  // ragged chunk: zero the staged k entries [kc, kc4)
      const int kc4 = (kc + 3) & ~3;
      for (int e = tid; e < kRT * 4; e += kThreads) {
        const int kk = kc + (e & 3);
        if (kk < kc4) {
          L.B[e >> 2][kk] = 0.0;
          L.R[kk][e >> 2] = 0.0;
        }
      }
      __syncthreads();
    }
    for (int k = 0; k < kc; k += 4) {
      double af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = L.B[wr + 16 * i + lr][k + lk];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = L.R[k + lk][wc + 16 * j + lr];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  }
  // epilogue: A rows r0 + wr + 16 i + 4 v + lk, columns c0 + wc + 16 j + lr
  const int64_t arow = r0 + wr + lk, acol = c0 + wc + lr;
  const T* ap = A + arow * lda + acol;
  auto load_a = [&](int i, T (&dst)[4][4]) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t off = (int64_t)(16 * i + 4 * v) * lda + 16 * j;
        if (EDGE) dst[j][v] = (arow + 16 * i + 4 * v < m && acol + 16 * j < n) ? ap[off] : (T)0;
        else dst[j][v] = ap[off];
      }
  };
  double emax = 0.0, esq = 0.0, asq = 0.0;
  auto reduce = [&](int i, const T (&src)[4][4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double av = (double)src[j][v];
        const double e = av - acc[i][j][v];
        emax = nan_max(emax, fabs(e));
        esq = fma(e, e, esq);
        asq = fma(av, av, asq);
      }
  };
  T pa0[4][4], pa1[4][4];
  load_a(0, pa0);
  reduce(0, pa0);
  load_a(1, pa1);
  load_a(2, pa0);
  reduce(1, pa1);
  load_a(3, pa1);
  reduce(2, pa0);
  reduce(3, pa1);
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
    const int64_t bid = (int64_t)ty * gxall + tx;
    part[3 * bid + 0] = emax;
    part[3 * bid + 1] = esq;
    part[3 * bid + 2] = asq;
  }
}

// Bm = C U on FP64 MFMA (C m x kd, U kd x r; kd = r for the square cross, c
// for a rectangular one), one 128-row x 128-column tile of Bm per block
// (r <= 128 columns, so one column tile), the same operand staging and lane
// layout as k_resid_mfma with C as the row operand and U as the column
// operand.  Loads take clamped indices and carry no bounds test: rows past m
// and columns past r only feed outputs that are not stored, and the staged k
// entries [kc, kc rounded up to 4) of a ragged chunk are zeroed.
template <typename T>
__global__ __launch_bounds__(kThreads, 2) void k_cu_mfma(const T* __restrict__ C, const double* __restrict__ U,
                                                         int64_t m, int kd, int r, double* __restrict__ Bm) {
  __shared__ ResidLds L;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * kRT;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  f64x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  // staging: element q of thread t is C[r0 + 8 q + (t >> 5)][k0 + (t & 31)] and
  // U[k0 + 2 q + (t >> 7)][t & 127]
  const int ucol = min(tid & 127, r - 1);
  for (int k0 = 0; k0 < kd; k0 += kKC) {
    const int kc = min(kKC, kd - k0);
    const int bk = k0 + min(tid & 31, kc - 1);
    double vb[16], vr[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) vb[q] = (double)C[min(r0 + 8 * q + (tid >> 5), m - 1) * kd + bk];
#pragma unroll
    for (int q = 0; q < 16; ++q) vr[q] = U[(int64_t)(k0 + min(2 * q + (tid >> 7), kc - 1)) * r + ucol];
    __syncthreads();  // the previous chunk's fragments have been read
#pragma unroll
    for (int q = 0; q < 16; ++q) L.B[8 * q + (tid >> 5)][tid & 31] = vb[q];
#pragma unroll
    for (int q = 0; q < 16; ++q) L.R[2 * q + (tid >> 7)][tid & 127] = vr[q];
    __syncthreads();
    if (kc & 3) {  // ragged chunk: zero the staged k entries [kc, kc4)
      const int kc4 = (kc + 3) & ~3;
      for (int e = tid; e < kRT * 4; e += kThreads) {
        const int kk = kc + (e & 3);
        if (kk < kc4) {
          L.B[e >> 2][kk] = 0.0;
          L.R[kk][e >> 2] = 0.0;
        }
      }
      __syncthreads();
    }
    for (int k = 0; k < kc; k += 4) {
      double af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = L.B[wr + 16 * i + lr][k + lk];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = L.R[k + lk][wc + 16 * j + lr];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + wr + 16 * i + 4 * v + lk;
      if (row >= m) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = wc + 16 * j + lr;
        if (col < r) Bm[row * r + col] = acc[i][j][v];
      }
    }
}

// Deterministic reduction of tile partials {max, sum, sum} (fixed order):
// block g reduces entries [g chunk, (g + 1) chunk) into out[3 g ..].  Run once
// with many blocks over the tile partials and once with one block over theirs.
constexpr int kRedBlocks = 1024;
__global__ __launch_bounds__(kThreads) void k_resid_reduce(const double* part, int64_t nb, int64_t chunk,
                                                           double* out) {
  const int64_t b0 = (int64_t)blockIdx.x * chunk, b1 = min(nb, b0 + chunk);
  double emax = 0.0, esq = 0.0, asq = 0.0;
  for (int64_t b = b0 + threadIdx.x; b < b1; b += kThreads) {
    emax = nan_max(emax, part[3 * b]);
    esq += part[3 * b + 1];
    asq += part[3 * b + 2];
  }
  __shared__ double s[3][kThreads];
  s[0][threadIdx.x] = emax;
  s[1][threadIdx.x] = esq;
  s[2][threadIdx.x] = asq;
  __syncthreads();
  for (int w = kThreads / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s[0][threadIdx.x] = nan_max(s[0][threadIdx.x], s[0][threadIdx.x + w]);
      s[1][threadIdx.x] += s[1][threadIdx.x + w];
      s[2][threadIdx.x] += s[2][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[3 * blockIdx.x + 0] = s[0][0];
    out[3 * blockIdx.x + 1] = s[1][0];
    out[3 * blockIdx.x + 2] = s[2][0];
  }
}

// Scratch of one residual call: [Bm FP64 m x r (native form only) | tile
// partials | final sums | reduced-precision operands].
static size_t residual_need(int64_t m, int64_t n, int r, int prec) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const bool mp = prec != CUR_PREC_NATIVE;
  const int64_t nb = mp ? residual_mp_tiles(m, n) : ((n + kRT - 1) / kRT) * ((m + kRT - 1) / kRT);
  return (mp ? 0 : al(sizeof(double) * m * r)) + al(sizeof(double) * 3 * nb) + al(sizeof(double) * 3 * kRedBlocks) +
         256 + (mp ? residual_mp_scratch(m, n, r, prec) : 0);
}

// The residual with its temporaries at `base` (residual_need bytes).
template <typename T>
static cur_status residual_core(cur_ctx ctx, const T* A, int64_t m, int64_t n, int64_t lda, int r,
                                const T* C, const double* U, const T* R, int prec, double* cheb,
                                double* fro_rel, char* base, int kd = 0) {
  if (kd == 0) kd = r;  // columns of C: r, or c for a rectangular cross (native form only)
  hipStream_t s = ctx->stream;
  const bool mp = prec != CUR_PREC_NATIVE;  // FP32 input only (checked by the API)
  const int64_t gx = (n + kRT - 1) / kRT, gy = (m + kRT - 1) / kRT;
  const int64_t nb = mp ? residual_mp_tiles(m, n) : gx * gy;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t sbm = mp ? 0 : al(sizeof(double) * m * r), spart = al(sizeof(double) * 3 * nb);
  const size_t smp = mp ? residual_mp_scratch(m, n, r, prec) : 0;
  const size_t smid = al(sizeof(double) * 3 * kRedBlocks);
  double* Bm = (double*)base;
  double* part = (double*)(base + sbm);
  double* mid = (double*)(base + sbm + spart);
  double* out = (double*)(base + sbm + spart + smid);
  const int64_t gm = (m + kRT - 1) / kRT;
  if (gm > 0x7fffffff) {
    set_error("matrix too tall for the residual grid");
    return CUR_ERR_ARG;
  }
  int64_t nparts = nb;
  if (mp) {
    if constexpr (std::is_same<T, float>::value) {
      cur_status st = residual_mp_launch(ctx, A, m, n, lda, r, C, U, R, prec, base + sbm + spart + smid + 256, smp,
                                         part, &nparts);
      if (st != CUR_OK) return st;
    } else {
      set_error("reduced-precision residual needs FP32 input");
      return CUR_ERR_ARG;
    }
  } else {
    if (gy > 65535) {
      set_error("matrix too tall for the residual grid");
      return CUR_ERR_ARG;
    }
    hipLaunchKernelGGL((k_cu_mfma<T>), dim3((unsigned)gm), dim3(kThreads), 0, s, C, U, m, kd, r, Bm);
    // interior tiles without bounds tests, then the ragged right strip (corner
    // included) and bottom strip with them
    const int nf = (int)(n / kRT), mf = (int)(m / kRT);
    if (nf > 0 && mf > 0)
      hipLaunchKernelGGL((k_resid_mfma<T, false>), dim3((unsigned)nf, (unsigned)mf), dim3(kThreads), 0, s, A, m,
                         n, lda, r, Bm, R, part, 0, 0, (int)gx);
    if (n % kRT)
      hipLaunchKernelGGL((k_resid_mfma<T, true>), dim3(1u, (unsigned)gy), dim3(kThreads), 0, s, A, m, n, lda, r,
                         Bm, R, part, nf, 0, (int)gx);
    if (m % kRT && nf > 0)
      hipLaunchKernelGGL((k_resid_mfma<T, true>), dim3((unsigned)nf, 1u), dim3(kThreads), 0, s, A, m, n, lda, r,
                         Bm, R, part, 0, mf, (int)gx);
  }
  const int64_t g = std::max<int64_t>(1, std::min<int64_t>(kRedBlocks, (nparts + kThreads - 1) / kThreads));
  const int64_t chunk = (nparts + g - 1) / g;
  hipLaunchKernelGGL(k_resid_reduce, dim3((unsigned)g), dim3(kThreads), 0, s, part, nparts, chunk, mid);
  hipLaunchKernelGGL(k_resid_reduce, dim3(1), dim3(kThreads), 0, s, mid, g, g, out);
  CUR_HIP_CHECK(hipGetLastError());
  double h[3];
  CUR_HIP_CHECK(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s));
  CUR_HIP_CHECK(hipStreamSynchronize(s));
  *cheb = h[0];
  if (fro_rel) *fro_rel = h[2] > 0.0 ? std::sqrt(h[1]) / std::sqrt(h[2]) : 0.0;
  if (!std::isfinite(h[0])) {
    set_error("A - C U R has a NaN or infinite entry");
    return CUR_ERR_NONFINITE;
  }
  return CUR_OK;
}

template <typename T>
static cur_status residual_impl(cur_ctx ctx, const T* A, int64_t m, int64_t n, int64_t lda, int r,
                                const T* C, const double* U, const T* R, int prec, double* cheb,
                                double* fro_rel) {
  cur_status st = ensure_arena(ctx, residual_need(m, n, r, prec));
  if (st != CUR_OK) return st;
  return residual_core<T>(ctx, A, m, n, lda, r, C, U, R, prec, cheb, fro_rel, (char*)ctx->arena);
}

// ---- the entry point that allocates nothing ----
// Its temporaries live in this fixed device array (one copy per GPU, held from
// module load until the process ends).  Host code never passes `scratch`
// itself (in host code that name is a stand-in, not a device address): the
// device address of each GPU's copy is looked up once per device, with that
// device current, by noalloc_init (called by cur_create) and kept in
// g_noalloc_ptr.
static __device__ __align__(256) unsigned char scratch[CUR_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static void* g_noalloc_ptr[kMaxDevices];
static std::mutex g_noalloc_mu;

cur_status noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device index beyond the library's per-device table");
    return CUR_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return CUR_OK;
  void* p = nullptr;
  CUR_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) {
    set_error("hipGetSymbolAddress returned NULL for the no-allocation scratch");
    return CUR_ERR_DEVICE;
  }
  g_noalloc_ptr[device] = p;
  return CUR_OK;
}

size_t residual_noalloc_need(int64_t m, int64_t n, int r, int prec) { return residual_need(m, n, r, prec); }

cur_status residual_noalloc_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n, int64_t lda,
                                     int r, const void* C, const double* U, const void* R, int prec, double* cheb,
                                     double* fro_rel) {
  void* p;
  {
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    p = (ctx->device >= 0 && ctx->device < kMaxDevices) ? g_noalloc_ptr[ctx->device] : nullptr;
  }
  if (!p) {
    set_error("no-allocation scratch not set up for this device (cur_create did not complete)");
    return CUR_ERR_DEVICE;
  }
  if (dtype == CUR_F64)
    return residual_core<double>(ctx, (const double*)A, m, n, lda, r, (const double*)C, U, (const double*)R, prec,
                                 cheb, fro_rel, (char*)p);
  return residual_core<float>(ctx, (const float*)A, m, n, lda, r, (const float*)C, U, (const float*)R, prec, cheb,
                              fro_rel, (char*)p);
}

// The native residual of a rectangular cross: C m x c, U c x r, R r x n.
cur_status residual_rect_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n, int64_t lda,
                                  int r, int c, const void* C, const double* U, const void* R, double* cheb,
                                  double* fro_rel) {
  cur_status st = ensure_arena(ctx, residual_need(m, n, r, CUR_PREC_NATIVE));
  if (st != CUR_OK) return st;
  if (dtype == CUR_F64)
    return residual_core<double>(ctx, (const double*)A, m, n, lda, r, (const double*)C, U, (const double*)R,
                                 CUR_PREC_NATIVE, cheb, fro_rel, (char*)ctx->arena, c);
  return residual_core<float>(ctx, (const float*)A, m, n, lda, r, (const float*)C, U, (const float*)R,
                              CUR_PREC_NATIVE, cheb, fro_rel, (char*)ctx->arena, c);
}

cur_status residual_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n, int64_t lda,
                             int r, const void* C, const double* U, const void* R, int prec, double* cheb,
                             double* fro_rel) {
  if (dtype == CUR_F64)
    return residual_impl<double>(ctx, (const double*)A, m, n, lda, r, (const double*)C, U,
                                 (const double*)R, prec, cheb, fro_rel);
  return residual_impl<float>(ctx, (const float*)A, m, n, lda, r, (const float*)C, U, (const float*)R,
                              prec, cheb, fro_rel);
}

}  // namespace cur
