// Residual of the CUR form (Thm 1 Chebyshev norm, Sec. 3.1 Frobenius error):
// E = A - (C U) R, reduced on the fly (E is never stored).
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "cur_device.hpp"
#include "cur_internal.hpp"

namespace cur {

// Bm = C U (m x r, FP64), sums over l ascending.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cu(const T* __restrict__ C, const double* __restrict__ U,
                                                 int64_t m, int r, double* __restrict__ Bm) {
  const int64_t total = m * r;
  for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * kThreads) {
    const int64_t i = idx / r;
    const int k = (int)(idx - i * r);
    const T* c = C + i * r;
    double s = 0.0;
    for (int l = 0; l < r; ++l) s = fma((double)c[l], U[l * r + k], s);
    Bm[idx] = s;
  }
}

// One 64 x 64 tile of E per block; each thread owns a 4 x 4 sub-grid with
// stride 16 (rows ty + 16a, columns tx + 16b) so that A is read coalesced.
// part[3*block] = {max|E|, sum E^2, sum A^2} of the tile.
constexpr int kRT = 64, kKC = 32;
template <typename T>
__global__ __launch_bounds__(kThreads) void k_resid_f64(const T* __restrict__ A, int64_t m, int64_t n,
                                                        int64_t lda, int r, const double* __restrict__ Bm,
                                                        const T* __restrict__ R, double* part) {
  __shared__ double sB[kRT][kKC + 1];
  __shared__ double sR[kKC][kRT + 1];
  __shared__ double red[3][kThreads / 64];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int64_t i0 = (int64_t)blockIdx.y * kRT, j0 = (int64_t)blockIdx.x * kRT;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int k0 = 0; k0 < r; k0 += kKC) {
    const int kc = min(kKC, r - k0);
    for (int idx = tid; idx < kRT * kKC; idx += kThreads) {
      const int ii = idx / kKC, kk = idx % kKC;
      const int64_t i = i0 + ii;
      sB[ii][kk] = (i < m && kk < kc) ? Bm[i * r + k0 + kk] : 0.0;
    }
    for (int idx = tid; idx < kKC * kRT; idx += kThreads) {
      const int kk = idx / kRT, jj = idx % kRT;
      const int64_t j = j0 + jj;
      sR[kk][jj] = (j < n && kk < kc) ? (double)R[(int64_t)(k0 + kk) * n + j] : 0.0;
    }
    __syncthreads();
    for (int kk = 0; kk < kc; ++kk) {
      double bv[4], rv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) bv[a] = sB[ty + 16 * a][kk];
#pragma unroll
      for (int b = 0; b < 4; ++b) rv[b] = sR[kk][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(bv[a], rv[b], acc[a][b]);
    }
    __syncthreads();
  }
  double emax = 0.0, esq = 0.0, asq = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t i = i0 + ty + 16 * a;
    if (i >= m) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t j = j0 + tx + 16 * b;
      if (j >= n) continue;
      const double av = (double)A[i * lda + j];
      const double e = av - acc[a][b];
      emax = fmax(emax, fabs(e));
      esq = fma(e, e, esq);
      asq = fma(av, av, asq);
    }
  }
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
    emax = fmax(emax, __shfl_xor(emax, s, 64));
    esq += __shfl_xor(esq, s, 64);
    asq += __shfl_xor(asq, s, 64);
  }
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = emax;
    red[1][tid >> 6] = esq;
    red[2][tid >> 6] = asq;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < kThreads / 64; ++w) {
      emax = fmax(emax, red[0][w]);
      esq += red[1][w];
      asq += red[2][w];
    }
    const int64_t bid = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    part[3 * bid + 0] = emax;
    part[3 * bid + 1] = esq;
    part[3 * bid + 2] = asq;
  }
}

// Deterministic final reduction of the tile partials (fixed order).
__global__ __launch_bounds__(kThreads) void k_resid_final(const double* part, int64_t nb, double* out) {
  double emax = 0.0, esq = 0.0, asq = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += kThreads) {
    emax = fmax(emax, part[3 * b]);
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
      s[0][threadIdx.x] = fmax(s[0][threadIdx.x], s[0][threadIdx.x + w]);
      s[1][threadIdx.x] += s[1][threadIdx.x + w];
      s[2][threadIdx.x] += s[2][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s[0][0];
    out[1] = s[1][0];
    out[2] = s[2][0];
  }
}

template <typename T>
static cur_status residual_impl(cur_ctx ctx, const T* A, int64_t m, int64_t n, int64_t lda, int r,
                                const T* C, const double* U, const T* R, int prec, double* cheb,
                                double* fro_rel) {
  hipStream_t s = ctx->stream;
  (void)prec;
  const int64_t gx = (n + kRT - 1) / kRT, gy = (m + kRT - 1) / kRT;
  const int64_t nb = gx * gy;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t bytes = al(sizeof(double) * m * r) + al(sizeof(double) * 3 * nb) + 256;
  cur_status st = ensure_arena(ctx, bytes);
  if (st != CUR_OK) return st;
  char* base = (char*)ctx->arena;
  double* Bm = (double*)base;
  double* part = (double*)(base + al(sizeof(double) * m * r));
  double* out = (double*)(base + al(sizeof(double) * m * r) + al(sizeof(double) * 3 * nb));
  const int g1 = (int)std::min<int64_t>((m * r + kThreads - 1) / kThreads, 16384);
  hipLaunchKernelGGL((k_cu<T>), dim3(std::max(g1, 1)), dim3(kThreads), 0, s, C, U, m, r, Bm);
  if (gy > 65535) {
    set_error("matrix too tall for the residual grid");
    return CUR_ERR_ARG;
  }
  hipLaunchKernelGGL((k_resid_f64<T>), dim3((unsigned)gx, (unsigned)gy), dim3(kThreads), 0, s, A, m, n,
                     lda, r, Bm, R, part);
  hipLaunchKernelGGL(k_resid_final, dim3(1), dim3(kThreads), 0, s, part, nb, out);
  CUR_HIP_CHECK(hipGetLastError());
  double h[3];
  CUR_HIP_CHECK(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s));
  CUR_HIP_CHECK(hipStreamSynchronize(s));
  *cheb = h[0];
  if (fro_rel) *fro_rel = h[2] > 0.0 ? std::sqrt(h[1]) / std::sqrt(h[2]) : 0.0;
  return CUR_OK;
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
