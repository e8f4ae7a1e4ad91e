// CUR assembly (Sec. 1.1): C = A(:,J), R = A(I,:), U = A(I,J)^+.
#include <hip/hip_runtime.h>

#include <vector>

#include "cur_device.hpp"
#include "cur_internal.hpp"

namespace cur {

template <typename T>
__global__ __launch_bounds__(kThreads) void k_gather_C(const T* __restrict__ A, int64_t m, int64_t lda,
                                                       int r, const int64_t* __restrict__ J, T* C) {
  const int64_t total = m * r;
  for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * kThreads) {
    const int64_t i = idx / r;
    const int k = (int)(idx - i * r);
    C[idx] = A[i * lda + J[k]];
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_gather_R(const T* __restrict__ A, int64_t n, int64_t lda,
                                                       const int64_t* __restrict__ I, T* R) {
  const int k = blockIdx.y;
  const T* src = A + I[k] * lda;
  T* dst = R + (int64_t)k * n;
  for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < n; j += (int64_t)gridDim.x * kThreads)
    dst[j] = src[j];
}

template <int RMAX, bool REG = (RMAX <= 64)>
struct AsmLu : LuScratch {};
template <int RMAX>
struct AsmLu<RMAX, false> {};

template <int RMAX>
struct AsmLds {
  static constexpr int CH = RMAX <= 64 ? RMAX : 16;
  double A[RMAX * RMAX];
  double B[RMAX * CH];
  double lk[RMAX];
  int perm[RMAX];
  int spiv;
  int pinv;
  double cs[2];
  int rot;
  AsmLu<RMAX> lu;
};

// U = A(I,J)^{-1} by LU with partial pivoting, or the Jacobi pseudo-inverse
// when a pivot is zero or min|u_kk|/max|u_kk| < r 2^-52.  W, V: r x r global
// scratch for the Jacobi path.  flag[0] <- 1 if the pseudo-inverse was used.
template <typename T, int RMAX>
__global__ __launch_bounds__(kThreads) void k_assemble_U(const T* __restrict__ A, int64_t lda, int r,
                                                         const int64_t* I, const int64_t* J, double* U,
                                                         double* W, double* V, double* sg, int* flag) {
  __shared__ AsmLds<RMAX> L;
  const int tid = threadIdx.x;
  // U(k,k) of the factorization: register LU for r <= 64, LDS LU otherwise
  [[maybe_unused]] LuRegs<(RMAX <= 64 ? RMAX : 64)> R;
  bool ok;
  const double* diag;
  int dstride;
  if constexpr (RMAX <= 64) {
    const GPtr<const T> Ag = (GPtr<const T>)A;
    const GPtr<const int64_t> Ig = (GPtr<const int64_t>)I, Jg = (GPtr<const int64_t>)J;
    ok = lu_fwd_reg<RMAX>([&](int p, int c) { return (double)Ag[Ig[p] * lda + Jg[c]]; }, r, R, L.B, L.lu);
    diag = L.lu.diag;
    dstride = 1;
  } else {
    for (int idx = tid; idx < r * r; idx += kThreads) {
      const int a = idx / r, b = idx % r;
      L.A[idx] = (double)A[I[a] * lda + J[b]];
    }
    __syncthreads();
    ok = block_gepp(L.A, r, L.perm, L.lk, &L.spiv);
    diag = L.A;
    dstride = r + 1;
  }
  if (tid == 0) {
    int use_pinv = 1;
    if (ok) {
      double umin = HUGE_VAL, umax = 0.0;
      for (int k = 0; k < r; ++k) {
        const double u = fabs(diag[k * dstride]);
        umin = fmin(umin, u);
        umax = fmax(umax, u);
      }
      use_pinv = (umin / umax < (double)r * 0x1p-52) ? 1 : 0;
    }
    L.pinv = use_pinv;
    flag[0] = use_pinv;
  }
  __syncthreads();
  if (!L.pinv) {
    if constexpr (RMAX <= 64)
      lu_back_reg<RMAX>(r, R, L.B, L.lu, U, nullptr);
    else
      block_lu_inverse<AsmLds<RMAX>::CH>(L.A, L.perm, r, L.B, U);
    return;
  }
  // ---- one-sided Jacobi: W = G V with orthogonal columns (cyclic pairs, <= 60 sweeps)
  for (int idx = tid; idx < r * r; idx += kThreads) {
    const int a = idx / r, b = idx % r;
    W[idx] = (double)A[I[a] * lda + J[b]];
    V[idx] = (a == b) ? 1.0 : 0.0;
  }
  block_global_sync();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) L.rot = 0;
    __syncthreads();
    for (int p = 0; p < r - 1; ++p)
      for (int q = p + 1; q < r; ++q) {
        if (tid == 0) {
          double al = 0.0, be = 0.0, ga = 0.0;
          for (int i = 0; i < r; ++i) {
            const double wp = W[i * r + p], wq = W[i * r + q];
            al = fma(wp, wp, al);
            be = fma(wq, wq, be);
            ga = fma(wp, wq, ga);
          }
          L.cs[0] = 0.0;
          L.cs[1] = 0.0;
          if (!(ga == 0.0 || fabs(ga) <= 0x1p-52 * sqrt(al * be))) {
            const double zeta = (be - al) / (2.0 * ga);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + t * t);
            L.cs[0] = c;
            L.cs[1] = c * t;
            L.rot = 1;
          }
        }
        __syncthreads();
        const double c = L.cs[0], s = L.cs[1];
        if (c != 0.0) {
          for (int i = tid; i < r; i += kThreads) {
            const double wp = W[i * r + p], wq = W[i * r + q];
            W[i * r + p] = c * wp - s * wq;
            W[i * r + q] = s * wp + c * wq;
            const double vp = V[i * r + p], vq = V[i * r + q];
            V[i * r + p] = c * vp - s * vq;
            V[i * r + q] = s * vp + c * vq;
          }
        }
        block_global_sync();
      }
    if (!L.rot) break;
  }
  if (tid == 0) {
    double smax = 0.0;
    for (int j = 0; j < r; ++j) {
      double s = 0.0;
      for (int i = 0; i < r; ++i) s = fma(W[i * r + j], W[i * r + j], s);
      sg[j] = sqrt(s);
      smax = fmax(smax, sg[j]);
    }
    L.cs[0] = (double)r * 0x1p-52 * smax;
  }
  block_global_sync();
  const double cut = L.cs[0];
  for (int idx = tid; idx < r * r; idx += kThreads) {
    const int a = idx / r, b = idx % r;
    double s = 0.0;
    for (int j = 0; j < r; ++j) {
      if (!(sg[j] > cut)) continue;
      s = fma(V[a * r + j], W[b * r + j] / (sg[j] * sg[j]), s);
    }
    U[idx] = s;
  }
}

template <typename T>
static cur_status assemble_impl(cur_ctx ctx, const T* A, int64_t m, int64_t n, int64_t lda, int r,
                                const int64_t* I, const int64_t* J, T* C, double* U, T* R) {
  hipStream_t s = ctx->stream;
  const size_t scratch = 3 * (size_t)r * r * sizeof(double) + 4096;
  cur_status st = ensure_arena(ctx, scratch);
  if (st != CUR_OK) return st;
  char* base = (char*)ctx->arena;
  int* flag = (int*)base;
  double* W = (double*)(base + 4096);
  double* V = W + (size_t)r * r;
  double* sg = V + (size_t)r * r;
  const int gc = (int)std::min<int64_t>((m * r + kThreads - 1) / kThreads, 8192);
  hipLaunchKernelGGL((k_gather_C<T>), dim3(std::max(gc, 1)), dim3(kThreads), 0, s, A, m, lda, r, J, C);
  const int gr = (int)std::min<int64_t>((n + kThreads - 1) / kThreads, 1024);
  hipLaunchKernelGGL((k_gather_R<T>), dim3(std::max(gr, 1), r), dim3(kThreads), 0, s, A, n, lda, I, R);
  if (r <= 32)
    hipLaunchKernelGGL((k_assemble_U<T, 32>), dim3(1), dim3(kThreads), 0, s, A, lda, r, I, J, U, W, V, sg, flag);
  else if (r <= 64)
    hipLaunchKernelGGL((k_assemble_U<T, 64>), dim3(1), dim3(kThreads), 0, s, A, lda, r, I, J, U, W, V, sg, flag);
  else
    hipLaunchKernelGGL((k_assemble_U<T, 128>), dim3(1), dim3(kThreads), 0, s, A, lda, r, I, J, U, W, V, sg, flag);
  CUR_HIP_CHECK(hipGetLastError());
  int hflag = 0;
  CUR_HIP_CHECK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  CUR_HIP_CHECK(hipStreamSynchronize(s));
  ctx->last_pinv = hflag;
  return CUR_OK;
}

// ---------------------------------------------------------------- rectangular cross
// U = A(I,J)^+ for r rows and c columns (c x r, row-major), one block: the
// one-sided Jacobi pseudo-inverse on the taller of G = A(I,J) and G^T
// (p x q, p >= q, p <= 128, q <= 64), W and V held in LDS.  Cyclic sweeps over
// column pairs (a < b) in order; thread 0 forms the pair's three sums over
// the p rows ascending (one fma per term) and the rotation, the block
// rotates the rows of W and V; sigma_j = ||W(:,j)||, G^+ = V diag(1/sigma^2)
// W^T over sigma_j > p 2^-52 sigma_max.  These are the oracle's operations
// in its order, so U is reproduced bit for bit.
constexpr int kPinvP = 128, kPinvQ = 64;
struct PinvLds {
  double W[kPinvP * kPinvQ];
  double V[kPinvQ * kPinvQ];
  double sg[kPinvQ];
  double cs[3];
  int rot;
};

template <typename T>
__global__ __launch_bounds__(kThreads) void k_pinv_rect(const T* __restrict__ A, int64_t lda, int r, int c,
                                                        const int64_t* __restrict__ I, const int64_t* __restrict__ J,
                                                        double* __restrict__ U) {
  __shared__ PinvLds L;
  const int tid = threadIdx.x;
  const bool tall = r >= c;  // G (r x c) itself, else its transpose
  const int p = tall ? r : c, q = tall ? c : r;
  for (int idx = tid; idx < p * q; idx += kThreads) {
    const int i = idx / q, j = idx % q;  // W(i, j) = G(i, j), or G(j, i)
    L.W[idx] = tall ? (double)A[I[i] * lda + J[j]] : (double)A[I[j] * lda + J[i]];
  }
  for (int idx = tid; idx < q * q; idx += kThreads) L.V[idx] = (idx / q == idx % q) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) L.rot = 0;
    __syncthreads();
    for (int a = 0; a < q - 1; ++a)
      for (int b = a + 1; b < q; ++b) {
        if (tid == 0) {
          double al = 0.0, be = 0.0, ga = 0.0;
          for (int i = 0; i < p; ++i) {
            const double wa = L.W[i * q + a], wb = L.W[i * q + b];
            al = fma(wa, wa, al);
            be = fma(wb, wb, be);
            ga = fma(wa, wb, ga);
          }
          L.cs[0] = 0.0;
          L.cs[1] = 0.0;
          if (!(ga == 0.0 || fabs(ga) <= 0x1p-52 * sqrt(al * be))) {
            const double zeta = (be - al) / (2.0 * ga);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cc = 1.0 / sqrt(1.0 + t * t);
            L.cs[0] = cc;
            L.cs[1] = cc * t;
            L.rot = 1;
          }
        }
        __syncthreads();
        const double cc = L.cs[0], sn = L.cs[1];
        if (cc != 0.0) {
          for (int i = tid; i < p; i += kThreads) {
            const double wa = L.W[i * q + a], wb = L.W[i * q + b];
            L.W[i * q + a] = cc * wa - sn * wb;
            L.W[i * q + b] = sn * wa + cc * wb;
          }
          for (int i = tid; i < q; i += kThreads) {
            const double va = L.V[i * q + a], vb = L.V[i * q + b];
            L.V[i * q + a] = cc * va - sn * vb;
            L.V[i * q + b] = sn * va + cc * vb;
          }
        }
        __syncthreads();
      }
    const int rot = L.rot;
    __syncthreads();  // every wavefront has read the flag before it is reset
    if (!rot) break;
  }
  if (tid == 0) {
    double smax = 0.0;
    for (int j = 0; j < q; ++j) {
      double sum = 0.0;
      for (int i = 0; i < p; ++i) sum = fma(L.W[i * q + j], L.W[i * q + j], sum);
      L.sg[j] = sqrt(sum);
      smax = fmax(smax, L.sg[j]);
    }
    L.cs[2] = (double)p * 0x1p-52 * smax;
  }
  __syncthreads();
  const double cut = L.cs[2];
  // P = W^+ of the working orientation (q x p); U = P (tall) or P^T
  for (int idx = tid; idx < q * p; idx += kThreads) {
    const int a = idx / p, b = idx % p;
    double sum = 0.0;
    for (int j = 0; j < q; ++j) {
      if (!(L.sg[j] > cut)) continue;
      sum = fma(L.V[a * q + j], L.W[b * q + j] / (L.sg[j] * L.sg[j]), sum);
    }
    if (tall) U[(int64_t)a * r + b] = sum;  // U is c x r = q x p
    else U[(int64_t)b * r + a] = sum;       // U(b, a): c = p rows, r = q columns
  }
}

template <typename T>
static cur_status assemble_rect_impl(cur_ctx ctx, const T* A, int64_t m, int64_t n, int64_t lda, int r, int c,
                                     const int64_t* I, const int64_t* J, T* C, double* U, T* R) {
  hipStream_t s = ctx->stream;
  const int gc = (int)std::min<int64_t>((m * c + kThreads - 1) / kThreads, 8192);
  hipLaunchKernelGGL((k_gather_C<T>), dim3(std::max(gc, 1)), dim3(kThreads), 0, s, A, m, lda, c, J, C);
  const int gr = (int)std::min<int64_t>((n + kThreads - 1) / kThreads, 1024);
  hipLaunchKernelGGL((k_gather_R<T>), dim3(std::max(gr, 1), r), dim3(kThreads), 0, s, A, n, lda, I, R);
  hipLaunchKernelGGL((k_pinv_rect<T>), dim3(1), dim3(kThreads), 0, s, A, lda, r, c, I, J, U);
  CUR_HIP_CHECK(hipGetLastError());
  CUR_HIP_CHECK(hipStreamSynchronize(s));
  return CUR_OK;
}

cur_status assemble_rect_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n, int64_t lda,
                                  int r, int c, const int64_t* I, const int64_t* J, void* C, double* U, void* R) {
  if (dtype == CUR_F64)
    return assemble_rect_impl<double>(ctx, (const double*)A, m, n, lda, r, c, I, J, (double*)C, U, (double*)R);
  return assemble_rect_impl<float>(ctx, (const float*)A, m, n, lda, r, c, I, J, (float*)C, U, (float*)R);
}

cur_status assemble_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n, int64_t lda,
                             int r, const int64_t* I, const int64_t* J, void* C, double* U, void* R) {
  if (dtype == CUR_F64)
    return assemble_impl<double>(ctx, (const double*)A, m, n, lda, r, I, J, (double*)C, U, (double*)R);
  return assemble_impl<float>(ctx, (const float*)A, m, n, lda, r, I, J, (float*)C, U, (float*)R);
}

}  // namespace cur
