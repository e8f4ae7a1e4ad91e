// Learned candidate proposal for the leaves of the selection tree.
//
// A small MLP scores every (leaf, row) pair from four features; the 4r rows
// of highest score of each leaf are the candidates of a restricted start:
// adaptive cross approximation (Alg. 1) on the 4r x |block| submatrix of the
// candidate rows, held in LDS, replaces the r streaming elimination passes over
// all m rows.  The leaf then enters the ordinary swap loop from that (I, J):
// its first row phase forms the interpolation matrix over all m rows (the
// verification) and swaps in any row of |B| > 1 + tau (the fallback to plain
// maxvol), so every node still ends dominant.  A leaf whose candidate
// elimination meets a pivot at or below the rank threshold, or whose candidate
// submatrix does not fit LDS, keeps the plain start.
//
// Features of row i in leaf k (block columns B_k, width w_k), FP32:
//   f0 = log2 ||A(i, B_k)||^2 - log2 max_i ||A(i, B_k)||^2   (block-local norm)
//   f1 = log2(l_i m / s)                                      (leverage)
//   f2 = log2(lb_ki m / w_k)                                  (block leverage)
//   f3 = share of the leaf's rows with a larger f2            (its rank in the leaf)
// with l_i the leverage of row i in the column space of the Gaussian sketch
// Y = A Omega (Omega n x s, s = 2r), computed by CholeskyQR2: G = Y^T Y = L L^T,
// Q1 = Y L^-T, G2 = Q1^T Q1 = L2 L2^T, Q = Q1 L2^-T, l_i = ||Q(i, :)||^2, and
// lb_ki the ridge leverage of row i in the block itself,
// ||A(i, B_k) L_k^-T||^2 with A(:, B_k)^T A(:, B_k) + lambda_k I = L_k L_k^T,
// lambda_k = 2^-20 max_j ||A(:, j in B_k)||^2 (directions far below the
// block's leading ones, such as noise, add little).  The rank
// comes from a 1024-bin histogram (rows of one bin share the rank of the
// bin's midpoint), so every feature is deterministic.
//
// MLP: s(x) = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 with W1 128 x 4,
// W2 128 x 128, w3 128 in FP16 and the biases in FP32; every product is
// accumulated in FP32.  Training minimizes the weighted logistic loss
//   L = (1/N) sum_i [ pw y_i softplus(-s_i) + (1 - y_i) softplus(s_i) ]
// (y_i = 1 when the plain method selects row i in leaf k), with gradients from
// k_mlp_grad and Adam updates of an FP32 master copy (k_mlp_adam), which also
// writes the FP16 weights the forward pass uses.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "cur_device.hpp"
#include "cur_internal.hpp"

namespace cur {

// ---------------------------------------------------------------- MLP blob
constexpr int kF = CUR_MLP_FEATURES;  // 4
constexpr int kH = CUR_MLP_HIDDEN;    // 128
constexpr int kOffW1 = 0;                        // fp16 [kH][kF]
constexpr int kOffW2 = kOffW1 + 2 * kH * kF;     // fp16 [kH][kH]
constexpr int kOffW3 = kOffW2 + 2 * kH * kH;     // fp16 [kH]
constexpr int kOffB1 = kOffW3 + 2 * kH;          // f32 [kH]
constexpr int kOffB2 = kOffB1 + 4 * kH;          // f32 [kH]
constexpr int kOffB3 = kOffB2 + 4 * kH;          // f32 [1]
static_assert(kOffB3 + 4 <= CUR_MLP_BLOB_BYTES, "blob layout");
// parameter vector (FP32 master copy and gradients): W1, b1, W2, b2, w3, b3
constexpr int kPW1 = 0, kPB1 = kPW1 + kH * kF, kPW2 = kPB1 + kH, kPB2 = kPW2 + kH * kH, kPW3 = kPB2 + kH,
              kPB3 = kPW3 + kH, kParams = kPB3 + 1;
static_assert(kParams == CUR_MLP_PARAMS, "parameter count");

// ---------------------------------------------------------------- counter-based Gaussian
// SplitMix64 (Steele, Lea and Flood's mixing of a Weyl sequence) applied to a
// counter, two 53-bit uniforms, Box-Muller: gauss(seed, idx) is a pure
// function of its arguments.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double gauss(uint64_t seed, uint64_t idx) {
  const uint64_t a = splitmix64(seed ^ (2 * idx)), b = splitmix64(seed ^ (2 * idx + 1));
  const double u1 = ((double)(a >> 11) + 1.0) * 0x1p-53;  // (0, 1]
  const double u2 = (double)(b >> 11) * 0x1p-53;          // [0, 1)
  return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

// Omega (n x s, row-major): Omega(j, c) = gauss(seed, j s + c).
__global__ __launch_bounds__(kThreads) void k_gauss(double* __restrict__ Om, int64_t total, uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total; i += (int64_t)gridDim.x * kThreads)
    Om[i] = gauss(seed, (uint64_t)i);
}

// ---------------------------------------------------------------- FP64 MFMA GEMM
// C[z](i, j) = sum over k in split z of A(i, k) B(k, j), with A(i, k) =
// a[i sai + k sak] (element TA) and B(k, j) = b[k sbk + j sbj] (element TB):
// the sketch Y = A Omega, the Grams Y^T Y and A_k^T A_k, Y L^-T and
// A_k L_k^-T.  TM x TM tiles (TM = 128, or 64 for the 64-wide leaf blocks),
// grid (column tiles, row tiles, batch x splits); operands staged in padded
// LDS 32 values of k at a time; v_mfma_f64_16x16x4f64, wavefront w on the
// TM/2 x TM/2 quadrant (w >> 1, w & 1).  Out-of-range rows, columns and k
// are zero operands.
constexpr int kGT = 128, kGK = 32;
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <int TM>
struct GemmLds {
  double A[TM][kGK + 1];
  double B[kGK][TM + 1];
};

// grid.z = batch x nsplit: product `batch` reads a + batch za and b + batch zb,
// split `z % nsplit` covers k in [split kchunk, +kchunk), and each z writes
// c + z cstride (the splits of one product are then summed by k_sum_splits).
// Row-norm epilogue (rsq != nullptr; one column tile, N <= TM, no split):
// instead of C, rsq[batch ostride + i] = sum_j C(i, j)^2 and, with esq,
// esq[batch ostride + i] = sum_k A(i, k)^2, both summed in FP64 and stored
// as FP32.
template <typename TA, typename TB, int TM>
__global__ __launch_bounds__(kThreads, 2) void k_gemm_f64(const TA* __restrict__ a, int64_t sai, int64_t sak,
                                                          const TB* __restrict__ b, int64_t sbk, int64_t sbj,
                                                          double* __restrict__ c, int64_t ldc, int64_t M, int64_t N,
                                                          int64_t K, int64_t kchunk, int64_t cstride, int nsplit,
                                                          int64_t za, int64_t zb, float* __restrict__ rsq,
                                                          float* __restrict__ esq, int64_t ostride) {
  constexpr int V = TM * kGK / kThreads;  // operand values each thread stages (16 or 8)
  constexpr int QM = TM / 2, NF = QM / 16;
  __shared__ GemmLds<TM> L;
  __shared__ double red[TM][2];
  double e2 = 0.0;  // this thread's share of sum_k A(i, k)^2 for its staging row
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t i0 = (int64_t)blockIdx.y * TM, j0 = (int64_t)blockIdx.x * TM;
  const int batch = (int)blockIdx.z / nsplit, split = (int)blockIdx.z % nsplit;
  a += (int64_t)batch * za;
  b += (int64_t)batch * zb;
  const int64_t kb = (int64_t)split * kchunk, ke = min(K, kb + kchunk);
  const int wr = (w >> 1) * QM, wc = (w & 1) * QM;
  f64x4 acc[NF][NF];
#pragma unroll
  for (int i = 0; i < NF; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  // A: thread t -> row t / (kGK / V), k values V (t % (kGK / V)) + q;
  // B: k row t / (TM / V), columns V (t % (TM / V)) + q
  const int ar = tid / (kGK / V), ak = V * (tid % (kGK / V));
  const int bk = tid / (TM / V), bc = V * (tid % (TM / V));
  // a chunk whose rows, columns and k values all lie inside the operands loads
  // without bounds tests (a lane-divergent tested load compiles to a branch
  // with a wait for its data, one memory latency per load); the others keep
  // the tests (their zeros feed the row sums of squares)
  const bool inner_mn = i0 + TM <= M && j0 + TM <= N;
  for (int64_t k0 = kb; k0 < ke; k0 += kGK) {
    double va[V], vb[V];
    if (inner_mn && k0 + kGK <= ke) {
#pragma unroll
      for (int q = 0; q < V; ++q) {
        va[q] = (double)a[(i0 + ar) * sai + (k0 + ak + q) * sak];
        vb[q] = (double)b[(k0 + bk) * sbk + (j0 + bc + q) * sbj];
      }
    } else {
#pragma unroll
      for (int q = 0; q < V; ++q) {
        const int64_t i = i0 + ar, k = k0 + ak + q;
        va[q] = (i < M && k < ke) ? (double)a[i * sai + k * sak] : 0.0;
        const int64_t kk = k0 + bk, j = j0 + bc + q;
        vb[q] = (kk < ke && j < N) ? (double)b[kk * sbk + j * sbj] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < V; ++q) {
      L.A[ar][ak + q] = va[q];
      L.B[bk][bc + q] = vb[q];
      e2 = fma(va[q], va[q], e2);
    }
    __syncthreads();
#pragma unroll 2
    for (int k = 0; k < kGK; k += 4) {
      double af[NF], bf[NF];
#pragma unroll
      for (int i = 0; i < NF; ++i) af[i] = L.A[wr + 16 * i + lr][k + lk];
#pragma unroll
      for (int j = 0; j < NF; ++j) bf[j] = L.B[k + lk][wc + 16 * j + lr];
#pragma unroll
      for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int j = 0; j < NF; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  }
  if (rsq) {
    // row sums of squares: over the 16 columns of a fragment row (lanes lr),
    // the fragments j, then the two column halves of the tile (w & 1)
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double q = 0.0;
#pragma unroll
        for (int j = 0; j < NF; ++j) q = fma(acc[i][j][v], acc[i][j][v], q);
#pragma unroll
        for (int sh = 1; sh < 16; sh <<= 1) q += __shfl_xor(q, sh, 64);
        if (lr == 0) red[wr + 16 * i + 4 * v + lk][w & 1] = q;
      }
    constexpr int TPR = kGK / V;  // staging threads per row of A
#pragma unroll
    for (int sh = 1; sh < TPR; sh <<= 1) e2 += __shfl_xor(e2, sh, 64);
    __syncthreads();
    const int64_t o = (int64_t)batch * ostride;
    if (tid < TM && i0 + tid < M) rsq[o + i0 + tid] = (float)(red[tid][0] + red[tid][1]);
    if (esq && tid % TPR == 0 && i0 + ar < M) esq[o + i0 + ar] = (float)e2;
    return;
  }
  double* cz = c + (int64_t)blockIdx.z * cstride;
#pragma unroll
  for (int i = 0; i < NF; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = i0 + wr + 16 * i + 4 * v + lk;
      if (row >= M) continue;
#pragma unroll
      for (int j = 0; j < NF; ++j) {
        const int64_t col = j0 + wc + 16 * j + lr;
        if (col < N) cz[row * ldc + col] = acc[i][j][v];
      }
    }
}

// out[q count + e] = sum over z of part[(q nz + z) cstride + e], z ascending
// (product q = blockIdx.y, e < count).
__global__ __launch_bounds__(kThreads) void k_sum_splits(const double* __restrict__ part, int64_t cstride, int nz,
                                                         int64_t count, double* __restrict__ out) {
  const int q = blockIdx.y;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < count; e += (int64_t)gridDim.x * kThreads) {
    double s = 0.0;
    for (int z = 0; z < nz; ++z) s += part[((int64_t)q * nz + z) * cstride + e];
    out[(int64_t)q * count + e] = s;
  }
}

// ---------------------------------------------------------------- Cholesky and triangular inverse
// One block of 1024 threads per matrix: G (s x s, row-major, s <= kLdsChol)
// -> G + ridge d I = L L^T (d the largest diagonal entry of G), then
// Li = L^-1 (lower, row-major, upper triangle zero).  Pivots below 2^-40 d are
// raised to it (the Gram of a numerically rank-deficient matrix), so L is
// always invertible.  The matrix is held in LDS, M = G in place, rows padded
// to s + 1 doubles so that column reads fall in distinct banks.  Step k of the Cholesky
// updates the trailing lower triangle with the unscaled column k and the
// pivot d_k = max(M(k, k), floor) (M(i, j) -= M(i, k) M(j, k) / d_k; thread
// (y, x) of a 32 x 32 grid takes rows i = k + 1 + y + 32 p and columns
// j = k + 1 + x + 32 q <= i), then scales column k by 1 / sqrt(d_k): one
// barrier per step.  The inverse is formed in place row by row (row i of
// L^-1 needs row i of L and the rows k < i of L^-1 already written over L):
// Li(i, j) = (delta_ij - sum over j <= k < i of L(i, k) Li(k, j)) / L(i, i),
// each j by a team of 8 lanes (k strided by 8, combined by xor shuffles).
constexpr int kLdsChol = 128;
__global__ __launch_bounds__(1024) void k_chol_inv(const double* __restrict__ G, int s, double ridge,
                                                       double* __restrict__ Li) {
  __shared__ double M[kLdsChol * (kLdsChol + 1)];
  __shared__ double sred[16];
  G += (int64_t)blockIdx.x * s * s;
  Li += (int64_t)blockIdx.x * s * s;
  const int tid = threadIdx.x, ld = s + 1;
  for (int e = tid; e < s * s; e += 1024) M[(e / s) * ld + e % s] = G[e];
  double dm = 0.0;
  for (int k = tid; k < s; k += 1024) dm = fmax(dm, G[(int64_t)k * s + k]);
#pragma unroll
  for (int sh = 32; sh >= 1; sh >>= 1) dm = fmax(dm, __shfl_xor(dm, sh, 64));
  if ((tid & 63) == 0) sred[tid >> 6] = dm;
  __syncthreads();
  dm = sred[0];
  for (int q = 1; q < 16; ++q) dm = fmax(dm, sred[q]);
  const double fl = dm > 0.0 ? dm * 0x1p-40 : 1.0;
  if (ridge > 0.0)
    for (int k = tid; k < s; k += 1024) M[k * ld + k] += ridge * dm;
  __syncthreads();
  const int ty = tid >> 5, tx = tid & 31;
  for (int k = 0; k < s; ++k) {
    const double d = fmax(M[k * ld + k], fl);
    const double rd = 1.0 / d;
    for (int i = k + 1 + ty; i < s; i += 32) {
      const double li = M[i * ld + k] * rd;
      for (int j = k + 1 + tx; j <= i; j += 32) M[i * ld + j] = fma(-li, M[j * ld + k], M[i * ld + j]);
    }
    __syncthreads();
    const double p = sqrt(d);
    for (int i = k + 1 + tid; i < s; i += 1024) M[i * ld + k] /= p;
    if (tid == 0) M[k * ld + k] = p;
    // the next step reads column k + 1 and the diagonal, which this scaling does not touch
  }
  __syncthreads();
  const int team = tid >> 3, t = tid & 7;
  for (int i = 0; i < s; ++i) {
    double v = 0.0;
    const int j = team;
    if (j <= i) {
      double acc = 0.0;
      for (int k = j + t; k < i; k += 8) acc = fma(M[i * ld + k], M[k * ld + j], acc);
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      acc += __shfl_xor(acc, 4, 64);
      v = ((j == i ? 1.0 : 0.0) - acc) / M[i * ld + i];
    }
    __syncthreads();
    if (j <= i && t == 0) M[i * ld + j] = v;
    __syncthreads();
  }
  for (int e = tid; e < s * s; e += 1024) {
    const int i = e / s, j = e % s;
    Li[e] = j <= i ? M[i * ld + j] : 0.0;
  }
}

// ---------------------------------------------------------------- features
constexpr int kBins = 1024;
constexpr float kLogLo = -64.0f;  // log2 range of the binned features: [kLogLo, kLogLo + 96)
__device__ __forceinline__ int log_bin(float v) {
  const float t = (v - kLogLo) * (kBins / 96.0f);
  return (int)fminf(fmaxf(t, 0.0f), (float)(kBins - 1));
}

// Per leaf g, one block over the values v = vals(g, :).
// mode 0: gmax(g) = log2 max_i v_i (the leaf's largest block energy);
// mode 1: rank(g, bin) = (count above + count in bin / 2) / m over the values
//         log2(v_i m / w_g) (the normalised block leverage, w_g the leaf's
//         width: w, or wl for the last leaf).
__global__ __launch_bounds__(kThreads) void k_group_rank(const float* __restrict__ vals, int64_t m, int mode, int w,
                                                         int wl, float* __restrict__ gmax, float* __restrict__ rank) {
  const int g = blockIdx.x;
  const float* v = vals + (int64_t)g * m;
  if (mode == 0) {
    __shared__ float smax[kThreads / 64];
    float mx = 0.0f;
    for (int64_t i = threadIdx.x; i < m; i += kThreads) mx = fmaxf(mx, v[i]);
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) mx = fmaxf(mx, __shfl_xor(mx, sh, 64));
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      mx = smax[0];
      for (int q = 1; q < kThreads / 64; ++q) mx = fmaxf(mx, smax[q]);
      gmax[g] = log2f(fmaxf(mx, 1e-38f));
    }
    return;
  }
  __shared__ unsigned cnt[kBins];
  for (int q = threadIdx.x; q < kBins; q += kThreads) cnt[q] = 0;
  __syncthreads();
  const float norm = (float)m / (float)(g == (int)gridDim.x - 1 ? wl : w);
  for (int64_t i = threadIdx.x; i < m; i += kThreads) atomicAdd(&cnt[log_bin(log2f(fmaxf(v[i] * norm, 1e-38f)))], 1u);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned above = 0;
    for (int q = kBins - 1; q >= 0; --q) {
      const unsigned c = cnt[q];
      rank[(int64_t)g * kBins + q] = ((float)above + 0.5f * (float)c) / (float)m;
      above += c;
    }
  }
}

// Feature rows F((k m + i) 4 + f) for every leaf k and row i (levb: the
// leaves' block leverages, leaf-major; lbn(k) = m / w_k).
__global__ __launch_bounds__(kThreads) void k_features(const float* __restrict__ E, const float* __restrict__ lev,
                                                       const float* __restrict__ levb, int64_t m, int b, int w,
                                                       int wl, float lev_norm, const float* __restrict__ lmax,
                                                       const float* __restrict__ rankb, float* __restrict__ F) {
  const int64_t total = (int64_t)b * m;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total; e += (int64_t)gridDim.x * kThreads) {
    const int k = (int)(e / m);
    const int64_t i = e - (int64_t)k * m;
    const float lbn = (float)m / (float)(k == b - 1 ? wl : w);
    float4 out;
    out.x = log2f(fmaxf(E[e], 1e-38f)) - lmax[k];
    out.y = log2f(fmaxf(lev[i] * lev_norm, 1e-38f));
    out.z = log2f(fmaxf(levb[e] * lbn, 1e-38f));
    out.w = rankb[(int64_t)k * kBins + log_bin(out.z)];
    *(float4*)(F + e * kF) = out;
  }
}

// ---------------------------------------------------------------- MLP
// The block's weights in LDS (FP16 as stored, biases FP32).
struct MlpLds {
  __half W1[kH * kF];
  __half W2[kH * kH];
  __half W3[kH];
  float b1[kH], b2[kH], b3;
};

__device__ void mlp_load(MlpLds& W, const uint8_t* blob) {
  const __half* w1 = (const __half*)(blob + kOffW1);
  const __half* w2 = (const __half*)(blob + kOffW2);
  const __half* w3 = (const __half*)(blob + kOffW3);
  const float* b1 = (const float*)(blob + kOffB1);
  const float* b2 = (const float*)(blob + kOffB2);
  for (int q = threadIdx.x; q < kH * kF; q += blockDim.x) W.W1[q] = w1[q];
  for (int q = threadIdx.x; q < kH * kH; q += blockDim.x) W.W2[q] = w2[q];
  for (int q = threadIdx.x; q < kH; q += blockDim.x) {
    W.W3[q] = w3[q];
    W.b1[q] = b1[q];
    W.b2[q] = b2[q];
  }
  if (threadIdx.x == 0) W.b3 = *(const float*)(blob + kOffB3);
}

// Rows are processed 64 at a time by 256 threads: thread t works on row
// t >> 2 and on the hidden units 32 (t & 3) .. + 32 of each layer.
constexpr int kMR = 64;
struct MlpRows {
  float X[kMR][kF];
  float H1[kMR][kH + 1];  // relu(W1 x + b1)
  float H2[kMR][kH + 1];  // relu(W2 h1 + b2), then g2 (backward)
  float G1[kMR][kH + 1];  // backward: g1
  float ds[kMR];
};

// Forward of the block's current kMR rows (X staged): H1, H2 and the scores
// (s_out[row]); every sum in FP32, in ascending unit order per thread, the
// four quarter-sums of the output added in quarter order.
__device__ void mlp_forward_rows(const MlpLds& W, MlpRows& R, float* s_out) {
  const int tid = threadIdx.x, row = tid >> 2, q0 = 32 * (tid & 3);
  for (int u = q0; u < q0 + 32; ++u) {
    float a = W.b1[u];
#pragma unroll
    for (int f = 0; f < kF; ++f) a = fmaf(__half2float(W.W1[u * kF + f]), R.X[row][f], a);
    R.H1[row][u] = fmaxf(a, 0.0f);
  }
  __syncthreads();
  float part = 0.0f;
  for (int u = q0; u < q0 + 32; ++u) {
    float a = W.b2[u];
    const __half* w = W.W2 + u * kH;
    for (int k = 0; k < kH; ++k) a = fmaf(__half2float(w[k]), R.H1[row][k], a);
    const float h = fmaxf(a, 0.0f);
    R.H2[row][u] = h;
    part = fmaf(__half2float(W.W3[u]), h, part);
  }
  // the four quarters of the row are lanes 4 (l >> 2) .. + 3 of the wavefront
  const int base = (tid & 63) & ~3;
  const float p0 = __shfl(part, base, 64), p1 = __shfl(part, base + 1, 64);
  const float p2 = __shfl(part, base + 2, 64), p3 = __shfl(part, base + 3, 64);
  const float s = W.b3 + ((p0 + p1) + (p2 + p3));
  if ((tid & 3) == 0) s_out[row] = s;
  __syncthreads();
}

// Scores of `count` feature rows.
__global__ __launch_bounds__(kThreads) void k_mlp_forward(const uint8_t* __restrict__ blob, const float* __restrict__ F,
                                                          int64_t count, float* __restrict__ score) {
  __shared__ MlpLds W;
  __shared__ MlpRows R;
  __shared__ float sc[kMR];
  mlp_load(W, blob);
  for (int64_t r0 = (int64_t)blockIdx.x * kMR; r0 < count; r0 += (int64_t)gridDim.x * kMR) {
    __syncthreads();
    for (int q = threadIdx.x; q < kMR * kF; q += kThreads) {
      const int64_t e = r0 + q / kF;
      R.X[q / kF][q % kF] = e < count ? F[e * kF + q % kF] : 0.0f;
    }
    __syncthreads();
    mlp_forward_rows(W, R, sc);
    for (int q = threadIdx.x; q < kMR; q += kThreads)
      if (r0 + q < count) score[r0 + q] = sc[q];
  }
}

__device__ __forceinline__ float softplus(float x) { return x > 0.0f ? x + log1pf(expf(-x)) : log1pf(expf(x)); }
__device__ __forceinline__ float sigmoid(float x) { return 1.0f / (1.0f + expf(-x)); }

// Gradient of the mean weighted logistic loss over `count` rows.  Block g
// handles rows [g chunk, (g + 1) chunk) in groups of kMR and writes its
// parameter-gradient sums (FP32, in the parameter order) to part[g] and its
// loss sum to lpart[g]; k_mlp_grad_sum adds the blocks in order.
__global__ __launch_bounds__(kThreads) void k_mlp_grad(const uint8_t* __restrict__ blob, const float* __restrict__ F,
                                                       const float* __restrict__ Y, int64_t count, int64_t chunk,
                                                       float pw, float* __restrict__ part, double* __restrict__ lpart) {
  __shared__ MlpLds W;
  __shared__ MlpRows R;
  __shared__ float sc[kMR];
  mlp_load(W, blob);
  const int tid = threadIdx.x, row = tid >> 2, q0 = 32 * (tid & 3);
  const float inv_n = 1.0f / (float)count;
  // thread t owns W2 entries (u, k) = (t >> 1, 64 (t & 1) + c), c < 64
  const int ou = tid >> 1, ok0 = 64 * (tid & 1);
  float gW2[64];
#pragma unroll
  for (int c = 0; c < 64; ++c) gW2[c] = 0.0f;
  float gW1[2] = {0.0f, 0.0f}, gb1 = 0.0f, gb2 = 0.0f, gw3 = 0.0f, gb3 = 0.0f;
  double lsum = 0.0;
  const int64_t b0 = (int64_t)blockIdx.x * chunk, b1e = min(count, b0 + chunk);
  for (int64_t r0 = b0; r0 < b1e; r0 += kMR) {
    __syncthreads();
    for (int q = tid; q < kMR * kF; q += kThreads) {
      const int64_t e = r0 + q / kF;
      R.X[q / kF][q % kF] = e < b1e ? F[e * kF + q % kF] : 0.0f;
    }
    __syncthreads();
    mlp_forward_rows(W, R, sc);
    // dL/ds per row (rows past the range contribute nothing)
    if ((tid & 3) == 0) {
      const int64_t e = r0 + row;
      float d = 0.0f;
      if (e < b1e) {
        const float y = Y[e], s = sc[row];
        d = (-pw * y * sigmoid(-s) + (1.0f - y) * sigmoid(s)) * inv_n;
        lsum += (double)(pw * y * softplus(-s) + (1.0f - y) * softplus(s));
      }
      R.ds[row] = d;
    }
    __syncthreads();
    // w3, b3 gradients (thread u < kH over the rows), then g2 = ds w3 [h2 > 0] in place of H2
    if (tid < kH) {
      for (int q = 0; q < kMR; ++q) gw3 = fmaf(R.ds[q], R.H2[q][tid], gw3);
    }
    if (tid == 0)
      for (int q = 0; q < kMR; ++q) gb3 += R.ds[q];
    __syncthreads();
    for (int u = q0; u < q0 + 32; ++u) {
      const float h = R.H2[row][u];
      R.H2[row][u] = h > 0.0f ? R.ds[row] * __half2float(W.W3[u]) : 0.0f;
    }
    __syncthreads();
    // g1 = (W2^T g2) [h1 > 0]
    for (int k = q0; k < q0 + 32; ++k) {
      float a = 0.0f;
      for (int u = 0; u < kH; ++u) a = fmaf(__half2float(W.W2[u * kH + k]), R.H2[row][u], a);
      R.G1[row][k] = R.H1[row][k] > 0.0f ? a : 0.0f;
    }
    __syncthreads();
    // W2, b2: sums over the rows of g2(u) h1(k)
    for (int q = 0; q < kMR; ++q) {
      const float g = R.H2[q][ou];
#pragma unroll
      for (int c = 0; c < 64; ++c) gW2[c] = fmaf(g, R.H1[q][ok0 + c], gW2[c]);
    }
    if (tid < kH)
      for (int q = 0; q < kMR; ++q) gb2 += R.H2[q][tid];
    // W1, b1: thread t owns W1 entries 2t, 2t + 1 (unit t >> 1, features 2 (t & 1) + 0/1)
    {
      const int u = tid >> 1, f0 = 2 * (tid & 1);
      for (int q = 0; q < kMR; ++q) {
        const float g = R.G1[q][u];
        gW1[0] = fmaf(g, R.X[q][f0], gW1[0]);
        gW1[1] = fmaf(g, R.X[q][f0 + 1], gW1[1]);
      }
    }
    if (tid < kH)
      for (int q = 0; q < kMR; ++q) gb1 += R.G1[q][tid];
  }
  float* P = part + (int64_t)blockIdx.x * kParams;
#pragma unroll
  for (int c = 0; c < 64; ++c) P[kPW2 + ou * kH + ok0 + c] = gW2[c];
  P[kPW1 + 2 * tid] = gW1[0];
  P[kPW1 + 2 * tid + 1] = gW1[1];
  if (tid < kH) {
    P[kPB1 + tid] = gb1;
    P[kPB2 + tid] = gb2;
    P[kPW3 + tid] = gw3;
  }
  if (tid == 0) P[kPB3] = gb3;
  // loss: sum over the block's rows (each row's term was added by its lane 4 row)
  double l = lsum;
#pragma unroll
  for (int sh = 32; sh >= 1; sh >>= 1) l += __shfl_xor(l, sh, 64);
  __shared__ double lred[kThreads / 64];
  if ((tid & 63) == 0) lred[tid >> 6] = l;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) t += lred[q];
    lpart[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kThreads) void k_mlp_grad_sum(const float* __restrict__ part, int nb,
                                                           const double* __restrict__ lpart, int64_t count,
                                                           float* __restrict__ grad, double* __restrict__ loss) {
  for (int e = blockIdx.x * kThreads + threadIdx.x; e < kParams; e += gridDim.x * kThreads) {
    float s = 0.0f;
    for (int g = 0; g < nb; ++g) s += part[(int64_t)g * kParams + e];
    grad[e] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double t = 0.0;
    for (int g = 0; g < nb; ++g) t += lpart[g];
    *loss = t / (double)count;
  }
}

// Adam on the FP32 master copy p with moments m1, m2 (bias-corrected with the
// step count t >= 1); the FP16 weights and FP32 biases of the blob follow.
__global__ __launch_bounds__(kThreads) void k_mlp_adam(uint8_t* __restrict__ blob, float* __restrict__ p,
                                                       float* __restrict__ m1, float* __restrict__ m2,
                                                       const float* __restrict__ g, int t, float lr, float beta1,
                                                       float beta2, float eps) {
  const float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
  for (int e = blockIdx.x * kThreads + threadIdx.x; e < kParams; e += gridDim.x * kThreads) {
    const float ge = g[e];
    const float a = beta1 * m1[e] + (1.0f - beta1) * ge;
    const float v = beta2 * m2[e] + (1.0f - beta2) * ge * ge;
    m1[e] = a;
    m2[e] = v;
    const float x = p[e] - lr * (a / c1) / (sqrtf(v / c2) + eps);
    p[e] = x;
    if (e < kPB1) ((__half*)(blob + kOffW1))[e - kPW1] = __float2half(x);
    else if (e < kPW2) ((float*)(blob + kOffB1))[e - kPB1] = x;
    else if (e < kPB2) ((__half*)(blob + kOffW2))[e - kPW2] = __float2half(x);
    else if (e < kPW3) ((float*)(blob + kOffB2))[e - kPB2] = x;
    else if (e < kPB3) ((__half*)(blob + kOffW3))[e - kPW3] = __float2half(x);
    else *(float*)(blob + kOffB3) = x;
  }
}

// ---------------------------------------------------------------- candidates and the restricted start
// Order-preserving key of a score (larger score -> larger key); NaN lowest,
// -0 the same as +0.
__device__ __forceinline__ uint32_t score_key(float x) {
  if (x != x) return 0u;
  if (x == 0.0f) x = 0.0f;
  const uint32_t u = __float_as_uint(x);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// One block per leaf: the rows of the kc largest scores (ties: smaller row
// first), ascending, into cand[leaf * kc ..].  Radix select of the kc-th
// largest key (4 passes of 8 bits), then an ordered compaction.
__global__ __launch_bounds__(kThreads) void k_topk(const float* __restrict__ score, int64_t m, int kc,
                                                   int32_t* __restrict__ cand) {
  const int g = blockIdx.x, tid = threadIdx.x;
  const float* sv = score + (int64_t)g * m;
  __shared__ unsigned hist[256];
  __shared__ uint32_t sprefix, smask;
  __shared__ int sneed;
  if (tid == 0) {
    sprefix = 0;
    smask = 0;
    sneed = kc;  // rows still to take at and below the current prefix
  }
  for (int pass = 3; pass >= 0; --pass) {
    for (int q = tid; q < 256; q += kThreads) hist[q] = 0;
    __syncthreads();
    const uint32_t pre = sprefix, msk = smask;
    for (int64_t i = tid; i < m; i += kThreads) {
      const uint32_t k = score_key(sv[i]);
      if ((k & msk) == pre) atomicAdd(&hist[(k >> (8 * pass)) & 255u], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      int need = sneed;
      int d = 255;
      for (; d > 0; --d) {
        if ((int)hist[d] >= need) break;
        need -= (int)hist[d];
      }
      sprefix = pre | ((uint32_t)d << (8 * pass));
      smask = msk | (255u << (8 * pass));
      sneed = need;
    }
    __syncthreads();
  }
  // threshold key T = sprefix: take every key > T and the first `sneed` rows with key == T
  const uint32_t T = sprefix;
  const int need_eq = sneed;
  // ordered compaction: thread t scans rows [t seg, (t + 1) seg)
  const int64_t seg = (m + kThreads - 1) / kThreads;
  const int64_t a = min(m, (int64_t)tid * seg), e = min(m, a + seg);
  int cgt = 0, ceq = 0;
  for (int64_t i = a; i < e; ++i) {
    const uint32_t k = score_key(sv[i]);
    cgt += k > T;
    ceq += k == T;
  }
  __shared__ int pgt[kThreads], peq[kThreads];
  pgt[tid] = cgt;
  peq[tid] = ceq;
  __syncthreads();
  if (tid == 0) {
    int sg = 0, se = 0;
    for (int q = 0; q < kThreads; ++q) {
      const int x = pgt[q], y = peq[q];
      pgt[q] = sg;
      peq[q] = se;
      sg += x;
      se += y;
    }
  }
  __syncthreads();
  int og = pgt[tid], oe = peq[tid];
  // output position of row i = (rows taken before it): greater-keys before it plus
  // taken equal-keys before it
  for (int64_t i = a; i < e; ++i) {
    const uint32_t k = score_key(sv[i]);
    if (k > T) {
      const int pos = og + min(oe, need_eq);
      cand[(int64_t)g * kc + pos] = (int32_t)i;
      ++og;
    } else if (k == T) {
      if (oe < need_eq) cand[(int64_t)g * kc + og + oe] = (int32_t)i;
      ++oe;
    }
  }
}

// One block per leaf: ACA (Alg. 1) on the candidate rows x the leaf's columns,
// held in LDS as R[c][j] (FP64, candidate-major), r steps: the pivot is the
// first largest |R| in the scan order candidate ascending, then column
// ascending (candidates are ascending rows, so this is the row-major scan
// order of the original rows); R -= R(:, j) R(i, :) / p, then the pivot row
// and column are set to zero.  On success the leaf's I, Jp hold the r pivots
// and the leaf opens its swap loop (ST_START_SWAP); a pivot at or below the
// rank threshold leaves the leaf to the plain start.
constexpr int kCandCap = 16384;  // doubles of the candidate submatrix held in LDS (128 KiB)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cand_aca(Node* nodes, const int32_t* __restrict__ cand, int kc) {
  Node& nd = nodes[blockIdx.x];
  const int nc = nd.nc, r = nd.r;
  if ((int64_t)kc * nc > kCandCap || kc < r || r > 64 || nc > 256) return;  // does not fit: plain start
  __shared__ double Rm[kCandCap];
  __shared__ double sf[256];
  __shared__ Cand sc[kThreads / 64];
  __shared__ int s_row[64], s_col[64];
  __shared__ int s_ok;
  const int64_t m = nd.m;
  const T* P = (const T*)nd.panel;
  const int32_t* cd = cand + (int64_t)blockIdx.x * kc;
  const int tid = threadIdx.x;
  for (int64_t e = tid; e < (int64_t)kc * nc; e += kThreads) {
    const int c = (int)(e / nc), j = (int)(e % nc);
    Rm[e] = (double)P[(int64_t)j * m + cd[c]];
  }
  if (tid == 0) s_ok = 1;
  __syncthreads();
  const int total = kc * nc;
  for (int t = 0; t < r; ++t) {
    Cand best = cand_none();
    for (int e = tid; e < total; e += kThreads) {
      const double x = Rm[e];
      const double ax = fabs(x);
      if (x == x && cand_better(ax, e, best.val, best.key)) {
        best.val = ax;
        best.sval = x;
        best.key = e;
      }
    }
    best = block_argmax(best, sc);
    const int ci = (int)(best.key / nc), cj = (int)(best.key % nc);
    if (best.key == INT64_MAX || !(best.val > nd.theta)) {
      if (tid == 0) s_ok = 0;
      break;
    }
    const double p = best.sval;
    if (tid == 0) {
      s_row[t] = cd[ci];
      s_col[t] = cj;
    }
    // f_j = R(ci, j) / p for all j, then R(a, j) -= R(a, cj) f_j; pivot row/column zeroed
    for (int j = tid; j < nc; j += kThreads) sf[j] = Rm[(int64_t)ci * nc + j] / p;
    __syncthreads();
    for (int e = tid; e < total; e += kThreads) {
      const int a = e / nc, j = e % nc;
      if (a == ci || j == cj) continue;
      Rm[e] = fma(-Rm[(int64_t)a * nc + cj], sf[j], Rm[e]);
    }
    __syncthreads();
    for (int j = tid; j < nc; j += kThreads) Rm[(int64_t)ci * nc + j] = 0.0;
    for (int a = tid; a < kc; a += kThreads) Rm[(int64_t)a * nc + cj] = 0.0;
    __syncthreads();
  }
  __syncthreads();
  if (tid == 0 && s_ok) {
    for (int t = 0; t < r; ++t) {
      nd.I[t] = s_row[t];
      nd.Jp[t] = s_col[t];
    }
    nd.t = r;
    nd.q = r;
    nd.st = ST_START_SWAP;
  }
}

// ---------------------------------------------------------------- host side
static int64_t grid_of(int64_t work, int64_t per) { return std::max<int64_t>(1, std::min<int64_t>((work + per - 1) / per, 65536)); }

constexpr double kBlockRidge = 0x1p-20;  // ridge of the block Grams, relative to their largest diagonal entry
static int block_ksplit(int64_t m) { return (int)std::max<int64_t>(1, std::min<int64_t>(8, m / 1024)); }

// Splits of the sketch product over the n columns (partial sketches of at
// most kYBytes together, summed in order), enough for ~1024 blocks.
constexpr int64_t kYBytes = 64ll << 20;
static int sketch_splits(int64_t m, int64_t n, int64_t s) {
  const int64_t tiles = ((s + kGT - 1) / kGT) * ((m + kGT - 1) / kGT);
  return (int)std::max<int64_t>(1, std::min<int64_t>({8, (1024 + tiles - 1) / tiles, n / 256, kYBytes / (8 * m * s)}));
}

size_t propose_scratch(int64_t m, int64_t n, int r, int b) {
  const int64_t s = 2 * (int64_t)r;
  const int64_t w = std::max<int64_t>(1, n / b), W = n - (b - 1) * w;  // uniform and last leaf widths (W >= w)
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const int ksplit = 32, kb = block_ksplit(m), ys = sketch_splits(m, n, s);
  return al(8 * (size_t)n * s)                    // Omega
         + 2 * al(8 * (size_t)m * s)              // Y, Q1
         + (ys > 1 ? al(8 * (size_t)ys * m * s) : 0)  // partial sketches
         + al(8 * (size_t)ksplit * s * s)         // Gram partials
         + 2 * al(8 * (size_t)s * s)              // G, L^-1
         + al(8 * (size_t)b * kb * W * W)         // block Gram partials
         + 2 * al(8 * (size_t)b * W * W)          // block Grams, their L^-1
         + al(4 * (size_t)b * m)                  // E
         + al(4 * (size_t)m)                      // leverage
         + al(4 * (size_t)b * m)                  // block leverage
         + al(4 * (size_t)b) + al(4 * (size_t)b * kBins)  // leaf maxima, rank tables
         + al(4 * (size_t)b * m * kF)             // features
         + al(4 * (size_t)b * m)                  // scores
         + al(4 * (size_t)b * 4 * r)              // candidates
         + 4096;
}

// G + ridge d I = L L^T and Li = L^-1 for `count` matrices of order s.
// (s <= 128: the sketch has 2r <= 128 columns and a leaf at most 127.)
static void chol_inv(hipStream_t st, double* G, int s, double ridge, double* Li, int count) {
  hipLaunchKernelGGL(k_chol_inv, dim3((unsigned)count), dim3(1024), 0, st, G, s, ridge, Li);
}

// `batch` products (operands offset by za, zb per product), each split over
// k into nsplit partial results: C[z] at c + z cstride, z = product nsplit +
// split.  64 x 64 tiles when the product has at most 64 rows or columns,
// else 128 x 128.
// With rsq, the row-norm epilogue (N <= 128, nsplit = 1) replaces C.
template <typename TA, typename TB>
static void gemm(hipStream_t st, const TA* a, int64_t sai, int64_t sak, const TB* b, int64_t sbk, int64_t sbj,
                 double* c, int64_t ldc, int64_t M, int64_t N, int64_t K, int nsplit, int batch, int64_t cstride,
                 int64_t za, int64_t zb, float* rsq = nullptr, float* esq = nullptr, int64_t ostride = 0) {
  const int64_t kchunk = (K + nsplit - 1) / nsplit;
  const unsigned z = (unsigned)(batch * nsplit);
  // the epilogue needs all N columns in one tile
  if (rsq ? N <= 64 : (M <= 64 || N <= 64))
    hipLaunchKernelGGL((k_gemm_f64<TA, TB, 64>), dim3((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), z),
                       dim3(kThreads), 0, st, a, sai, sak, b, sbk, sbj, c, ldc, M, N, K, kchunk, cstride, nsplit, za, zb,
                       rsq, esq, ostride);
  else
    hipLaunchKernelGGL((k_gemm_f64<TA, TB, kGT>), dim3((unsigned)((N + kGT - 1) / kGT), (unsigned)((M + kGT - 1) / kGT), z),
                       dim3(kThreads), 0, st, a, sai, sak, b, sbk, sbj, c, ldc, M, N, K, kchunk, cstride, nsplit, za, zb,
                       rsq, esq, ostride);
}

// Leverage of Y's rows by CholeskyQR2 (two Cholesky-QR passes).
static cur_status leverage(cur_ctx ctx, double* Y, double* Q1, int64_t m, int s, double* gpart, double* G,
                           double* Li, float* lev) {
  hipStream_t st = ctx->stream;
  const int ksplit = (int)std::min<int64_t>(32, std::max<int64_t>(1, m / 256));
  const int64_t ss = (int64_t)s * s;
  double* src = Y;
  double* dst[2] = {Q1, nullptr};
  for (int pass = 0; pass < 2; ++pass) {
    // G = src^T src (split over rows), summed in order
    gemm<double, double>(st, src, 1, s, src, s, 1, gpart, s, s, s, m, ksplit, 1, ss, 0, 0);
    hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)grid_of(ss, kThreads), 1), dim3(kThreads), 0, st, gpart, ss,
                       ksplit, ss, G);
    chol_inv(st, G, s, 0.0, Li, 1);
    // dst = src L^-T (B(k, j) = Li(j, k)); the second pass keeps only the row norms
    if (pass == 0)
      gemm<double, double>(st, src, s, 1, Li, 1, s, dst[pass], s, m, s, s, 1, 1, 0, 0, 0);
    else
      gemm<double, double>(st, src, s, 1, Li, 1, s, nullptr, s, m, s, s, 1, 1, 0, 0, 0, lev, nullptr, 0);
    src = dst[pass];
  }
  CUR_HIP_CHECK(hipGetLastError());
  return CUR_OK;
}

// Ridge block leverage of every leaf: lb(k, i) = ||A(i, B_k) L_k^-T||^2 with
// A(:, B_k)^T A(:, B_k) + lambda_k I = L_k L_k^T, and the block energies
// E(k, i) = ||A(i, B_k)||^2 from the same pass over A.  Leaves 0 .. b-2 (width w) run as
// batches, the last leaf (width wl) on its own.
template <typename T>
static cur_status block_leverage(cur_ctx ctx, const T* A, int64_t m, int64_t lda, int w, int wl, int b, double* gpart,
                                 double* Gb, double* Lb, float* levb, float* E) {
  hipStream_t st = ctx->stream;
  const int kb = block_ksplit(m);
  for (int grp = 0; grp < 2; ++grp) {
    const int first = grp == 0 ? 0 : b - 1, cnt = grp == 0 ? b - 1 : 1, wk = grp == 0 ? w : wl;
    if (cnt <= 0) continue;
    const int64_t ww = (int64_t)wk * wk;
    const T* a0 = A + (int64_t)first * w;
    double* G = Gb + (int64_t)first * ww;
    double* Li = Lb + (int64_t)first * ww;
    for (int c0 = 0; c0 < cnt; c0 += 16384 / kb) {  // grid.z <= 16384
      const int cc = std::min(cnt - c0, 16384 / kb);
      // Grams, split over rows, then summed per leaf in order
      gemm<T, T>(st, a0 + (int64_t)c0 * w, 1, lda, a0 + (int64_t)c0 * w, lda, 1, gpart, wk, wk, wk, m, kb, cc, ww, w,
                 w);
      hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)grid_of(ww, kThreads), (unsigned)cc), dim3(kThreads), 0, st,
                         gpart, ww, kb, ww, G + (int64_t)c0 * ww);
    }
    chol_inv(st, G, wk, kBlockRidge, Li, cnt);
    // the row norms of A_k L_k^-T (B(k', j) = Li(j, k')) and of A_k
    for (int c0 = 0; c0 < cnt; c0 += 16384) {
      const int cc = std::min(cnt - c0, 16384);
      gemm<T, double>(st, a0 + (int64_t)c0 * w, lda, 1, Li + (int64_t)c0 * ww, 1, wk, nullptr, wk, m, wk, wk, 1, cc, 0,
                      w, ww, levb + (int64_t)(first + c0) * m, E + (int64_t)(first + c0) * m, m);
    }
  }
  CUR_HIP_CHECK(hipGetLastError());
  return CUR_OK;
}

// Features of every (leaf, row) of A into F (b m x 4 FP32); scratch as laid
// out by propose_scratch.  Returns the scratch pointers the later steps use.
struct ProposeBufs {
  float* F;
  float* score;
  int32_t* cand;
};

template <typename T>
static cur_status features_impl(cur_ctx ctx, const T* A, int64_t m, int64_t n, int64_t lda, int r, int w, int b,
                                uint64_t seed, char* scratch, ProposeBufs* out, float* F_ext) {
  hipStream_t st = ctx->stream;
  const int s = 2 * r;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const int ksplit = 32;
  char* p = scratch;
  auto take = [&](size_t bytes) {
    char* q = p;
    p += al(bytes);
    return q;
  };
  const int wl = (int)(n - (int64_t)(b - 1) * w), kb = block_ksplit(m), ys = sketch_splits(m, n, s);
  double* Om = (double*)take(8 * (size_t)n * s);
  double* Y = (double*)take(8 * (size_t)m * s);
  double* Q1 = (double*)take(8 * (size_t)m * s);
  double* ypart = ys > 1 ? (double*)take(8 * (size_t)ys * m * s) : nullptr;
  double* gpart = (double*)take(8 * (size_t)ksplit * s * s);
  double* G = (double*)take(8 * (size_t)s * s);
  double* Li = (double*)take(8 * (size_t)s * s);
  double* gbpart = (double*)take(8 * (size_t)b * kb * wl * wl);
  double* Gb = (double*)take(8 * (size_t)b * wl * wl);
  double* Lb = (double*)take(8 * (size_t)b * wl * wl);
  float* E = (float*)take(4 * (size_t)b * m);
  float* lev = (float*)take(4 * (size_t)m);
  float* levb = (float*)take(4 * (size_t)b * m);
  float* lmax = (float*)take(4 * (size_t)b);
  float* ranks = (float*)take(4 * (size_t)b * kBins);
  float* F = (float*)take(4 * (size_t)b * m * kF);
  float* score = (float*)take(4 * (size_t)b * m);
  int32_t* cand = (int32_t*)take(4 * (size_t)b * 4 * r);
  if (F_ext) F = F_ext;
  // the sketch Y = A Omega, split over the n columns and summed in order
  hipLaunchKernelGGL(k_gauss, dim3((unsigned)grid_of(n * s, kThreads)), dim3(kThreads), 0, st, Om, n * s, seed);
  gemm<T, double>(st, A, lda, 1, Om, s, 1, ys > 1 ? ypart : Y, s, m, s, n, ys, 1, m * s, 0, 0);
  if (ys > 1)
    hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)grid_of(m * s, kThreads), 1), dim3(kThreads), 0, st, ypart, m * s,
                       ys, m * s, Y);
  cur_status rc = leverage(ctx, Y, Q1, m, s, gpart, G, Li, lev);
  if (rc != CUR_OK) return rc;
  rc = block_leverage<T>(ctx, A, m, lda, w, wl, b, gbpart, Gb, Lb, levb, E);
  if (rc != CUR_OK) return rc;
  const float lev_norm = (float)((double)m / (double)s);
  hipLaunchKernelGGL(k_group_rank, dim3((unsigned)b), dim3(kThreads), 0, st, E, m, 0, w, wl, lmax, ranks);
  hipLaunchKernelGGL(k_group_rank, dim3((unsigned)b), dim3(kThreads), 0, st, levb, m, 1, w, wl, lmax, ranks);
  hipLaunchKernelGGL(k_features, dim3((unsigned)grid_of((int64_t)b * m, kThreads)), dim3(kThreads), 0, st, E, lev,
                     levb, m, b, w, wl, lev_norm, lmax, ranks, F);
  CUR_HIP_CHECK(hipGetLastError());
  if (out) {
    out->F = F;
    out->score = score;
    out->cand = cand;
  }
  return CUR_OK;
}

cur_status propose_features(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n, int64_t lda, int r, int w,
                            uint64_t seed, float* F) {
  const int b = (int)std::max<int64_t>(1, n / w);
  cur_status st = ensure_arena(ctx, propose_scratch(m, n, r, b));
  if (st != CUR_OK) return st;
  if (dtype == CUR_F64)
    return features_impl<double>(ctx, (const double*)A, m, n, lda, r, w, b, seed, (char*)ctx->arena, nullptr, F);
  return features_impl<float>(ctx, (const float*)A, m, n, lda, r, w, b, seed, (char*)ctx->arena, nullptr, F);
}

// The proposal for the leaves of one tree (leaves = the first b nodes of the
// level-0 table): features, scores, top 4r rows, restricted start.
template <typename T>
cur_status propose_leaves(cur_ctx ctx, const T* A, int64_t m, int64_t n, int64_t lda, int r, int w, int b,
                          const void* mlp, uint64_t seed, Node* leaves, char* scratch) {
  hipStream_t st = ctx->stream;
  ProposeBufs pb;
  cur_status rc = features_impl<T>(ctx, A, m, n, lda, r, w, b, seed, scratch, &pb, nullptr);
  if (rc != CUR_OK) return rc;
  const int64_t count = (int64_t)b * m;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)grid_of(count, kMR)), dim3(kThreads), 0, st, (const uint8_t*)mlp,
                     pb.F, count, pb.score);
  const int kc = (int)std::min<int64_t>(4 * (int64_t)r, m);
  hipLaunchKernelGGL(k_topk, dim3((unsigned)b), dim3(kThreads), 0, st, pb.score, m, kc, pb.cand);
  hipLaunchKernelGGL((k_cand_aca<T>), dim3((unsigned)b), dim3(kThreads), 0, st, leaves, pb.cand, kc);
  CUR_HIP_CHECK(hipGetLastError());
  return CUR_OK;
}
template cur_status propose_leaves<double>(cur_ctx, const double*, int64_t, int64_t, int64_t, int, int, int, const void*,
                                           uint64_t, Node*, char*);
template cur_status propose_leaves<float>(cur_ctx, const float*, int64_t, int64_t, int64_t, int, int, int, const void*,
                                          uint64_t, Node*, char*);

cur_status mlp_forward_dispatch(cur_ctx ctx, const void* blob, const float* F, int64_t count, float* score) {
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)grid_of(count, kMR)), dim3(kThreads), 0, ctx->stream,
                     (const uint8_t*)blob, F, count, score);
  CUR_HIP_CHECK(hipGetLastError());
  return CUR_OK;
}

cur_status mlp_grad_dispatch(cur_ctx ctx, const void* blob, const float* F, const float* Y, int64_t count, float pw,
                             float* grad, double* loss) {
  const int nb = (int)std::min<int64_t>(256, std::max<int64_t>(1, (count + 4 * kMR - 1) / (4 * kMR)));
  const int64_t chunk = ((count + nb - 1) / nb + kMR - 1) / kMR * kMR;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  cur_status st = ensure_arena(ctx, al(4 * (size_t)nb * kParams) + al(8 * (size_t)nb) + 256);
  if (st != CUR_OK) return st;
  float* part = (float*)ctx->arena;
  double* lpart = (double*)((char*)ctx->arena + al(4 * (size_t)nb * kParams));
  double* dloss = lpart + nb;
  hipStream_t s = ctx->stream;
  hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)nb), dim3(kThreads), 0, s, (const uint8_t*)blob, F, Y, count, chunk, pw,
                     part, lpart);
  hipLaunchKernelGGL(k_mlp_grad_sum, dim3((unsigned)grid_of(kParams, kThreads)), dim3(kThreads), 0, s, part, nb, lpart,
                     count, grad, dloss);
  CUR_HIP_CHECK(hipGetLastError());
  double h = 0.0;
  CUR_HIP_CHECK(hipMemcpyAsync(&h, dloss, sizeof(double), hipMemcpyDeviceToHost, s));
  CUR_HIP_CHECK(hipStreamSynchronize(s));
  if (loss) *loss = h;
  return CUR_OK;
}

cur_status mlp_adam_dispatch(cur_ctx ctx, void* blob, float* p, float* m1, float* m2, const float* g, int t, float lr,
                             float beta1, float beta2, float eps) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)grid_of(kParams, kThreads)), dim3(kThreads), 0, ctx->stream,
                     (uint8_t*)blob, p, m1, m2, g, t, lr, beta1, beta2, eps);
  CUR_HIP_CHECK(hipGetLastError());
  return CUR_OK;
}

}  // namespace cur
