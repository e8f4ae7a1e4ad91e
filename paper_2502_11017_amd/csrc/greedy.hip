// Norm-greedy selection of rows and columns (Alg. 2 with Alg. 3): on each
// axis, r times, the vector (row or column) of largest Euclidean norm is
// chosen and projected out of every other vector, v <- v - ((s.v)/(s.s)) s.
// The block partition of Alg. 3 only distributes the work; here each step is
// an argmax launch over all candidates and an update launch with one
// wavefront per vector.
//
// Every sum over a vector (dot products, squared norms) is split over one
// wavefront: lane l accumulates elements i = l, l + 64, ... ascending with
// fma, then the 64 partials are combined by a xor butterfly (distances
// 32 .. 1).  That order differs from a plain ascending sum by rounding only, so
// a choice can differ from one made with plain sums only where the two best
// squared norms of a step lie within that rounding of each other.  Each
// element update is one fma with the coefficient (s.v) / (s.s).  Norms are
// compared squared; a chosen vector is no candidate again and is not updated;
// the axis stops, rank-short, once the largest remaining squared norm is at
// most (max(m,n) 2^-52)^2 times the largest initial one.
//
// Working copies are FP64 (FP32 input is converted exactly), one contiguous
// vector each: the rows as they are, the columns transposed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "cur_device.hpp"
#include "cur_internal.hpp"

namespace cur {

// State of one axis in device memory.
struct GreedyState {
  double theta;  // stop threshold on squared norms (set at step 0)
  int64_t j;     // vector chosen at the current step
  int count;     // vectors chosen so far
  int stop;      // 1: no further step (rank reached short or non-finite input)
  int nonfinite; // a squared norm was not finite
  int pad;
};

// Lane-ordered sum of a[i] * b[i] over one wavefront, returned in every lane.
__device__ __forceinline__ double wave_lane_dot(const double* a, const double* b, int64_t len) {
  const int lane = threadIdx.x & 63;
  double p = 0.0;
  for (int64_t i = lane; i < len; i += 64) p = fma(a[i], b[i], p);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) p = p + __shfl_xor(p, d, 64);
  return p;
}

// Rows of A as contiguous FP64 vectors: W[i * n + j] = A(i, j).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gr_load_rows(const T* __restrict__ A, int64_t m, int64_t n,
                                                           int64_t lda, double* __restrict__ W) {
  for (int64_t i = blockIdx.y; i < m; i += gridDim.y)
    for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < n; j += (int64_t)gridDim.x * kThreads)
      W[i * n + j] = (double)A[i * lda + j];
}

// Columns of A as contiguous FP64 vectors: W[j * m + i] = A(i, j), through a
// 64 x 64 LDS tile so that both the reads and the writes are coalesced.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gr_load_cols(const T* __restrict__ A, int64_t m, int64_t n,
                                                           int64_t lda, double* __restrict__ W) {
  __shared__ double tile[64][65];
  const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int q = ty; q < 64; q += kThreads / 64) {
    const int64_t i = i0 + q, j = j0 + tx;
    tile[q][tx] = (i < m && j < n) ? (double)A[i * lda + j] : 0.0;
  }
  __syncthreads();
  for (int q = ty; q < 64; q += kThreads / 64) {
    const int64_t j = j0 + q, i = i0 + tx;
    if (i < m && j < n) W[j * m + i] = tile[tx][q];
  }
}

// Squared norm of every vector (one wavefront per vector).
__global__ __launch_bounds__(kThreads) void k_gr_norms(const double* __restrict__ W, int64_t len, int64_t cnt,
                                                       double* __restrict__ nrm) {
  const int64_t v = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (v >= cnt) return;
  const double* w = W + v * len;
  const double s = wave_lane_dot(w, w, len);
  if ((threadIdx.x & 63) == 0) nrm[v] = s;
}

// One step's choice: the largest squared norm over the vectors not chosen,
// ties to the smaller index.  Step 0 also sets the stop threshold.
__global__ __launch_bounds__(kThreads) void k_gr_argmax(const double* __restrict__ nrm, uint8_t* sel, int64_t cnt,
                                                        double eps2, int t, GreedyState* st, int64_t* order) {
  if (st->stop) return;
  double best = -1.0;
  int64_t bi = -1;
  int bad = 0;
  for (int64_t v = threadIdx.x; v < cnt; v += kThreads) {  // ascending per thread: strict '>'
    const double x = nrm[v];
    if (!(x == x) || x == HUGE_VAL) bad = 1;
    if (!sel[v] && x > best) {
      best = x;
      bi = v;
    }
  }
  __shared__ double sb[kThreads];
  __shared__ int64_t si[kThreads];
  __shared__ int sbad;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  if (bad) sbad = 1;
  sb[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < kThreads; ++q)
      if (si[q] >= 0 && (sb[q] > best || (sb[q] == best && (bi < 0 || si[q] < bi)))) {
        best = sb[q];
        bi = si[q];
      }
    if (t == 0) {
      st->theta = eps2 * best;  // at step 0 nothing is chosen: best is the largest initial norm
      if (sbad) st->nonfinite = 1;
    }
    if (sbad || bi < 0 || !(best > st->theta)) {
      st->stop = 1;
    } else {
      sel[bi] = 1;
      order[t] = bi;
      st->j = bi;
      st->count = t + 1;
    }
  }
}

// One step's projection: every vector not chosen, v <- v - ((s.v)/(s.s)) s,
// then its new squared norm (one wavefront per vector; the chosen vector s is
// read-only here).
__global__ __launch_bounds__(kThreads) void k_gr_update(double* __restrict__ W, int64_t len, int64_t cnt,
                                                        double* __restrict__ nrm, const uint8_t* __restrict__ sel,
                                                        const GreedyState* __restrict__ st) {
  if (st->stop) return;
  const int64_t v = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (v >= cnt || sel[v]) return;
  const int64_t j = st->j;
  const double* s = W + j * len;
  double* w = W + v * len;
  const double c = wave_lane_dot(s, w, len) / nrm[j];
  for (int64_t i = threadIdx.x & 63; i < len; i += 64) w[i] = fma(-c, s[i], w[i]);
  const double q = wave_lane_dot(w, w, len);
  if ((threadIdx.x & 63) == 0) nrm[v] = q;
}

template <typename T>
static cur_status greedy_impl(cur_ctx ctx, const T* A, int64_t m, int64_t n, int64_t lda, int rr, int rc,
                              int64_t* I, int64_t* J, cur_info* info, cur_trace* trace) {
  cur_status st = ensure_groups(ctx);
  if (st != CUR_OK) return st;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t mn = (size_t)m * (size_t)n;
  const size_t need = 2 * al(sizeof(double) * mn) + al(sizeof(double) * m) + al(sizeof(double) * n) + al(m) + al(n) +
                      2 * al(sizeof(GreedyState)) + al(sizeof(int64_t) * rr) + al(sizeof(int64_t) * rc);
  st = ensure_arena(ctx, need);
  if (st != CUR_OK) return st;
  Arena ar{(char*)ctx->arena, ctx->arena_bytes, 0};
  double* Wr = (double*)ar.take(sizeof(double) * mn);
  double* Wc = (double*)ar.take(sizeof(double) * mn);
  double* nr = (double*)ar.take(sizeof(double) * m);
  double* nc = (double*)ar.take(sizeof(double) * n);
  uint8_t* selr = (uint8_t*)ar.take(m);
  uint8_t* selc = (uint8_t*)ar.take(n);
  GreedyState* str = (GreedyState*)ar.take(sizeof(GreedyState));
  GreedyState* stc = (GreedyState*)ar.take(sizeof(GreedyState));
  int64_t* ordr = (int64_t*)ar.take(sizeof(int64_t) * rr);
  int64_t* ordc = (int64_t*)ar.take(sizeof(int64_t) * rc);
  if (!ordc) {
    set_error("workspace layout overflow");
    return CUR_ERR_INTERNAL;
  }
  hipStream_t s0 = ctx->stream;
  CUR_HIP_CHECK(hipMemsetAsync(selr, 0, m, s0));
  CUR_HIP_CHECK(hipMemsetAsync(selc, 0, n, s0));
  CUR_HIP_CHECK(hipMemsetAsync(str, 0, sizeof(GreedyState), s0));
  CUR_HIP_CHECK(hipMemsetAsync(stc, 0, sizeof(GreedyState), s0));
  CUR_HIP_CHECK(hipEventRecord(ctx->gfork, s0));
  hipStream_t sr = ctx->gstream[0], sc = ctx->gstream[1];
  CUR_HIP_CHECK(hipStreamWaitEvent(sr, ctx->gfork, 0));
  CUR_HIP_CHECK(hipStreamWaitEvent(sc, ctx->gfork, 0));
  const double eps = (double)std::max(m, n) * std::ldexp(1.0, -52);
  const double eps2 = eps * eps;
  // rows: m vectors of length n; columns: n vectors of length m
  {
    const unsigned gx = (unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 64);
    const unsigned gy = (unsigned)std::min<int64_t>(m, 65535);
    hipLaunchKernelGGL((k_gr_load_rows<T>), dim3(gx, gy), dim3(kThreads), 0, sr, A, m, n, lda, Wr);
    const int64_t tby = (m + 63) / 64, tbx = (n + 63) / 64;
    if (tby > 65535) {
      set_error("matrix too tall for the column transpose grid");
      return CUR_ERR_ARG;
    }
    hipLaunchKernelGGL((k_gr_load_cols<T>), dim3((unsigned)tbx, (unsigned)tby), dim3(kThreads), 0, sc, A, m, n, lda,
                       Wc);
  }
  auto axis = [&](double* W, int64_t len, int64_t cnt, int steps, double* nrm, uint8_t* sel, GreedyState* gs,
                  int64_t* ord, hipStream_t s) {
    const unsigned nb = (unsigned)((cnt + kThreads / 64 - 1) / (kThreads / 64));
    hipLaunchKernelGGL(k_gr_norms, dim3(nb), dim3(kThreads), 0, s, W, len, cnt, nrm);
    for (int t = 0; t < steps; ++t) {
      hipLaunchKernelGGL(k_gr_argmax, dim3(1), dim3(kThreads), 0, s, nrm, sel, cnt, eps2, t, gs, ord);
      if (t + 1 < steps) hipLaunchKernelGGL(k_gr_update, dim3(nb), dim3(kThreads), 0, s, W, len, cnt, nrm, sel, gs);
    }
  };
  axis(Wr, n, m, rr, nr, selr, str, ordr, sr);
  axis(Wc, m, n, rc, nc, selc, stc, ordc, sc);
  CUR_HIP_CHECK(hipGetLastError());
  CUR_HIP_CHECK(hipEventRecord(ctx->gjoin[0], sr));
  CUR_HIP_CHECK(hipEventRecord(ctx->gjoin[1], sc));
  CUR_HIP_CHECK(hipStreamWaitEvent(s0, ctx->gjoin[0], 0));
  CUR_HIP_CHECK(hipStreamWaitEvent(s0, ctx->gjoin[1], 0));
  GreedyState hs[2];
  std::vector<int64_t> hr(rr, -1), hc(rc, -1);
  CUR_HIP_CHECK(hipMemcpyAsync(&hs[0], str, sizeof(GreedyState), hipMemcpyDeviceToHost, s0));
  CUR_HIP_CHECK(hipMemcpyAsync(&hs[1], stc, sizeof(GreedyState), hipMemcpyDeviceToHost, s0));
  CUR_HIP_CHECK(hipMemcpyAsync(hr.data(), ordr, sizeof(int64_t) * rr, hipMemcpyDeviceToHost, s0));
  CUR_HIP_CHECK(hipMemcpyAsync(hc.data(), ordc, sizeof(int64_t) * rc, hipMemcpyDeviceToHost, s0));
  CUR_HIP_CHECK(hipStreamSynchronize(s0));
  if (hs[0].nonfinite || hs[1].nonfinite) {
    set_error("A holds NaN or Inf");
    return CUR_ERR_NONFINITE;
  }
  const int qr = hs[0].count, qc = hs[1].count;
  std::vector<int64_t> oI(rr, -1), oJ(rc, -1);
  for (int t = 0; t < qr; ++t) oI[t] = hr[t];
  for (int t = 0; t < qc; ++t) oJ[t] = hc[t];
  std::sort(oI.begin(), oI.begin() + qr);
  std::sort(oJ.begin(), oJ.begin() + qc);
  CUR_HIP_CHECK(hipMemcpyAsync(I, oI.data(), sizeof(int64_t) * rr, hipMemcpyHostToDevice, s0));
  CUR_HIP_CHECK(hipMemcpyAsync(J, oJ.data(), sizeof(int64_t) * rc, hipMemcpyHostToDevice, s0));
  CUR_HIP_CHECK(hipStreamSynchronize(s0));
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->rank = std::min(qr, qc);
    info->logvol = std::nan("");
  }
  if (trace) {  // one record: rows and columns in the order chosen (square calls only)
    int64_t* mt = trace->meta;
    for (int f = 0; f < kMetaFields; ++f) mt[f] = 0;
    mt[2] = std::min(qr, qc);
    mt[3] = (qr < rr || qc < rc) ? 1 : 0;
    trace->vol_mant[0] = 0.0;
    for (int t = 0; t < rr; ++t) trace->I[t] = t < qr ? hr[t] : -1;
    for (int t = 0; t < rc; ++t) trace->J[t] = t < qc ? hc[t] : -1;
    trace->count = 1;
  }
  if (qr < rr || qc < rc) {
    set_error("fewer vectors above the rank threshold than asked for");
    return CUR_ERR_RANK;
  }
  return CUR_OK;
}

cur_status greedy_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n, int64_t lda, int r,
                           int64_t* I, int64_t* J, cur_info* info, cur_trace* trace) {
  if (dtype == CUR_F64) return greedy_impl<double>(ctx, (const double*)A, m, n, lda, r, r, I, J, info, trace);
  return greedy_impl<float>(ctx, (const float*)A, m, n, lda, r, r, I, J, info, trace);
}

cur_status greedy_rect_dispatch(cur_ctx ctx, cur_dtype dtype, const void* A, int64_t m, int64_t n, int64_t lda,
                                int r, int c, int64_t* I, int64_t* J, cur_info* info) {
  if (dtype == CUR_F64) return greedy_impl<double>(ctx, (const double*)A, m, n, lda, r, c, I, J, info, nullptr);
  return greedy_impl<float>(ctx, (const float*)A, m, n, lda, r, c, I, J, info, nullptr);
}

}  // namespace cur
