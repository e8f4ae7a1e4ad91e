// Microbenchmarks of the two limits the roofline figures are quoted against:
// HBM streaming bandwidth (read, write, copy) and dense MFMA throughput for
// the instruction shapes the kernels use (FP64 16x16x4, BF16 16x16x32, FP8
// e4m3 16x16x32).  Built as its own library (libcurbench.so), not part of the
// selection ABI; each entry point allocates, times with HIP events on its own
// stream and frees.
//
// Bandwidth: float4 loads/stores, each thread handling 4 vectors per trip of a
// grid-stride loop (independent requests in flight), 2048 workgroups of 256.
// MFMA: 8 independent accumulator chains per wavefront (enough to cover the
// instruction's dependent-issue latency), operands in registers, 4 wavefronts
// per workgroup and 8 workgroups per compute unit; the accumulators are
// written out so that nothing is removed.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kT = 256;

__global__ __launch_bounds__(kT) void k_read(const float4* __restrict__ x, int64_t n4, float* __restrict__ out) {
  float s = 0.0f;
  const int64_t stride = (int64_t)gridDim.x * kT;
  int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  for (; i + 3 * stride < n4; i += 4 * stride) {
    const float4 a = x[i], b = x[i + stride], c = x[i + 2 * stride], d = x[i + 3 * stride];
    s += (a.x + b.y) + (c.z + d.w);
  }
  for (; i < n4; i += stride) s += x[i].x;
  if (s == 12345.678f) out[blockIdx.x * kT + threadIdx.x] = s;  // keeps the loads
}

__global__ __launch_bounds__(kT) void k_write(float4* __restrict__ y, int64_t n4, float v) {
  const int64_t stride = (int64_t)gridDim.x * kT;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n4; i += stride) y[i] = make_float4(v, v, v, v);
}

__global__ __launch_bounds__(kT) void k_copy(const float4* __restrict__ x, float4* __restrict__ y, int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * kT;
  int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  for (; i + 3 * stride < n4; i += 4 * stride) {
    const float4 a = x[i], b = x[i + stride], c = x[i + 2 * stride], d = x[i + 3 * stride];
    y[i] = a;
    y[i + stride] = b;
    y[i + 2 * stride] = c;
    y[i + 3 * stride] = d;
  }
  for (; i < n4; i += stride) y[i] = x[i];
}

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(kT) void k_mfma_f64(int iters, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const double a = 1.0 + lane * 1e-3, b = 1.0 - lane * 1e-3;
  f64x4 acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = f64x4{0.0, 0.0, 0.0, (double)c};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * kT + threadIdx.x] = s;
}

__global__ __launch_bounds__(kT) void k_mfma_bf16(int iters, float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(1.0f + 0.01f * (lane + e));
    b[e] = (__bf16)(1.0f - 0.01f * (lane - e));
  }
  f32x4 acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = f32x4{0.0f, 0.0f, 0.0f, (float)c};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * kT + threadIdx.x] = s;
}

__global__ __launch_bounds__(kT) void k_mfma_fp8(int iters, float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  // eight e4m3 values per operand register pair: 0x38 = 1.0, 0x3c = 1.5
  const long a = (long)(0x3838383838383838ull ^ (uint64_t)(lane & 3));
  const long b = (long)0x3c3c3c3c3c3c3c3cull;
  f32x4 acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = f32x4{0.0f, 0.0f, 0.0f, (float)c};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * kT + threadIdx.x] = s;
}

struct Timer {
  hipEvent_t a, b;
  hipStream_t s;
  int ok;
  Timer() : ok(0) {
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
    ok = 1;
  }
  ~Timer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipStreamDestroy(s);
  }
};

}  // namespace

extern "C" {

/* Bandwidth of one kind of stream (0 read, 1 write, 2 copy) over `bytes`
 * bytes per buffer, best of `reps` timed launches after one warm-up: GB/s
 * (read + written bytes / time) in *gbs, the best launch in *ms.  Returns 0,
 * or -1 on a HIP error (allocation included). */
int curbench_stream(int kind, int64_t bytes, int reps, double* gbs, double* ms) {
  Timer t;
  if (!t.ok || kind < 0 || kind > 2 || bytes < 16 || reps < 1) return -1;
  const int64_t n4 = bytes / 16;
  float4 *x = nullptr, *y = nullptr;
  float* out = nullptr;
  const int grid = 2048;
  auto release = [&]() {
    if (x) (void)hipFree(x);
    if (y) (void)hipFree(y);
    if (out) (void)hipFree(out);
  };
  if (hipMalloc(&x, n4 * 16) != hipSuccess || (kind == 2 && hipMalloc(&y, n4 * 16) != hipSuccess) ||
      hipMalloc(&out, (size_t)grid * kT * sizeof(float)) != hipSuccess) {
    release();
    return -1;
  }
  hipLaunchKernelGGL(k_write, dim3(grid), dim3(kT), 0, t.s, x, n4, 1.0f);
  if (y) hipLaunchKernelGGL(k_write, dim3(grid), dim3(kT), 0, t.s, y, n4, 0.0f);
  float best = 1e30f;
  for (int k = 0; k <= reps; ++k) {
    (void)hipEventRecord(t.a, t.s);
    if (kind == 0) hipLaunchKernelGGL(k_read, dim3(grid), dim3(kT), 0, t.s, x, n4, out);
    else if (kind == 1) hipLaunchKernelGGL(k_write, dim3(grid), dim3(kT), 0, t.s, x, n4, 2.0f);
    else hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kT), 0, t.s, x, y, n4);
    (void)hipEventRecord(t.b, t.s);
    if (hipEventSynchronize(t.b) != hipSuccess) {
      release();
      return -1;
    }
    float e = 0.0f;
    (void)hipEventElapsedTime(&e, t.a, t.b);
    if (k > 0 && e < best) best = e;
  }
  const double moved = (double)n4 * 16.0 * (kind == 2 ? 2.0 : 1.0);
  *ms = best;
  *gbs = moved / (best * 1e-3) / 1e9;
  release();
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

/* Dense MFMA throughput (0: FP64 16x16x4, 1: BF16 16x16x32, 2: FP8 e4m3
 * 16x16x32), `iters` trips of 8 instructions per wavefront, `blocks`
 * workgroups of 4 wavefronts; best of `reps` after one warm-up: TFLOP/s in
 * *tflops (2 m n k per instruction), the best launch in *ms. */
int curbench_mfma(int kind, int iters, int blocks, int reps, double* tflops, double* ms) {
  Timer t;
  if (!t.ok || kind < 0 || kind > 2 || iters < 1 || blocks < 1 || reps < 1) return -1;
  void* out = nullptr;
  if (hipMalloc(&out, (size_t)blocks * kT * sizeof(double)) != hipSuccess) return -1;
  float best = 1e30f;
  for (int k = 0; k <= reps; ++k) {
    (void)hipEventRecord(t.a, t.s);
    if (kind == 0) hipLaunchKernelGGL(k_mfma_f64, dim3(blocks), dim3(kT), 0, t.s, iters, (double*)out);
    else if (kind == 1) hipLaunchKernelGGL(k_mfma_bf16, dim3(blocks), dim3(kT), 0, t.s, iters, (float*)out);
    else hipLaunchKernelGGL(k_mfma_fp8, dim3(blocks), dim3(kT), 0, t.s, iters, (float*)out);
    (void)hipEventRecord(t.b, t.s);
    if (hipEventSynchronize(t.b) != hipSuccess) {
      (void)hipFree(out);
      return -1;
    }
    float e = 0.0f;
    (void)hipEventElapsedTime(&e, t.a, t.b);
    if (k > 0 && e < best) best = e;
  }
  const double per_instr = kind == 0 ? 2.0 * 16 * 16 * 4 : 2.0 * 16 * 16 * 32;
  const double flops = per_instr * 8.0 * iters * (double)blocks * (kT / 64);
  *ms = best;
  *tflops = flops / (best * 1e-3) / 1e12;
  (void)hipFree(out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // extern "C"
