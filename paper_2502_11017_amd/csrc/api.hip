// C ABI front end: argument validation (host, before any device work),
// context and workspace management, error strings.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "cur_internal.hpp"

namespace cur {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error() { return g_last_error.c_str(); }

cur_status ensure_arena(cur_ctx ctx, size_t bytes) {
  if (ctx->arena_bytes >= bytes) return CUR_OK;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) {
    set_error(std::string("hipSetDevice: ") + hipGetErrorString(e));
    return CUR_ERR_DEVICE;
  }
  if (ctx->arena) {
    hipStreamSynchronize(ctx->stream);
    hipFree(ctx->arena);
    ctx->arena = nullptr;
    ctx->arena_bytes = 0;
  }
  size_t want = bytes + bytes / 8 + (1 << 20);
  e = hipMalloc(&ctx->arena, want);
  if (e != hipSuccess) {
    ctx->arena = nullptr;
    set_error("device workspace of " + std::to_string(want) + " bytes: " + hipGetErrorString(e));
    return CUR_ERR_NOMEM;
  }
  ctx->arena_bytes = want;
  return CUR_OK;
}

static cur_status arg_error(const std::string& msg) {
  set_error(msg);
  return CUR_ERR_ARG;
}

static cur_status check_matrix(int32_t dtype, const void* A, int64_t m, int64_t n, int64_t lda, int32_t r) {
  if (dtype != CUR_F64 && dtype != CUR_F32) return arg_error("dtype must be CUR_F64 or CUR_F32");
  if (!A) return arg_error("A is NULL");
  if (m < 1 || n < 1) return arg_error("m and n must be >= 1");
  if (lda < n) return arg_error("lda must be >= n");
  if (r < 1 || (int64_t)r > m || (int64_t)r > n) return arg_error("r must satisfy 1 <= r <= min(m, n)");
  if (r > 128) return arg_error("r > 128 is not supported (kernels are instantiated for r <= 128)");
  if (m > ((int64_t)1 << 40) || n > ((int64_t)1 << 40)) return arg_error("matrix dimensions too large");
  return CUR_OK;
}

// The selection's row kernels address a column of the working matrices with a
// 32-bit byte offset: one column must stay below 4 GiB, in FP64 for either
// input type (the elimination residual is FP64).
static cur_status check_select_rows(cur_dtype dtype, int64_t m) {
  (void)dtype;
  if (m * 8 >= ((int64_t)1 << 32)) return arg_error("m x 8 bytes must be below 4 GiB for selection");
  return CUR_OK;
}

// Resolve the options (defaults filled in) or report an argument error.
static cur_status resolve_opts(const cur_opts* in, cur_dtype dtype, int32_t r, int64_t n, cur_opts* out) {
  cur_opts o;
  std::memset(&o, 0, sizeof(o));
  o.struct_size = sizeof(cur_opts);
  if (in) {
    if (in->struct_size != (int32_t)sizeof(cur_opts)) return arg_error("cur_opts.struct_size mismatch");
    o = *in;
  }
  if (o.col_block < 0) return arg_error("col_block must be >= 0");
  if (o.col_block == 0) o.col_block = r > 64 ? r : 64;
  if (o.col_block < r) return arg_error("col_block must be >= r");
  if (!(o.tau >= 0.0)) return arg_error("tau must be >= 0");
  if (o.tau == 0.0) o.tau = 1e-13;
  (void)dtype;
  if (o.max_swaps < 0) return arg_error("max_swaps must be >= 0");
  if (o.max_swaps == 0) o.max_swaps = 64 * r;
  if (o.prec < CUR_PREC_NATIVE || o.prec > CUR_PREC_FP8) return arg_error("prec out of range");
  if (o.propose != 0 && o.propose != 1) return arg_error("propose must be 0 (none) or 1 (learned proposal)");
  if (o.propose == 1) {
    if (!o.mlp) return arg_error("propose == 1 needs the weight blob in mlp");
    if (r > 64) return arg_error("propose == 1 supports r <= 64");
    if (o.col_block > 64) return arg_error("propose == 1 supports col_block <= 64");
    if (o.method != 0) return arg_error("propose == 1 applies to the maximal-volume method only");
  }
  if (o.groups < 0 || o.groups > 3) return arg_error("groups must be 0 (autotuned) or 1..3");
  if (o.method != 0 && o.method != 1) return arg_error("method must be 0 (maximal volume) or 1 (norm-greedy)");
  if (o.propose == 0 && o.mlp != nullptr) return arg_error("mlp must be NULL when propose == 0");
  if (o.polish != 0 && o.polish != 1) return arg_error("polish must be 0 or 1");
  if (o.polish == 1 && o.method != 0) return arg_error("polish == 1 applies to the maximal-volume method only");
  if (o.polish == 1 && (int64_t)r * n > 0x7fffffff) return arg_error("polish == 1 needs r * n < 2^31");
  if (o.trace) {
    int64_t b = n / o.col_block;
    if (b < 1) b = 1;
    int64_t tot = 0;
    for (int64_t c = b;;) {
      tot += c;
      if (c <= 1) break;
      c = (c + 1) / 2;
    }
    if (o.method == 1) tot = 1;  // one record: the choice orders
    else if (o.polish == 1) tot += 1;  // the polish record
    if (!o.trace->meta || !o.trace->vol_mant || !o.trace->I || !o.trace->J)
      return arg_error("cur_trace arrays must be non-NULL");
    if (o.trace->capacity < tot) return arg_error("cur_trace.capacity too small for the tree");
  }
  (void)n;
  *out = o;
  return CUR_OK;
}

}  // namespace cur

using namespace cur;

extern "C" {

void cur_opts_init(cur_opts* opts) {
  if (!opts) return;
  std::memset(opts, 0, sizeof(*opts));
  opts->struct_size = sizeof(cur_opts);
}

const char* cur_strerror(cur_status s) {
  switch (s) {
    case CUR_OK: return "ok";
    case CUR_WARN_NOCONV: return "swap budget exhausted; dominance not certified";
    case CUR_ERR_ARG: return "invalid argument";
    case CUR_ERR_RANK: return "matrix rank below r";
    case CUR_ERR_NONFINITE: return "non-finite input";
    case CUR_ERR_DEVICE: return "HIP device error";
    case CUR_ERR_NOMEM: return "out of device memory";
    case CUR_ERR_INTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* cur_last_error(void) { return last_error(); }

cur_status cur_create(cur_ctx* out, int device, void* hip_stream) {
  if (!out) return arg_error("out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count < 1) {
    set_error(std::string("no HIP device: ") + (e == hipSuccess ? "count 0" : hipGetErrorString(e)));
    return CUR_ERR_DEVICE;
  }
  if (device < 0 || device >= count) return arg_error("device index out of range");
  CUR_HIP_CHECK(hipSetDevice(device));
  cur_ctx c = new cur_ctx_s();
  c->device = device;
  c->arena = nullptr;
  c->arena_bytes = 0;
  c->last_pinv = 0;
  c->rect_discard = nullptr;
  c->prof_on = 0;
  c->prof_bytes = nullptr;
  c->prof_ev = new std::vector<hipEvent_t>();
  c->prof_kind = new std::vector<int>();
  std::memset(&c->prof, 0, sizeof(c->prof));
  c->groups_ready = 0;
  c->tune = new std::vector<cur::TuneEntry>();
  c->stream = (hipStream_t)hip_stream;  // NULL: the null stream
  c->own_stream = false;
  e = hipHostMalloc((void**)&c->host_flag, 64, hipHostMallocDefault);
  if (e != hipSuccess) {
    if (c->own_stream) hipStreamDestroy(c->stream);
    delete c;
    set_error(std::string("hipHostMalloc: ") + hipGetErrorString(e));
    return CUR_ERR_DEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->cu_count = prop.multiProcessorCount;
  else c->cu_count = 256;
  cur_status ns = noalloc_init(device);  // device address of this GPU's no-allocation scratch
  if (ns != CUR_OK) {
    hipHostFree(c->host_flag);
    delete c->prof_ev;
    delete c->prof_kind;
    delete c->tune;
    delete c;
    return ns;
  }
  *out = c;
  return CUR_OK;
}

cur_status cur_destroy(cur_ctx ctx) {
  if (!ctx) return arg_error("ctx is NULL");
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  if (ctx->arena) hipFree(ctx->arena);
  if (ctx->host_flag) hipHostFree(ctx->host_flag);
  if (ctx->own_stream) hipStreamDestroy(ctx->stream);
  if (ctx->prof_bytes) hipFree(ctx->prof_bytes);
  if (ctx->rect_discard) hipFree(ctx->rect_discard);
  for (hipEvent_t e : *ctx->prof_ev) hipEventDestroy(e);
  if (ctx->groups_ready) {
    for (int g = 0; g < 4; ++g) {
      hipStreamSynchronize(ctx->gstream[g]);
      hipStreamDestroy(ctx->gstream[g]);
      hipEventDestroy(ctx->gjoin[g]);
    }
    hipEventDestroy(ctx->gfork);
  }
  delete ctx->prof_ev;
  delete ctx->prof_kind;
  delete ctx->tune;
  delete ctx;
  return CUR_OK;
}

cur_status cur_select(cur_ctx ctx, int32_t dtype_in, const void* A, int64_t m, int64_t n, int64_t lda,
                      int32_t r, const cur_opts* opts, int64_t* I, int64_t* J, cur_info* info) {
  cur_status st = check_matrix(dtype_in, A, m, n, lda, r);
  if (st != CUR_OK) return st;
  const cur_dtype dtype = (cur_dtype)dtype_in;  // a valid enumerator from here on
  st = check_select_rows(dtype, m);
  if (st != CUR_OK) return st;
  if (!I || !J) return arg_error("I and J must be non-NULL device pointers");
  cur_opts o;
  st = resolve_opts(opts, dtype, r, n, &o);
  if (st != CUR_OK) return st;
  if (!ctx) return arg_error("ctx is NULL");
  CUR_HIP_CHECK(hipSetDevice(ctx->device));
  set_error("");
  if (o.method == 1) return greedy_dispatch(ctx, dtype, A, m, n, lda, r, I, J, info, o.trace);
  return select_dispatch(ctx, dtype, A, m, n, lda, r, o, I, J, info);
}

cur_status cur_assemble(cur_ctx ctx, int32_t dtype_in, const void* A, int64_t m, int64_t n, int64_t lda,
                        int32_t r, const int64_t* I, const int64_t* J, void* C, double* U, void* R) {
  cur_status st = check_matrix(dtype_in, A, m, n, lda, r);
  if (st != CUR_OK) return st;
  const cur_dtype dtype = (cur_dtype)dtype_in;
  if (!I || !J || !C || !U || !R) return arg_error("I, J, C, U and R must be non-NULL device pointers");
  if (!ctx) return arg_error("ctx is NULL");
  CUR_HIP_CHECK(hipSetDevice(ctx->device));
  // indices must be in range: checked on a host copy (r values each)
  std::vector<int64_t> hI(r), hJ(r);
  CUR_HIP_CHECK(hipMemcpyAsync(hI.data(), I, sizeof(int64_t) * r, hipMemcpyDeviceToHost, ctx->stream));
  CUR_HIP_CHECK(hipMemcpyAsync(hJ.data(), J, sizeof(int64_t) * r, hipMemcpyDeviceToHost, ctx->stream));
  CUR_HIP_CHECK(hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < r; ++k)
    if (hI[k] < 0 || hI[k] >= m || hJ[k] < 0 || hJ[k] >= n) return arg_error("I or J entry out of range");
  set_error("");
  return assemble_dispatch(ctx, dtype, A, m, n, lda, r, I, J, C, U, R);
}

cur_status cur_residual(cur_ctx ctx, int32_t dtype_in, const void* A, int64_t m, int64_t n, int64_t lda,
                        int32_t r, const void* C, const double* U, const void* R, int32_t prec,
                        double* cheb, double* fro_rel) {
  cur_status st = check_matrix(dtype_in, A, m, n, lda, r);
  if (st != CUR_OK) return st;
  const cur_dtype dtype = (cur_dtype)dtype_in;
  if (!C || !U || !R) return arg_error("C, U and R must be non-NULL device pointers");
  if (!cheb) return arg_error("cheb must be a non-NULL host pointer");
  if (prec < CUR_PREC_NATIVE || prec > CUR_PREC_FP8) return arg_error("prec out of range");
  if (dtype == CUR_F64 && prec != CUR_PREC_NATIVE) return arg_error("FP64 input takes CUR_PREC_NATIVE");
  if (!ctx) return arg_error("ctx is NULL");
  CUR_HIP_CHECK(hipSetDevice(ctx->device));
  set_error("");
  return residual_dispatch(ctx, dtype, A, m, n, lda, r, C, U, R, prec, cheb, fro_rel);
}

cur_status cur_residual_noalloc(cur_ctx ctx, int32_t dtype_in, const void* A, int64_t m, int64_t n, int64_t lda,
                                int32_t r, const void* C, const double* U, const void* R, int32_t prec,
                                double* cheb, double* fro_rel) {
  cur_status st = check_matrix(dtype_in, A, m, n, lda, r);
  if (st != CUR_OK) return st;
  const cur_dtype dtype = (cur_dtype)dtype_in;
  if (!C || !U || !R) return arg_error("C, U and R must be non-NULL device pointers");
  if (!cheb) return arg_error("cheb must be a non-NULL host pointer");
  if (prec < CUR_PREC_NATIVE || prec > CUR_PREC_FP8) return arg_error("prec out of range");
  if (dtype == CUR_F64 && prec != CUR_PREC_NATIVE) return arg_error("FP64 input takes CUR_PREC_NATIVE");
  const size_t need = residual_noalloc_need(m, n, r, prec);
  if (need > CUR_NOALLOC_SCRATCH_BYTES)
    return arg_error("the call needs " + std::to_string(need) + " bytes of scratch, more than the " +
                     std::to_string(CUR_NOALLOC_SCRATCH_BYTES) + " bytes of CUR_NOALLOC_SCRATCH_BYTES");
  if (!ctx) return arg_error("ctx is NULL");
  CUR_HIP_CHECK(hipSetDevice(ctx->device));
  set_error("");
  return residual_noalloc_dispatch(ctx, dtype, A, m, n, lda, r, C, U, R, prec, cheb, fro_rel);
}

// ---- rectangular cross: r rows, c columns
static cur_status check_rect(int32_t dtype, const void* A, int64_t m, int64_t n, int64_t lda, int32_t r, int32_t c) {
  cur_status st = check_matrix(dtype, A, m, n, lda, 1);
  if (st != CUR_OK) return st;
  const int64_t mn = std::min(m, n);
  if (r < 1 || c < 1 || r > mn || c > mn) return arg_error("r and c must satisfy 1 <= r, c <= min(m, n)");
  if (r > 128 || c > 128) return arg_error("r, c > 128 are not supported (kernels are instantiated for <= 128)");
  return CUR_OK;
}

cur_status cur_select_rect(cur_ctx ctx, int32_t dtype_in, const void* A, int64_t m, int64_t n, int64_t lda, int32_t r,
                           int32_t c, const cur_opts* opts, int64_t* I, int64_t* J, cur_info* info) {
  cur_status st = check_rect(dtype_in, A, m, n, lda, r, c);
  if (st != CUR_OK) return st;
  const cur_dtype dtype = (cur_dtype)dtype_in;
  st = check_select_rows(dtype, std::max(m, n));  // the row tree runs on A^T (n rows)
  if (st != CUR_OK) return st;
  if (!I || !J) return arg_error("I and J must be non-NULL device pointers");
  cur_opts o;
  st = resolve_opts(opts, dtype, std::max(r, c), n, &o);  // the leaf width must hold either rank
  if (st != CUR_OK) return st;
  if (o.trace) return arg_error("cur_select_rect takes no trace");
  if (o.propose != 0) return arg_error("cur_select_rect takes no learned proposal");
  if (o.polish != 0 && r != c) return arg_error("cur_select_rect: polish needs r == c");
  if (!ctx) return arg_error("ctx is NULL");
  CUR_HIP_CHECK(hipSetDevice(ctx->device));
  set_error("");
  if (o.method == 1) return greedy_rect_dispatch(ctx, dtype, A, m, n, lda, r, c, I, J, info);
  if (!ctx->rect_discard) CUR_HIP_CHECK(hipMalloc(&ctx->rect_discard, 256 * sizeof(int64_t)));
  return select_rect_dispatch(ctx, dtype, A, m, n, lda, r, c, o, I, J, ctx->rect_discard, info);
}

cur_status cur_assemble_rect(cur_ctx ctx, int32_t dtype_in, const void* A, int64_t m, int64_t n, int64_t lda,
                             int32_t r, int32_t c, const int64_t* I, const int64_t* J, void* C, double* U, void* R) {
  cur_status st = check_rect(dtype_in, A, m, n, lda, r, c);
  if (st != CUR_OK) return st;
  if (std::min(r, c) > 64) return arg_error("cur_assemble_rect needs min(r, c) <= 64");
  const cur_dtype dtype = (cur_dtype)dtype_in;
  if (!I || !J || !C || !U || !R) return arg_error("I, J, C, U and R must be non-NULL device pointers");
  if (!ctx) return arg_error("ctx is NULL");
  CUR_HIP_CHECK(hipSetDevice(ctx->device));
  std::vector<int64_t> hI(r), hJ(c);
  CUR_HIP_CHECK(hipMemcpyAsync(hI.data(), I, sizeof(int64_t) * r, hipMemcpyDeviceToHost, ctx->stream));
  CUR_HIP_CHECK(hipMemcpyAsync(hJ.data(), J, sizeof(int64_t) * c, hipMemcpyDeviceToHost, ctx->stream));
  CUR_HIP_CHECK(hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < r; ++k)
    if (hI[k] < 0 || hI[k] >= m) return arg_error("I entry out of range");
  for (int k = 0; k < c; ++k)
    if (hJ[k] < 0 || hJ[k] >= n) return arg_error("J entry out of range");
  set_error("");
  return assemble_rect_dispatch(ctx, dtype, A, m, n, lda, r, c, I, J, C, U, R);
}

cur_status cur_residual_rect(cur_ctx ctx, int32_t dtype_in, const void* A, int64_t m, int64_t n, int64_t lda,
                             int32_t r, int32_t c, const void* C, const double* U, const void* R, double* cheb,
                             double* fro_rel) {
  cur_status st = check_rect(dtype_in, A, m, n, lda, r, c);
  if (st != CUR_OK) return st;
  if (!C || !U || !R) return arg_error("C, U and R must be non-NULL device pointers");
  if (!cheb) return arg_error("cheb must be a non-NULL host pointer");
  if (!ctx) return arg_error("ctx is NULL");
  CUR_HIP_CHECK(hipSetDevice(ctx->device));
  set_error("");
  return residual_rect_dispatch(ctx, (cur_dtype)dtype_in, A, m, n, lda, r, c, C, U, R, cheb, fro_rel);
}

cur_status cur_mlp_features(cur_ctx ctx, int32_t dtype_in, const void* A, int64_t m, int64_t n, int64_t lda, int32_t r,
                            int32_t col_block, uint64_t seed, float* F) {
  cur_status st = check_matrix(dtype_in, A, m, n, lda, r);
  if (st != CUR_OK) return st;
  if (r > 64) return arg_error("the proposal features support r <= 64");
  if (col_block < 0) return arg_error("col_block must be >= 0");
  const int w = col_block == 0 ? (r > 64 ? r : 64) : col_block;
  if (w < r) return arg_error("col_block must be >= r");
  if (w > 64) return arg_error("the proposal features support col_block <= 64");
  if (!F) return arg_error("F must be a non-NULL device pointer");
  if (!ctx) return arg_error("ctx is NULL");
  CUR_HIP_CHECK(hipSetDevice(ctx->device));
  set_error("");
  return propose_features(ctx, (cur_dtype)dtype_in, A, m, n, lda, r, w, seed, F);
}

cur_status cur_mlp_forward(cur_ctx ctx, const void* blob, const float* F, int64_t count, float* score) {
  if (!blob || !F || !score) return arg_error("blob, F and score must be non-NULL device pointers");
  if (count < 0) return arg_error("count must be >= 0");
  if (!ctx) return arg_error("ctx is NULL");
  if (count == 0) return CUR_OK;
  CUR_HIP_CHECK(hipSetDevice(ctx->device));
  set_error("");
  return mlp_forward_dispatch(ctx, blob, F, count, score);
}

cur_status cur_mlp_grad(cur_ctx ctx, const void* blob, const float* F, const float* y, int64_t count, float pos_weight,
                        float* grad, double* loss) {
  if (!blob || !F || !y || !grad) return arg_error("blob, F, y and grad must be non-NULL device pointers");
  if (count < 1) return arg_error("count must be >= 1");
  if (!(pos_weight > 0.0f)) return arg_error("pos_weight must be > 0");
  if (!ctx) return arg_error("ctx is NULL");
  CUR_HIP_CHECK(hipSetDevice(ctx->device));
  set_error("");
  return mlp_grad_dispatch(ctx, blob, F, y, count, pos_weight, grad, loss);
}

cur_status cur_mlp_adam(cur_ctx ctx, void* blob, float* params, float* m1, float* m2, const float* grad, int32_t step,
                        float lr, float beta1, float beta2, float eps) {
  if (!blob || !params || !m1 || !m2 || !grad) return arg_error("blob, params, m1, m2 and grad must be non-NULL");
  if (step < 1) return arg_error("step must be >= 1");
  if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return arg_error("Adam hyper-parameters out of range");
  if (!ctx) return arg_error("ctx is NULL");
  CUR_HIP_CHECK(hipSetDevice(ctx->device));
  set_error("");
  return mlp_adam_dispatch(ctx, blob, params, m1, m2, grad, step, lr, beta1, beta2, eps);
}

cur_status cur_tune_export(cur_ctx ctx, cur_tune_entry* out, int32_t cap, int32_t* count) {
  if (!ctx || !count) return arg_error("ctx and count must be non-NULL");
  if (cap < 0 || (cap > 0 && !out)) return arg_error("out must hold cap >= 0 entries");
  const std::vector<cur::TuneEntry>& t = *ctx->tune;
  *count = (int32_t)t.size();
  for (int32_t k = 0; k < cap && k < (int32_t)t.size(); ++k) {
    const cur::TuneEntry& e = t[k];
    cur_tune_entry& o = out[k];
    std::copy(e.key, e.key + 6, o.key);
    std::copy(e.ms, e.ms + 3, o.ms);
    o.tried = e.tried;
    o.groups = e.fixed > 0 ? e.fixed : (e.tried >= 3 ? cur::tune_best(e) : 0);
  }
  return CUR_OK;
}

cur_status cur_tune_import(cur_ctx ctx, const cur_tune_entry* in, int32_t count) {
  if (!ctx) return arg_error("ctx is NULL");
  if (count < 0 || (count > 0 && !in)) return arg_error("in must hold count >= 0 entries");
  std::vector<cur::TuneEntry> t;
  for (int32_t k = 0; k < count; ++k) {
    const cur_tune_entry& i = in[k];
    if (i.groups < 0 || i.groups > 3 || i.tried < 0 || i.tried > 3) return arg_error("tune entry out of range");
    cur::TuneEntry e;
    std::copy(i.key, i.key + 6, e.key);
    std::copy(i.ms, i.ms + 3, e.ms);
    e.tried = i.tried;
    e.fixed = i.groups;
    t.push_back(e);
  }
  *ctx->tune = t;
  return CUR_OK;
}

cur_status cur_profile_enable(cur_ctx ctx, int enable) {
  if (!ctx) return arg_error("ctx is NULL");
  if (enable < 0 || enable > 2) return arg_error("enable must be 0, 1 or 2");
  CUR_HIP_CHECK(hipSetDevice(ctx->device));
  if (enable && !ctx->prof_bytes)
    CUR_HIP_CHECK(hipMalloc((void**)&ctx->prof_bytes, sizeof(unsigned long long) * 2 * cur::kProfSlots));
  std::memset(&ctx->prof, 0, sizeof(ctx->prof));
  ctx->prof_on = enable;
  return CUR_OK;
}

cur_status cur_profile_read(cur_ctx ctx, cur_profile* out) {
  if (!ctx || !out) return arg_error("ctx and out must be non-NULL");
  *out = ctx->prof;  // accumulated at the end of every profiled selection
  return CUR_OK;
}

cur_status cur_select_batched(cur_ctx ctx, int32_t count, const cur_item* items, const cur_opts* opts,
                              cur_status* per_item) {
  if (count < 0) return arg_error("count must be >= 0");
  if (count > 0 && !items) return arg_error("items is NULL");
  if (opts && opts->trace) return arg_error("opts->trace must be NULL for batched selection");
  if (opts && opts->struct_size == (int32_t)sizeof(cur_opts) && opts->method != 0)
    return arg_error("batched selection supports the maximal-volume method only");
  if (opts && opts->struct_size == (int32_t)sizeof(cur_opts) && opts->propose != 0)
    return arg_error("batched selection supports no candidate proposal");
  for (int32_t i = 0; i < count; ++i) {
    const cur_item& it = items[i];
    cur_status st = check_matrix(it.dtype, it.A, it.m, it.n, it.lda, it.r);
    if (st == CUR_OK) st = check_select_rows((cur_dtype)it.dtype, it.m);
    if (st != CUR_OK) return arg_error("item " + std::to_string(i) + ": " + last_error());
    if (!it.I || !it.J) return arg_error("item " + std::to_string(i) + ": I and J must be non-NULL");
    cur_opts o;
    st = resolve_opts(opts, (cur_dtype)it.dtype, it.r, it.n, &o);
    if (st != CUR_OK) return arg_error("item " + std::to_string(i) + ": " + last_error());
  }
  if (!ctx) return arg_error("ctx is NULL");
  CUR_HIP_CHECK(hipSetDevice(ctx->device));
  std::vector<cur_opts> ro(count);
  for (int32_t i = 0; i < count; ++i) resolve_opts(opts, (cur_dtype)items[i].dtype, items[i].r, items[i].n, &ro[i]);
  std::vector<cur_status> st(count, CUR_OK);
  cur_status rc = select_batched_dispatch(ctx, count, items, ro, st.data());
  if (rc != CUR_OK) return rc;
  cur_status worst = CUR_OK;
  for (int32_t i = 0; i < count; ++i) {
    if (per_item) per_item[i] = st[i];
    if (st[i] < 0 && (worst >= 0 || st[i] < worst)) worst = st[i];
    else if (worst == CUR_OK && st[i] > 0) worst = st[i];
  }
  return worst;
}

}  // extern "C"
