// Host argument paths of libcur under AddressSanitizer and UBSan: every
// argument error of the C ABI is exercised with a NULL context (no device
// work is reached), plus context creation without a usable GPU.  Built and
// run by tests/test_sanitizers.py; prints OK and exits 0 when every call
// returns the documented status.
#include <cstdio>
#include <cstring>
#include "cur.h"
int main() {
  int bad = 0;
  cur_opts o; cur_opts_init(&o);
  int64_t dummy = 0;
  cur_info info;
  // select: every argument error path
  struct { int64_t m, n, lda; int r; const void* A; int dtype; } cs[] = {
    {10, 12, 12, 0, &dummy, 0}, {10, 12, 12, 11, &dummy, 0}, {0, 12, 12, 3, &dummy, 0},
    {10, 12, 5, 3, &dummy, 0}, {10, 12, 12, 3, nullptr, 0}, {10, 12, 12, 3, &dummy, 7},
    {300, 300, 300, 200, &dummy, 0}, {1ll << 29, 64, 64, 3, &dummy, 0}};
  for (auto& c : cs) bad |= cur_select(nullptr, (cur_dtype)c.dtype, c.A, c.m, c.n, c.lda, c.r, &o, &dummy, &dummy, &info) != CUR_ERR_ARG;
  for (int f = 0; f < 9; ++f) {
    cur_opts p; cur_opts_init(&p);
    switch (f) { case 0: p.col_block = 2; break; case 1: p.col_block = -1; break; case 2: p.tau = -1; break;
      case 3: p.max_swaps = -3; break; case 4: p.prec = 9; break; case 5: p.propose = 1; break;
      case 6: p.struct_size = 8; break; case 7: p.groups = 4; break; case 8: p.method = 2; break; }
    bad |= cur_select(nullptr, CUR_F64, &dummy, 10, 12, 12, 3, &p, &dummy, &dummy, &info) != CUR_ERR_ARG;
    bad |= std::strlen(cur_last_error()) == 0;
  }
  cur_trace tr; std::memset(&tr, 0, sizeof(tr)); tr.capacity = 1;
  cur_opts t; cur_opts_init(&t); t.trace = &tr;
  bad |= cur_select(nullptr, CUR_F64, &dummy, 10, 300, 300, 3, &t, &dummy, &dummy, &info) != CUR_ERR_ARG;
  bad |= cur_select(nullptr, CUR_F64, &dummy, 10, 12, 12, 3, &o, &dummy, &dummy, &info) != CUR_ERR_ARG;  // NULL ctx
  bad |= cur_assemble(nullptr, CUR_F64, &dummy, 10, 12, 12, 3, &dummy, &dummy, nullptr, (double*)&dummy, &dummy) != CUR_ERR_ARG;
  double cheb;
  bad |= cur_residual(nullptr, CUR_F64, &dummy, 10, 12, 12, 3, &dummy, (double*)&dummy, &dummy, CUR_PREC_FP8, &cheb, nullptr) != CUR_ERR_ARG;
  bad |= cur_residual_noalloc(nullptr, CUR_F64, &dummy, 40000, 64, 64, 64, &dummy, (double*)&dummy, &dummy, 0, &cheb,
                              nullptr) != CUR_ERR_ARG;  // beyond CUR_NOALLOC_SCRATCH_BYTES
  bad |= cur_residual_noalloc(nullptr, 9, &dummy, 100, 64, 64, 8, &dummy, (double*)&dummy, &dummy, 0, &cheb,
                              nullptr) != CUR_ERR_ARG;  // dtype out of range
  cur_item it[2]; std::memset(it, 0, sizeof(it));
  bad |= cur_select_batched(nullptr, 2, it, nullptr, nullptr) != CUR_ERR_ARG;
  bad |= cur_select_batched(nullptr, -1, nullptr, nullptr, nullptr) != CUR_ERR_ARG;
  int32_t cnt;
  bad |= cur_tune_export(nullptr, nullptr, 0, &cnt) != CUR_ERR_ARG;
  bad |= cur_tune_import(nullptr, nullptr, 0) != CUR_ERR_ARG;
  bad |= cur_profile_enable(nullptr, 1) != CUR_ERR_ARG;
  for (int s = -7; s <= 1; ++s) bad |= cur_strerror((cur_status)s) == nullptr;
  cur_ctx c = nullptr;
  cur_status cs2 = cur_create(&c, 0, nullptr);  // no GPU here: a device error, nothing leaked
  bad |= cs2 != CUR_ERR_DEVICE && cs2 != CUR_OK;
  if (c) cur_destroy(c);
  std::printf("%s\n", bad ? "FAIL" : "OK");
  return bad;
}
