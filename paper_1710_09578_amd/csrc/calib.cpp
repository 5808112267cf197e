// Run-time calibration of the evaluation path (section "Software
// description": the paper's classes time their algorithms at run time and
// pick the faster one per size and number of vectors). For a small operator
// (m, n <= 64) the library can apply either its structured transforms or a
// dense product with the operator's matrix; fm_op_calibrate times both on
// the caller's column count and keeps the faster for later applications. The
// dense matrix is materialised once, through the complex128 instantiation of
// the operator's own transforms applied to the identity, and rounded once
// for complex64.
#include <mutex>
#include <vector>

#include "runtime.h"

using namespace fm;

namespace {

std::mutex g_calib_mu;  // serialises building an operator's dense copy

fm_status build_dense(fm_op_s* a, hipStream_t s) {
  if (a->dense64.p != nullptr) return FM_OK;
  const int64_t m = a->m, n = a->n;
  DevBuf eye, d64, d32, wsb;
  std::vector<double> h(size_t(n * n) * 2, 0.0);
  for (int64_t j = 0; j < n; ++j) h[2 * size_t(j * n + j)] = 1.0;
  FM_TRY(eye.alloc(h.size() * 8));
  FM_HIP(hipMemcpyAsync(eye.p, h.data(), h.size() * 8, hipMemcpyHostToDevice, s));
  FM_TRY(d64.alloc(size_t(m * n) * 16));
  const Batch b{n, 1, 1, n, n, m, m};
  Workspace sz;
  sz.sizing = true;
  FM_TRY(exec(a, false, Elem::C128, b, nullptr, nullptr, false, sz, s));
  FM_TRY(wsb.alloc(sz.peak > 0 ? sz.peak : 1));
  Workspace w;
  w.base = static_cast<char*>(wsb.p);
  w.cap = wsb.bytes;
  FM_TRY(exec(a, false, Elem::C128, b, eye.p, d64.p, false, w, s));  // column j = A e_j
  if (a->dt == FM_C64) {
    FM_TRY(d32.alloc(size_t(m * n) * 8));
    FM_TRY(launch_c128_to_c64(m * n, d64.p, d32.p, s));
  }
  FM_HIP(hipStreamSynchronize(s));
  std::swap(a->dense64.p, d64.p);
  std::swap(a->dense64.bytes, d64.bytes);
  std::swap(a->dense32.p, d32.p);
  std::swap(a->dense32.bytes, d32.bytes);
  return FM_OK;
}

}  // namespace

extern "C" {

fm_status fm_op_set_path(fm_op a, int32_t path) {
  set_error("");
  FM_CHECK_ARG(a != nullptr, FM_E_INVALID, "operator handle is NULL");
  FM_CHECK_ARG(op_alive(a), FM_E_RELEASED, "operator handle was released");
  FM_CHECK_ARG(path == 0 || path == 1, FM_E_INVALID, "path must be 0 (structured) or 1 (dense)");
  if (path == 1) {
    FM_CHECK_ARG(is_complex(a->dt), FM_E_DTYPE, "dense path for a complex operator only");
    FM_CHECK_ARG(a->m <= 64 && a->n <= 64, FM_E_UNSUPPORTED, "dense path for operators up to 64 x 64");
    std::lock_guard<std::mutex> lk(g_calib_mu);
    a->path.store(0, std::memory_order_release);
    FM_TRY(build_dense(a, nullptr));
  }
  a->path.store(path, std::memory_order_release);
  return FM_OK;
}

fm_status fm_op_calibrate(fm_op a, int64_t ncols, int32_t* choice, double* ms_fast, double* ms_dense,
                          void* stream) {
  set_error("");
  FM_CHECK_ARG(a != nullptr, FM_E_INVALID, "operator handle is NULL");
  FM_CHECK_ARG(op_alive(a), FM_E_RELEASED, "operator handle was released");
  FM_CHECK_ARG(is_complex(a->dt), FM_E_DTYPE, "calibration of a complex operator only");
  FM_CHECK_ARG(a->m <= 64 && a->n <= 64, FM_E_UNSUPPORTED, "calibration for operators up to 64 x 64");
  FM_CHECK_ARG(ncols >= 1 && ncols <= (int64_t(1) << 20), FM_E_INVALID, "ncols must be in 1 .. 2^20");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const Elem e = elem_of(a->dt);
  const size_t es = elem_bytes(e);
  std::lock_guard<std::mutex> lk(g_calib_mu);
  a->path.store(0, std::memory_order_release);
  FM_TRY(build_dense(a, s));
  const int64_t m = a->m, n = a->n;
  DevBuf x, y, wsb;
  FM_TRY(x.alloc(size_t(ncols * n) * es));
  FM_TRY(y.alloc(size_t(ncols * m) * es));
  FM_HIP(hipMemsetAsync(x.p, 0, x.bytes, s));
  const Batch b{ncols, 1, 1, n, n, m, m};
  Workspace sz;
  sz.sizing = true;
  FM_TRY(exec(a, false, e, b, nullptr, nullptr, false, sz, s));
  FM_TRY(wsb.alloc(sz.peak > 0 ? sz.peak : 1));
  Workspace w;
  w.base = static_cast<char*>(wsb.p);
  w.cap = wsb.bytes;
  const void* dm = e == Elem::C64 ? a->dense32.p : a->dense64.p;
  hipEvent_t t0, t1;
  FM_HIP(hipEventCreate(&t0));
  FM_HIP(hipEventCreate(&t1));
  double times[2] = {0.0, 0.0};
  fm_status st = FM_OK;
  for (int path = 0; path < 2 && st == FM_OK; ++path) {
    auto run = [&]() -> fm_status {
      if (path == 0) return exec(a, false, e, b, x.p, y.p, false, w, s);
      return launch_dense(e, m, n, dm, m, 0, 0, b, x.p, y.p, 0, s);
    };
    constexpr int kWarm = 2, kReps = 5;
    for (int r = 0; r < kWarm && st == FM_OK; ++r) st = run();
    if (st != FM_OK) break;
    if (hipEventRecord(t0, s) != hipSuccess) st = FM_E_DEVICE;
    for (int r = 0; r < kReps && st == FM_OK; ++r) st = run();
    if (st == FM_OK && hipEventRecord(t1, s) != hipSuccess) st = FM_E_DEVICE;
    float ms = 0.f;
    if (st == FM_OK && (hipEventSynchronize(t1) != hipSuccess || hipEventElapsedTime(&ms, t0, t1) != hipSuccess))
      st = FM_E_DEVICE;
    times[path] = double(ms) / kReps;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  FM_TRY(st);
  const int pick = times[1] < times[0] ? 1 : 0;
  a->path.store(pick, std::memory_order_release);
  if (choice) *choice = pick;
  if (ms_fast) *ms_fast = times[0];
  if (ms_dense) *ms_dense = times[1];
  return FM_OK;
}

}  // extern "C"
