// Run-time calibration of the evaluation path (section "Software
// description": the paper's classes time their algorithms at run time and
// pick the faster one per size and number of vectors). For a small operator
// (m, n <= 64) the library can apply either its structured transforms or a
// dense product with the operator's matrix; fm_op_calibrate times both on
// the caller's column count and keeps the faster for later applications. The
// dense matrix is materialised once, through the complex128 instantiation of
// the operator's own transforms applied to the identity, and rounded once
// for complex64.
#include <algorithm>
#include <cmath>
#include <map>
#include <cstring>
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

// Times the structured and the dense evaluation of `a` on ncols columns of
// zeros (2 warm-up and 5 timed applications each); the dense copy must exist.
fm_status time_paths(fm_op_s* a, int64_t ncols, hipStream_t s, double times[2]) {
  const Elem e = elem_of(a->dt);
  const size_t es = elem_bytes(e);
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
  return st;
}

// ---------------------------------------------------------------- calibration model
// Per device: the structured and dense times of three operator classes
// (circulant, Toeplitz, Fourier) in both complex dtypes on a grid of sizes and
// column counts, measured once and consulted for any handle.
constexpr int kSizes[] = {8, 16, 32, 48, 64};
constexpr int64_t kCols[] = {1, 16, 256, 4096, 65536};
constexpr int kNS = 5, kNC = 5;

struct Model {
  std::vector<fm_calib_entry> e;
};
std::mutex g_model_mu;
std::map<int, Model> g_models;

int class_of(const fm_op_s* a) {
  switch (a->kind) {
    case Kind::Circulant: return FM_CAL_CIRCULANT;
    case Kind::Toeplitz: return FM_CAL_TOEPLITZ;
    case Kind::Fourier: return FM_CAL_FOURIER;
    default: return -1;
  }
}

// Deterministic complex test values (a 64-bit LCG) for the model's operators.
std::vector<double> lcg_values(size_t count, uint64_t seed) {
  std::vector<double> v(count);
  uint64_t z = seed * 0x9E3779B97F4A7C15ull + 1;
  for (size_t i = 0; i < count; ++i) {
    z = z * 6364136223846793005ull + 1442695040888963407ull;
    v[i] = double(z >> 11) / double(uint64_t(1) << 53) - 0.5;
  }
  return v;
}

fm_status make_class_op(int cls, fm_dtype dt, int n, hipStream_t s, fm_op* out) {
  if (cls == FM_CAL_FOURIER) return fm_op_create_fourier(out, n, dt);
  const size_t es = dt == FM_C64 ? 8 : 16;
  std::vector<double> v = lcg_values(size_t(4 * n), uint64_t(cls * 1000 + n));
  std::vector<unsigned char> h(size_t(2 * n) * es);
  for (int i = 0; i < 2 * n; ++i) {
    if (dt == FM_C64) {
      const float re = float(v[2 * i]), im = float(v[2 * i + 1]);
      std::memcpy(h.data() + size_t(i) * 8, &re, 4);
      std::memcpy(h.data() + size_t(i) * 8 + 4, &im, 4);
    } else {
      std::memcpy(h.data() + size_t(i) * 16, &v[2 * i], 8);
      std::memcpy(h.data() + size_t(i) * 16 + 8, &v[2 * i + 1], 8);
    }
  }
  DevBuf d;
  FM_TRY(d.alloc(h.size()));
  FM_HIP(hipMemcpy(d.p, h.data(), h.size(), hipMemcpyHostToDevice));
  if (cls == FM_CAL_CIRCULANT) return fm_op_create_circulant(out, n, d.p, dt, s);
  return fm_op_create_toeplitz(out, n, n, d.p, static_cast<char*>(d.p) + size_t(n) * es, dt, s);
}

// log(ms_dense / ms_fast) of class `cls`, dtype `dt` at (size n, ncols),
// bilinear in (n, log2 ncols) between the grid points, clamped to the grid.
bool model_ratio(const Model& md, int cls, fm_dtype dt, int64_t n, int64_t ncols, double* r) {
  double grid[kNS][kNC];
  bool have[kNS][kNC] = {};
  for (const auto& en : md.e) {
    if (en.cls != cls || en.dt != int32_t(dt)) continue;
    const int* ps = std::find(kSizes, kSizes + kNS, en.n);
    const int64_t* pc = std::find(kCols, kCols + kNC, en.ncols);
    if (ps == kSizes + kNS || pc == kCols + kNC || !(en.ms_fast > 0.0) || !(en.ms_dense > 0.0)) continue;
    grid[ps - kSizes][pc - kCols] = std::log(en.ms_dense / en.ms_fast);
    have[ps - kSizes][pc - kCols] = true;
  }
  for (int i = 0; i < kNS; ++i)
    for (int j = 0; j < kNC; ++j)
      if (!have[i][j]) return false;
  const double fn = std::min<double>(std::max<double>(double(n), kSizes[0]), kSizes[kNS - 1]);
  const double lc = std::log2(std::min<double>(std::max<double>(double(ncols), double(kCols[0])),
                                               double(kCols[kNC - 1])));
  int i = 0, j = 0;
  while (i + 2 < kNS && fn > kSizes[i + 1]) ++i;
  while (j + 2 < kNC && lc > std::log2(double(kCols[j + 1]))) ++j;
  const double tn = (fn - kSizes[i]) / double(kSizes[i + 1] - kSizes[i]);
  const double c0 = std::log2(double(kCols[j])), c1 = std::log2(double(kCols[j + 1]));
  const double tc = (lc - c0) / (c1 - c0);
  *r = (1 - tn) * (1 - tc) * grid[i][j] + tn * (1 - tc) * grid[i + 1][j] + (1 - tn) * tc * grid[i][j + 1] +
       tn * tc * grid[i + 1][j + 1];
  return true;
}

}  // namespace

extern "C" {

fm_status fm_calibration_build(void* stream) {
  set_error("");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int dev = 0;
  FM_HIP(hipGetDevice(&dev));
  Model md;
  for (fm_dtype dt : {FM_C64, FM_C128}) {
    for (int cls : {FM_CAL_CIRCULANT, FM_CAL_TOEPLITZ, FM_CAL_FOURIER}) {
      for (int n : kSizes) {
        fm_op op = nullptr;
        FM_TRY(make_class_op(cls, dt, n, s, &op));
        fm_status st = FM_OK;
        {
          std::lock_guard<std::mutex> lk(g_calib_mu);
          st = build_dense(op, s);
          for (int64_t c : kCols) {
            if (st != FM_OK) break;
            double t[2] = {0.0, 0.0};
            st = time_paths(op, c, s, t);
            md.e.push_back(fm_calib_entry{int32_t(cls), int32_t(dt), int32_t(n), 0, c, t[0], t[1]});
          }
        }
        fm_op_release(op);
        FM_TRY(st);
      }
    }
  }
  std::lock_guard<std::mutex> lk(g_model_mu);
  g_models[dev] = std::move(md);
  return FM_OK;
}

fm_status fm_calibration_entries(fm_calib_entry* out, int32_t cap, int32_t* count) {
  set_error("");
  FM_CHECK_ARG(count != nullptr, FM_E_INVALID, "NULL count");
  int dev = 0;
  FM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_model_mu);
  auto it = g_models.find(dev);
  const int32_t n = it == g_models.end() ? 0 : int32_t(it->second.e.size());
  *count = n;
  if (out) {
    FM_CHECK_ARG(cap >= n, FM_E_INVALID, "room for %d entries given, %d needed", cap, n);
    for (int32_t i = 0; i < n; ++i) out[i] = it->second.e[size_t(i)];
  }
  return FM_OK;
}

fm_status fm_calibration_load(const fm_calib_entry* in, int32_t count) {
  set_error("");
  FM_CHECK_ARG(count >= 0 && (in != nullptr || count == 0), FM_E_INVALID, "bad table");
  for (int32_t i = 0; i < count; ++i) {
    FM_CHECK_ARG(in[i].cls >= 0 && in[i].cls <= 2 && (in[i].dt == FM_C64 || in[i].dt == FM_C128),
                 FM_E_INVALID, "entry %d: unknown class or dtype", i);
    FM_CHECK_ARG(in[i].ms_fast > 0.0 && in[i].ms_dense > 0.0 && std::isfinite(in[i].ms_fast) &&
                     std::isfinite(in[i].ms_dense),
                 FM_E_INVALID, "entry %d: times must be positive", i);
  }
  int dev = 0;
  FM_HIP(hipGetDevice(&dev));
  Model md;
  md.e.assign(in, in + count);
  std::lock_guard<std::mutex> lk(g_model_mu);
  g_models[dev] = std::move(md);
  return FM_OK;
}

fm_status fm_op_choose_path(fm_op a, int64_t ncols, int32_t* choice) {
  set_error("");
  FM_CHECK_ARG(a != nullptr, FM_E_INVALID, "operator handle is NULL");
  FM_CHECK_ARG(op_alive(a), FM_E_RELEASED, "operator handle was released");
  FM_CHECK_ARG(is_complex(a->dt), FM_E_DTYPE, "path choice for a complex operator only");
  FM_CHECK_ARG(a->m <= 64 && a->n <= 64, FM_E_UNSUPPORTED, "path choice for operators up to 64 x 64");
  FM_CHECK_ARG(ncols >= 1, FM_E_INVALID, "ncols must be positive");
  const int cls = class_of(a);
  FM_CHECK_ARG(cls >= 0, FM_E_UNSUPPORTED, "no model class for this operator kind (use fm_op_calibrate)");
  int dev = 0;
  FM_HIP(hipGetDevice(&dev));
  double r = 0.0;
  {
    std::lock_guard<std::mutex> lk(g_model_mu);
    auto it = g_models.find(dev);
    FM_CHECK_ARG(it != g_models.end(), FM_E_INVALID,
                 "no calibration model on this device (fm_calibration_build or fm_calibration_load)");
    FM_CHECK_ARG(model_ratio(it->second, cls, a->dt, std::max(a->m, a->n), ncols, &r), FM_E_INVALID,
                 "the calibration model lacks grid points for this class and dtype");
  }
  const int pick = r < 0.0 ? 1 : 0;
  FM_TRY(fm_op_set_path(a, pick));
  if (choice) *choice = pick;
  return FM_OK;
}

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
  std::lock_guard<std::mutex> lk(g_calib_mu);
  a->path.store(0, std::memory_order_release);
  FM_TRY(build_dense(a, s));
  double times[2] = {0.0, 0.0};
  FM_TRY(time_paths(a, ncols, s, times));
  const int pick = times[1] < times[0] ? 1 : 0;
  a->path.store(pick, std::memory_order_release);
  if (choice) *choice = pick;
  if (ms_fast) *ms_fast = times[0];
  if (ms_dense) *ms_dense = times[1];
  return FM_OK;
}

}  // extern "C"
