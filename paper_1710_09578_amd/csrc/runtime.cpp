// Runtime support: error text, device buffers, twiddle tables, live-handle
// registry and the per-precision split of long transforms.
#include <cstdlib>
#include "runtime.h"

#include <cmath>
#include <cstdarg>
#include <map>
#include <mutex>
#include <unordered_set>

namespace fm {

// ---------------------------------------------------------------- errors
namespace {
thread_local char g_err[512] = "";
}
void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
const char* last_error() { return g_err; }

// ---------------------------------------------------------------- buffers
fm_status DevBuf::alloc(size_t n) {
  reset();
  if (n == 0) return FM_OK;
  hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) {
    p = nullptr;
    set_error("hipMalloc(%zu) failed: %s", n, hipGetErrorName(e));
    return e == hipErrorOutOfMemory ? FM_E_NOMEM : FM_E_DEVICE;
  }
  bytes = n;
  return FM_OK;
}
void DevBuf::reset() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

Elem elem_of(fm_dtype dt) {
  switch (dt) {
    case FM_C64: return Elem::C64;
    case FM_C128: return Elem::C128;
    case FM_I32: return Elem::I32;
    default: return Elem::I64;
  }
}

int conv_max_fuse() {
  static const int v = [] {
    const char* e = std::getenv("FM_MAX_FUSE");
    int k = e ? std::atoi(e) : 3;  // measured best on a log-uniform Toeplitz mix
    return k < 0 ? 0 : (k > 5 ? 5 : k);
  }();
  return v;
}

Split split_for(Elem e, int logL) {
  Split s;
  s.logL = logL;
  const int lim = fft_lds_max_log(e);
  if (logL <= lim) {
    s.log1 = logL;
    s.log2 = 0;
  } else {
    // the contiguous factor takes the full single-pass length; the strided
    // factor (2^1 .. 2^8 for L up to 2^20) lets a strided pass cover many
    // neighbouring vectors per work-group, i.e. long contiguous runs
    s.log1 = lim;
    s.log2 = logL - lim;
  }
  s.n2 = 1 << s.log2;
  return s;
}

bool mixed_n2_ok(int n2) {
  switch (n2) {
    case 3: case 5: case 6: case 9: case 10: case 12: case 20: case 24: case 30:
      return true;
    default:
      return false;
  }
}

Split split_mixed(int64_t L) {
  Split s;
  s.logL = -1;
  s.log1 = 12;
  s.log2 = -1;
  s.n2 = int(L >> 12);
  return s;
}

// ---------------------------------------------------------------- twiddles
namespace {
constexpr int kTwiddleLogMax = 20;

struct Tables {
  void* t32 = nullptr;
  void* t64 = nullptr;
};
std::mutex g_tw_mu;
std::map<int, Tables> g_tw;

}  // namespace

// exp(-2 pi j k / size), reduced to an angle of at most pi/4 before calling
// cos/sin, then rotated by whole quadrants (exact).
void root_of_unity(int64_t k, int64_t size, double* re, double* im) {
  if (size == 1) {
    *re = 1.0;
    *im = 0.0;
    return;
  }
  if (size == 2) {
    *re = k ? -1.0 : 1.0;
    *im = 0.0;
    return;
  }
  const int64_t quarter = size / 4;
  const int64_t q = k / quarter, r = k % quarter;
  double c, s;  // cos, sin of 2 pi r / size, r < size/4
  if (2 * r <= quarter) {
    const double a = 2.0 * M_PI * double(r) / double(size);
    c = std::cos(a);
    s = std::sin(a);
  } else {
    const double a = 2.0 * M_PI * double(quarter - r) / double(size);
    c = std::sin(a);
    s = std::cos(a);
  }
  for (int64_t i = 0; i < q; ++i) {  // add a quarter turn: (c, s) -> (-s, c)
    const double t = c;
    c = -s;
    s = t;
  }
  *re = c;
  *im = (s == 0.0) ? 0.0 : -s;
}

const void* twiddle_table(Elem e, int logmax) {
  if (logmax > kTwiddleLogMax) {
    set_error("twiddle table: length 2^%d above 2^%d", logmax, kTwiddleLogMax);
    return nullptr;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_error("twiddle table: hipGetDevice failed");
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_tw_mu);
  Tables& t = g_tw[dev];
  if (!t.t64) {
    const int64_t total = int64_t(2) << kTwiddleLogMax;
    std::vector<double> h64(2 * total, 0.0);
    std::vector<float> h32(2 * total, 0.0f);
    for (int l = 0; l <= kTwiddleLogMax; ++l) {
      const int64_t size = int64_t(1) << l;
      for (int64_t k = 0; k < size; ++k) {
        double re, im;
        root_of_unity(k, size, &re, &im);
        h64[2 * (size + k)] = re;
        h64[2 * (size + k) + 1] = im;
        h32[2 * (size + k)] = float(re);
        h32[2 * (size + k) + 1] = float(im);
      }
    }
    void *d64 = nullptr, *d32 = nullptr;
    if (hipMalloc(&d64, h64.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&d32, h32.size() * sizeof(float)) != hipSuccess ||
        hipMemcpy(d64, h64.data(), h64.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d32, h32.data(), h32.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
      if (d64) (void)hipFree(d64);
      if (d32) (void)hipFree(d32);
      set_error("twiddle table: allocation or upload failed");
      return nullptr;
    }
    t.t64 = d64;
    t.t32 = d32;
  }
  return e == Elem::C64 ? t.t32 : t.t64;
}

namespace {
struct MixedTables {
  std::map<int64_t, void*> t32, t64;
};
std::map<int, MixedTables> g_twm;
}  // namespace

const void* twiddle_table_L(Elem e, int64_t L) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_error("twiddle table: hipGetDevice failed");
    return nullptr;
  }
  if (L % 4096 != 0 || !mixed_n2_ok(int(L / 4096))) {
    set_error("twiddle table: unsupported mixed length %lld", (long long)L);
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_tw_mu);
  MixedTables& mt = g_twm[dev];
  auto& slot = e == Elem::C64 ? mt.t32 : mt.t64;
  auto it = slot.find(L);
  if (it != slot.end()) return it->second;
  std::vector<double> h64(size_t(2 * L));
  std::vector<float> h32(size_t(2 * L));
  for (int64_t k = 0; k < L; ++k) {
    double re, im;
    root_of_unity(k, L, &re, &im);
    h64[2 * k] = re;
    h64[2 * k + 1] = im;
    h32[2 * k] = float(re);
    h32[2 * k + 1] = float(im);
  }
  void* d = nullptr;
  const size_t bytes = e == Elem::C64 ? h32.size() * sizeof(float) : h64.size() * sizeof(double);
  const void* src = e == Elem::C64 ? static_cast<const void*>(h32.data()) : static_cast<const void*>(h64.data());
  if (hipMalloc(&d, bytes) != hipSuccess || hipMemcpy(d, src, bytes, hipMemcpyHostToDevice) != hipSuccess) {
    if (d) (void)hipFree(d);
    set_error("twiddle table: allocation or upload failed");
    return nullptr;
  }
  slot[L] = d;
  return d;
}

// ---------------------------------------------------------------- live handles
namespace {
std::mutex g_live_mu;
std::unordered_set<const fm_op_s*>& live() {
  static std::unordered_set<const fm_op_s*> s;
  return s;
}
}  // namespace
void register_op(const fm_op_s* op) {
  std::lock_guard<std::mutex> lock(g_live_mu);
  live().insert(op);
}
void unregister_op(const fm_op_s* op) {
  std::lock_guard<std::mutex> lock(g_live_mu);
  live().erase(op);
}
bool op_alive(const fm_op_s* op) {
  std::lock_guard<std::mutex> lock(g_live_mu);
  return live().count(op) != 0;
}

}  // namespace fm
