// fm_apply_noalloc: fm_apply with its workspace (the four-step intermediates
// of long transforms) taken from a fixed device array of this library instead
// of the caller or the stream-ordered allocator, for callers that cannot
// allocate device memory.
//
// The array is a file-scope __device__ variable: every GPU the library runs on
// holds its own copy, at its own address, until the process ends. Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in): the device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept here.
#include <mutex>

#include "runtime.h"

namespace {

constexpr size_t kScratchBytes = size_t(FM_NOALLOC_SCRATCH_BYTES);
static_assert(kScratchBytes % 256 == 0, "scratch size must keep 256-byte alignment");

__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
fm_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    fm::set_error("device %d: at most %d devices are supported", dev, kMaxDevices);
    return FM_E_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      fm::set_error("hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorName(e));
      return FM_E_DEVICE;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return FM_OK;
}

}  // namespace

extern "C" fm_status fm_apply_noalloc(fm_op a, fm_dir dir, int64_t ncols, const void* x, int64_t ldx, void* y,
                                      int64_t ldy, void* stream) {
  fm::set_error("");
  int dev = 0;
  FM_HIP(hipGetDevice(&dev));
  void* ws = nullptr;
  FM_TRY(scratch_address(dev, &ws));
  return fm::apply_op(a, dir, ncols, x, ldx, y, ldy, ws, kScratchBytes, false, stream);
}
