// Shared definitions of the HIP library: complex element types, status and
// error helpers, and small device utilities. gfx950 only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "fm.h"

namespace fm {

// Interleaved complex value (matches torch.complex64 / complex128 storage).
template <typename R>
struct alignas(2 * sizeof(R)) Cx {
  R x, y;
};
using c64 = Cx<float>;
using c128 = Cx<double>;

template <typename R>
__host__ __device__ __forceinline__ Cx<R> cadd(Cx<R> a, Cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__host__ __device__ __forceinline__ Cx<R> csub(Cx<R> a, Cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__host__ __device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename R>
__host__ __device__ __forceinline__ Cx<R> cmulc(Cx<R> a, Cx<R> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename R>
__host__ __device__ __forceinline__ Cx<R> cconj(Cx<R> a) { return {a.x, -a.y}; }
template <typename R>
__host__ __device__ __forceinline__ Cx<R> cscale(Cx<R> a, R s) { return {a.x * s, a.y * s}; }

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
const char* last_error();

#define FM_CHECK_ARG(cond, code, ...)     \
  do {                                    \
    if (!(cond)) {                        \
      ::fm::set_error(__VA_ARGS__);       \
      return code;                        \
    }                                     \
  } while (0)

#define FM_HIP(call)                                                                        \
  do {                                                                                      \
    hipError_t _e = (call);                                                                 \
    if (_e != hipSuccess) {                                                                 \
      ::fm::set_error("HIP error %s at %s:%d: %s", hipGetErrorName(_e), __FILE__, __LINE__, \
                      #call);                                                               \
      return _e == hipErrorOutOfMemory ? FM_E_NOMEM : FM_E_DEVICE;                          \
    }                                                                                       \
  } while (0)

#define FM_TRY(expr)                   \
  do {                                 \
    fm_status _s = (expr);             \
    if (_s != FM_OK) return _s;        \
  } while (0)

// Checks the launch that was just enqueued.
#define FM_LAUNCHED() FM_HIP(hipGetLastError())

inline size_t elem_size(fm_dtype dt) {
  switch (dt) {
    case FM_C64: return 8;
    case FM_C128: return 16;
    case FM_I32: return 4;
    case FM_I64: return 8;
  }
  return 0;
}
inline bool is_complex(fm_dtype dt) { return dt == FM_C64 || dt == FM_C128; }

inline int ilog2(int64_t n) {
  int l = 0;
  while ((int64_t(1) << l) < n) ++l;
  return l;
}
inline bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }
inline int64_t next_pow2(int64_t n) {
  int64_t p = 1;
  while (p < n) p <<= 1;
  return p;
}
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace fm
