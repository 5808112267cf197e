// Fast Walsh-Hadamard transform y = H_N x, H_N = H_2 (x) ... (x) H_2 in
// natural (Sylvester) order, entries +-1, unnormalised.
//
// Since H_N is a Kronecker power, its factors act on independent bit-digits of
// the index and can be applied in any order, in place. Thread t of T = N/16
// holds positions t + T*k (k = 0..15); the top 4-bit digit is transformed in
// registers straight after the coalesced load, the remaining digits in LDS
// (each thread owns the 16 (or fewer) positions that differ in that digit),
// and the result is read back in the natural layout for a coalesced store.
// Integer element types wrap modulo 2^w (two's complement), so the result is
// exact and independent of the order of the additions.
#include "kernels.h"

namespace fm {
namespace {

template <typename V>
struct Arith;
template <>
struct Arith<c64> {
  static __device__ __forceinline__ c64 add(c64 a, c64 b) { return cadd(a, b); }
  static __device__ __forceinline__ c64 sub(c64 a, c64 b) { return csub(a, b); }
  static __device__ __forceinline__ c64 zero() { return {0.f, 0.f}; }
};
template <>
struct Arith<c128> {
  static __device__ __forceinline__ c128 add(c128 a, c128 b) { return cadd(a, b); }
  static __device__ __forceinline__ c128 sub(c128 a, c128 b) { return csub(a, b); }
  static __device__ __forceinline__ c128 zero() { return {0.0, 0.0}; }
};
template <>
struct Arith<int32_t> {
  static __device__ __forceinline__ int32_t add(int32_t a, int32_t b) {
    return int32_t(uint32_t(a) + uint32_t(b));
  }
  static __device__ __forceinline__ int32_t sub(int32_t a, int32_t b) {
    return int32_t(uint32_t(a) - uint32_t(b));
  }
  static __device__ __forceinline__ int32_t zero() { return 0; }
};
template <>
struct Arith<int64_t> {
  static __device__ __forceinline__ int64_t add(int64_t a, int64_t b) {
    return int64_t(uint64_t(a) + uint64_t(b));
  }
  static __device__ __forceinline__ int64_t sub(int64_t a, int64_t b) {
    return int64_t(uint64_t(a) - uint64_t(b));
  }
  static __device__ __forceinline__ int64_t zero() { return 0; }
};

// In-register H_R on a[0..R) (natural order).
template <int W, typename V>
__device__ __forceinline__ void hadamard_regs(V* a) {
#pragma unroll
  for (int bit = 0; bit < W; ++bit) {
#pragma unroll
    for (int r = 0; r < (1 << W); ++r) {
      if (!(r & (1 << bit))) {
        const V u = a[r], w = a[r | (1 << bit)];
        a[r] = Arith<V>::add(u, w);
        a[r | (1 << bit)] = Arith<V>::sub(u, w);
      }
    }
  }
}

__device__ __forceinline__ int pad16(int pos) { return pos + (pos >> 4); }

template <int LOGN, int LE_>
struct WPlan {
  static constexpr int N = 1 << LOGN;
  static constexpr int LE = LE_;
  static constexpr int E = 1 << LE;
  static constexpr int T = N / E;
  static constexpr int LOW = LOGN - LE;  // bits handled in LDS
  static constexpr int lds_elems() { return LOW > 0 ? N + (N >> 4) : 1; }
};

// Offset (in values) between the LDS regions of the B = THREADS / T
// transforms of a work-group. Strided layout: the lanes of a wave are
// min(B, 64) transforms, all at the same offsets inside their regions, and
// the plain 17 N / 16 (a multiple of 64 values from N = 1024) puts them in the
// same banks. The padding was chosen by timing the exchanges alone with
// strides base + 0..32 for the work-group shapes below (2048 to 8192 points
// with 8-byte values, 1024 to 4096 with 16-byte ones; 2-8x faster than +0
// where B >= 4), the smallest odd stride of at least base + 2 elsewhere.
// Contiguous layout: the plain stride.
template <typename V, int LOGN, int LE, bool STRIDED, int THREADS>
constexpr int w_stride() {
  using PL = WPlan<LOGN, LE>;
  const int base = PL::lds_elems();
  if (!STRIDED || PL::LOW == 0 || THREADS / PL::T <= 1) return base;
  if (sizeof(V) == 8 && LE == 4 && LOGN >= 10 && LOGN <= 13)
    return base + (LOGN == 10 ? 3 : LOGN == 11 ? 6 : LOGN == 12 ? 4 : 8);
  if (sizeof(V) == 16 && LE == 4 && LOGN >= 10 && LOGN <= 12) return base + (LOGN == 12 ? 4 : 2);
  return (base + 2) | 1;
}

// One lower digit: bits [S, S+W) of the index.
template <typename V, int LOGN, int LE, int S, int W>
__device__ __forceinline__ void digit_pass(V* lds, int t) {
  using PL = WPlan<LOGN, LE>;
  constexpr int R = 1 << W;
  constexpr int M = PL::E / R;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int g = t + PL::T * m;
    const int base = (g & ((1 << S) - 1)) | ((g >> S) << (S + W));
    V a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = lds[pad16(base + (r << S))];
    hadamard_regs<W>(a);
#pragma unroll
    for (int r = 0; r < R; ++r) lds[pad16(base + (r << S))] = a[r];
  }
  __syncthreads();
}

template <typename V, int LOGN, int LE, int S>
__device__ __forceinline__ void lower_digits(V* lds, int t) {
  using PL = WPlan<LOGN, LE>;
  if constexpr (S < PL::LOW) {
    constexpr int W = (PL::LOW - S) < 4 ? (PL::LOW - S) : 4;
    digit_pass<V, LOGN, LE, S, W>(lds, t);
    lower_digits<V, LOGN, LE, S + W>(lds, t);
  }
}

// Elements per thread and work-group size, as for the FFT. Strided: 16
// fibres per work-group where the threads and the LDS allow (128-byte row
// segments for 8-byte values, so a tile fetches whole lines), up to 1024
// threads (512 for 16-byte values): 16 fibres of 1024 points in 1024 threads
// ran the Kronecker workload's Hadamard pass in 1.95 ms against 2.36 ms for
// 8 fibres in 512.
constexpr int w_le(int logn) { return logn < 4 ? logn : (logn - 9 > 4 ? logn - 9 : 4); }
constexpr int w_threads(int logn, bool strided, int esize) {
  const int t = 1 << (logn - w_le(logn));
  if (!strided) return t > 256 ? t : 256;
  const int n = 1 << logn;
  const int fit = (160 * 1024) / ((n + n / 16 + 64) * esize);  // regions the LDS holds (padding <= 64)
  const int cap = (esize >= 16 ? 512 : 1024) / t;
  int b = 16 * t > 256 ? 16 : 256 / t;
  if (b > cap) b = cap;
  if (b > fit) b = fit;
  if (b < 1) b = 1;
  return t * b;
}

struct WArgs {
  const void* x;
  void* y;
  int64_t ncols, outer, inner;
  int64_t ldx, xvs, ldy, yvs;
  int accumulate, B;
};

template <typename V, int LOGN, int LE, bool STRIDED, int THREADS>
__global__ __launch_bounds__(THREADS) void fwht_kernel(WArgs a) {
  using PL = WPlan<LOGN, LE>;
  extern __shared__ unsigned char smem_raw[];
  V* smem = reinterpret_cast<V*>(smem_raw);
  const int tid = threadIdx.x;
  int t, b;
  int64_t c, o, i;
  bool valid;
  if constexpr (!STRIDED) {
    b = tid >> (LOGN - LE);
    t = tid & (PL::T - 1);
    const int64_t q = int64_t(blockIdx.x) * a.B + b;
    valid = q < a.ncols * a.outer;
    c = q / a.outer;
    o = q - c * a.outer;
    i = 0;
  } else {
    b = tid % a.B;
    t = tid / a.B;
    const int64_t tiles = (a.inner + a.B - 1) / a.B;
    int64_t bid = blockIdx.x;
    // A tile's row segments are B values, shorter than a 128-byte line when
    // B sizeof(V) < 128: then the P tiles that share each line are given to
    // work-groups on one XCD (work-group g runs on XCD g mod 8; groups of 8 P
    // consecutive indices are permuted), so the line is fetched into that
    // XCD's L2 once instead of once per XCD.
    constexpr int P = (THREADS / PL::T) * int(sizeof(V)) < 128 ? 128 / ((THREADS / PL::T) * int(sizeof(V))) : 1;
    if constexpr (P > 1) {
      constexpr int64_t grp = 8 * P;
      if (bid < int64_t(gridDim.x) / grp * grp) {
        const int64_t q = bid / grp, r = bid % grp;
        bid = q * grp + (r % 8) * P + r / 8;
      }
    }
    const int64_t it = bid % tiles;
    bid /= tiles;
    o = bid % a.outer;
    c = bid / a.outer;
    i = it * a.B + b;
    valid = i < a.inner;
  }
  const int64_t inner = STRIDED ? a.inner : 1;
  V v[PL::E];
  const V* X = reinterpret_cast<const V*>(a.x) + c * a.ldx + o * a.xvs + i;
#pragma unroll
  for (int k = 0; k < PL::E; ++k) v[k] = valid ? X[int64_t(t + PL::T * k) * inner] : Arith<V>::zero();
  hadamard_regs<PL::LE>(v);
  if constexpr (PL::LOW > 0) {
    V* lds = smem + b * w_stride<V, LOGN, LE, STRIDED, THREADS>();
#pragma unroll
    for (int k = 0; k < PL::E; ++k) lds[pad16(t + PL::T * k)] = v[k];
    __syncthreads();
    lower_digits<V, LOGN, LE, 0>(lds, t);
#pragma unroll
    for (int k = 0; k < PL::E; ++k) v[k] = lds[pad16(t + PL::T * k)];
  }
  if (valid) {
    V* Y = reinterpret_cast<V*>(a.y) + c * a.ldy + o * a.yvs + i;
#pragma unroll
    for (int k = 0; k < PL::E; ++k) {
      const int64_t off = int64_t(t + PL::T * k) * inner;
      Y[off] = a.accumulate ? Arith<V>::add(Y[off], v[k]) : v[k];
    }
  }
}

template <typename V, int LOGN, int LE, bool STRIDED, int THREADS>
fm_status wlaunch_one(const Batch& bt, WArgs wa, hipStream_t s) {
  using PL = WPlan<LOGN, LE>;
  const size_t per = size_t(w_stride<V, LOGN, LE, STRIDED, THREADS>()) * sizeof(V);
  const int B = THREADS / PL::T;
  int64_t blocks;
  if (!STRIDED)
    blocks = cdiv(bt.ncols * bt.outer, B);
  else
    blocks = bt.ncols * bt.outer * cdiv(bt.inner, B);
  FM_CHECK_ARG(blocks > 0 && blocks < (int64_t(1) << 31), FM_E_UNSUPPORTED,
               "fwht: grid of %lld work-groups is out of range", (long long)blocks);
  wa.B = B;
  const size_t shmem = size_t(B) * per;
  FM_CHECK_ARG(shmem <= 160 * 1024, FM_E_UNSUPPORTED, "fwht: LDS request of %zu bytes", shmem);
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&fwht_kernel<V, LOGN, LE, STRIDED, THREADS>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL((fwht_kernel<V, LOGN, LE, STRIDED, THREADS>), dim3(unsigned(blocks)), dim3(B * PL::T),
                     shmem, s, wa);
  FM_LAUNCHED();
  return FM_OK;
}

template <typename V, int LOGN>
fm_status wdispatch(const Batch& bt, const WArgs& wa, int logn, hipStream_t s) {
  if constexpr (LOGN >= 0) {
    if (logn == LOGN) {
      if (bt.inner > 1) return wlaunch_one<V, LOGN, w_le(LOGN), true, w_threads(LOGN, true, sizeof(V))>(bt, wa, s);
      return wlaunch_one<V, LOGN, w_le(LOGN), false, w_threads(LOGN, false, sizeof(V))>(bt, wa, s);
    }
    if constexpr (LOGN > 0) return wdispatch<V, LOGN - 1>(bt, wa, logn, s);
  }
  set_error("fwht: unsupported length 2^%d", logn);
  return FM_E_UNSUPPORTED;
}

}  // namespace

fm_status launch_fwht(Elem e, int logn, const Batch& b, const void* x, void* y, int accumulate,
                      hipStream_t s) {
  if (b.ncols == 0 || b.outer == 0 || b.inner == 0) return FM_OK;
  FM_CHECK_ARG(logn <= fwht_lds_max_log(e), FM_E_UNSUPPORTED, "fwht: length above LDS limit");
  WArgs wa{x, y, b.ncols, b.outer, b.inner, b.ldx, b.xvs, b.ldy, b.yvs, accumulate, 1};
  switch (e) {
    case Elem::C64: return wdispatch<c64, 14>(b, wa, logn, s);
    case Elem::C128: return wdispatch<c128, 13>(b, wa, logn, s);
    case Elem::I32: return wdispatch<int32_t, 14>(b, wa, logn, s);
    case Elem::I64: return wdispatch<int64_t, 14>(b, wa, logn, s);
  }
  return FM_E_DTYPE;
}

}  // namespace fm
