// Per-operator FFT kernels: the fast transform behind the DFT of eq. (1) and
// the cyclic convolution of eq. (5), on a strided batch of vectors, with the
// engine of xform.h (one work-group = 4096 complex values).
#include "kernels.h"
#include "runtime.h"
#include "mixed.h"
#include "xform.h"

#include <mutex>

namespace fm {
namespace {

using namespace xf;

struct KArgs {
  const void* x;
  void* y;
  int64_t ncols, outer, inner;
  int64_t ldx, xvs, ldy, yvs;
  int in_limit, out_limit;
  const void* spec;
  int64_t spec_ostride;
  const void* tw;
  const void* twl;
  int mode, spec_conj, tw_log, tw_inv, accumulate, logn, fuse_n2;
  int layout;  // contiguous: 0 transforms = columns, 1 packed (ncols*outer), 2 per column
  int64_t tiles;  // work-groups per column (layout 2) / per vector (strided)
  const int* omap;  // OMAP: a row selection's inverse index map for the store
};

// Store epilogue of a row selection applied to the result: position e of a
// transform's output vector goes to row omap[e] of its column (added with
// acc), and nowhere where omap[e] < 0. Y: the column of transform 0 (strided
// items: the one column of the work-group, stride 0).
template <typename R>
struct MapStoreEp {
  static constexpr bool kOn = true;
  Cx<R>* Y;
  int64_t ystride;
  const int* omap;
  int acc;
  int mk[kE];
  __device__ __forceinline__ void pre(int k, int, int e, Cx<R>*) { mk[k] = omap[e]; }
  __device__ __forceinline__ void put(int k, int, int b, int, Cx<R>*, Cx<R> v) {
    if (mk[k] < 0) return;
    Cx<R>* dst = Y + int64_t(b) * ystride + mk[k];
    *dst = acc ? cadd(*dst, v) : v;
  }
};

constexpr int kXcdCount = 8;  // work-group g runs on XCD g mod 8
// Contiguous transforms of up to 2^FM_SMALL_LOGW points run in work-groups of
// 2^FM_SMALL_LOGW values (one wave at 10): with four work-groups' barriers
// per CU replaced by sixteen, the loads of one overlap the arithmetic of the
// others (1024-point convolution of 65536 columns: 0.535 -> 0.505 ms per
// forward + adjoint; 2^11: 0.514).
#ifndef FM_SMALL_LOGW
#define FM_SMALL_LOGW 10
#endif
// Fewest columns for which the rows of a column are grouped on one XCD: with
// fewer, grouping leaves XCDs idle in a launch that is short anyway.
#ifndef FM_XCD_GROUP_MIN_COLS
#define FM_XCD_GROUP_MIN_COLS 64
#endif

// XG (layout 2 only): the work-groups of column c take the indices = c (mod 8).
// The complex64 strided form is held to 128 VGPRs (four work-groups per CU; it
// spills 6 registers there and measured faster than at three).
// FIX > 0: the transform length 2^FIX is a compile-time constant (a.logn ==
// FIX), so the steps unroll and every LDS and twiddle index folds into
// immediate offsets; the arithmetic is the same as the run-time form's, so
// both give the same bits.
// PRE (compile-time lengths only): the spectrum and the twiddle seeds are
// loaded together with the input (the engine's PRETW), one dependent memory
// round trip less per work-group, for launches too small to hide it (fewer
// work-groups than CUs); more registers live, same arithmetic and bits.
// OMAP (run-time lengths only): the result is stored through a row
// selection's inverse map (MapStoreEp): the selection of a product S C
// applied inside the transform's last pass.
template <typename R, bool STRIDED, int LOGW, bool XG = false, int FIX = 0, bool PRE = false, bool OMAP = false>
__global__ __launch_bounds__(Geo<LOGW>::kThreads, (!PRE && (STRIDED || FIX > 0) && sizeof(R) == 4) ? 4 : 1) void fft_kernel(KArgs a) {
  extern __shared__ unsigned char smem_raw[];
  Cx<R>* lds = reinterpret_cast<Cx<R>*>(smem_raw);
  const int logn = FIX > 0 ? FIX : a.logn;
  const int tpw = 1 << (LOGW - logn);  // transforms per work-group
  Job<R> jb;
  jb.in_limit = a.in_limit;
  jb.out_limit = a.out_limit;
  const Cx<R>* X = reinterpret_cast<const Cx<R>*>(a.x);
  Cx<R>* Y = reinterpret_cast<Cx<R>*>(a.y);
  const Cx<R>* S = reinterpret_cast<const Cx<R>*>(a.spec);
  Cx<R>* ycol = Y;
  int64_t ystr = 0;
  if constexpr (STRIDED) {
    int64_t bid = blockIdx.x;
    // tiles whose row segments (tpw values) are shorter than a 128-byte line
    // share lines: the P tiles of a line go to work-groups on one XCD
    // (work-group g runs on XCD g mod 8), which then fetches it once
    const int seg = tpw * int(sizeof(Cx<R>));
    if (seg < 128) {
      const int P = 128 / seg;
      const int64_t grp = 8 * P;
      if (bid < int64_t(gridDim.x) / grp * grp) {
        const int64_t q = bid / grp, r = bid % grp;
        bid = q * grp + (r % 8) * P + r / 8;
      }
    }
    const int64_t it = bid % a.tiles;
    bid /= a.tiles;
    const int64_t o = bid % a.outer, c = bid / a.outer;
    const int64_t i0 = it * tpw;
    jb.x = X + c * a.ldx + o * a.xvs + i0;
    jb.y = Y + c * a.ldy + o * a.yvs + i0;
    ycol = Y + c * a.ldy + o * a.yvs;
    ystr = 0;
    jb.xbstride = jb.ybstride = 1;
    jb.inner = int(a.inner);
    jb.nvalid = int(a.inner - i0 < tpw ? a.inner - i0 : tpw);
    jb.i0 = int(i0);
    jb.S = S;
    jb.sbstride = 0;
    jb.q0 = int(i0);
  } else {
    jb.inner = 1;
    jb.i0 = 0;
    if (a.layout == 0) {  // one vector per column
      const int64_t c0 = int64_t(blockIdx.x) * tpw;
      jb.x = X + c0 * a.ldx;
      jb.y = Y + c0 * a.ldy;
      ycol = jb.y;
      ystr = a.ldy;
      jb.xbstride = a.ldx;
      jb.ybstride = a.ldy;
      jb.nvalid = int(a.ncols - c0 < tpw ? a.ncols - c0 : tpw);
      jb.S = S;
      jb.sbstride = 0;
      jb.q0 = 0;
    } else if (a.layout == 1) {  // (column, outer) pairs packed at stride xvs
      const int64_t q0 = int64_t(blockIdx.x) * tpw;
      jb.x = X + q0 * a.xvs;
      jb.y = Y + q0 * a.yvs;
      ycol = jb.y;
      ystr = a.yvs;
      jb.xbstride = a.xvs;
      jb.ybstride = a.yvs;
      const int64_t total = a.ncols * a.outer;
      jb.nvalid = int(total - q0 < tpw ? total - q0 : tpw);
      jb.S = S;
      jb.sbstride = 0;
      jb.q0 = 0;
    } else {  // work-groups inside one column
      int64_t c = blockIdx.x / a.tiles, o0 = (blockIdx.x % a.tiles) * tpw;
      if constexpr (XG) {  // rows of one column on one XCD, where they share it in L2
        const int64_t g = blockIdx.x, r = g / kXcdCount;
        c = (r / a.tiles) * kXcdCount + g % kXcdCount;
        o0 = (r % a.tiles) * tpw;
        if (c >= a.ncols) return;  // padding of the last group of 8 columns
      }
      jb.x = X + c * a.ldx + o0 * a.xvs;
      jb.y = Y + c * a.ldy + o0 * a.yvs;
      ycol = jb.y;
      ystr = a.yvs;
      jb.xbstride = a.xvs;
      jb.ybstride = a.yvs;
      jb.nvalid = int(a.outer - o0 < tpw ? a.outer - o0 : tpw);
      jb.S = S + o0 * a.spec_ostride;
      jb.sbstride = a.spec_ostride;
      jb.q0 = int(o0);
    }
  }
  jb.fuse_n2 = a.fuse_n2;
  jb.twl = reinterpret_cast<const Cx<R>*>(a.twl);
  const Mode md{a.mode, a.spec_conj, a.tw_log, a.tw_inv, a.accumulate};
  const Cx<R>* tw = reinterpret_cast<const Cx<R>*>(a.tw);
  if constexpr (OMAP) {
    MapStoreEp<R> ep;
    ep.Y = ycol;
    ep.ystride = ystr;
    ep.omap = a.omap;
    ep.acc = a.accumulate;
    run_job<R, STRIDED, LOGW, (FIX > 0), MapStoreEp<R>, false, false, PRE>(jb, md, logn, lds, tw, &ep);
  } else {
    run_job<R, STRIDED, LOGW, (FIX > 0), NoEp, false, false, PRE>(jb, md, logn, lds, tw);
  }
}

// Contiguous transforms of 2^kFixMin .. 2^LOGW points run the compile-time
// length forms.
constexpr int kFixMin = 4;
template <typename R, int LOGW, bool PRE = false, int LG = LOGW>
const void* fixed_kernel(int lg) {
  if constexpr (LG < kFixMin) {
    return nullptr;
  } else {
    if (lg == LG) return reinterpret_cast<const void*>(&fft_kernel<R, false, LOGW, false, LG, PRE>);
    return fixed_kernel<R, LOGW, PRE, LG - 1>(lg);
  }
}
// Run-time-length kernels that store through a row selection (contiguous,
// and strided at 4096-value work-groups, where the four-step passes run);
// NULL where there is none.
template <typename R, int LOGW>
const void* omap_kernel(bool strided, bool xg) {
  if (xg) return nullptr;
  if (!strided) return reinterpret_cast<const void*>(&fft_kernel<R, false, LOGW, false, 0, false, true>);
  if constexpr (LOGW == 12) return reinterpret_cast<const void*>(&fft_kernel<R, true, LOGW, false, 0, false, true>);
  return nullptr;
}

// Launches of at most this many work-groups take the PRE forms (one-wave
// work-groups only).
#ifndef FM_PRE_MAX_WG
#define FM_PRE_MAX_WG 256
#endif

template <typename R, int LOGW>
fm_status launch_typed(const FftLaunch& L, KArgs ka, hipStream_t s) {
  const int tpw = 1 << (LOGW - L.logn);
  const bool strided = L.b.inner > 1;
  int64_t blocks;
  if (strided) {
    ka.tiles = cdiv(L.b.inner, tpw);
    blocks = L.b.ncols * L.b.outer * ka.tiles;
  } else if (L.b.outer == 1) {
    ka.layout = 0;
    blocks = cdiv(L.b.ncols, tpw);
  } else if (L.spec_ostride == 0 && L.tw_log == 0 && L.fuse_n2 == 0 &&
             (L.b.ncols == 1 || (L.b.ldx == L.b.outer * L.b.xvs && L.b.ldy == L.b.outer * L.b.yvs))) {
    ka.layout = 1;
    blocks = cdiv(L.b.ncols * L.b.outer, tpw);
  } else {
    ka.layout = 2;
    ka.tiles = cdiv(L.b.outer, tpw);
    blocks = L.b.ncols * ka.tiles;
  }
  // the rows of a column re-read it: keep them on one XCD
  const bool xg = !strided && ka.layout == 2 && L.fuse_n2 > 0 && L.b.ncols >= FM_XCD_GROUP_MIN_COLS;
  if (xg) blocks = cdiv(L.b.ncols, kXcdCount) * kXcdCount * ka.tiles;
  FM_CHECK_ARG(blocks > 0 && blocks < (int64_t(1) << 31), FM_E_UNSUPPORTED,
               "fft: grid of %lld work-groups is out of range", (long long)blocks);
  FM_CHECK_ARG((int64_t(1) << L.logn) * L.b.inner < (int64_t(1) << 30), FM_E_UNSUPPORTED,
               "fft: vector span above 2^30 elements");
  FM_CHECK_ARG(L.fuse_n2 == 0 || (!strided && ka.layout == 2 && L.logn == LOGW && L.fuse_n2 <= 32),
               FM_E_UNSUPPORTED, "fft: fused column transform needs a full-size row per work-group");
  static std::once_flag attr_once;
  std::call_once(attr_once, [] {
    for (const void* f : {reinterpret_cast<const void*>(&fft_kernel<R, true, LOGW>),
                          reinterpret_cast<const void*>(&fft_kernel<R, false, LOGW>),
                          reinterpret_cast<const void*>(&fft_kernel<R, false, LOGW, true>),
                          reinterpret_cast<const void*>(&fft_kernel<R, false, LOGW, true, LOGW>)})
      (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    for (int lg = kFixMin; lg <= LOGW; ++lg)
      (void)hipFuncSetAttribute(fixed_kernel<R, LOGW>(lg), hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    for (const void* f : {omap_kernel<R, LOGW>(false, false), omap_kernel<R, LOGW>(true, false)})
      if (f) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  });
  const dim3 wg(Geo<LOGW>::kThreads);
  if (L.omap != nullptr) {
    const void* fn = omap_kernel<R, LOGW>(strided, xg);
    FM_CHECK_ARG(fn != nullptr, FM_E_UNSUPPORTED, "fft: row selection at the store not available for this pass");
    ka.omap = L.omap;
    void* args[] = {&ka};
    FM_HIP(hipLaunchKernel(fn, dim3(unsigned(blocks)), wg, args, job_lds_bytes<R, LOGW>(), s));
    FM_LAUNCHED();
    return FM_OK;
  }
  if (strided)
    hipLaunchKernelGGL((fft_kernel<R, true, LOGW>), dim3(unsigned(blocks)), wg, (job_lds_bytes<R, LOGW>()), s, ka);
  else if (xg && L.logn == LOGW)
    hipLaunchKernelGGL((fft_kernel<R, false, LOGW, true, LOGW>), dim3(unsigned(blocks)), wg,
                       (job_lds_bytes<R, LOGW>()), s, ka);
  else if (xg)
    hipLaunchKernelGGL((fft_kernel<R, false, LOGW, true>), dim3(unsigned(blocks)), wg, (job_lds_bytes<R, LOGW>()), s,
                       ka);
  else if (L.logn >= kFixMin) {
    void* args[] = {&ka};
    const bool pre = LOGW == FM_SMALL_LOGW && blocks <= FM_PRE_MAX_WG;
    FM_HIP(hipLaunchKernel(pre ? fixed_kernel<R, FM_SMALL_LOGW, true>(L.logn) : fixed_kernel<R, LOGW>(L.logn),
                           dim3(unsigned(blocks)), wg, args, job_lds_bytes<R, LOGW>(), s));
  } else
    hipLaunchKernelGGL((fft_kernel<R, false, LOGW>), dim3(unsigned(blocks)), wg, (job_lds_bytes<R, LOGW>()), s, ka);
  FM_LAUNCHED();
  return FM_OK;
}

}  // namespace

fm_status launch_fft(const FftLaunch& L, hipStream_t s) {
  if (L.b.ncols == 0 || L.b.outer == 0 || L.b.inner == 0) return FM_OK;
  FM_CHECK_ARG(L.elem == Elem::C64 || L.elem == Elem::C128, FM_E_DTYPE, "fft: integer element type");
  FM_CHECK_ARG(L.logn >= 0 && L.logn <= fft_lds_max_log(L.elem), FM_E_UNSUPPORTED,
               "fft: length 2^%d above the single-pass limit", L.logn);
  KArgs ka{};
  ka.x = L.x;
  ka.y = L.y;
  ka.ncols = L.b.ncols;
  ka.outer = L.b.outer;
  ka.inner = L.b.inner;
  ka.ldx = L.b.ldx;
  ka.xvs = L.b.xvs;
  ka.ldy = L.b.ldy;
  ka.yvs = L.b.yvs;
  ka.in_limit = int(L.in_limit < (int64_t(1) << 30) ? L.in_limit : (int64_t(1) << 30));
  ka.out_limit = int(L.out_limit < (int64_t(1) << 30) ? L.out_limit : (int64_t(1) << 30));
  ka.spec = L.spec;
  ka.spec_ostride = L.spec_ostride;
  ka.mode = L.mode;
  ka.spec_conj = L.spec_conj;
  ka.tw_log = L.tw_log;
  ka.tw_inv = L.tw_inv;
  ka.accumulate = L.accumulate;
  ka.logn = L.logn;
  ka.fuse_n2 = L.fuse_n2;
  const bool own_table = L.twl == nullptr && L.tw_log > 0;
  int need_log = own_table && L.tw_log > L.logn ? L.tw_log : L.logn;
  ka.tw = twiddle_table(L.elem, need_log);
  FM_CHECK_ARG(ka.tw != nullptr, FM_E_DEVICE, "fft: twiddle table unavailable: %s", last_error());
  FM_CHECK_ARG(L.fuse_n2 == 0 || L.tw_log > 0, FM_E_INVALID, "fft: a fused row needs its twiddle table");
  // W_L of the twiddle epilogue / fused row: the caller's table, or the
  // power-of-two table of length 2^tw_log
  ka.twl = L.twl ? L.twl
                 : own_table ? static_cast<const char*>(ka.tw) + (size_t(1) << L.tw_log) * elem_bytes(L.elem)
                             : nullptr;
  // small work-groups: same arithmetic, so the same bits
  const bool small = L.b.inner == 1 && L.logn <= FM_SMALL_LOGW && L.fuse_n2 == 0;
  if (L.elem == Elem::C128) return small ? launch_typed<double, FM_SMALL_LOGW>(L, ka, s) : launch_typed<double, 12>(L, ka, s);
  return small ? launch_typed<float, FM_SMALL_LOGW>(L, ka, s) : launch_typed<float, 12>(L, ka, s);
}

// ---------------------------------------------------------------- mixed strided passes
namespace {
struct MArgs {
  const void* x;
  int64_t ldx, in_limit;
  void* y;
  int64_t ldy, out_limit;
  const void* twl;
  int64_t L, ncols;
  int n2, inverse, acc;
};

// Tile blockIdx.x of every column (one or two threads per column position),
// one instantiation per strided factor.
template <typename R, int N2>
__global__ __launch_bounds__(256) void mixed_kernel(MArgs a) {
  extern __shared__ __align__(16) unsigned char mixed_lds[];
  for (int64_t c = blockIdx.y; c < a.ncols; c += gridDim.y) {
    const Cx<R>* x = static_cast<const Cx<R>*>(a.x) + c * a.ldx;
    Cx<R>* y = static_cast<Cx<R>*>(a.y) + c * a.ldy;
    mixed_tile_n<N2, R, NoEp>(int(blockIdx.x), x, a.in_limit, y, a.out_limit, a.inverse != 0,
                              static_cast<const Cx<R>*>(a.twl), a.L, a.acc, static_cast<NoEp*>(nullptr),
                              reinterpret_cast<Cx<R>*>(mixed_lds));
    if constexpr (N2 > 12) __syncthreads();  // the pair buffers are reused by the next column
  }
}

template <typename R>
void launch_mixed_n(int n2, dim3 g, size_t lds, hipStream_t s, const MArgs& a) {
  switch (n2) {
#define FM_MIXED_LAUNCH(N) \
  case N:                  \
    hipLaunchKernelGGL((mixed_kernel<R, N>), g, dim3(256), lds, s, a); \
    break;
    FM_MIXED_LAUNCH(3)
    FM_MIXED_LAUNCH(5)
    FM_MIXED_LAUNCH(6)
    FM_MIXED_LAUNCH(9)
    FM_MIXED_LAUNCH(10)
    FM_MIXED_LAUNCH(12)
    FM_MIXED_LAUNCH(20)
    FM_MIXED_LAUNCH(24)
    FM_MIXED_LAUNCH(30)
#undef FM_MIXED_LAUNCH
    default:
      break;
  }
}
}  // namespace

fm_status launch_mixed(Elem e, int n2, int inverse, int64_t ncols, const void* x, int64_t ldx, int64_t in_limit,
                       void* y, int64_t ldy, int64_t out_limit, const void* twl, int64_t L, int acc, hipStream_t s) {
  if (ncols == 0) return FM_OK;
  FM_CHECK_ARG(mixed_n2_ok(n2) && L == int64_t(4096) * n2, FM_E_UNSUPPORTED, "mixed pass: strided factor %d", n2);
  FM_CHECK_ARG(twl != nullptr, FM_E_INVALID, "mixed pass: no twiddle table");
  MArgs a{x, ldx, in_limit, y, ldy, out_limit, twl, L, ncols, n2, inverse, acc};
  const dim3 g(unsigned(mixed_tiles(n2)), unsigned(ncols < 65535 ? ncols : 65535));
  const size_t lds = mixed_threads(n2) > 1 ? size_t(256 / mixed_threads(n2)) * (n2 + 1) * elem_bytes(e) : 0;
  if (e == Elem::C64)
    launch_mixed_n<float>(n2, g, lds, s, a);
  else if (e == Elem::C128)
    launch_mixed_n<double>(n2, g, lds, s, a);
  else {
    set_error("mixed pass: integer element type");
    return FM_E_DTYPE;
  }
  FM_LAUNCHED();
  return FM_OK;
}

// ---------------------------------------------------------------- transpose
namespace {
template <typename V>
__global__ __launch_bounds__(256) void transpose_kernel(const V* __restrict__ x, int64_t ldx,
                                                        V* __restrict__ y, int64_t ldy, int64_t rows,
                                                        int64_t cols, int acc) {
  __shared__ V tile[32][33];
  const int64_t col = blockIdx.z;
  const int64_t tr = blockIdx.y, tc = blockIdx.x;
  const V* X = x + col * ldx;
  V* Y = y + col * ldy;
  const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;  // 32 x 8
  for (int k = 0; k < 32; k += 8) {
    const int64_t i = tr * 32 + ly + k, j = tc * 32 + lx;
    if (i < rows && j < cols) tile[ly + k][lx] = X[i * cols + j];
  }
  __syncthreads();
  for (int k = 0; k < 32; k += 8) {
    const int64_t j = tc * 32 + ly + k, i = tr * 32 + lx;
    if (i < rows && j < cols) {
      if (acc)
        Y[j * rows + i] = cadd(Y[j * rows + i], tile[lx][ly + k]);
      else
        Y[j * rows + i] = tile[lx][ly + k];
    }
  }
}
}  // namespace

fm_status launch_transpose(Elem e, int64_t ncols, int64_t rows, int64_t cols, const void* x,
                           int64_t ldx, void* y, int64_t ldy, int acc, hipStream_t s) {
  if (ncols == 0) return FM_OK;
  FM_CHECK_ARG(ncols < 65536, FM_E_UNSUPPORTED, "transpose: too many columns");
  dim3 grid(unsigned(cdiv(cols, 32)), unsigned(cdiv(rows, 32)), unsigned(ncols));
  switch (e) {
    case Elem::C64:
      hipLaunchKernelGGL(transpose_kernel<c64>, grid, dim3(256), 0, s, (const c64*)x, ldx, (c64*)y,
                         ldy, rows, cols, acc);
      break;
    case Elem::C128:
      hipLaunchKernelGGL(transpose_kernel<c128>, grid, dim3(256), 0, s, (const c128*)x, ldx,
                         (c128*)y, ldy, rows, cols, acc);
      break;
    default:
      set_error("transpose: integer element type");
      return FM_E_DTYPE;
  }
  FM_LAUNCHED();
  return FM_OK;
}

}  // namespace fm
