// LDS-staged Stockham FFT for gfx950 (the fast transform behind the DFT of
// eq. (1) and the cyclic convolution of eq. (5)).
//
// One transform of N = 2^LOGN points is held by T = N/E threads, E = 16
// elements per thread in registers, thread t holding positions t + T*k. Each
// pass is a radix-R Stockham step (R = 16, plus one smaller radix when LOGN is
// not a multiple of 4): butterfly j reads positions j + r*N/R -- which are in
// the thread's own registers -- applies the twiddles W_{Ns R}^{(j mod Ns) r},
// does a radix-R DFT in registers and writes result q to position
// (j div Ns)*Ns*R + (j mod Ns) + q*Ns. Between passes the results go through
// LDS (padded by one slot every 16 to spread the banks); after the last pass
// the results are already back in the natural register layout, so global loads
// and stores are coalesced and a spectral product between a forward and an
// inverse transform needs no exchange at all.
//
// A work-group holds B transforms. Contiguous vectors map lanes as b*T + t,
// strided vectors (stride `inner`) as t*B + b so that B neighbouring vectors
// are read and written as contiguous runs.
#include "kernels.h"
#include "runtime.h"

namespace fm {
namespace {

// cos and sin of 2 pi m / 16, m = 0..4
__device__ constexpr double kCos16[5] = {1.0, 0.92387953251128675613, 0.70710678118654752440,
                                         0.38268343236508977173, 0.0};

// a * exp(-+ 2 pi j e / 16): sign - for the forward transform, + for the inverse.
template <bool INV, typename R>
__device__ __forceinline__ Cx<R> rot16(Cx<R> a, int e) {
  e &= 15;
  if (e == 0) return a;
  if (e == 8) return {-a.x, -a.y};
  // forward: multiply by (cos, -sin); inverse by (cos, +sin)
  if (e == 4) return INV ? Cx<R>{-a.y, a.x} : Cx<R>{a.y, -a.x};
  if (e == 12) return INV ? Cx<R>{a.y, -a.x} : Cx<R>{-a.y, a.x};
  // general angle: cos/sin from the quadrant of e
  const int q = e >> 2, r = e & 3;
  R c = R(kCos16[r]), sn = R(kCos16[4 - r]);  // cos, sin of 2 pi r/16
  // rotate by q quarter turns: (c, s) -> (-s, c)
  for (int k = 0; k < q; ++k) {
    R t = c;
    c = -sn;
    sn = t;
  }
  if (!INV) sn = -sn;
  return {a.x * c - a.y * sn, a.x * sn + a.y * c};
}

// In-register DFT of RAD points (natural order in and out).
template <int RAD, bool INV, typename R>
__device__ __forceinline__ void dft(Cx<R>* a) {
  if constexpr (RAD == 2) {
    Cx<R> t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  } else if constexpr (RAD == 4) {
    Cx<R> t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    Cx<R> t2 = cadd(a[1], a[3]), d = csub(a[1], a[3]);
    Cx<R> t3 = INV ? Cx<R>{-d.y, d.x} : Cx<R>{d.y, -d.x};  // d * (-+j)
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
  } else if constexpr (RAD == 8 || RAD == 16) {
    // RAD = P*Q, n = Q*n1 + n2, k = k1 + P*k2:
    // X[k1 + P k2] = sum_n2 W_Q^{n2 k2} W_RAD^{n2 k1} sum_n1 x[Q n1 + n2] W_P^{n1 k1}
    constexpr int P = RAD == 8 ? 2 : 4;
    constexpr int Q = RAD / P;
    Cx<R> b[RAD];
#pragma unroll
    for (int n2 = 0; n2 < Q; ++n2) {
      Cx<R> t[P];
#pragma unroll
      for (int n1 = 0; n1 < P; ++n1) t[n1] = a[Q * n1 + n2];
      dft<P, INV>(t);
#pragma unroll
      for (int k1 = 0; k1 < P; ++k1) b[n2 * P + k1] = rot16<INV>(t[k1], n2 * k1 * (16 / RAD));
    }
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) {
      Cx<R> t[Q];
#pragma unroll
      for (int n2 = 0; n2 < Q; ++n2) t[n2] = b[n2 * P + k1];
      dft<Q, INV>(t);
#pragma unroll
      for (int k2 = 0; k2 < Q; ++k2) a[k1 + P * k2] = t[k2];
    }
  }
}

template <int LOGN, int LE_>
struct Plan {
  static constexpr int N = 1 << LOGN;
  static constexpr int LE = LE_;  // log2 elements per thread
  static constexpr int E = 1 << LE;
  static constexpr int T = N / E;  // threads per transform
  static constexpr int FIRST = LOGN >= 4 ? (LOGN & 3) : LOGN;  // log radix of a short first pass
  static constexpr int NPASS = LOGN == 0 ? 0 : (LOGN < 4 ? 1 : (LOGN >> 2) + (FIRST ? 1 : 0));
  static constexpr int log_radix(int p) { return (LOGN < 4) ? LOGN : ((FIRST && p == 0) ? FIRST : 4); }
  static constexpr int log_ns(int p) {
    int s = 0;
    for (int i = 0; i < p; ++i) s += log_radix(i);
    return s;
  }
  static constexpr int lds_elems() { return N + (N >> 4); }
};

// Elements per thread: 16, more only where a transform would need more than
// 512 threads. Work-group size: at least 256 threads (several short
// transforms per group); strided groups aim at 16 neighbouring vectors.
constexpr int fft_le(int logn) { return logn < 4 ? logn : (logn - 9 > 4 ? logn - 9 : 4); }
constexpr int fft_threads(int logn, bool strided) {
  const int t = 1 << (logn - fft_le(logn));
  if (!strided) return t > 256 ? t : 256;
  const int want = 16 * t > 256 ? 16 * t : 256;
  return want > 512 ? (t > 512 ? t : 512) : want;
}

__device__ __forceinline__ int pad16(int pos) { return pos + (pos >> 4); }

// Twiddles W^(jj r), r = 1..RR-1, from four table entries W^(jj), W^(2jj),
// W^(4jj), W^(8jj) (products of at most three of them).
template <int RR, typename R>
__device__ __forceinline__ void pass_twiddles(const Cx<R>* __restrict__ tab, int jj, Cx<R>* w) {
  w[1] = tab[jj];
  if constexpr (RR > 2) {
    w[2] = tab[2 * jj];
    w[3] = cmul(w[1], w[2]);
  }
  if constexpr (RR > 4) {
    w[4] = tab[4 * jj];
    w[5] = cmul(w[1], w[4]);
    w[6] = cmul(w[2], w[4]);
    w[7] = cmul(w[3], w[4]);
  }
  if constexpr (RR > 8) {
    w[8] = tab[8 * jj];
#pragma unroll
    for (int r = 9; r < 16; ++r) w[r] = cmul(w[r - 8], w[8]);
  }
}

template <typename R, int LOGN, int LE, int P, bool INV>
__device__ __forceinline__ void fft_pass(Cx<R>* v, Cx<R>* lds, int t, const Cx<R>* __restrict__ tw) {
  using PL = Plan<LOGN, LE>;
  constexpr int LR = PL::log_radix(P);
  constexpr int RR = 1 << LR;
  constexpr int LNS = PL::log_ns(P);
  constexpr int NS = 1 << LNS;
  constexpr bool LAST = (P == PL::NPASS - 1);
  constexpr int M = PL::E / RR;  // butterflies per thread
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int j = t + PL::T * m;
    Cx<R> a[RR];
#pragma unroll
    for (int r = 0; r < RR; ++r) a[r] = v[m + r * M];
    if constexpr (NS > 1) {
      Cx<R> w[RR];
      pass_twiddles<RR>(tw + NS * RR, j & (NS - 1), w);  // table of W_{NS*RR}
#pragma unroll
      for (int r = 1; r < RR; ++r) a[r] = INV ? cmulc(a[r], w[r]) : cmul(a[r], w[r]);
    }
    dft<RR, INV>(a);
    if constexpr (LAST) {
#pragma unroll
      for (int q = 0; q < RR; ++q) v[m + q * M] = a[q];
    } else {
      const int idxd = ((j >> LNS) << (LNS + LR)) | (j & (NS - 1));
#pragma unroll
      for (int q = 0; q < RR; ++q) lds[pad16(idxd + q * NS)] = a[q];
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PL::E; ++k) v[k] = lds[pad16(t + PL::T * k)];
    __syncthreads();
  }
}

template <typename R, int LOGN, int LE, int P, bool INV>
__device__ __forceinline__ void fft_passes_from(Cx<R>* v, Cx<R>* lds, int t, const Cx<R>* tw) {
  if constexpr (P < Plan<LOGN, LE>::NPASS) {
    fft_pass<R, LOGN, LE, P, INV>(v, lds, t, tw);
    fft_passes_from<R, LOGN, LE, P + 1, INV>(v, lds, t, tw);
  }
}

struct KArgs {
  const void* x;
  void* y;
  int64_t ncols, outer, inner;
  int64_t ldx, xvs, ldy, yvs;
  int64_t in_limit, out_limit;
  const void* spec;
  int64_t spec_ostride;
  const void* tw;
  int mode, spec_conj, tw_log, tw_inv, accumulate, B;
};

template <typename R, int LOGN, int LE, bool STRIDED, int THREADS>
__global__ __launch_bounds__(THREADS) void fft_kernel(KArgs a) {
  using PL = Plan<LOGN, LE>;
  extern __shared__ unsigned char smem_raw[];
  Cx<R>* smem = reinterpret_cast<Cx<R>*>(smem_raw);
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
    const int64_t it = bid % tiles;
    bid /= tiles;
    o = bid % a.outer;
    c = bid / a.outer;
    i = it * a.B + b;
    valid = i < a.inner;
  }
  Cx<R>* lds = smem + b * PL::lds_elems();
  const Cx<R>* tw = reinterpret_cast<const Cx<R>*>(a.tw);
  // 32-bit offsets inside one vector (checked on the host)
  const int inner = STRIDED ? int(a.inner) : 1;
  const int ii = int(i);

  Cx<R> v[PL::E];
  const Cx<R>* X = reinterpret_cast<const Cx<R>*>(a.x) + c * a.ldx + o * a.xvs + i;
  const int in_limit = int(a.in_limit < (int64_t(1) << 30) ? a.in_limit : (int64_t(1) << 30));
#pragma unroll
  for (int k = 0; k < PL::E; ++k) {
    const int p = t + PL::T * k;
    v[k] = (valid && p * inner + ii < in_limit) ? X[p * inner] : Cx<R>{R(0), R(0)};
  }

  if (a.mode == FFT_INV) {
    fft_passes_from<R, LOGN, LE, 0, true>(v, lds, t, tw);
  } else {
    fft_passes_from<R, LOGN, LE, 0, false>(v, lds, t, tw);
    if (a.mode == FFT_CONV) {
      const Cx<R>* S = reinterpret_cast<const Cx<R>*>(a.spec) + (STRIDED ? 0 : o * a.spec_ostride);
#pragma unroll
      for (int k = 0; k < PL::E; ++k) {
        const Cx<R> s = S[t + PL::T * k];
        v[k] = a.spec_conj ? cmulc(v[k], s) : cmul(v[k], s);
      }
      fft_passes_from<R, LOGN, LE, 0, true>(v, lds, t, tw);
    }
  }

  if (a.tw_log > 0) {
    const int twn = 1 << a.tw_log;
    const Cx<R>* tab = tw + twn;
    const int qq = STRIDED ? ii : int(o);
#pragma unroll
    for (int k = 0; k < PL::E; ++k) {
      const int p = t + PL::T * k;
      const Cx<R> w = tab[(p * qq) & (twn - 1)];
      v[k] = a.tw_inv ? cmulc(v[k], w) : cmul(v[k], w);
    }
  }

  if (valid) {
    Cx<R>* Y = reinterpret_cast<Cx<R>*>(a.y) + c * a.ldy + o * a.yvs + i;
    const int out_limit = int(a.out_limit < (int64_t(1) << 30) ? a.out_limit : (int64_t(1) << 30));
#pragma unroll
    for (int k = 0; k < PL::E; ++k) {
      const int p = t + PL::T * k;
      if (p * inner + ii < out_limit) {
        if (a.accumulate) {
          Cx<R> old = Y[p * inner];
          Y[p * inner] = cadd(old, v[k]);
        } else {
          Y[p * inner] = v[k];
        }
      }
    }
  }
}

template <typename R, int LOGN, int LE, bool STRIDED, int THREADS>
fm_status launch_one(const FftLaunch& L, KArgs ka, hipStream_t s) {
  using PL = Plan<LOGN, LE>;
  const size_t per = size_t(PL::lds_elems()) * sizeof(Cx<R>);
  const int B = THREADS / PL::T;
  int64_t blocks;
  if (!STRIDED)
    blocks = cdiv(L.b.ncols * L.b.outer, B);
  else
    blocks = L.b.ncols * L.b.outer * cdiv(L.b.inner, B);
  FM_CHECK_ARG(blocks > 0 && blocks < (int64_t(1) << 31), FM_E_UNSUPPORTED,
               "fft: grid of %lld work-groups is out of range", (long long)blocks);
  FM_CHECK_ARG(int64_t(PL::N) * L.b.inner < (int64_t(1) << 30), FM_E_UNSUPPORTED,
               "fft: vector span above 2^30 elements");
  ka.B = B;
  const size_t shmem = size_t(B) * per;
  FM_CHECK_ARG(shmem <= 160 * 1024, FM_E_UNSUPPORTED, "fft: LDS request of %zu bytes", shmem);
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&fft_kernel<R, LOGN, LE, STRIDED, THREADS>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL((fft_kernel<R, LOGN, LE, STRIDED, THREADS>), dim3(unsigned(blocks)), dim3(B * PL::T),
                     shmem, s, ka);
  FM_LAUNCHED();
  return FM_OK;
}

template <typename R, int LOGN>
fm_status dispatch_logn(const FftLaunch& L, const KArgs& ka, bool strided, int logn, hipStream_t s) {
  if constexpr (LOGN >= 0) {
    if (logn == LOGN) {
      if (strided) return launch_one<R, LOGN, fft_le(LOGN), true, fft_threads(LOGN, true)>(L, ka, s);
      return launch_one<R, LOGN, fft_le(LOGN), false, fft_threads(LOGN, false)>(L, ka, s);
    }
    if constexpr (LOGN > 0) return dispatch_logn<R, LOGN - 1>(L, ka, strided, logn, s);
  }
  set_error("fft: unsupported length 2^%d", logn);
  return FM_E_UNSUPPORTED;
}

}  // namespace

fm_status launch_fft(const FftLaunch& L, hipStream_t s) {
  if (L.b.ncols == 0 || L.b.outer == 0 || L.b.inner == 0) return FM_OK;
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
  ka.in_limit = L.in_limit;
  ka.out_limit = L.out_limit;
  ka.spec = L.spec;
  ka.spec_ostride = L.spec_ostride;
  ka.mode = L.mode;
  ka.spec_conj = L.spec_conj;
  ka.tw_log = L.tw_log;
  ka.tw_inv = L.tw_inv;
  ka.accumulate = L.accumulate;
  const bool strided = L.b.inner > 1;
  const int need_log = L.tw_log > L.logn ? L.tw_log : L.logn;
  if (L.elem == Elem::C64) {
    FM_CHECK_ARG(L.logn <= 13, FM_E_UNSUPPORTED, "fft: c64 LDS length limit exceeded");
    ka.tw = twiddle_table(Elem::C64, need_log);
    FM_CHECK_ARG(ka.tw != nullptr, FM_E_DEVICE, "fft: twiddle table unavailable: %s", last_error());
    return dispatch_logn<float, 13>(L, ka, strided, L.logn, s);
  }
  if (L.elem == Elem::C128) {
    FM_CHECK_ARG(L.logn <= 13, FM_E_UNSUPPORTED, "fft: c128 LDS length limit exceeded");
    ka.tw = twiddle_table(Elem::C128, need_log);
    FM_CHECK_ARG(ka.tw != nullptr, FM_E_DEVICE, "fft: twiddle table unavailable: %s", last_error());
    return dispatch_logn<double, 13>(L, ka, strided, L.logn, s);
  }
  set_error("fft: integer element type");
  return FM_E_DTYPE;
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
