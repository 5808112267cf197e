// Fused Kronecker slab pass: the last two factors of a Kronecker product,
// a Fourier matrix F_nF and a small dense matrix G (m x n), applied to each
// slab of nF x n values (eq. (7) structure, first factor slowest) in one
// read and one write of the slab:
//   forward:  Y[o, kF, r] = sum_pF W^(pF kF) sum_k G[r, k] X[o, pF, k]
//   adjoint:  Y[o, pF, k] = sum_kF W^-(pF kF) sum_r conj(G[r, k]) X[o, kF, r]
// A work-group of 512 threads stages the slab in LDS (coalesced loads),
// applies op(G) to every row in place (each row is read into registers
// first; op(G) sits in LDS and is read by broadcast), and then runs the nF-
// point transforms along the rows' other axis with the register/LDS engine,
// one transform per output column, storing coalesced rows of the result.
#include <algorithm>

#include "runtime.h"
#include "xform.h"

namespace fm {
namespace {

using namespace xf;

constexpr int kKW = 13;                    // 8192 values per work-group
constexpr int kKT = Geo<kKW>::kThreads;    // 512 threads
constexpr int kMaxG = 32;                  // largest dense dimension

struct KronArgs {
  const c64* x;
  c64* y;
  const c64* g;  // column-major m x n, leading dimension lda
  int64_t lda;
  int m, n;      // shape of G
  int lognf;
  int64_t outer;     // slabs per column
  int64_t ldx, ldy;  // column strides
  const c64* tw;
  int adj, real, acc;
};

template <int NIN>
__global__ __launch_bounds__(kKT) void kron_fg_kernel(KronArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nF = 1 << a.lognf;
  const int nin = a.adj ? a.m : a.n, nout = a.adj ? a.n : a.m;
  const int S = (nin > nout ? nin : nout) + 1;  // padded row stride of the slab
  c64* slab = reinterpret_cast<c64*>(smem_raw);
  const size_t slab_vals = size_t(nF) * S > size_t(Geo<kKW>::kVals + Geo<kKW>::kVals / 16)
                               ? size_t(nF) * S
                               : size_t(Geo<kKW>::kVals + Geo<kKW>::kVals / 16);
  c64* gm = slab + slab_vals;  // op(G) rows: gm[r * NIN + k]
  const int tid = threadIdx.x;
  const int64_t col = blockIdx.x / a.outer, o = blockIdx.x % a.outer;
  const c64* X = a.x + col * a.ldx + o * int64_t(nF) * nin;
  c64* Y = a.y + col * a.ldy + o * int64_t(nF) * nout;
  // op(G), zero-padded to NIN columns
  for (int i = tid; i < nout * NIN; i += kKT) {
    const int r = i / NIN, k = i - r * NIN;
    c64 v = {0.f, 0.f};
    if (k < nin) {
      v = a.adj ? a.g[k + int64_t(r) * a.lda] : a.g[r + int64_t(k) * a.lda];
      if (a.adj) v.y = -v.y;
    }
    gm[i] = v;
  }
  // slab rows (coalesced): element e = p*nin + k, at most 16 per thread; all
  // loads are issued before the first LDS store
  {
    c64 ld[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int e = tid + kKT * i;
      ld[i] = e < nF * nin ? X[e] : c64{0.f, 0.f};
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int e = tid + kKT * i;
      if (e < nF * nin) {
        const int p = e / nin, k = e - p * nin;
        slab[p * S + k] = ld[i];
      }
    }
  }
  __syncthreads();
  // op(G) along each row: tpr = 512 / nF threads per row share its outputs
  {
    const int tpr = kKT / nF;
    const int row = tid / tpr, part = tid % tpr;
    c64 xr[NIN];
#pragma unroll
    for (int k = 0; k < NIN; ++k) xr[k] = k < nin ? slab[row * S + k] : c64{0.f, 0.f};
    __syncthreads();  // every row is read before any is overwritten
    for (int r = part; r < nout; r += tpr) {
      const c64* gr = gm + r * NIN;
      float sr = 0.f, si = 0.f;
      if (a.real) {
#pragma unroll
        for (int k = 0; k < NIN; ++k) {
          sr += gr[k].x * xr[k].x;
          si += gr[k].x * xr[k].y;
        }
      } else {
#pragma unroll
        for (int k = 0; k < NIN; ++k) {
          sr += gr[k].x * xr[k].x - gr[k].y * xr[k].y;
          si += gr[k].x * xr[k].y + gr[k].y * xr[k].x;
        }
      }
      slab[row * S + r] = c64{sr, si};
    }
    __syncthreads();
  }
  // nF-point transforms along the slab's first axis, one per output column r:
  // thread (b = tid % B, t = tid / B) holds points t + T*k of transform b
  const int T = nF >> 4;
  const int B = kKT / T;
  const int b = tid % B, t = tid / B;
  c64 v[kE];
#pragma unroll
  for (int k = 0; k < kE; ++k) v[k] = b < nout ? slab[(t + T * k) * S + b] : c64{0.f, 0.f};
  __syncthreads();  // the slab is free: its LDS becomes the transforms' exchange space
  c64* my = slab + b * (nF + T);
  if (a.adj) conj_all(v);
  forward(v, a.lognf, t, my, a.tw);
  if (a.adj) conj_all(v);
  if (b < nout) {
#pragma unroll
    for (int k = 0; k < kE; ++k) {
      c64* dst = Y + int64_t(t + T * k) * nout + b;
      *dst = a.acc ? cadd(*dst, v[k]) : v[k];
    }
  }
}

}  // namespace

bool kron_fg_supported(Elem e, int lognf, int64_t m, int64_t n) {
  const int64_t nF = int64_t(1) << lognf;
  const int64_t mx = m > n ? m : n;
  // nF <= 512: every row has at least one thread in the op(G) step
  return e == Elem::C64 && lognf >= 4 && lognf <= 9 && m <= kMaxG && n <= kMaxG && nF * mx <= (int64_t(1) << kKW) &&
         m >= 1 && n >= 1;
}

fm_status launch_kron_fg(int lognf, int64_t m, int64_t n, const void* g, int64_t lda, int adjoint, int real_g,
                         int64_t ncols, int64_t outer, const void* x, int64_t ldx, void* y, int64_t ldy, int acc,
                         hipStream_t s) {
  FM_CHECK_ARG(kron_fg_supported(Elem::C64, lognf, m, n), FM_E_UNSUPPORTED, "fused Kronecker slab: shape");
  if (ncols == 0 || outer == 0) return FM_OK;
  const int64_t blocks = ncols * outer;
  FM_CHECK_ARG(blocks < (int64_t(1) << 31), FM_E_UNSUPPORTED, "fused Kronecker slab: grid too large");
  KronArgs a;
  a.x = static_cast<const c64*>(x);
  a.y = static_cast<c64*>(y);
  a.g = static_cast<const c64*>(g);
  a.lda = lda;
  a.m = int(m);
  a.n = int(n);
  a.lognf = lognf;
  a.outer = outer;
  a.ldx = ldx;
  a.ldy = ldy;
  a.tw = static_cast<const c64*>(twiddle_table(Elem::C64, lognf));
  FM_CHECK_ARG(a.tw != nullptr, FM_E_DEVICE, "twiddle table unavailable");
  a.adj = adjoint;
  a.real = real_g;
  a.acc = acc;
  const int64_t nF = int64_t(1) << lognf;
  const int nin = int(adjoint ? m : n), nout = int(adjoint ? n : m);
  const int S = (nin > nout ? nin : nout) + 1;
  const int NIN = nin <= 8 ? 8 : nin <= 16 ? 16 : 32;
  const size_t slab_vals = std::max<size_t>(size_t(nF) * S, size_t(Geo<kKW>::kVals + Geo<kKW>::kVals / 16));
  const size_t lds = (slab_vals + size_t(nout) * NIN) * sizeof(c64);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&kron_fg_kernel<8>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&kron_fg_kernel<16>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&kron_fg_kernel<32>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr = true;
  }
  const dim3 grid{unsigned(blocks)};
  if (NIN == 8)
    hipLaunchKernelGGL(kron_fg_kernel<8>, grid, dim3(kKT), lds, s, a);
  else if (NIN == 16)
    hipLaunchKernelGGL(kron_fg_kernel<16>, grid, dim3(kKT), lds, s, a);
  else
    hipLaunchKernelGGL(kron_fg_kernel<32>, grid, dim3(kKT), lds, s, a);
  FM_LAUNCHED();
  return FM_OK;
}

}  // namespace fm
