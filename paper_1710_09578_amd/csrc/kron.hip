// Fused Kronecker slab pass: the last two factors of a Kronecker product,
// a Fourier matrix F_nF and a small dense matrix G (m x n), applied to each
// slab of nF x n values (eq. (7) structure, first factor slowest) in one
// read and one write of the slab:
//   forward:  Y[o, kF, r] = sum_pF W^(pF kF) sum_k G[r, k] X[o, pF, k]
//   adjoint:  Y[o, pF, k] = sum_kF W^-(pF kF) sum_r conj(G[r, k]) X[o, kF, r]
// A work-group of 512 threads stages the slab in LDS (coalesced loads),
// applies op(G) to every row in place as a matrix product on the matrix
// cores (MFMA, fp32), and then runs the nF-point transforms along the rows'
// other axis with the register/LDS engine, one transform per output column,
// storing coalesced rows of the result.
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

// Register budget of four waves per SIMD: two 512-thread work-groups per CU,
// as many as the slab's LDS allows (the complex 32-column form spills 10
// registers there and runs 1.2x faster than at one work-group per CU).
template <int NIN, bool REAL>
__global__ __launch_bounds__(kKT, 4) void kron_fg_kernel(KronArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nF = 1 << a.lognf;
  const int nin = a.adj ? a.m : a.n, nout = a.adj ? a.n : a.m;
  const int S = (nin > nout ? nin : nout) + 1;  // padded row stride of the slab
  c64* slab = reinterpret_cast<c64*>(smem_raw);
  // op(G) rows: gm[r * GS + k]; the odd row stride spreads the 32 rows a wave
  // reads together over the banks (NIN values, a multiple of 64 bytes, folded
  // them onto one to four banks)
  constexpr int GS = NIN + 1;
  c64* gm = slab + size_t(nF) * S;
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
    gm[r * GS + k] = v;
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
        const int p = nin == NIN ? e / NIN : e / nin;  // a shift when op(G) needs no padding
        const int k = e - p * nin;
        slab[p * S + k] = ld[i];
      }
    }
  }
  __syncthreads();
  // op(G) along each row as a matrix product on the matrix cores
  // (v_mfma_f32_32x32x2_f32: lane l supplies A[l % 32][l / 32] and
  // B[l / 32][l % 32]; value v of lane l is D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32]).
  //   real op(G):    rows m = 2p + part (re / im of slab row p), K = NIN, N = 32:
  //                  D[m][r] = sum_k X_part[p][k] op(G)[r][k]
  //   complex op(G): rows m = p, K = 2 NIN ([X_re | X_im]), N = 64 ([Y_re | Y_im]),
  //                  B = [[Gr^T, Gi^T], [-Gi^T, Gr^T]]
  {
    typedef float v16 __attribute__((ext_vector_type(16)));
    const float* sf = reinterpret_cast<const float*>(slab);
    const float* gf = reinterpret_cast<const float*>(gm);
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 31, lk = lane >> 5;
    const int mt_count = REAL ? (2 * nF + 31) / 32 : (nF + 31) / 32;
    const int nt_count = REAL ? 1 : 2;
    const int ntiles = mt_count * nt_count;
    // operands of a tile are gathered from LDS before its products are
    // issued; real op(G): the two tiles of a wave advance together (B is the
    // same for both); complex op(G): one tile at a time
    v16 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = v16{};
    if constexpr (REAL) {
      constexpr int KS = NIN / 2;
      float bf[KS];
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        const int k = 2 * kk + lk;
        bf[kk] = li < nout ? gf[2 * (li * GS + k)] : 0.f;  // k >= nin: zero padding of op(G)
      }
#pragma unroll
      for (int j0 = 0; j0 < 4; j0 += 2) {
        if (wave + 8 * j0 >= ntiles) break;  // uniform across the wave
        float af[2][KS];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          const int tile = wave + 8 * (j0 + jj);
          const int m = tile * 32 + li;
          const int p = m >> 1, part = m & 1;
#pragma unroll
          for (int kk = 0; kk < KS; ++kk) {
            const int k = 2 * kk + lk;
            af[jj][kk] = (tile < ntiles && p < nF && k < nin) ? sf[2 * (p * S + k) + part] : 0.f;
          }
        }
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
          acc[j0] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[0][kk], bf[kk], acc[j0], 0, 0, 0);
          acc[j0 + 1] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[1][kk], bf[kk], acc[j0 + 1], 0, 0, 0);
        }
      }
    } else {
      constexpr int KS = NIN;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int tile = wave + 8 * j;
        if (tile < ntiles) {
          const int mt = tile / nt_count, nt = tile % nt_count;
          const int m = mt * 32 + li;
          float af[KS], bf[KS];
#pragma unroll
          for (int kk = 0; kk < KS; ++kk) {
            const int k = 2 * kk + lk;
            const int kr = k < NIN ? k : k - NIN, kpart = k < NIN ? 0 : 1;
            af[kk] = (m < nF && kr < nin) ? sf[2 * (m * S + kr) + kpart] : 0.f;
            const int n = nt * 32 + li;
            const int nr = n & 31, npart = n >> 5;
            float bv = 0.f;
            if (nr < nout) {
              const float gr = gf[2 * (nr * GS + kr)], gi = gf[2 * (nr * GS + kr) + 1];
              bv = kpart == 0 ? (npart == 0 ? gr : gi) : (npart == 0 ? -gi : gr);
            }
            bf[kk] = bv;
          }
#pragma unroll
          for (int kk = 0; kk < KS; ++kk)
            acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[kk], bf[kk], acc[j], 0, 0, 0);
        }
      }
    }
    __syncthreads();  // every product has read the slab: write the results in place
    float* so = reinterpret_cast<float*>(slab);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int tile = wave + 8 * j;
      if (tile < ntiles) {
        const int mt = tile / nt_count, nt = tile % nt_count;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int m = mt * 32 + 8 * (v / 4) + 4 * lk + (v % 4);
          const int n = nt * 32 + li;
          if (REAL) {
            const int p = m >> 1, part = m & 1;
            if (p < nF && n < nout) so[2 * (p * S + n) + part] = acc[j][v];
          } else {
            const int nr = n & 31, npart = n >> 5;
            if (m < nF && nr < nout) so[2 * (m * S + nr) + npart] = acc[j][v];
          }
        }
      }
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
  __syncthreads();  // slab and op(G) are free: their LDS becomes the transforms' exchange space
  c64* my = slab + b * region_stride(a.lognf, B, true);
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
  // the slab and op(G), later the exchange regions of the 8192 / nF transforms
  const int B = int((int64_t(1) << kKW) / nF);
  const size_t lds = std::max<size_t>(size_t(nF) * S + size_t(nout) * (NIN + 1), size_t(B) * region_stride(lognf, B, true)) *
                     sizeof(c64);
  const dim3 grid{unsigned(blocks)};
#define FM_KRON_LAUNCH(N, RL)                                                                           \
  do {                                                                                                 \
    static bool attr = false;                                                                          \
    if (!attr) {                                                                                       \
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&kron_fg_kernel<N, RL>),                 \
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);               \
      attr = true;                                                                                     \
    }                                                                                                  \
    hipLaunchKernelGGL((kron_fg_kernel<N, RL>), grid, dim3(kKT), lds, s, a);                           \
  } while (0)
  if (real_g) {
    if (NIN == 8) FM_KRON_LAUNCH(8, true);
    else if (NIN == 16) FM_KRON_LAUNCH(16, true);
    else FM_KRON_LAUNCH(32, true);
  } else {
    if (NIN == 8) FM_KRON_LAUNCH(8, false);
    else if (NIN == 16) FM_KRON_LAUNCH(16, false);
    else FM_KRON_LAUNCH(32, false);
  }
#undef FM_KRON_LAUNCH
  FM_LAUNCHED();
  return FM_OK;
}

}  // namespace fm
