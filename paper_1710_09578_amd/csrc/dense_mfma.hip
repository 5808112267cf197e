// Dense complex64 product of a small matrix (both sides <= 64) with many
// vectors on the matrix cores: y_q = op(A) x_q for every vector q of a batch
// (the dense product of eq. (2), the candidate the run-time calibration
// weighs against an operator's fast transform).
//
// The complex product is a real one on interleaved values: with
// X[q][2k + p] the real (p = 0) or imaginary (p = 1) part of x_q[k] and
// Y[q][2i + p] likewise,
//   Y[q][rho] = sum_kappa X[q][kappa] Ar[rho][kappa],
//   Ar[2i][2k] = Ar[2i+1][2k+1] = Re op(A)[i][k], Ar[2i][2k+1] = -Im, Ar[2i+1][2k] = Im,
// so a block of vectors is an M = vectors, N = 2 rows_out, K = 2 rows_in real
// product. A work-group of 256 threads takes 64 vectors: they are loaded
// coalesced into LDS (row stride 2 NI + 1 floats: the 32 lanes that read one
// K index of 32 vectors hit 32 banks), op(A) goes to LDS once, each wave
// computes 32 x 32 output tiles with v_mfma_f32_32x32x2_f32 (lane l supplies
// A[l % 32][l / 32] and B[l / 32][l % 32]; value v of lane l is
// D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32]), the tiles go back through LDS,
// and the outputs leave coalesced.
#include <algorithm>

#include "kernels.h"
#include "runtime.h"

namespace fm {
namespace {

constexpr int kDM = 64;  // vectors per work-group

struct DmArgs {
  const c64* a;  // column-major m x n, leading dimension lda
  int64_t lda;
  int m, n, adj, acc;
  Batch b;
  const c64* x;
  c64* y;
  int64_t P;  // vectors (ncols * outer)
};

// NI, NO: rows in / out rounded up to 16, 32 or 64.
template <int NI, int NO>
__global__ __launch_bounds__(256) void dense_mfma_kernel(DmArgs a) {
  typedef float v16 __attribute__((ext_vector_type(16)));
  constexpr int SX = 2 * NI + 1;  // floats per staged input vector
  constexpr int SY = 2 * NO + 1;  // floats per staged output vector
  constexpr int SA = NI + 1;      // complex per row of op(A)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* xs = reinterpret_cast<float*>(smem_raw);  // kDM x SX, reused for the outputs (kDM x SY)
  constexpr int kStage = (kDM * (SX > SY ? SX : SY) + 3) & ~3;
  c64* as = reinterpret_cast<c64*>(xs + kStage);  // NO x SA
  const int tid = threadIdx.x;
  const int rin = a.adj ? a.m : a.n, rout = a.adj ? a.n : a.m;
  const int64_t q0 = int64_t(blockIdx.x) * kDM;
  const int nq = int(a.P - q0 < kDM ? a.P - q0 : kDM);
  // op(A), zero-padded to NO x NI
  for (int e = tid; e < NO * NI; e += 256) {
    const int i = e / NI, k = e - i * NI;
    c64 v = {0.f, 0.f};
    if (i < rout && k < rin) {
      v = a.adj ? a.a[k + int64_t(i) * a.lda] : a.a[i + int64_t(k) * a.lda];
      if (a.adj) v.y = -v.y;
    }
    as[i * SA + k] = v;
  }
  // the block of vectors (vector q at column q / outer, slab q % outer)
  for (int e = tid; e < kDM * NI; e += 256) {
    const int q = e / NI, k = e - q * NI;
    c64 v = {0.f, 0.f};
    if (q < nq && k < rin) {
      const int64_t g = q0 + q;
      const int64_t c = a.b.outer == 1 ? g : g / a.b.outer, o = g - c * a.b.outer;
      v = a.x[c * a.b.ldx + o * a.b.xvs + k];
    }
    xs[q * SX + 2 * k] = v.x;
    xs[q * SX + 2 * k + 1] = v.y;
  }
  __syncthreads();
  // tiles: M = 64 vectors (2 tiles), N = 2 NO (NO / 16 tiles), K = 2 NI (NI steps)
  constexpr int MT = kDM / 32, NT = 2 * NO / 32, TILES = MT * NT;
  constexpr int TPW = (TILES + 3) / 4;  // tiles per wave
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, lk = lane >> 5;
  v16 acc[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) acc[j] = v16{};
  // per tile: the lane's operand rows, and the part / sign of op(A) it needs
  // (Ar[rho][2s + lk] is Re when lk == rho % 2, else -Im (rho even) or +Im)
  int xoff[TPW], aoff[TPW];
  bool take_re[TPW];
  float sgn[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    const int tile = wave + 4 * j;
    const int mt = (tile < TILES ? tile : 0) / NT, nt = (tile < TILES ? tile : 0) % NT;
    const int rho = nt * 32 + li, po = rho & 1;
    xoff[j] = (mt * 32 + li) * SX + lk;
    aoff[j] = (rho >> 1) * SA;
    take_re[j] = lk == po;
    sgn[j] = (lk != po && po == 0) ? -1.f : 1.f;
  }
  // the wave's tiles advance together (independent accumulators in flight);
  // the operands of 4 K steps are read from LDS before their products issue
  const bool on_last = TILES % 4 == 0 || wave + 4 * (TPW - 1) < TILES;  // uniform across the wave
  constexpr int U = 4;
  for (int s0 = 0; s0 < NI; s0 += U) {
    float af[TPW][U];
    c64 av[TPW][U];
#pragma unroll
    for (int j = 0; j < TPW; ++j)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        // A operand: X[q][2s + lk]; B operand from op(A)[rho / 2][s]
        af[j][u] = xs[xoff[j] + 2 * (s0 + u)];
        av[j][u] = as[aoff[j] + s0 + u];
      }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int j = 0; j < TPW; ++j) {
        if (j < TPW - 1 || on_last) {
          const float bf = (take_re[j] ? av[j][u].x : av[j][u].y) * sgn[j];
          acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[j][u], bf, acc[j], 0, 0, 0);
        }
      }
  }
  __syncthreads();  // every product has read the staged inputs
  float* ys = xs;
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    const int tile = wave + 4 * j;
    if (tile < TILES) {
      const int mt = tile / NT, nt = tile % NT;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int q = mt * 32 + 8 * (v / 4) + 4 * lk + (v % 4);
        ys[q * SY + nt * 32 + li] = acc[j][v];
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < kDM * NO; e += 256) {
    const int q = e / NO, i = e - q * NO;
    if (q < nq && i < rout) {
      const int64_t g = q0 + q;
      const int64_t c = a.b.outer == 1 ? g : g / a.b.outer, o = g - c * a.b.outer;
      c64* dst = a.y + c * a.b.ldy + o * a.b.yvs + i;
      const c64 v = {ys[q * SY + 2 * i], ys[q * SY + 2 * i + 1]};
      *dst = a.acc ? cadd(*dst, v) : v;
    }
  }
}

template <int NI, int NO>
size_t dm_lds() {
  constexpr int SX = 2 * NI + 1, SY = 2 * NO + 1, SA = NI + 1;
  constexpr int kStage = (kDM * (SX > SY ? SX : SY) + 3) & ~3;
  return size_t(kStage) * 4 + size_t(NO) * SA * 8;
}

template <int NI, int NO>
fm_status launch_dm(const DmArgs& a, hipStream_t s) {
  static bool attr = false;
  const size_t lds = dm_lds<NI, NO>();
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dense_mfma_kernel<NI, NO>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr = true;
  }
  hipLaunchKernelGGL((dense_mfma_kernel<NI, NO>), dim3(unsigned(cdiv(a.P, kDM))), dim3(256), lds, s, a);
  FM_LAUNCHED();
  return FM_OK;
}

int pad16(int v) { return v <= 16 ? 16 : v <= 32 ? 32 : 64; }

}  // namespace

bool dense_mfma_supported(Elem e, int64_t m, int64_t n, const Batch& b) {
  return e == Elem::C64 && m >= 1 && n >= 1 && m <= 64 && n <= 64 && b.inner == 1 && b.ncols * b.outer >= 1 &&
         b.ncols * b.outer < (int64_t(1) << 37);
}

fm_status launch_dense_mfma(int64_t m, int64_t n, const void* A, int64_t lda, int adjoint, const Batch& b,
                            const void* x, void* y, int acc, hipStream_t s) {
  FM_CHECK_ARG(dense_mfma_supported(Elem::C64, m, n, b), FM_E_UNSUPPORTED, "dense (matrix cores): shape");
  const int64_t P = b.ncols * b.outer;
  if (P == 0) return FM_OK;
  DmArgs a{static_cast<const c64*>(A), lda, int(m), int(n), adjoint, acc, b, static_cast<const c64*>(x),
           static_cast<c64*>(y), P};
  const int ni = pad16(int(adjoint ? m : n)), no = pad16(int(adjoint ? n : m));
#define FM_DM(I, O) \
  if (ni == I && no == O) return launch_dm<I, O>(a, s);
  FM_DM(16, 16) FM_DM(16, 32) FM_DM(16, 64)
  FM_DM(32, 16) FM_DM(32, 32) FM_DM(32, 64)
  FM_DM(64, 16) FM_DM(64, 32) FM_DM(64, 64)
#undef FM_DM
  set_error("dense (matrix cores): no kernel for %d x %d", no, ni);
  return FM_E_UNSUPPORTED;
}

}  // namespace fm
