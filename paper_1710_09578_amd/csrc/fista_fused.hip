// Fused per-operator proximal-gradient solver (fm_fista) for A = C and
// A = S C, C a circulant or Toeplitz operator (eq. (5), eq. (7)) and S a row
// selection: the iteration of eq. (8) with its accelerated form, where the
// time goes to the forward and backward transforms. Each iteration is the
// convolution's passes in each direction plus one stop check:
//   forward:  the passes of C y; the last pass stores r = S (C y) - b (the
//             selection and the subtraction of b in its store);
//   adjoint:  the passes of C^H (S^H r), S^H applied at the first pass's
//             load (the inverse index map of S); the last pass applies the
//             update z = y - g/L, x+ = soft(z, lam/L), y+ = x+ + beta (x+ - x)
//             in place of storing g, with the stopping rule's partial sums;
//   stop:     per column, freeze when ||x+ - x|| <= tol ||x+|| and advance the
//             device iteration counter that selects the next momentum weight.
// The passes and their work items are those of the batched stage kernel (the
// same engine calls and epilogues), so a complex64 solve gives the same bits
// as the same problem solved in a batch. A = S C (never a batch problem) with
// one or two columns and a power-of-two length L >= 65536 takes 1024-point
// rows instead (L = 1024 n2, one-wave work-groups, the spectrum reordered for
// that split once per solve): a single column then spreads each pass over
// n2 >= 64 work-groups instead of L / 4096. The launches of a chunk of steady
// iterations (10 by default) are captured once per solve into a HIP graph and
// replayed; the first iteration and a remainder shorter than a chunk are
// launched directly.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "epi.h"
#include "mixed.h"
#include "runtime.h"
#include "solve.h"
#include "xform.h"

namespace fm {
namespace {

using namespace xf;

// FS31 / FS3U1: the last strided pass of one direction and the first strided
// pass of the next in one work-group. Both cover the same column positions
// (tile i0 .. i0 + n1 / n2 of every strided transform), and a thread holds
// the same points of its transform in both, so the first pass's epilogue
// keeps the values the second loads (S^H r after the residual, y after the
// update) in registers: one launch and one read of them fewer, same bits.
enum FKind : int {
  FK_SINGLE = 0, FK_ROWF = 1, FK_FS1 = 2, FK_FS2 = 3, FK_FS3 = 4, FK_MX1 = 5, FK_MX3 = 6,
  FK_FS31 = 7,   // forward FS3 with the residual, then the adjoint's FS1
  FK_FS3U1 = 8   // adjoint FS3 with the update, then the next forward FS1
};

template <typename R>
struct FArgs {
  const Cx<R>* in;  // the direction's input block: y (forward) or r (adjoint)
  int64_t ldin;
  Cx<R>* slot;      // L values per column
  const Cx<R>* spec;
  const Cx<R>* tw;   // power-of-two twiddle tables
  const Cx<R>* twl;  // W_L of the four-step length
  int logL, n2, adj;
  int64_t L;
  int in_rows, out_rows;  // rows of C's input and output in this direction
  const int* imap;        // adjoint: C's output row -> row of r (or -1)
  const int* omap;        // forward: the same map, for the store of r
  const Cx<R>* b;
  int64_t ldb;
  Cx<R>* r;
  int64_t ldr;
  Cx<R>* yv;  // y iterate
  int64_t ldy;
  Cx<R>* x;   // x iterate
  int64_t ldx;
  const double* lam;
  double invL;
  const int* active;
  int* status;
  const int64_t* pbase;
  double* partial;
  const R* beta;
  const int* iter;
  int momentum;
  int64_t ncols;
  // chained iterations: the forward's first launch (FS2) also runs the
  // previous iteration's stop check (check), the next launch (FS31) advances
  // the iteration counter (bump); see launch_chained
  int check, bump, nslot;
  double stop_tol;
  int* active_w;
  int* iters;
  int* iter_w;
};

// Stop rule of one column after an iteration: freeze when it met a
// non-finite value or when ||x+ - x|| <= tol * max(||x+||, 1e-30), with the
// partial sums taken in slot order.
__device__ __forceinline__ bool freeze_now(const double* partial, const int64_t* pbase, int nslot, int64_t c,
                                           double tol, const int* status) {
  if (status[c]) return true;
  if (tol <= 0.0) return false;
  double dx = 0.0, nx = 0.0;
  for (int t = 0; t < nslot; ++t) {
    dx += partial[2 * (pbase[c] + t)];
    nx += partial[2 * (pbase[c] + t) + 1];
  }
  const double nrm = sqrt(nx);
  return sqrt(dx) <= tol * (nrm > 1e-30 ? nrm : 1e-30);
}

template <typename R, bool CAP = false>
__device__ __forceinline__ FistaEpT<R, CAP> update_ep(const FArgs<R>& a, int64_t col, bool strided, int lg) {
  FistaEpT<R, CAP> ep;
  ep.X = a.x + col * a.ldx;
  ep.xstride = strided ? 0 : a.ldx;
  ep.gcol0 = col;
  ep.colstride = strided ? 0 : 1;
  ep.active = a.active;
  ep.lam = a.lam;
  ep.invLd = a.invL;
  ep.invL = R(a.invL);
  ep.beta = a.beta[*a.iter];
  ep.momentum = a.momentum;
  ep.status = a.status;
  ep.flush_per_slot = !strided && lg < 4;
  ep.pbase = a.pbase;
  ep.partial = a.partial;
  return ep;
}

// EPI: 0 slot pass, 1 residual store (forward's last pass), 2 update (adjoint's
// last pass). IMAP: the input goes through imap; MAP: r is stored through omap.
// LOGW: log2 of the four-step row length n1 (12: 4096-point rows in
// 256-thread work-groups; 10: 1024-point rows in one-wave work-groups, for the
// separate power-of-two strided passes only).
template <typename R, int KIND, int EPI, bool IMAP, bool MAP, int LOGW = 12>
__global__ __launch_bounds__(256) void ff_kernel(FArgs<R> a) {
  static_assert(LOGW == 12 || KIND == FK_FS1 || KIND == FK_FS2 || KIND == FK_FS3 || KIND == FK_FS31 ||
                    KIND == FK_FS3U1,
                "shorter rows: separate power-of-two strided passes only");
  constexpr int N1 = 1 << LOGW;
  constexpr int NT = Geo<LOGW>::kThreads;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Cx<R>* smem = reinterpret_cast<Cx<R>*>(smem_raw);
  if constexpr (KIND == FK_SINGLE) {
    // whole zero-padded convolutions of length 2^logL, 4096 / 2^logL columns
    const int lg = a.logL;
    const int tpw = 1 << (12 - lg);
    const int64_t c0 = int64_t(blockIdx.x) * tpw;
    const int cnt = int(a.ncols - c0 < tpw ? a.ncols - c0 : tpw);
    if (a.active) {
      bool any = false;
      for (int c = 0; c < cnt; ++c) any |= a.active[c0 + c] != 0;
      if (!any) return;
    }
    Job<R> jb;
    jb.x = a.in + c0 * a.ldin;
    jb.xbstride = a.ldin;
    jb.imap = a.imap;
    if constexpr (EPI == 2) {
      jb.y = a.yv + c0 * a.ldy;
      jb.ybstride = a.ldy;
    } else {
      jb.y = a.r + c0 * a.ldr;
      jb.ybstride = a.ldr;
    }
    jb.inner = 1;
    jb.nvalid = cnt;
    jb.in_limit = a.in_rows;
    jb.out_limit = a.out_rows;
    jb.i0 = 0;
    jb.S = a.spec;
    jb.sbstride = 0;
    jb.q0 = 0;
    const Mode md{FFT_CONV, a.adj, 0, 0, 0};
    if constexpr (EPI == 1) {
      ResidualEpT<R, MAP> ep{a.b + c0 * a.ldb, a.ldb, a.r + c0 * a.ldr, a.omap, a.ldr};
      run_job<R, false, 12, true, ResidualEpT<R, MAP>, IMAP>(jb, md, lg, smem, a.tw, &ep);
    } else {
      FistaEpT<R> ep = update_ep(a, c0, false, lg);
      run_job<R, false, 12, true, FistaEpT<R>, IMAP>(jb, md, lg, smem, a.tw, &ep);
      fista_partials<256>(ep, false, lg, cnt, 0, smem);
    }
    return;
  }
  const int64_t c = blockIdx.y;
  if constexpr (KIND == FK_FS31) {  // advance the counter once per launch (frozen columns included)
    if (a.bump && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *a.iter_w = *a.iter + 1;
  }
  if (a.active && !a.active[c]) return;
  if constexpr (KIND == FK_FS2) {
    // the previous iteration's stop check, taken by every work-group of the
    // column alike (the same sums in the same order); the first one records
    // it. The row pass of a column frozen here is computed and not used.
    if (a.check && blockIdx.x == 0 && threadIdx.x == 0 &&
        freeze_now(a.partial, a.pbase, a.nslot, c, a.stop_tol, a.status)) {
      a.active_w[c] = 0;
      a.iters[c] = *a.iter + 1;
    }
  }
  Cx<R>* w = a.slot + c * a.L;
  const Cx<R>* xin = a.in + c * a.ldin;
  if constexpr (KIND == FK_ROWF || KIND == FK_FS2) {
    // row k2 of the four-step split: transform, spectral product, inverse,
    // twiddles W_L^-(n1 k2), into the slot (ROWF forms the row from the input)
    const int k2 = blockIdx.x;
    Cx<R>* row = w + (int64_t(k2) << LOGW);
    Job<R> jb;
    jb.twl = a.twl;
    if constexpr (KIND == FK_ROWF) {
      jb.x = xin;
      jb.in_limit = a.in_rows;
      jb.fuse_n2 = a.n2;
      jb.imap = a.imap;
    } else {
      jb.x = row;
      jb.in_limit = N1;
    }
    jb.y = row;
    jb.xbstride = jb.ybstride = 0;
    jb.inner = 1;
    jb.nvalid = 1;
    jb.out_limit = N1;
    jb.i0 = 0;
    jb.S = a.spec + (int64_t(k2) << LOGW);
    jb.sbstride = 0;
    jb.q0 = k2;
    const Mode md{FFT_CONV, a.adj, a.logL, 1, 0};
    // rows are latency-bound launches of n2 work-groups per column: the
    // twiddle seeds go out with the input loads (PRETW)
    run_job<R, false, LOGW, true, NoEp, KIND == FK_ROWF && IMAP, false, true>(jb, md, LOGW, smem, a.tw);
    return;
  } else if constexpr (KIND == FK_FS31 || KIND == FK_FS3U1) {
    // the direction's inverse strided pass with its epilogue (capturing; its
    // operand loads issued first), then the next direction's forward strided
    // pass on the captured values
    const int lg = 31 - __builtin_clz(a.n2);
    const int tpw = 1 << (LOGW - lg);
    const int i0 = int(blockIdx.x) * tpw;
    Job<R> jb;
    jb.xbstride = jb.ybstride = 1;
    jb.inner = N1;
    jb.nvalid = tpw;
    jb.i0 = i0;
    jb.S = nullptr;
    jb.sbstride = 0;
    jb.q0 = i0;
    jb.twl = a.twl;
    jb.x = w + i0;
    jb.y = (KIND == FK_FS3U1 ? a.yv + c * a.ldy : a.r + c * a.ldr) + i0;
    jb.in_limit = int(a.L);
    jb.out_limit = a.out_rows;
    const Mode mi{FFT_INV, 0, 0, 0, 0};
    const Mode mf{FFT_FWD, 0, a.logL, 0, 0};
    Job<R> jf = jb;  // the second pass: from registers into the slot
    jf.x = nullptr;
    jf.y = w + i0;
    jf.out_limit = int(a.L);
    if constexpr (KIND == FK_FS31) {
      ResidualEpT<R, MAP, true> ep{a.b + c * a.ldb, 0, a.r + c * a.ldr, a.omap, 0};
      run_job<R, true, LOGW, true, ResidualEpT<R, MAP, true>, false, false, false, true>(jb, mi, lg, smem, a.tw, &ep);
      __syncthreads();  // every thread is past the first pass's LDS use
      jf.rin = ep.cap;
      run_job<R, true, LOGW, true, NoEp, false, true>(jf, mf, lg, smem, a.tw);
    } else {
      FistaEpT<R, true> ep = update_ep<R, true>(a, c, true, lg);
      run_job<R, true, LOGW, true, FistaEpT<R, true>, false, false, false, true>(jb, mi, lg, smem, a.tw, &ep);
      fista_partials<NT>(ep, true, lg, tpw, int(blockIdx.x), smem);
      __syncthreads();  // the partial sums have left the LDS
      jf.rin = ep.cap;
      run_job<R, true, LOGW, true, NoEp, false, true>(jf, mf, lg, smem, a.tw);
    }
    return;
  } else if constexpr (KIND == FK_FS1 || KIND == FK_FS3) {
    // strided 2^lg-point transforms at stride n1 over n1 / 2^lg positions
    const int lg = 31 - __builtin_clz(a.n2);
    const int tpw = 1 << (LOGW - lg);
    const int i0 = int(blockIdx.x) * tpw;
    Job<R> jb;
    jb.xbstride = jb.ybstride = 1;
    jb.inner = N1;
    jb.nvalid = tpw;
    jb.i0 = i0;
    jb.S = nullptr;
    jb.sbstride = 0;
    jb.q0 = i0;
    jb.twl = a.twl;
    if constexpr (KIND == FK_FS1) {
      jb.x = xin + i0;
      jb.xcol = xin;
      jb.imap = a.imap;
      jb.y = w + i0;
      jb.in_limit = a.in_rows;
      jb.out_limit = int(a.L);
      const Mode md{FFT_FWD, 0, a.logL, 0, 0};
      run_job<R, true, LOGW, true, NoEp, IMAP>(jb, md, lg, smem, a.tw);
    } else {
      jb.x = w + i0;
      jb.y = (EPI == 2 ? a.yv + c * a.ldy : a.r + c * a.ldr) + i0;
      jb.in_limit = int(a.L);
      jb.out_limit = a.out_rows;
      const Mode md{FFT_INV, 0, 0, 0, 0};
      if constexpr (EPI == 1) {
        ResidualEpT<R, MAP> ep{a.b + c * a.ldb, 0, a.r + c * a.ldr, a.omap, 0};
        run_job<R, true, LOGW, true, ResidualEpT<R, MAP>, false, false, false, true>(jb, md, lg, smem, a.tw, &ep);
      } else {
        FistaEpT<R> ep = update_ep(a, c, true, lg);
        run_job<R, true, LOGW, true, FistaEpT<R>, false, false, false, true>(jb, md, lg, smem, a.tw, &ep);
        fista_partials<NT>(ep, true, lg, tpw, int(blockIdx.x), smem);
      }
    }
    return;
  } else {
    // mixed strided passes (L = 4096 n2, n2 not a power of two)
    const int tile = blockIdx.x;
    if constexpr (KIND == FK_MX1) {
      mixed_tile<R, NoEp, IMAP>(a.n2, tile, xin, a.in_rows, w, a.L, false, a.twl, a.L, 0,
                                static_cast<NoEp*>(nullptr), smem, a.imap);
    } else {
      Cx<R>* ycol = EPI == 2 ? a.yv + c * a.ldy : a.r + c * a.ldr;
      if constexpr (EPI == 1) {
        ResidualEpT<R, MAP> ep{a.b + c * a.ldb, 0, a.r + c * a.ldr, a.omap, 0};
        mixed_tile<R, ResidualEpT<R, MAP>>(a.n2, tile, w, a.L, ycol, a.out_rows, true, a.twl, a.L, 0, &ep, smem);
      } else {
        FistaEpT<R> ep = update_ep(a, c, true, 12);
        mixed_tile<R, FistaEpT<R>>(a.n2, tile, w, a.L, ycol, a.out_rows, true, a.twl, a.L, 0, &ep, smem);
        fista_partials<256>(ep, true, 12, 0, tile, smem);
      }
    }
  }
}

// Stop check of one iteration (one work-group): freezes column c when
// ||x+ - x|| <= tol * max(||x+||, 1e-30) (partial sums in slot order) or when
// it met a non-finite value, records the count, and advances the iteration
// counter the next iteration's momentum weight is read with.
__global__ __launch_bounds__(256) void ff_stop_kernel(const double* partial, const int64_t* pbase, int nslot,
                                                      int64_t ncols, double tol, int* active, int* iters,
                                                      const int* status, int* iter) {
  const int k = *iter;
  for (int64_t c = threadIdx.x; c < ncols; c += blockDim.x) {
    if (!active[c]) continue;
    if (freeze_now(partial, pbase, nslot, c, tol, status)) {
      active[c] = 0;
      iters[c] = k + 1;
    }
  }
  __syncthreads();  // every thread has read the counter
  if (threadIdx.x == 0) *iter = k + 1;
}

__global__ __launch_bounds__(256) void ff_pbase_kernel(int64_t ncols, int nslot, int64_t* pbase) {
  const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (c < ncols) pbase[c] = c * nslot;
}

template <typename R, int KIND, int EPI, bool IMAP, bool MAP, int LOGW = 12>
fm_status launch_ff(dim3 grid, const FArgs<R>& a, hipStream_t s) {
  auto fn = &ff_kernel<R, KIND, EPI, IMAP, MAP, LOGW>;
  static std::once_flag once;
  std::call_once(once, [fn] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
  });
  hipLaunchKernelGGL(fn, grid, dim3(Geo<LOGW>::kThreads), (job_lds_bytes<R, LOGW>()), s, a);
  FM_LAUNCHED();
  return FM_OK;
}

// One direction's passes. fwd: input y, last pass stores r; adj: input r
// (through the selection map), last pass updates x and y.
template <typename R, bool SEL>
fm_status launch_direction(const FArgs<R>& a, bool adj, int fuse_max, hipStream_t s) {
  const unsigned nc = unsigned(a.ncols);
  if (a.L <= 4096) {
    const unsigned g = unsigned(cdiv(a.ncols, int64_t(1) << (12 - a.logL)));
    if (!adj) return launch_ff<R, FK_SINGLE, 1, false, SEL>(dim3(g), a, s);
    return launch_ff<R, FK_SINGLE, 2, SEL, false>(dim3(g), a, s);
  }
  const int n2 = a.n2;
  const bool mixed = (n2 & (n2 - 1)) != 0;
  const bool fold = n2 <= fuse_max;
  const unsigned rows = unsigned(n2);
  const unsigned tiles = unsigned(mixed ? mixed_tiles(n2) : n2);
  if (!adj) {
    if (fold) {
      FM_TRY((launch_ff<R, FK_ROWF, 0, false, false>(dim3(rows, nc), a, s)));
    } else {
      if (mixed)
        FM_TRY((launch_ff<R, FK_MX1, 0, false, false>(dim3(tiles, nc), a, s)));
      else
        FM_TRY((launch_ff<R, FK_FS1, 0, false, false>(dim3(tiles, nc), a, s)));
      FM_TRY((launch_ff<R, FK_FS2, 0, false, false>(dim3(rows, nc), a, s)));
    }
    if (mixed) return launch_ff<R, FK_MX3, 1, false, SEL>(dim3(tiles, nc), a, s);
    return launch_ff<R, FK_FS3, 1, false, SEL>(dim3(tiles, nc), a, s);
  }
  if (fold) {
    FM_TRY((launch_ff<R, FK_ROWF, 0, SEL, false>(dim3(rows, nc), a, s)));
  } else {
    if (mixed)
      FM_TRY((launch_ff<R, FK_MX1, 0, SEL, false>(dim3(tiles, nc), a, s)));
    else
      FM_TRY((launch_ff<R, FK_FS1, 0, SEL, false>(dim3(tiles, nc), a, s)));
    FM_TRY((launch_ff<R, FK_FS2, 0, false, false>(dim3(rows, nc), a, s)));
  }
  if (mixed) return launch_ff<R, FK_MX3, 2, false, false>(dim3(tiles, nc), a, s);
  return launch_ff<R, FK_FS3, 2, false, false>(dim3(tiles, nc), a, s);
}

// The stop kernel of one iteration.
fm_status launch_stop_check(const FusedRun& run, int nslot, hipStream_t s) {
  hipLaunchKernelGGL(ff_stop_kernel, dim3(1), dim3(256), 0, s, run.partial, run.pbase, nslot, run.ncols,
                     run.stop_tol, run.active, run.iters, run.status, run.iter);
  FM_LAUNCHED();
  return FM_OK;
}

// Separate power-of-two strided passes of at least 16 points: the chained
// form (one pass before the first iteration, then FS2, FS31, FS2 and FS3U1
// per iteration with the stop check inside them: four launches instead of
// seven).
template <typename R>
bool chained(const FArgs<R>& a, int fuse_max) {
  const int n2 = a.n2;
  return a.L > 4096 && n2 > fuse_max && (n2 & (n2 - 1)) == 0 && n2 >= 16;
}

// One iteration. Chained form: FS2 (forward rows; from the second iteration
// on also the previous iteration's stop check), FS31 (advances the counter
// from the second iteration on), FS2 (adjoint rows), FS3U1; the check of the
// last iteration is a stop kernel after the loop (launch_stop_check). Other
// forms: the direction's passes and a stop kernel.
// LOGW 10 (1024-point rows) runs the chained form only.
template <typename R, int LOGW = 12>
fm_status launch_iteration(const FArgs<R>& fa, const FArgs<R>& aa, const FusedRun& run, int fuse_max, int nslot,
                           bool first, hipStream_t s) {
  if (LOGW != 12 || chained(fa, fuse_max)) {
    const dim3 grid(unsigned(fa.n2), unsigned(fa.ncols));  // n2 rows / n2 tiles per column
    FArgs<R> f = fa;
    f.check = f.bump = first ? 0 : 1;
    FM_TRY((launch_ff<R, FK_FS2, 0, false, false, LOGW>(grid, f, s)));
    if (run.sel_map)
      FM_TRY((launch_ff<R, FK_FS31, 1, false, true, LOGW>(grid, f, s)));
    else
      FM_TRY((launch_ff<R, FK_FS31, 1, false, false, LOGW>(grid, f, s)));
    FM_TRY((launch_ff<R, FK_FS2, 0, false, false, LOGW>(grid, aa, s)));
    return launch_ff<R, FK_FS3U1, 2, false, false, LOGW>(grid, aa, s);
  } else if (run.sel_map) {
    FM_TRY((launch_direction<R, true>(fa, false, fuse_max, s)));
    FM_TRY((launch_direction<R, true>(aa, true, fuse_max, s)));
  } else {
    FM_TRY((launch_direction<R, false>(fa, false, fuse_max, s)));
    FM_TRY((launch_direction<R, false>(aa, true, fuse_max, s)));
  }
  return launch_stop_check(run, nslot, s);
}

// Iterations per captured graph (FM_FISTA_GRAPH; 0: direct launches).
int graph_chunk() {
  static const int v = [] {
    const char* e = std::getenv("FM_FISTA_GRAPH");
    const int k = e ? std::atoi(e) : 10;
    return k < 0 ? 0 : (k > 1000 ? 1000 : k);
  }();
  return v;
}

// Capture stream per device (default priority, non-blocking).
std::mutex g_cap_mu;
hipStream_t g_cap[64] = {};

hipStream_t capture_stream() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(g_cap_mu);
  if (!g_cap[dev] && hipStreamCreateWithFlags(&g_cap[dev], hipStreamNonBlocking) != hipSuccess) g_cap[dev] = nullptr;
  return g_cap[dev];
}

template <typename R, int LOGW>
fm_status iterate(const FArgs<R>& fa, const FArgs<R>& aa, const FusedRun& run, int fuse_max, int nslot,
                  hipStream_t s);

// The convolution's spectrum in the order of the split with 1024-point rows
// (L = 1024 n2): row k2 holds the frequencies k2 + n2 k1, k1 = 0..1023, as
// the row pass reads them (complex64: in pair order, values k and k + 1 of a
// thread adjacent for one 16-byte load). Read from the complex128 copy, which
// is stored for 4096-point rows (row k2' holds k2' + (L / 4096) k1'), and
// rounded once, as the complex64 copy is: the same values, reordered.
template <typename R>
__global__ __launch_bounds__(256) void narrow_spectrum_kernel(int64_t L, const Cx<double>* __restrict__ p64,
                                                              Cx<R>* out) {
  const int64_t f = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (f >= L) return;
  const int64_t n2 = L >> 10, n2w = L >> 12;
  const int64_t k1 = f & 1023, k2 = f >> 10;
  const int64_t g = k2 + n2 * k1;
  const Cx<double> v = p64[g / n2w + 4096 * (g % n2w)];
  int64_t o = f;
  if constexpr (sizeof(R) == 4) {
    const int64_t t = k1 & 63, k = k1 >> 6;  // position t + 64 k of the row's 64 threads
    o = (k2 << 10) + 2 * (t + 64 * (k >> 1)) + (k & 1);
  }
  out[o] = Cx<R>{R(v.x), R(v.y)};
}

template <typename R>
fm_status run_typed(const FusedRun& run, hipStream_t s) {
  const fm_op_s* C = run.conv;
  const Split& sp = sizeof(R) == 4 ? C->s32 : C->s64;
  FArgs<R> fa{};
  fa.slot = static_cast<Cx<R>*>(run.slot);
  fa.spec = static_cast<const Cx<R>*>(sizeof(R) == 4 ? C->p32.p : C->p64.p);
  const Elem e = sizeof(R) == 4 ? Elem::C64 : Elem::C128;
  fa.tw = static_cast<const Cx<R>*>(twiddle_table(e, 20));
  FM_CHECK_ARG(fa.tw != nullptr, FM_E_DEVICE, "twiddle table unavailable: %s", last_error());
  fa.L = C->L;
  fa.logL = ilog2(C->L);
  fa.n2 = sp.four_step() ? sp.n2 : 1;
  if (sp.four_step()) {
    fa.twl = sp.mixed() ? static_cast<const Cx<R>*>(twiddle_table_L(e, C->L)) : fa.tw + C->L;
    FM_CHECK_ARG(fa.twl != nullptr, FM_E_DEVICE, "twiddle table unavailable: %s", last_error());
  }
  fa.b = static_cast<const Cx<R>*>(run.b);
  fa.ldb = run.ldb;
  fa.r = static_cast<Cx<R>*>(run.r);
  fa.ldr = run.m;
  fa.yv = static_cast<Cx<R>*>(run.y);
  fa.ldy = run.n;
  fa.x = static_cast<Cx<R>*>(run.x);
  fa.ldx = run.ldx;
  fa.lam = run.lam;
  fa.invL = run.invL;
  fa.active = run.active;
  fa.status = run.status;
  fa.pbase = run.pbase;
  fa.partial = run.partial;
  fa.beta = static_cast<const R*>(run.beta);
  fa.iter = run.iter;
  fa.momentum = run.momentum;
  fa.ncols = run.ncols;
  fa.check = fa.bump = 0;
  const int nslot = fused_nslot(FusedForm{C, run.sel_map, run.narrow}, e);
  fa.nslot = nslot;
  fa.stop_tol = run.stop_tol;
  fa.active_w = run.active;
  fa.iters = run.iters;
  fa.iter_w = run.iter;
  FArgs<R> aa = fa;
  // forward: C y (C's input rows n_C), r = S (C y) - b
  fa.in = fa.yv;
  fa.ldin = run.n;
  fa.adj = 0;
  fa.in_rows = int(C->n);
  fa.out_rows = int(C->m);
  fa.omap = run.sel_map;
  fa.imap = nullptr;
  // adjoint: C^H (S^H r), then the update
  aa.in = fa.r;
  aa.ldin = run.m;
  aa.adj = 1;
  aa.in_rows = int(C->m);
  aa.out_rows = int(C->n);
  aa.imap = run.sel_map;
  aa.omap = nullptr;
  if (run.narrow) {  // 1024-point rows: n2 = L / 1024, the spectrum in that split's order
    fa.n2 = aa.n2 = int(C->L >> 10);
    Cx<R>* ns = static_cast<Cx<R>*>(run.nspec);
    hipLaunchKernelGGL(narrow_spectrum_kernel<R>, dim3(unsigned(cdiv(C->L, 256))), dim3(256), 0, s, C->L,
                       static_cast<const Cx<double>*>(C->p64.p), ns);
    FM_LAUNCHED();
    fa.spec = aa.spec = ns;
  }
  const int fuse_max = 1 << conv_max_fuse();
  hipLaunchKernelGGL(ff_pbase_kernel, dim3(unsigned(cdiv(run.ncols, 256))), dim3(256), 0, s, run.ncols, nslot,
                     run.pbase);
  FM_LAUNCHED();
  if (run.max_iters <= 0) return FM_OK;
  if (run.narrow) return iterate<R, 10>(fa, aa, run, fuse_max, nslot, s);
  return iterate<R, 12>(fa, aa, run, fuse_max, nslot, s);
}

// The iterations: the chained form's first strided pass and first iteration
// directly, then chunks replayed from a graph, then the remainder directly.
template <typename R, int LOGW>
fm_status iterate(const FArgs<R>& fa, const FArgs<R>& aa, const FusedRun& run, int fuse_max, int nslot,
                  hipStream_t s) {
  const bool ch = LOGW != 12 || chained(fa, fuse_max);
  int k = 0;
  if (ch) {  // the first forward strided pass and the first iteration (no check before it)
    FM_TRY((launch_ff<R, FK_FS1, 0, false, false, LOGW>(dim3(unsigned(fa.n2), unsigned(fa.ncols)), fa, s)));
    FM_TRY((launch_iteration<R, LOGW>(fa, aa, run, fuse_max, nslot, true, s)));
    k = 1;
  }
  // `chunk` iterations captured once and replayed (0: direct launches)
  const int chunk = std::min(graph_chunk(), run.max_iters - k);
  hipGraphExec_t exec = nullptr;
  hipStream_t cs = chunk > 0 ? capture_stream() : nullptr;
  if (cs && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    fm_status st = FM_OK;
    for (int j = 0; j < chunk && st == FM_OK; ++j)
      st = launch_iteration<R, LOGW>(fa, aa, run, fuse_max, nslot, false, cs);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &g);
    if (st == FM_OK && ec == hipSuccess && g) {
      if (hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) != hipSuccess) exec = nullptr;
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
  }
  fm_status st = FM_OK;
  for (; exec && k + chunk <= run.max_iters && st == FM_OK; k += chunk) {
    if (hipGraphLaunch(exec, s) != hipSuccess) {
      set_error("hipGraphLaunch failed");
      st = FM_E_DEVICE;
    }
  }
  for (; k < run.max_iters && st == FM_OK; ++k) st = launch_iteration<R, LOGW>(fa, aa, run, fuse_max, nslot, false, s);
  if (ch && st == FM_OK) st = launch_stop_check(run, nslot, s);  // the last iteration's check
  if (exec) {
    (void)hipStreamSynchronize(s);  // the replays have finished before the graph goes
    (void)hipGraphExecDestroy(exec);
  }
  return st;
}

}  // namespace

// 1024-point rows for S C (FM_FISTA_NARROW=0: never).
bool narrow_enabled() {
  static const bool v = [] {
    const char* e = std::getenv("FM_FISTA_NARROW");
    return !(e && e[0] == '0');
  }();
  return v;
}

FusedForm fused_form(const fm_op_s* a, int64_t ncols) {
  FusedForm f;
  auto conv_ok = [](const fm_op_s* c) {
    if (c->kind != Kind::Circulant && c->kind != Kind::Toeplitz) return false;
    if (!c->terms.empty() || c->path.load() != 0 || c->L <= 0) return false;
    if (c->dt != FM_C64 && c->dt != FM_C128) return false;
    const Split& sp = c->dt == FM_C64 ? c->s32 : c->s64;
    if (!sp.four_step()) return c->L <= 4096;
    return sp.log1 == 12 && sp.n2 <= 32 && c->L == (int64_t(sp.n2) << 12);
  };
  if (a->path.load() != 0) return f;
  if (conv_ok(a)) {
    f.conv = a;
    return f;
  }
  if (a->kind == Kind::Product && a->terms.size() == 2) {
    const fm_op_s* S = a->terms[0];
    const fm_op_s* C = a->terms[1];
    if (S->kind == Kind::Select && S->path.load() == 0 && S->m > 0 && S->n == C->m && S->inv.p && conv_ok(C) &&
        S->dt == C->dt) {
      f.conv = C;
      f.sel_map = static_cast<const int*>(S->inv.p);
      // a separate power-of-two strided pass, few columns: 1024-point rows
      // (four times the work-groups per pass, one wave each)
      const Split& s32 = C->s32;
      const Split& s64 = C->s64;
      f.narrow = narrow_enabled() && ncols <= kNarrowMaxCols && C->p64.p && s64.four_step() && !s64.mixed() &&
                 s64.log1 == 12 && s32.log1 == 12 && s32.n2 == s64.n2 && s64.n2 >= 16 && C->L <= (int64_t(1) << 20);
    }
  }
  return f;
}

int fused_nslot(const FusedForm& f, Elem e) {
  if (f.narrow) return int(f.conv->L >> 10);
  const Split& sp = e == Elem::C64 ? f.conv->s32 : f.conv->s64;
  if (!sp.four_step()) return 1;
  return sp.mixed() ? mixed_tiles(sp.n2) : sp.n2;
}

fm_status fista_fused_run(const FusedRun& run, hipStream_t s) {
  if (run.ncols == 0) return FM_OK;
  if (run.e == Elem::C64) return run_typed<float>(run, s);
  return run_typed<double>(run, s);
}

hipStream_t solver_capture_stream() { return capture_stream(); }

// w = A^H (A v) for the power iteration on A = S C (complex128) through the
// solver's passes with 1024-point rows: the forward's last pass stores A v
// through the selection and runs the adjoint's first pass on the same
// values, and the adjoint's last pass stores w; both last passes use the
// residual store with b = 0 (a value minus 0 is the value exactly). Five
// launches instead of the executor's seven.
fm_status narrow_prepare(const NarrowForm& p, Elem e, hipStream_t s) {
  const fm_op_s* C = p.conv;
  const dim3 g(unsigned(cdiv(C->L, 256)));
  const Cx<double>* p64 = static_cast<const Cx<double>*>(C->p64.p);
  if (e == Elem::C64)
    hipLaunchKernelGGL(narrow_spectrum_kernel<float>, g, dim3(256), 0, s, C->L, p64, static_cast<Cx<float>*>(p.nspec));
  else
    hipLaunchKernelGGL(narrow_spectrum_kernel<double>, g, dim3(256), 0, s, C->L, p64,
                       static_cast<Cx<double>*>(p.nspec));
  FM_LAUNCHED();
  return launch_zero2d(e, std::max(p.m, p.n), 1, p.zeros, std::max(p.m, p.n), s);
}

namespace {
template <typename R>
fm_status narrow_args(const NarrowForm& p, int64_t ncols, FArgs<R>* a) {
  const fm_op_s* C = p.conv;
  FArgs<R> fa{};
  fa.slot = static_cast<Cx<R>*>(p.slot);
  fa.spec = static_cast<const Cx<R>*>(p.nspec);
  fa.tw = static_cast<const Cx<R>*>(twiddle_table(sizeof(R) == 4 ? Elem::C64 : Elem::C128, 20));
  FM_CHECK_ARG(fa.tw != nullptr, FM_E_DEVICE, "twiddle table unavailable: %s", last_error());
  fa.L = C->L;
  fa.logL = ilog2(C->L);
  fa.n2 = int(C->L >> 10);
  fa.twl = fa.tw + C->L;
  fa.b = static_cast<const Cx<R>*>(p.zeros);
  fa.ldb = 0;
  fa.ncols = ncols;
  fa.check = fa.bump = 0;
  *a = fa;
  return FM_OK;
}

}  // namespace

fm_status power_product(const NarrowForm& p, const void* v, void* av, void* w, hipStream_t s) {
  const fm_op_s* C = p.conv;
  FArgs<double> fa;
  FM_TRY(narrow_args<double>(p, 1, &fa));
  FArgs<double> aa = fa;
  fa.in = static_cast<const Cx<double>*>(v);
  fa.ldin = p.n;
  fa.adj = 0;
  fa.in_rows = int(C->n);
  fa.out_rows = int(C->m);
  fa.omap = p.sel_map;
  fa.r = static_cast<Cx<double>*>(av);
  fa.ldr = p.m;
  aa.in = static_cast<const Cx<double>*>(av);
  aa.ldin = p.m;
  aa.adj = 1;
  aa.in_rows = int(C->m);
  aa.out_rows = int(C->n);
  aa.imap = p.sel_map;
  aa.r = static_cast<Cx<double>*>(w);
  aa.ldr = p.n;
  const dim3 grid(unsigned(fa.n2), 1u);
  FM_TRY((launch_ff<double, FK_FS1, 0, false, false, 10>(grid, fa, s)));
  FM_TRY((launch_ff<double, FK_FS2, 0, false, false, 10>(grid, fa, s)));
  FM_TRY((launch_ff<double, FK_FS31, 1, false, true, 10>(grid, fa, s)));
  FM_TRY((launch_ff<double, FK_FS2, 0, false, false, 10>(grid, aa, s)));
  return launch_ff<double, FK_FS3, 1, false, false, 10>(grid, aa, s);
}
bool solver_graphs_enabled() { return graph_chunk() > 0; }

}  // namespace fm
