// Host driver of the proximal-gradient solver and of the FP64 power
// iteration. The solver is the iteration the paper states for eq. (8) (ISTA:
// a gradient step on 1/2||Ax - b||^2 followed by soft thresholding) in its
// accelerated form (FISTA, the variant the paper runs for its results), with
// the constant step 1/L, L >= ||A||_2^2. Every operator product goes through
// the operator executor; everything else runs in the kernels of solve.hip.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "runtime.h"
#include "solve.h"

using namespace fm;

namespace {

// Workspace layout of one solve (byte offsets), from one sizing pass.
struct FistaPlan {
  size_t r, g, y, lam, active, status, iters, partial, exec, total;
  size_t slot, pbase, beta, iter, nspec;  // fused solver only
  int64_t ntiles;
  int per_thread;
  FusedForm fused;
};

// FM_FISTA_FUSED=0 runs every operator through the general loop.
bool fused_enabled() {
  static const bool v = [] {
    const char* e = std::getenv("FM_FISTA_FUSED");
    return !(e && e[0] == '0');
  }();
  return v;
}

size_t up(size_t v) { return (v + 255) & ~size_t(255); }

fm_status plan_fista(const fm_op_s* a, int64_t ncols, int max_iters, FistaPlan* p) {
  const Elem e = elem_of(a->dt);
  const size_t es = elem_bytes(e);
  const int64_t m = a->m, n = a->n;
  p->fused = fused_enabled() ? fused_form(a, ncols) : FusedForm{};
  p->ntiles = update_tiles(n, &p->per_thread);
  size_t off = 0;
  p->r = off;
  off += up(size_t(m * ncols) * es);
  p->g = off;
  off += up(size_t(n * ncols) * es);
  p->y = off;
  off += up(size_t(n * ncols) * es);
  p->lam = off;
  off += up(size_t(ncols) * 8);
  p->active = off;
  off += up(size_t(ncols) * 4);
  p->status = off;
  off += up(size_t(ncols) * 4);
  p->iters = off;
  off += up(size_t(ncols) * 4);
  p->partial = off;
  int64_t nslot = p->ntiles;
  if (p->fused.conv) nslot = std::max<int64_t>(nslot, fused_nslot(p->fused, e));
  off += up(size_t(2 * nslot * ncols) * 8);
  p->slot = p->pbase = p->beta = p->iter = p->nspec = off;
  if (p->fused.conv) {
    p->slot = off;
    if (p->fused.conv->L > 4096) off += up(size_t(p->fused.conv->L * ncols) * es);
    p->pbase = off;
    off += up(size_t(ncols) * 8);
    p->beta = off;
    off += up(size_t(std::max(max_iters, 1)) * (es / 2));
    p->iter = off;
    off += up(4);
    p->nspec = off;
    if (p->fused.narrow) off += up(size_t(p->fused.conv->L) * es);
  }
  p->exec = off;
  size_t ex = 0;
  for (int adj = 0; adj < 2; ++adj) {
    Batch b{ncols, 1, 1, in_rows(a, adj), in_rows(a, adj), out_rows(a, adj), out_rows(a, adj)};
    Workspace ws;
    ws.sizing = true;
    FM_TRY(exec(a, adj != 0, e, b, nullptr, nullptr, false, ws, nullptr));
    ex = std::max(ex, ws.peak);
  }
  p->total = off + up(ex);
  return FM_OK;
}

// Power iteration in complex128 on A^H A; sizes of its buffers.
// Power iterations run in chunks of this many between host checks of the
// convergence test: each keeps its two norms in a device history, and the
// host applies the test to the history in order, so the estimate and the
// iteration count are those of a check after every iteration.
constexpr int kPowerChunk = 16;
static_assert(kPowerChunk % 2 == 0, "a captured chunk leaves v and w in place");

struct PowerPlan {
  size_t v, av, w, partial, scal, slot, nspec, zeros, exec, total;
  int nparts;
  FusedForm fused;  // narrow: the products run through the solver's passes
};

fm_status plan_power(const fm_op_s* a, PowerPlan* p) {
  const int64_t m = a->m, n = a->n;
  p->nparts = 256;
  size_t off = 0;
  p->v = off;
  off += up(size_t(n) * 16);
  p->av = off;
  off += up(size_t(m) * 16);
  p->w = off;
  off += up(size_t(n) * 16);
  p->partial = off;
  off += up(size_t(2 * p->nparts) * 8);  // partial sums of ||w||^2, then of ||A v||^2
  p->scal = off;
  off += up(size_t(2 * kPowerChunk + 2) * 8);
  p->fused = fused_enabled() ? fused_form(a, 1) : FusedForm{};
  p->slot = p->nspec = p->zeros = off;
  if (p->fused.narrow) {
    p->slot = off;
    off += up(size_t(p->fused.conv->L) * 16);
    p->nspec = off;
    off += up(size_t(p->fused.conv->L) * 16);
    p->zeros = off;
    off += up(size_t(std::max(m, n)) * 16);
  }
  p->exec = off;
  size_t ex = 0;
  for (int adj = 0; adj < 2; ++adj) {
    Batch b{1, 1, 1, in_rows(a, adj), in_rows(a, adj), out_rows(a, adj), out_rows(a, adj)};
    Workspace ws;
    ws.sizing = true;
    FM_TRY(exec(a, adj != 0, Elem::C128, b, nullptr, nullptr, false, ws, nullptr));
    ex = std::max(ex, ws.peak);
  }
  p->total = off + up(ex);
  return FM_OK;
}

fm_status power_iteration(const fm_op_s* a, const void* v0, uint64_t seed, int max_iters, double tol, double* L_out,
                          int* iters_out, hipStream_t s) {
  PowerPlan p;
  FM_TRY(plan_power(a, &p));
  void* base = nullptr;
  FM_HIP(hipMallocAsync(&base, p.total, s));
  char* B = static_cast<char*>(base);
  auto cleanup = [&]() { (void)hipFreeAsync(base, s); };
  c128* v = reinterpret_cast<c128*>(B + p.v);
  c128* av = reinterpret_cast<c128*>(B + p.av);
  c128* w = reinterpret_cast<c128*>(B + p.w);
  double* partial = reinterpret_cast<double*>(B + p.partial);
  double* scal = reinterpret_cast<double*>(B + p.scal);
  const int64_t n = a->n, m = a->m;
  fm_status st = FM_OK;
  hipGraphExec_t gexec = nullptr;  // one chunk of iterations, captured once
  bool captured = false;
  auto run = [&]() -> fm_status {
    if (v0)
      FM_HIP(hipMemcpyAsync(v, v0, size_t(n) * 16, hipMemcpyDeviceToDevice, s));
    else
      FM_TRY(launch_start_vector(n, seed, v, s));
    FM_TRY(launch_norm2(n, v, partial, p.nparts, scal, s));
    FM_TRY(launch_normalize(n, v, scal, s));
    Workspace ws;
    ws.base = B + p.exec;
    ws.cap = p.total - p.exec;
    const Batch bf{1, 1, 1, n, n, m, m}, ba{1, 1, 1, m, m, n, n};
    double prev = 0.0, lk = 0.0;
    int it = 0;  // iterations whose test has been applied
    bool done = false;
    const NarrowForm pf{p.fused.conv, p.fused.sel_map, m, n, B + p.slot, B + p.nspec, B + p.zeros};
    if (p.fused.narrow) FM_TRY(narrow_prepare(pf, Elem::C128, s));
    // iteration j of a chunk: ||A v||^2 -> scal[2j], ||A^H A v|| -> scal[2j+1]
    auto launch_chunk = [&](int chunk, hipStream_t q) -> fm_status {
      for (int j = 0; j < chunk; ++j) {
        double* part_w = partial;
        double* part_a = partial + p.nparts;
        if (p.fused.narrow) {
          FM_TRY(power_product(pf, v, av, w, q));
          FM_TRY(launch_norm2_partial(m, av, part_a, p.nparts, q));
        } else {
          FM_TRY(exec(a, false, Elem::C128, bf, v, av, false, ws, q));
          FM_TRY(launch_norm2_partial(m, av, part_a, p.nparts, q));
          FM_TRY(exec(a, true, Elem::C128, ba, av, w, false, ws, q));
        }
        FM_TRY(launch_norm2_partial(n, w, part_w, p.nparts, q));
        // both final sums and w / ||w|| in one launch (iterates past a stop are discarded)
        FM_TRY(launch_normalize_final(n, w, p.nparts, part_w, part_a, scal + 2 * j + 1, scal + 2 * j, q));
        std::swap(v, w);
      }
      return FM_OK;
    };
    while (!done && it < max_iters) {
      const int chunk = std::min(kPowerChunk, max_iters - it);
      // full chunks after the first (which has set up whatever the launches
      // create on first use) replay one captured graph: a chunk has an even
      // number of iterations, so v and w are back in place at its end
      if (it > 0 && chunk == kPowerChunk && !captured && solver_graphs_enabled()) {
        captured = true;
        hipStream_t cs = solver_capture_stream();
        if (cs && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
          c128* const v_at = v;
          c128* const w_at = w;
          const size_t ws_at = ws.mark();
          const fm_status sc = launch_chunk(chunk, cs);
          v = v_at;  // also where the capture stopped part way
          w = w_at;
          ws.release(ws_at);
          hipGraph_t g = nullptr;
          const hipError_t ec = hipStreamEndCapture(cs, &g);
          if (sc == FM_OK && ec == hipSuccess && g &&
              hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0) != hipSuccess)
            gexec = nullptr;
          if (g) (void)hipGraphDestroy(g);
          (void)hipGetLastError();
        }
      }
      if (it > 0 && chunk == kPowerChunk && gexec) {
        FM_HIP(hipGraphLaunch(gexec, s));
      } else {
        FM_TRY(launch_chunk(chunk, s));
      }
      double h[2 * kPowerChunk];
      FM_HIP(hipMemcpyAsync(h, scal, size_t(2 * chunk) * 8, hipMemcpyDeviceToHost, s));
      FM_HIP(hipStreamSynchronize(s));
      for (int j = 0; j < chunk && !done; ++j) {
        ++it;
        lk = h[2 * j];
        if (h[2 * j + 1] == 0.0) {
          lk = 0.0;
          done = true;
        } else if (it > 1 && std::fabs(lk - prev) <= tol * lk) {
          done = true;
        }
        prev = lk;
      }
    }
    *L_out = lk;
    if (iters_out) *iters_out = it;
    return FM_OK;
  };
  st = run();
  if (gexec) {
    (void)hipStreamSynchronize(s);  // the replays have finished before the graph goes
    (void)hipGraphExecDestroy(gexec);
  }
  cleanup();
  if (st == FM_OK) FM_HIP(hipStreamSynchronize(s));
  return st;
}

}  // namespace

extern "C" {

fm_status fm_power_iteration(fm_op a, const void* v0, uint64_t seed, int32_t max_iters, double tol, double* L_out,
                             int32_t* iters_out, void* stream) {
  set_error("");
  FM_CHECK_ARG(a != nullptr, FM_E_INVALID, "operator handle is NULL");
  FM_CHECK_ARG(op_alive(a), FM_E_RELEASED, "operator handle was released");
  FM_CHECK_ARG(is_complex(a->dt), FM_E_DTYPE, "power iteration needs a complex operator");
  FM_CHECK_ARG(L_out != nullptr, FM_E_INVALID, "NULL output");
  FM_CHECK_ARG(max_iters >= 1, FM_E_INVALID, "max_iters must be positive");
  FM_CHECK_ARG(tol >= 0.0, FM_E_INVALID, "tol must be non-negative");
  int it = 0;
  FM_TRY(power_iteration(a, v0, seed, max_iters, tol, L_out, &it, reinterpret_cast<hipStream_t>(stream)));
  if (iters_out) *iters_out = it;
  return FM_OK;
}

fm_status fm_fista_workspace_size(fm_op a, int64_t ncols, const fm_fista_opts* opts, size_t* bytes) {
  set_error("");
  FM_CHECK_ARG(a != nullptr, FM_E_INVALID, "operator handle is NULL");
  FM_CHECK_ARG(op_alive(a), FM_E_RELEASED, "operator handle was released");
  FM_CHECK_ARG(bytes != nullptr && opts != nullptr, FM_E_INVALID, "NULL argument");
  FM_CHECK_ARG(ncols >= 0, FM_E_INVALID, "negative column count");
  FistaPlan p;
  FM_TRY(plan_fista(a, ncols, opts->max_iters, &p));
  *bytes = p.total;
  return FM_OK;
}

fm_status fm_fista(fm_op a, int64_t ncols, const void* b, int64_t ldb, void* x, int64_t ldx,
                   const fm_fista_opts* o, fm_fista_stat* stats, void* ws, size_t ws_bytes, void* stream) {
  set_error("");
  FM_CHECK_ARG(a != nullptr, FM_E_INVALID, "operator handle is NULL");
  FM_CHECK_ARG(op_alive(a), FM_E_RELEASED, "operator handle was released");
  FM_CHECK_ARG(o != nullptr, FM_E_INVALID, "NULL options");
  FM_CHECK_ARG(is_complex(a->dt), FM_E_DTYPE, "the solver needs a complex operator");
  FM_CHECK_ARG(ncols >= 0, FM_E_INVALID, "negative column count");
  FM_CHECK_ARG(o->max_iters >= 0, FM_E_INVALID, "max_iters must be non-negative");
  FM_CHECK_ARG(o->lambda_abs > 0.0 || o->lambda_rel > 0.0, FM_E_INVALID,
               "set lambda_abs > 0 or lambda_rel > 0");
  FM_CHECK_ARG(ncols < 65536, FM_E_UNSUPPORTED, "at most 65535 columns per call");
  if (ncols == 0) return FM_OK;
  const int64_t m = a->m, n = a->n;
  FM_CHECK_ARG(b != nullptr && x != nullptr, FM_E_INVALID, "NULL data pointer");
  FM_CHECK_ARG(ldb >= m && ldx >= n, FM_E_SHAPE, "leading dimensions too small");
  int dev = 0;
  FM_HIP(hipGetDevice(&dev));
  FM_CHECK_ARG(dev == a->device, FM_E_DEVICE, "operator lives on device %d, current is %d", a->device, dev);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const Elem e = elem_of(a->dt);
  // step constant
  double L = o->L;
  if (!(L > 0.0)) {
    const int pit = o->power_max_iters > 0 ? o->power_max_iters : 500;
    const double ptol = o->power_tol > 0.0 ? o->power_tol : 1e-13;
    FM_TRY(power_iteration(a, nullptr, o->seed, pit, ptol, &L, nullptr, s));
    FM_CHECK_ARG(L > 0.0, FM_E_INVALID, "the operator is zero (power iteration gave L = 0)");
  }
  FistaPlan p;
  FM_TRY(plan_fista(a, ncols, o->max_iters, &p));
  void* base = ws;
  bool own = false;
  if (ws == nullptr && ws_bytes == 0) {
    FM_HIP(hipMallocAsync(&base, p.total, s));
    own = true;
  } else {
    FM_CHECK_ARG(ws != nullptr && ws_bytes >= p.total, FM_E_WORKSPACE, "workspace of %zu bytes given, %zu needed",
                 ws_bytes, p.total);
  }
  char* B = static_cast<char*>(base);
  void* r = B + p.r;
  void* g = B + p.g;
  void* y = B + p.y;
  double* lam = reinterpret_cast<double*>(B + p.lam);
  int* active = reinterpret_cast<int*>(B + p.active);
  int* status = reinterpret_cast<int*>(B + p.status);
  int* iters = reinterpret_cast<int*>(B + p.iters);
  double* partial = o->stop_tol > 0.0 ? reinterpret_cast<double*>(B + p.partial) : nullptr;
  Workspace w;
  w.base = B + p.exec;
  w.cap = p.total - p.exec;
  const Batch bf{ncols, 1, 1, n, n, m, m}, ba{ncols, 1, 1, m, m, n, n};
  auto body = [&]() -> fm_status {
    // regularisation weight per column
    if (o->lambda_abs > 0.0) {
      FM_TRY(launch_fill_double(ncols, lam, o->lambda_abs, s));
    } else {
      const Batch bb{ncols, 1, 1, ldb, m, n, n};
      FM_TRY(exec(a, true, e, bb, b, g, false, w, s));
      FM_TRY(launch_colmax(e, n, ncols, g, n, o->lambda_rel, lam, s));
    }
    // start
    if (o->x0_given) {
      FM_TRY(launch_copy2d(e, n, ncols, x, ldx, y, n, s));
    } else {
      FM_TRY(launch_zero2d(e, n, ncols, x, ldx, s));
      FM_TRY(launch_zero2d(e, n, ncols, y, n, s));
    }
    FM_TRY(launch_fill_int(ncols, active, 1, s));
    FM_TRY(launch_fill_int(ncols, status, 0, s));
    FM_TRY(launch_fill_int(ncols, iters, o->max_iters, s));
    if (p.fused.conv) {
      // the fused iteration: the convolution's passes with the residual and
      // the update in their last passes, replayed from a captured graph
      const std::vector<double> w = fista_momentum_weights(o->max_iters);
      std::vector<float> w32(w.size());
      for (size_t k = 0; k < w.size(); ++k) w32[k] = float(w[k]);
      if (!w.empty()) {
        const void* src = e == Elem::C64 ? static_cast<const void*>(w32.data()) : static_cast<const void*>(w.data());
        FM_HIP(hipMemcpyAsync(B + p.beta, src, w.size() * (e == Elem::C64 ? 4 : 8), hipMemcpyHostToDevice, s));
        FM_HIP(hipStreamSynchronize(s));  // the host vector is freed on return
      }
      FM_TRY(launch_fill_int(1, reinterpret_cast<int*>(B + p.iter), 0, s));
      FusedRun run{};
      run.e = e;
      run.conv = p.fused.conv;
      run.sel_map = p.fused.sel_map;
      run.narrow = p.fused.narrow;
      run.nspec = B + p.nspec;
      run.ncols = ncols;
      run.m = m;
      run.n = n;
      run.b = b;
      run.ldb = ldb;
      run.x = x;
      run.ldx = ldx;
      run.r = r;
      run.y = y;
      run.slot = B + p.slot;
      run.invL = 1.0 / L;
      run.lam = lam;
      run.active = active;
      run.status = status;
      run.iters = iters;
      run.partial = reinterpret_cast<double*>(B + p.partial);
      run.pbase = reinterpret_cast<int64_t*>(B + p.pbase);
      run.beta = B + p.beta;
      run.iter = reinterpret_cast<int*>(B + p.iter);
      run.momentum = o->momentum != 0;
      run.max_iters = o->max_iters;
      run.stop_tol = o->stop_tol;
      FM_TRY(fista_fused_run(run, s));
    }
    const std::vector<double> betas = fista_momentum_weights(o->max_iters);
    for (int k = 0; !p.fused.conv && k < o->max_iters; ++k) {
      const double beta = betas[size_t(k)];
      FM_TRY(exec(a, false, e, bf, y, r, false, w, s));             // r = A y
      FM_TRY(launch_sub(e, m, ncols, b, ldb, r, m, active, s));     // r = A y - b
      FM_TRY(exec(a, true, e, ba, r, g, false, w, s));              // g = A^H r
      UpdateArgs ua{};
      ua.x = x;
      ua.y = y;
      ua.g = g;
      ua.ldx = ldx;
      ua.ldy = n;
      ua.ldg = n;
      ua.rows = n;
      ua.invL = 1.0 / L;
      ua.lam = lam;
      ua.beta = beta;
      ua.momentum = o->momentum != 0;
      ua.active = active;
      ua.status = status;
      ua.partial = partial;
      ua.ntiles = p.ntiles;
      ua.per_thread = p.per_thread;
      FM_TRY(launch_update(e, ua, ncols, s));
      FM_TRY(launch_stop(partial, p.ntiles, ncols, o->stop_tol, k, active, iters, status, s));
    }
    if (stats) {
      std::vector<int> hi(ncols), hs(ncols);
      std::vector<double> hl(ncols);
      FM_HIP(hipMemcpyAsync(hi.data(), iters, size_t(ncols) * 4, hipMemcpyDeviceToHost, s));
      FM_HIP(hipMemcpyAsync(hs.data(), status, size_t(ncols) * 4, hipMemcpyDeviceToHost, s));
      FM_HIP(hipMemcpyAsync(hl.data(), lam, size_t(ncols) * 8, hipMemcpyDeviceToHost, s));
      FM_HIP(hipStreamSynchronize(s));
      for (int64_t j = 0; j < ncols; ++j) stats[j] = fm_fista_stat{hi[j], hs[j], L, hl[j]};
    }
    return FM_OK;
  };
  fm_status st = body();
  if (own) (void)hipFreeAsync(base, s);
  return st;
}

}  // extern "C"
