// The proximal-gradient solver (FISTA / ISTA, as in fm_fista) for every column
// of every operator of a batch at once. Each iteration is one batched forward
// launch sequence whose last pass stores r = A y - b, one batched adjoint
// sequence whose last pass applies the update (z = y - g/L, soft threshold,
// momentum) in place of storing g, and one stop check, all over the whole
// batch. A column that meets the stopping rule (or a non-finite value) is
// frozen: the epilogues leave it alone and the batched launches skip its work
// items, so finished problems stop costing time.
#include <cmath>
#include <cstring>
#include <vector>

#include "batch.h"
#include "solve.h"

namespace fm {
namespace {

constexpr int kTPB = 256;
constexpr int kTile = 1024;  // elements per update / residual tile

struct SCol {  // one batch column
  int32_t op, col;
  int32_t n, m;     // rows of x (and y, g) and of b (and r)
  int64_t yoff, roff;  // offsets into the packed y/g and r buffers
  int64_t pbase;    // first partial-sum slot of the column
  int32_t nslot;    // slots: 1, or the column-pass tiles of a four-step column (fs3_tiles)
};
struct STile {
  int32_t g;     // batch column
  int32_t tile;  // tile index inside the column
};

__global__ __launch_bounds__(256) void bstop_kernel(const SCol* cols, int64_t ncols, const double* partial,
                                                    double tol, int k, int* active, int* iters, const int* status,
                                                    int* iter) {
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi == 0) *iter = k + 1;  // the next iteration's momentum weight
  if (gi >= ncols || !active[gi]) return;
  if (status[gi]) {
    active[gi] = 0;
    iters[gi] = k + 1;
    return;
  }
  if (tol <= 0.0) return;
  const SCol c = cols[gi];
  double dx = 0.0, nx = 0.0;
  for (int t = 0; t < c.nslot; ++t) {
    dx += partial[2 * (c.pbase + t)];
    nx += partial[2 * (c.pbase + t) + 1];
  }
  const double nrm = sqrt(nx);
  if (sqrt(dx) <= tol * (nrm > 1e-30 ? nrm : 1e-30)) {
    active[gi] = 0;
    iters[gi] = k + 1;
  }
}

__global__ __launch_bounds__(kTPB) void bcolmax_kernel(const SCol* cols, const c64* g, double rel, double* lam) {
  __shared__ double sm[kTPB];
  const SCol c = cols[blockIdx.x];
  const c64* G = g + c.yoff;
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < c.n; i += kTPB) {
    const double v = sqrt(double(G[i].x) * G[i].x + double(G[i].y) * G[i].y);
    m = v > m ? v : m;
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = kTPB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] = sm[threadIdx.x] > sm[threadIdx.x + w] ? sm[threadIdx.x] : sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) lam[blockIdx.x] = rel * sm[0];
}

// x0 handling: y = x (warm start) or x = y = 0, per tile
__global__ __launch_bounds__(kTPB) void binit_kernel(const STile* tiles, const SCol* cols, const User* user, c64* y,
                                                     int warm) {
  const STile t = tiles[blockIdx.x];
  const SCol c = cols[t.g];
  const User u = user[c.op];
  c64* X = u.x + int64_t(c.col) * u.ldx;
  c64* Y = y + c.yoff;
  for (int k = threadIdx.x; k < kTile; k += kTPB) {
    const int64_t i = int64_t(t.tile) * kTile + k;
    if (i >= c.n) break;
    if (warm) {
      Y[i] = X[i];
    } else {
      X[i] = {0.f, 0.f};
      Y[i] = {0.f, 0.f};
    }
  }
}

// max_k |p_k|^2 * scale^2 of one spectrum (complex128), one work-group
__global__ __launch_bounds__(kTPB) void spec_bound_kernel(int64_t n, const c128* p, double scale, double* out) {
  __shared__ double sm[kTPB];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kTPB) {
    const double v = p[i].x * p[i].x + p[i].y * p[i].y;
    m = v > m ? v : m;
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = kTPB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] = sm[threadIdx.x] > sm[threadIdx.x + w] ? sm[threadIdx.x] : sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0] * scale * scale;
}

template <typename V>
__global__ __launch_bounds__(kTPB) void bfill_kernel(int64_t n, V* p, V v) {
  const int64_t i = int64_t(blockIdx.x) * kTPB + threadIdx.x;
  if (i < n) p[i] = v;
}

fm_status ensure_state(fm_batch_s* b) {
  if (b->s_cols.p) return FM_OK;
  const int nops = int(b->ops.size());
  std::vector<SCol> cols;
  std::vector<STile> ut;
  std::vector<int64_t> pbase;
  int64_t yo = 0, ro = 0, slots = 0;
  b->s_yoff.assign(nops, 0);
  b->s_roff.assign(nops, 0);
  for (int i = 0; i < nops; ++i) {
    const fm_op_s* o = b->ops[i];
    b->s_yoff[i] = yo;
    b->s_roff[i] = ro;
    const int32_t nslot = o->L > (int64_t(1) << kLog1) ? fs3_tiles(int32_t(o->L >> kLog1)) : 1;
    for (int64_t c = 0; c < b->ncols[i]; ++c) {
      SCol sc{i, int32_t(c), int32_t(o->n), int32_t(o->m), yo + c * o->n, ro + c * o->m, slots, nslot};
      const int32_t gidx = int32_t(cols.size());
      for (int t = 0; t < int(cdiv(o->n, kTile)); ++t) ut.push_back(STile{gidx, t});
      pbase.push_back(slots);
      slots += nslot;
      cols.push_back(sc);
    }
    yo += b->ncols[i] * o->n;
    ro += b->ncols[i] * o->m;
  }
  const int64_t G = int64_t(cols.size());
  FM_TRY(b->s_y.alloc(size_t(std::max<int64_t>(yo, 1)) * 8));
  FM_TRY(b->s_g.alloc(size_t(std::max<int64_t>(yo, 1)) * 8));
  FM_TRY(b->s_r.alloc(size_t(std::max<int64_t>(ro, 1)) * 8));
  FM_TRY(b->s_lam.alloc(size_t(std::max<int64_t>(G, 1)) * 8));
  FM_TRY(b->s_L.alloc(size_t(nops) * 8));
  FM_TRY(b->s_active.alloc(size_t(std::max<int64_t>(G, 1)) * 4));
  FM_TRY(b->s_status.alloc(size_t(std::max<int64_t>(G, 1)) * 4));
  FM_TRY(b->s_iters.alloc(size_t(std::max<int64_t>(G, 1)) * 4));
  FM_TRY(b->s_partial.alloc(size_t(std::max<int64_t>(slots, 1)) * 16));
  FM_TRY(b->s_pbase.alloc(size_t(std::max<int64_t>(G, 1)) * 8));
  FM_TRY(b->s_cols.alloc(std::max<size_t>(cols.size(), 1) * sizeof(SCol)));
  FM_TRY(b->s_utiles.alloc(std::max<size_t>(ut.size(), 1) * sizeof(STile)));
  FM_TRY(b->s_user.alloc(size_t(nops) * sizeof(User)));
  FM_TRY(b->s_iter.alloc(sizeof(int)));
  if (!cols.empty()) {
    FM_HIP(hipMemcpy(b->s_cols.p, cols.data(), cols.size() * sizeof(SCol), hipMemcpyHostToDevice));
    FM_HIP(hipMemcpy(b->s_pbase.p, pbase.data(), pbase.size() * 8, hipMemcpyHostToDevice));
  }
  if (!ut.empty()) FM_HIP(hipMemcpy(b->s_utiles.p, ut.data(), ut.size() * sizeof(STile), hipMemcpyHostToDevice));
  b->s_nutiles = int64_t(ut.size());
  return FM_OK;
}

}  // namespace
}  // namespace fm

using namespace fm;

extern "C" fm_status fm_batch_fista(fm_batch b, const void* const* bvec, const int64_t* ldb, void* const* x,
                                    const int64_t* ldx, const fm_fista_opts* o, fm_fista_stat* stats, void* stream) {
  set_error("");
  FM_CHECK_ARG(b != nullptr, FM_E_INVALID, "batch handle is NULL");
  FM_CHECK_ARG(batch_alive(b), FM_E_RELEASED, "batch handle was released");
  FM_CHECK_ARG(o != nullptr, FM_E_INVALID, "NULL options");
  FM_CHECK_ARG(bvec != nullptr && ldb != nullptr && x != nullptr && ldx != nullptr, FM_E_INVALID,
               "batch: NULL pointer array");
  FM_CHECK_ARG(o->max_iters >= 0, FM_E_INVALID, "max_iters must be non-negative");
  FM_CHECK_ARG(o->lambda_abs > 0.0 || o->lambda_rel > 0.0, FM_E_INVALID, "set lambda_abs > 0 or lambda_rel > 0");
  const int nops = int(b->ops.size());
  std::vector<User> user(nops);
  for (int i = 0; i < nops; ++i) {
    const fm_op_s* op = b->ops[i];
    if (b->ncols[i] > 0) {
      FM_CHECK_ARG(bvec[i] != nullptr && x[i] != nullptr, FM_E_INVALID, "batch: NULL block for operator %d", i);
      FM_CHECK_ARG(ldb[i] >= op->m && ldx[i] >= op->n, FM_E_SHAPE, "batch: leading dimension of operator %d", i);
    }
    user[i] = User{static_cast<const c64*>(bvec[i]), static_cast<c64*>(x[i]), ldb[i], ldx[i]};
  }
  int dev = 0;
  FM_HIP(hipGetDevice(&dev));
  FM_CHECK_ARG(dev == b->device, FM_E_DEVICE, "batch lives on device %d, current is %d", b->device, dev);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  FM_TRY(ensure_state(b));
  const int64_t G = b->total_cols;
  if (G == 0) return FM_OK;
  FM_HIP(hipMemcpyAsync(b->s_user.p, user.data(), size_t(nops) * sizeof(User), hipMemcpyHostToDevice, s));
  double* Ld = static_cast<double*>(b->s_L.p);
  std::vector<double> Lh(nops);
  if (o->L > 0.0) {
    for (int i = 0; i < nops; ++i) Lh[i] = o->L;
  } else {
    // per operator: max_k |DFT_L(g)_k|^2 of its cyclic embedding, >= ||A||_2^2
    if (b->s_bound.empty()) {
      DevBuf tmp;
      FM_TRY(tmp.alloc(size_t(nops) * 8));
      for (int i = 0; i < nops; ++i) {
        const fm_op_s* op = b->ops[i];
        hipLaunchKernelGGL(spec_bound_kernel, dim3(1), dim3(kTPB), 0, s, op->L, static_cast<const c128*>(op->p64.p),
                           double(op->L), static_cast<double*>(tmp.p) + i);
        FM_LAUNCHED();
      }
      b->s_bound.resize(nops);
      FM_HIP(hipMemcpyAsync(b->s_bound.data(), tmp.p, size_t(nops) * 8, hipMemcpyDeviceToHost, s));
      FM_HIP(hipStreamSynchronize(s));
    }
    Lh = b->s_bound;
  }
  FM_HIP(hipMemcpyAsync(Ld, Lh.data(), size_t(nops) * 8, hipMemcpyHostToDevice, s));
  c64* y = static_cast<c64*>(b->s_y.p);
  c64* r = static_cast<c64*>(b->s_r.p);
  c64* g = static_cast<c64*>(b->s_g.p);
  double* lam = static_cast<double*>(b->s_lam.p);
  int* active = static_cast<int*>(b->s_active.p);
  int* status = static_cast<int*>(b->s_status.p);
  int* iters = static_cast<int*>(b->s_iters.p);
  double* partial = static_cast<double*>(b->s_partial.p);
  const SCol* cols = static_cast<const SCol*>(b->s_cols.p);
  const STile* ut = static_cast<const STile*>(b->s_utiles.p);
  const User* ud = static_cast<const User*>(b->s_user.p);
  auto table = [&](bool adj_in, const c64* in_base, const std::vector<int64_t>& in_off, bool in_m, c64* out_base,
                   const std::vector<int64_t>& out_off, bool out_m, const Ptrs** t) -> fm_status {
    (void)adj_in;
    b->cur.resize(nops);
    for (int i = 0; i < nops; ++i) {
      const fm_op_s* op = b->ops[i];
      b->cur[i] = Ptrs{in_base + in_off[i], out_base + out_off[i], in_m ? op->m : op->n, out_m ? op->m : op->n};
    }
    return batch_pointer_table(b, s, t);
  };
  // regularisation weights
  if (o->lambda_abs > 0.0) {
    hipLaunchKernelGGL(bfill_kernel<double>, dim3(unsigned(cdiv(G, kTPB))), dim3(kTPB), 0, s, G, lam, o->lambda_abs);
    FM_LAUNCHED();
  } else {
    b->cur.resize(nops);
    for (int i = 0; i < nops; ++i)
      b->cur[i] = Ptrs{user[i].b, g + b->s_yoff[i], user[i].ldb, b->ops[i]->n};
    const Ptrs* t = nullptr;
    FM_TRY(batch_pointer_table(b, s, &t));
    FM_TRY(batch_launch(b, true, t, nullptr, s));
    hipLaunchKernelGGL(bcolmax_kernel, dim3(unsigned(G)), dim3(kTPB), 0, s, cols, g, o->lambda_rel, lam);
    FM_LAUNCHED();
  }
  // start
  if (b->s_nutiles > 0) {
    hipLaunchKernelGGL(binit_kernel, dim3(unsigned(b->s_nutiles)), dim3(kTPB), 0, s, ut, cols, ud, y, o->x0_given);
    FM_LAUNCHED();
  }
  hipLaunchKernelGGL(bfill_kernel<int>, dim3(unsigned(cdiv(G, kTPB))), dim3(kTPB), 0, s, G, active, 1);
  hipLaunchKernelGGL(bfill_kernel<int>, dim3(unsigned(cdiv(G, kTPB))), dim3(kTPB), 0, s, G, status, 0);
  hipLaunchKernelGGL(bfill_kernel<int>, dim3(unsigned(cdiv(G, kTPB))), dim3(kTPB), 0, s, G, iters, o->max_iters);
  FM_LAUNCHED();
  // forward: y -> r (the epilogue subtracts b); adjoint: r -> y (the epilogue
  // reads y_k at the output position and replaces it by y_{k+1})
  const Ptrs *tf = nullptr, *ta = nullptr;
  FM_TRY(table(false, y, b->s_yoff, false, r, b->s_roff, true, &tf));
  FM_TRY(table(true, r, b->s_roff, true, y, b->s_yoff, false, &ta));
  // momentum weights of every iteration, read on the device through the
  // iteration counter the stop check advances (so the launches of every
  // iteration are the same and replay from one captured graph per direction)
  {
    std::vector<float> betas(size_t(std::max(o->max_iters, 1)), 0.f);
    const std::vector<double> w = fista_momentum_weights(o->max_iters);
    for (int k = 0; k < o->max_iters; ++k) betas[size_t(k)] = float(w[size_t(k)]);
    if (b->s_beta.bytes < betas.size() * 4) {
      FM_HIP(hipStreamSynchronize(s));  // earlier work may still read the old array
      b->s_beta.reset();
      FM_TRY(b->s_beta.alloc(betas.size() * 4));
      drop_graphs(b);
    }
    FM_HIP(hipMemcpyAsync(b->s_beta.p, betas.data(), betas.size() * 4, hipMemcpyHostToDevice, s));
    FM_HIP(hipStreamSynchronize(s));  // betas is host memory of this call
  }
  int* iter_dev = static_cast<int*>(b->s_iter.p);
  hipLaunchKernelGGL(bfill_kernel<int>, dim3(1), dim3(kTPB), 0, s, int64_t(1), iter_dev, 0);
  FM_LAUNCHED();
  EpiArgs ef, ea;
  ef.kind = 1;
  ef.user = ud;
  ea.kind = 2;
  ea.user = ud;
  ea.lam = lam;
  ea.L = Ld;
  ea.pbase = static_cast<const int64_t*>(b->s_pbase.p);
  ea.partial = partial;
  ea.status = status;
  ea.momentum = o->momentum != 0;
  ea.beta = static_cast<const float*>(b->s_beta.p);
  ea.iter = iter_dev;
  for (int k = 0; k < o->max_iters; ++k) {
    FM_TRY(batch_launch(b, false, tf, active, s, &ef));  // r = A y - b
    FM_TRY(batch_launch(b, true, ta, active, s, &ea));   // x, y updated from A^H r
    hipLaunchKernelGGL(bstop_kernel, dim3(unsigned(cdiv(G, 256))), dim3(256), 0, s, cols, G, partial, o->stop_tol, k,
                       active, iters, status, iter_dev);
    FM_LAUNCHED();
  }
  if (stats) {
    std::vector<int> hi(G), hs(G);
    std::vector<double> hl(G);
    FM_HIP(hipMemcpyAsync(hi.data(), iters, size_t(G) * 4, hipMemcpyDeviceToHost, s));
    FM_HIP(hipMemcpyAsync(hs.data(), status, size_t(G) * 4, hipMemcpyDeviceToHost, s));
    FM_HIP(hipMemcpyAsync(hl.data(), lam, size_t(G) * 8, hipMemcpyDeviceToHost, s));
    FM_HIP(hipStreamSynchronize(s));
    int64_t gi = 0;
    for (int i = 0; i < nops; ++i)
      for (int64_t c = 0; c < b->ncols[i]; ++c, ++gi) stats[gi] = fm_fista_stat{hi[gi], hs[gi], Lh[i], hl[gi]};
  } else {
    FM_HIP(hipStreamSynchronize(s));  // the caller's arrays outlive no further use of user[]
  }
  return FM_OK;
}
