// Store epilogues of the proximal-gradient solver (eq. (8): ISTA and its
// accelerated form FISTA), shared by the batched stage kernel and the fused
// per-operator solver, so that both take the same arithmetic on the same
// values:
//   residual (forward's last pass):  r = A y - b, b subtracted in the store;
//                                    with a row selection S on the output,
//                                    position p of the convolution goes to
//                                    r[omap[p]] (omap[p] < 0: not selected)
//   update (adjoint's last pass):    from g = A^H r: z = y - g/L,
//                                    x+ = soft(z, lam/L), y+ = x+ + beta (x+ - x),
//                                    x and y replaced in place, partial sums of
//                                    |x+ - x|^2 and |x+|^2 per slot for the
//                                    stopping rule, a status flag on a
//                                    non-finite value.
// An epilogue receives every result of run_job / mixed_tile in two rounds
// (pre: operand loads, put: arithmetic and stores); see xform.h.
#pragma once

#include "xform.h"

namespace fm {
namespace xf {

// Complex soft threshold: shrinks the modulus by s, keeps the phase; |z| <= s
// gives exactly 0.
template <typename R>
__device__ __forceinline__ Cx<R> soft_thr(Cx<R> z, R s) {
  const R mag = sqrt(z.x * z.x + z.y * z.y);
  if (!(mag > s)) return {R(0), R(0)};
  const R f = (mag - s) / mag;
  return {z.x * f, z.y * f};
}

// r = A y - b. Without a map: transform b of the item is column col0 + b
// (contiguous items, bstride = ldb) or every transform belongs to one column
// (strided items, bstride = 0; e then holds the transform's offset), and r is
// the store destination. With a map (MAP): position e of the column goes to
// Rr[omap[e]], with b read at the same index; unselected positions are not
// stored.
// CAP: the epilogue also keeps, per register index k, the value the adjoint
// reads at the same position through the selection (r where selected, 0
// elsewhere and at positions that are not stored), for a pass that continues
// from registers.
template <typename R, bool MAP = false, bool CAP = false>
struct ResidualEpT {
  static constexpr bool kOn = true;
  const Cx<R>* B;
  int64_t bstride;
  Cx<R>* Rr = nullptr;         // MAP: residual column base
  const int* omap = nullptr;   // MAP: position -> selected row, or -1
  int64_t rstride = 0;         // MAP: element offset between the residual columns of a contiguous item
  Cx<R> bv[16];
  int mk[MAP ? 16 : 1];
  Cx<R> cap[CAP ? 16 : 1] = {};
  __device__ __forceinline__ void pre(int k, int b, int e, Cx<R>*) {
    if constexpr (MAP) {
      const int m = omap[e];
      mk[k] = m;
      bv[k] = m >= 0 ? B[int64_t(b) * bstride + m] : Cx<R>{R(0), R(0)};
    } else {
      bv[k] = B[int64_t(b) * bstride + e];
    }
  }
  __device__ __forceinline__ void put(int k, int, int b, int, Cx<R>* dst, Cx<R> v) {
    const Cx<R> r = csub(v, bv[k]);
    if constexpr (MAP) {
      if (mk[k] >= 0) Rr[int64_t(b) * rstride + mk[k]] = r;
      if constexpr (CAP) cap[k] = mk[k] >= 0 ? r : Cx<R>{R(0), R(0)};
    } else {
      *dst = r;
      if constexpr (CAP) cap[k] = r;
    }
  }
};

// FISTA update from g = A^H r. Contiguous items: transform b is column
// gcol0 + b with x at X + b*xstride; strided items: one column. CAP: the
// epilogue also keeps, per register index k, the new y (the old one for a
// frozen column; 0 at positions that are not stored), the next forward
// pass's input at the same positions.
template <typename R, bool CAP = false>
struct FistaEpT {
  static constexpr bool kOn = true;
  Cx<R>* X;
  int64_t xstride;
  int64_t gcol0;
  int colstride;  // 1: contiguous, 0: strided
  const int* active;
  const double* lam;
  double invLd;
  R invL, beta;
  int momentum;
  int* status;
  // running sums of the current slot (tiny contiguous transforms flush when
  // the slot changes: one thread holds the whole transform)
  bool flush_per_slot;
  const int64_t* pbase;
  double* partial;
  int cur = -1;
  int64_t cur_col = -1;
  int64_t c_gc = -1;
  bool c_act = false;
  R c_s = R(0);
  double dx = 0.0, nx = 0.0;

  __device__ __forceinline__ void flush() {
    if (cur_col >= 0) {
      partial[2 * pbase[cur_col]] = dx;
      partial[2 * pbase[cur_col] + 1] = nx;
    }
    dx = nx = 0.0;
    cur_col = -1;
  }
  Cx<R> yk[16], xk[16];
  Cx<R> cap[CAP ? 16 : 1] = {};
  __device__ __forceinline__ void pre(int k, int b, int e, Cx<R>* dst) {
    yk[k] = *dst;
    xk[k] = X[int64_t(b) * xstride + e];
  }
  __device__ __forceinline__ void put(int k, int slot, int b, int e, Cx<R>* dst, Cx<R> g) {
    const int64_t gc = gcol0 + int64_t(b) * colstride;
    if (flush_per_slot && slot != cur) {
      flush();
      cur = slot;
    }
    if (gc != c_gc) {  // per-column values, reloaded only when the column changes
      c_gc = gc;
      c_act = !active || active[gc];
      c_s = R(lam[gc] * invLd);
    }
    if (!c_act) {
      if constexpr (CAP) cap[k] = yk[k];
      return;
    }
    if (flush_per_slot) cur_col = gc;
    const R s = c_s;
    const Cx<R> yv = yk[k];
    Cx<R>* xp = X + int64_t(b) * xstride + e;
    const Cx<R> xo = xk[k];
    const Cx<R> z = {yv.x - g.x * invL, yv.y - g.y * invL};
    const Cx<R> xn = soft_thr(z, s);
    const Cx<R> d = {xn.x - xo.x, xn.y - xo.y};
    *xp = xn;
    const Cx<R> yn = momentum ? Cx<R>{xn.x + beta * d.x, xn.y + beta * d.y} : xn;
    *dst = yn;
    if constexpr (CAP) cap[k] = yn;
    dx += double(d.x) * d.x + double(d.y) * d.y;
    nx += double(xn.x) * xn.x + double(xn.y) * xn.y;
    if (!(isfinite(z.x) && isfinite(z.y))) atomicOr(status + gc, 1);
  }
};

// Partial sums of a FistaEpT after run_job: per transform (contiguous items
// of >= 16 points: the T = 2^(lg-4) threads of transform b are tid / T == b),
// per item (strided items: one column, slot pbase + tile), or already flushed
// (contiguous transforms of < 16 points). kThreads: the work-group size.
template <int kThreads, typename R, bool CAP>
__device__ __forceinline__ void fista_partials(FistaEpT<R, CAP>& ep, bool strided, int lg, int nvalid, int tile,
                                               void* smem) {
  if (ep.flush_per_slot) {
    ep.flush();
    return;
  }
  __syncthreads();  // the transform's last LDS reads are done
  double2* red = reinterpret_cast<double2*>(smem);
  const int tid = threadIdx.x;
  red[tid] = make_double2(ep.dx, ep.nx);
  __syncthreads();
  // tree reduction over segments of T threads (the whole work-group for a
  // strided item), in a fixed order
  const int T = strided ? kThreads : 1 << (lg - 4);
  for (int w = T >> 1; w > 0; w >>= 1) {
    if ((tid & (T - 1)) < w) {
      red[tid].x += red[tid + w].x;
      red[tid].y += red[tid + w].y;
    }
    __syncthreads();
  }
  if ((tid & (T - 1)) != 0) return;
  if (strided) {
    if (!ep.active || ep.active[ep.gcol0]) {
      ep.partial[2 * (ep.pbase[ep.gcol0] + tile)] = red[0].x;
      ep.partial[2 * (ep.pbase[ep.gcol0] + tile) + 1] = red[0].y;
    }
    return;
  }
  const int b = tid / T;
  if (b < nvalid) {
    const int64_t gc = ep.gcol0 + b;
    if (!ep.active || ep.active[gc]) {
      ep.partial[2 * ep.pbase[gc]] = red[tid].x;
      ep.partial[2 * ep.pbase[gc] + 1] = red[tid].y;
    }
  }
}

}  // namespace xf
}  // namespace fm
