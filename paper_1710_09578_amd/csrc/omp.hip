// Orthogonal matching pursuit: the greedy sparse-recovery method the paper
// runs beside FISTA on the ultrasound model (section "Application to
// Ultrasonic Nondestructive Testing"; OMP after Tropp and Gilbert), built
// on the operator's transforms.
//
// Per column b (each column is one problem), k steps of
//   c = A^H r                        (one backward transform of the block)
//   j = argmax over unchosen i of |c_i|, first index on ties
//   a = A e_j                        (read from the stored generator for A = C or
//                                     S C, C a circulant or Toeplitz; otherwise one
//                                     forward transform of a one-hot block)
//   orthogonalise a against the basis Q of the chosen columns (classical
//   Gram-Schmidt, applied twice), append q = a'/||a'|| to Q and the
//   coefficients to the triangular factor R (A_S = Q R)
//   z_k = q^H r, r <- r - z_k q      (r = b - Q Q^H b stays orthogonal to Q)
// then x_S = R^{-1} z by back substitution, scattered into x. A column stops
// early when ||r|| <= tol ||b||, or when the chosen column depends on the
// earlier ones (status 2), or on a non-finite value (status 1).
//
// All columns advance together: the transforms run on the whole block, the
// selection, orthogonalisation and final solve take one work-group per column.
#include <algorithm>
#include <cmath>
#include <vector>

#include "runtime.h"
#include "solve.h"

namespace fm {
namespace {

size_t up(size_t v) { return (v + 255) & ~size_t(255); }

template <typename R>
__device__ __forceinline__ R wave_sum(R v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Sums G complex values over the work-group (NT threads); every thread gets
// the totals. red: LDS of 2 * G * (NT / 64) reals.
template <typename R, int G, int NT>
__device__ __forceinline__ void block_sum(Cx<R>* v, R* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = NT / 64;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const R sx = wave_sum(v[g].x), sy = wave_sum(v[g].y);
    if (lane == 0) {
      red[(2 * g) * NW + wave] = sx;
      red[(2 * g + 1) * NW + wave] = sy;
    }
  }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < G; ++g) {
    R sx = R(0), sy = R(0);
#pragma unroll 4
    for (int w = 0; w < NW; ++w) {
      sx += red[(2 * g) * NW + w];
      sy += red[(2 * g + 1) * NW + w];
    }
    v[g] = {sx, sy};
  }
  __syncthreads();
}

struct OmpState {
  int64_t m, n, k;       // rows, columns, atom budget
  const void* b;         // caller's right-hand sides (ldb)
  int64_t ldb;
  void* r;               // residuals, ncols x m
  void* c;               // correlations, ncols x n
  void* e;               // one-hot block, ncols x n
  void* acol;            // chosen columns A e_j, ncols x m
  void* q;               // orthonormal bases, ncols x k x m
  void* rf;              // triangular factors, ncols x k x k (column-major per column)
  void* z;               // Q^H b, ncols x k
  int* idx;              // chosen atoms, ncols x k (-1: unused)
  unsigned char* sel;    // chosen flags, ncols x n
  double* bnorm2;        // ||b||^2 per column
  double* rnorm2;        // ||r||^2 per column
  int* active;
  int* nsel;
  int* status;
  double tol2;
  // split Gram-Schmidt step (P > 1 work-groups per column, `chunk` rows each):
  // part: per column and work-group, k + 4 partial sums (projections, then
  // ||a||^2, ||a'||^2, q^H r, ||r'||^2); hbuf: the projections of a pass
  void* part;
  void* hbuf;
  int P;
  int64_t chunk;
  // split argmax (SP > 1 work-groups per column, schunk indices each): per
  // column and work-group the largest |c_i|^2 and its index
  double* sbest;
  int64_t* sidx;
  int SP;
  int64_t schunk;
};

template <typename R>
__global__ __launch_bounds__(256) void omp_init_kernel(OmpState s) {
  __shared__ R red[2 * 4];
  const int64_t col = blockIdx.x;
  const Cx<R>* B = static_cast<const Cx<R>*>(s.b) + col * s.ldb;
  Cx<R>* r = static_cast<Cx<R>*>(s.r) + col * s.m;
  Cx<R>* e = static_cast<Cx<R>*>(s.e) + col * s.n;
  Cx<R> acc[1] = {{R(0), R(0)}};
  for (int64_t t = threadIdx.x; t < s.m; t += 256) {
    const Cx<R> v = B[t];
    r[t] = v;
    acc[0].x += v.x * v.x + v.y * v.y;
  }
  for (int64_t t = threadIdx.x; t < s.n; t += 256) {
    e[t] = {R(0), R(0)};
    s.sel[col * s.n + t] = 0;
  }
  for (int64_t t = threadIdx.x; t < s.k; t += 256) s.idx[col * s.k + t] = -1;
  block_sum<R, 1, 256>(acc, red);
  if (threadIdx.x == 0) {
    s.bnorm2[col] = double(acc[0].x);
    s.rnorm2[col] = double(acc[0].x);
    s.nsel[col] = 0;
    s.status[col] = 0;
    s.active[col] = acc[0].x > R(0) && s.tol2 < 1.0 ? 1 : 0;
  }
}

// Largest |c_i|^2 over the unchosen i in [lo, hi) of one column and its index
// (first index on ties; -1 when every value there is chosen or NaN), by the
// whole work-group; the result is valid in thread 0.
template <typename R, int NT>
__device__ __forceinline__ void argmax_range(const Cx<R>* c, const unsigned char* sel, int64_t lo, int64_t hi,
                                             R* bv, int64_t* bi, R* best_out, int64_t* idx_out) {
  R best = R(-1);
  int64_t bj = -1;
  // strided order, 4 loads in flight: the first maximum of this thread wins
  constexpr int U = 4;
  int64_t j0 = lo + threadIdx.x;
  for (; j0 + (U - 1) * NT < hi; j0 += U * NT) {
    Cx<R> v[U];
    unsigned char sl[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u] = c[j0 + u * NT];
      sl[u] = sel[j0 + u * NT];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const R mag = v[u].x * v[u].x + v[u].y * v[u].y;
      if (!sl[u] && mag > best) {
        best = mag;
        bj = j0 + u * NT;
      }
    }
  }
  for (int64_t j = j0; j < hi; j += NT) {
    if (sel[j]) continue;
    const Cx<R> v = c[j];
    const R mag = v.x * v.x + v.y * v.y;
    if (mag > best) {
      best = mag;
      bj = j;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bj;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const R ov = bv[threadIdx.x + w];
      const int64_t oi = bi[threadIdx.x + w];
      const R mv = bv[threadIdx.x];
      const int64_t mi = bi[threadIdx.x];
      if (oi >= 0 && (mi < 0 || ov > mv || (ov == mv && oi < mi))) {
        bv[threadIdx.x] = ov;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  *best_out = bv[0];
  *idx_out = bi[0];
}

// Records the chosen index j of a column (thread 0): the one-hot entry moves
// to it, or the column stops (status 1) when there is none.
template <typename R>
__device__ __forceinline__ void record_choice(OmpState& s, int64_t col, int step, int64_t j) {
  Cx<R>* e = static_cast<Cx<R>*>(s.e) + col * s.n;
  if (step > 0) {
    const int prev = s.idx[col * s.k + step - 1];
    if (prev >= 0) e[prev] = {R(0), R(0)};
  }
  if (j < 0) {  // every unchosen correlation is NaN (k <= n leaves one unchosen)
    s.active[col] = 0;
    s.status[col] = 1;
    return;
  }
  s.idx[col * s.k + step] = int(j);
  s.sel[col * s.n + j] = 1;
  e[j] = {R(1), R(0)};
}

// Argmax of |c_i|^2 over unchosen i (first index on ties); moves the one-hot
// entry of the column to it. One work-group per column.
template <typename R, int NT>
__global__ __launch_bounds__(NT) void omp_select_kernel(OmpState s, int step) {
  __shared__ R bv[NT];
  __shared__ int64_t bi[NT];
  const int64_t col = blockIdx.x;
  if (!s.active[col]) return;
  R best;
  int64_t j;
  argmax_range<R, NT>(static_cast<const Cx<R>*>(s.c) + col * s.n, s.sel + col * s.n, 0, s.n, bv, bi, &best, &j);
  if (threadIdx.x == 0) record_choice<R>(s, col, step, j);
}

// The same argmax split over SP work-groups per column (grid SP x ncols):
// each takes its range of schunk indices.
template <typename R, int NT>
__global__ __launch_bounds__(NT) void omp_select_part_kernel(OmpState s) {
  __shared__ R bv[NT];
  __shared__ int64_t bi[NT];
  const int64_t col = blockIdx.y;
  if (!s.active[col]) return;
  const int64_t lo = int64_t(blockIdx.x) * s.schunk;
  const int64_t hi = lo + s.schunk < s.n ? lo + s.schunk : s.n;
  R best;
  int64_t j;
  argmax_range<R, NT>(static_cast<const Cx<R>*>(s.c) + col * s.n, s.sel + col * s.n, lo, hi, bv, bi, &best, &j);
  if (threadIdx.x == 0) {
    s.sbest[col * s.SP + blockIdx.x] = double(best);
    s.sidx[col * s.SP + blockIdx.x] = j;
  }
}

// Combines the SP partial maxima of each column in range order (the larger
// value, the smaller index on ties: the single work-group's choice) and
// records it. One thread per column.
template <typename R>
__global__ __launch_bounds__(64) void omp_select_fin_kernel(OmpState s, int64_t ncols, int step) {
  const int64_t col = int64_t(blockIdx.x) * 64 + threadIdx.x;
  if (col >= ncols || !s.active[col]) return;
  double best = -1.0;
  int64_t j = -1;
  for (int p = 0; p < s.SP; ++p) {
    const double v = s.sbest[col * s.SP + p];
    const int64_t i = s.sidx[col * s.SP + p];
    if (i >= 0 && (j < 0 || v > best)) {
      best = v;
      j = i;
    }
  }
  record_choice<R>(s, col, step, j);
}

// The chosen column a = A e_j of a (row-selected) circulant or Toeplitz
// operator read from its generator: A[i, j] = g[(rows[i] - j) mod L]
// (rows: the selection's indices, NULL for none), rounded once to the
// working precision, instead of a transform of the one-hot vector.
template <typename R>
__global__ __launch_bounds__(256) void omp_atom_kernel(OmpState s, int step, const c128* __restrict__ g, int64_t L,
                                                       const int* __restrict__ rows) {
  const int64_t col = blockIdx.y;
  if (!s.active[col]) return;
  const int j = s.idx[col * s.k + step];
  if (j < 0) return;
  Cx<R>* a = static_cast<Cx<R>*>(s.acol) + col * s.m;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < s.m; i += int64_t(gridDim.x) * 256) {
    int64_t d = (rows ? int64_t(rows[i]) : i) - j;
    if (d < 0) d += L;
    const c128 v = g[d];
    a[i] = {R(v.x), R(v.y)};
  }
}

// Gram-Schmidt step of one column (NT threads, G dot products per sweep).
template <typename R, int NT>
__global__ __launch_bounds__(NT) void omp_orth_kernel(OmpState s, int step, R dep2) {
  constexpr int G = 8;
  __shared__ R red[2 * G * (NT / 64)];
  extern __shared__ unsigned char smem[];
  Cx<R>* h = reinterpret_cast<Cx<R>*>(smem);            // step entries: projections of this pass
  Cx<R>* rcol = h + s.k;                                 // accumulated column of R
  const int64_t col = blockIdx.x;
  if (!s.active[col]) return;
  const int64_t m = s.m;
  Cx<R>* a = static_cast<Cx<R>*>(s.acol) + col * m;
  Cx<R>* Q = static_cast<Cx<R>*>(s.q) + col * s.k * m;
  Cx<R>* r = static_cast<Cx<R>*>(s.r) + col * m;
  for (int i = threadIdx.x; i < step; i += NT) rcol[i] = {R(0), R(0)};
  Cx<R> nrm[1] = {{R(0), R(0)}};
  for (int64_t t = threadIdx.x; t < m; t += NT) nrm[0].x += a[t].x * a[t].x + a[t].y * a[t].y;
  block_sum<R, 1, NT>(nrm, red);
  const R anorm2 = nrm[0].x;
  for (int pass = 0; pass < 2; ++pass) {
    for (int i0 = 0; i0 < step; i0 += G) {
      Cx<R> d[G];
#pragma unroll
      for (int g = 0; g < G; ++g) d[g] = {R(0), R(0)};
      for (int64_t t = threadIdx.x; t < m; t += NT) {
        const Cx<R> av = a[t];
#pragma unroll
        for (int g = 0; g < G; ++g)
          if (i0 + g < step) d[g] = cadd(d[g], cmulc(av, Q[int64_t(i0 + g) * m + t]));  // conj(q) a
      }
      block_sum<R, G, NT>(d, red);
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (int(threadIdx.x) == g && i0 + g < step) {
          h[i0 + g] = d[g];
          rcol[i0 + g] = cadd(rcol[i0 + g], d[g]);
        }
    }
    __syncthreads();
    for (int64_t t = threadIdx.x; t < m; t += NT) {
      Cx<R> av = a[t];
      int i = 0;
      for (; i + G <= step; i += G) {  // G loads in flight, subtracted in order
        Cx<R> qv[G];
#pragma unroll
        for (int g = 0; g < G; ++g) qv[g] = Q[int64_t(i + g) * m + t];
#pragma unroll
        for (int g = 0; g < G; ++g) av = csub(av, cmul(qv[g], h[i + g]));
      }
      for (; i < step; ++i) av = csub(av, cmul(Q[int64_t(i) * m + t], h[i]));
      a[t] = av;
    }
    __syncthreads();
  }
  nrm[0] = {R(0), R(0)};
  for (int64_t t = threadIdx.x; t < m; t += NT) nrm[0].x += a[t].x * a[t].x + a[t].y * a[t].y;
  block_sum<R, 1, NT>(nrm, red);
  const R rho2 = nrm[0].x;
  if (!(rho2 == rho2) || !(anorm2 == anorm2) || rho2 > R(3.0e38)) {
    if (threadIdx.x == 0) {
      s.active[col] = 0;
      s.status[col] = 1;
      s.idx[col * s.k + step] = -1;
    }
    return;
  }
  if (rho2 <= dep2 * anorm2 || rho2 <= R(0)) {  // depends on the chosen columns
    if (threadIdx.x == 0) {
      s.active[col] = 0;
      s.status[col] = 2;
      s.idx[col * s.k + step] = -1;
    }
    return;
  }
  const R inv = R(1) / sqrt(rho2);
  Cx<R>* qk = Q + int64_t(step) * m;
  Cx<R> zk[1] = {{R(0), R(0)}};
  for (int64_t t = threadIdx.x; t < m; t += NT) {
    const Cx<R> qv = cscale(a[t], inv);
    qk[t] = qv;
    zk[0] = cadd(zk[0], cmulc(r[t], qv));  // conj(q) r
  }
  block_sum<R, 1, NT>(zk, red);
  Cx<R> rn[1] = {{R(0), R(0)}};
  for (int64_t t = threadIdx.x; t < m; t += NT) {
    const Cx<R> rv = csub(r[t], cmul(qk[t], zk[0]));
    r[t] = rv;
    rn[0].x += rv.x * rv.x + rv.y * rv.y;
  }
  block_sum<R, 1, NT>(rn, red);
  Cx<R>* Rf = static_cast<Cx<R>*>(s.rf) + col * s.k * s.k + int64_t(step) * s.k;  // column `step`
  for (int i = threadIdx.x; i < step; i += NT) Rf[i] = rcol[i];
  if (threadIdx.x == 0) {
    Rf[step] = {sqrt(rho2), R(0)};
    static_cast<Cx<R>*>(s.z)[col * s.k + step] = zk[0];
    s.rnorm2[col] = double(rn[0].x);
    s.nsel[col] = step + 1;
    if (double(rn[0].x) <= s.tol2 * s.bnorm2[col]) s.active[col] = 0;
  }
}

// ---- Gram-Schmidt step split over P work-groups per column (few columns).
// The same arithmetic as omp_orth_kernel, with every sum over the rows taken
// as P chunk sums added in work-group order (deterministic; every work-group
// of a column forms the same totals, so all take the same decisions).
template <typename R>
__device__ __forceinline__ Cx<R>* split_part(const OmpState& s, int64_t col, int w) {
  return static_cast<Cx<R>*>(s.part) + (col * s.P + w) * (s.k + 4);
}

template <typename R>
__device__ __forceinline__ Cx<R> split_total(const OmpState& s, int64_t col, int64_t slot) {
  Cx<R> acc = {R(0), R(0)};
  for (int w = 0; w < s.P; ++w) acc = cadd(acc, split_part<R>(s, col, w)[slot]);
  return acc;
}

// Chunk sums of conj(q_i) a for the projections i0 = blockIdx.z * kSdotG ..
// i0 + kSdotG - 1 (i < step; one group per work-group, the groups side by
// side in the grid); pass 0, group 0 also ||a||^2.
constexpr int kSdotG = 8;

template <typename R, int NT>
__global__ __launch_bounds__(NT) void omp_sdot_kernel(OmpState s, int step, int pass) {
  constexpr int G = kSdotG;
  __shared__ R red[2 * G * (NT / 64)];
  const int64_t col = blockIdx.y;
  const int w = int(blockIdx.x);
  if (!s.active[col]) return;
  const int64_t m = s.m, t0 = int64_t(w) * s.chunk, t1 = t0 + s.chunk < m ? t0 + s.chunk : m;
  const Cx<R>* a = static_cast<const Cx<R>*>(s.acol) + col * m;
  const Cx<R>* Q = static_cast<const Cx<R>*>(s.q) + col * s.k * m;
  Cx<R>* part = split_part<R>(s, col, w);
  if (pass == 0 && blockIdx.z == 0) {
    Cx<R> nrm[1] = {{R(0), R(0)}};
    for (int64_t t = t0 + threadIdx.x; t < t1; t += NT) nrm[0].x += a[t].x * a[t].x + a[t].y * a[t].y;
    block_sum<R, 1, NT>(nrm, red);
    if (threadIdx.x == 0) part[s.k] = nrm[0];
  }
  const int i0 = int(blockIdx.z) * G;
  if (i0 >= step) return;  // uniform over the work-group
  Cx<R> d[G];
#pragma unroll
  for (int g = 0; g < G; ++g) d[g] = {R(0), R(0)};
  for (int64_t t = t0 + threadIdx.x; t < t1; t += NT) {
    const Cx<R> av = a[t];
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (i0 + g < step) d[g] = cadd(d[g], cmulc(av, Q[int64_t(i0 + g) * m + t]));
  }
  block_sum<R, G, NT>(d, red);
#pragma unroll
  for (int g = 0; g < G; ++g)
    if (int(threadIdx.x) == g && i0 + g < step) part[i0 + g] = d[g];
}

// Projections of the pass (h) and the accumulated column of R (column `step`
// of the factor, written in place; used only once the step succeeds).
template <typename R>
__global__ __launch_bounds__(256) void omp_sred_kernel(OmpState s, int step, int pass) {
  const int64_t col = blockIdx.x;
  if (!s.active[col]) return;
  Cx<R>* h = static_cast<Cx<R>*>(s.hbuf) + col * s.k;
  Cx<R>* Rf = static_cast<Cx<R>*>(s.rf) + col * s.k * s.k + int64_t(step) * s.k;
  for (int i = threadIdx.x; i < step; i += 256) {
    const Cx<R> v = split_total<R>(s, col, i);
    h[i] = v;
    Rf[i] = pass == 0 ? v : cadd(Rf[i], v);
  }
}

// a -= Q h over the chunk, projections subtracted in order.
template <typename R, int NT>
__global__ __launch_bounds__(NT) void omp_supd_kernel(OmpState s, int step) {
  extern __shared__ unsigned char smem[];
  Cx<R>* hs = reinterpret_cast<Cx<R>*>(smem);
  const int64_t col = blockIdx.y;
  const int w = int(blockIdx.x);
  if (!s.active[col]) return;
  const int64_t m = s.m, t0 = int64_t(w) * s.chunk, t1 = t0 + s.chunk < m ? t0 + s.chunk : m;
  const Cx<R>* h = static_cast<const Cx<R>*>(s.hbuf) + col * s.k;
  for (int i = threadIdx.x; i < step; i += NT) hs[i] = h[i];
  __syncthreads();
  Cx<R>* a = static_cast<Cx<R>*>(s.acol) + col * m;
  const Cx<R>* Q = static_cast<const Cx<R>*>(s.q) + col * s.k * m;
  constexpr int G = 8;
  for (int64_t t = t0 + threadIdx.x; t < t1; t += NT) {
    Cx<R> av = a[t];
    int i = 0;
    for (; i + G <= step; i += G) {
      Cx<R> qv[G];
#pragma unroll
      for (int g = 0; g < G; ++g) qv[g] = Q[int64_t(i + g) * m + t];
#pragma unroll
      for (int g = 0; g < G; ++g) av = csub(av, cmul(qv[g], hs[i + g]));
    }
    for (; i < step; ++i) av = csub(av, cmul(Q[int64_t(i) * m + t], hs[i]));
    a[t] = av;
  }
}

// Chunk sums of ||a'||^2 (slot k + 1).
template <typename R, int NT>
__global__ __launch_bounds__(NT) void omp_snorm_kernel(OmpState s) {
  __shared__ R red[2 * (NT / 64)];
  const int64_t col = blockIdx.y;
  const int w = int(blockIdx.x);
  if (!s.active[col]) return;
  const int64_t m = s.m, t0 = int64_t(w) * s.chunk, t1 = t0 + s.chunk < m ? t0 + s.chunk : m;
  const Cx<R>* a = static_cast<const Cx<R>*>(s.acol) + col * m;
  Cx<R> nrm[1] = {{R(0), R(0)}};
  for (int64_t t = t0 + threadIdx.x; t < t1; t += NT) nrm[0].x += a[t].x * a[t].x + a[t].y * a[t].y;
  block_sum<R, 1, NT>(nrm, red);
  if (threadIdx.x == 0) split_part<R>(s, col, w)[s.k + 1] = nrm[0];
}

// Outcome of the step from the summed norms: 0 ok, 1 non-finite, 2 the new
// column depends on the chosen ones. Every kernel after the norms derives it
// from the same sums; only omp_sfin_kernel records it, so no kernel changes
// `active` while work-groups of its own launch may still read it.
template <typename R>
__device__ __forceinline__ int split_outcome(const OmpState& s, int64_t col, R dep2, R* rho2_out) {
  const R anorm2 = split_total<R>(s, col, s.k).x;
  const R rho2 = split_total<R>(s, col, s.k + 1).x;
  *rho2_out = rho2;
  if (!(rho2 == rho2) || !(anorm2 == anorm2) || rho2 > R(3.0e38)) return 1;
  if (rho2 <= dep2 * anorm2 || rho2 <= R(0)) return 2;
  return 0;
}

// q = a'/||a'|| over the chunk and the chunk sums of conj(q) r (slot k + 2).
template <typename R, int NT>
__global__ __launch_bounds__(NT) void omp_sq_kernel(OmpState s, int step, R dep2) {
  __shared__ R red[2 * (NT / 64)];
  const int64_t col = blockIdx.y;
  const int w = int(blockIdx.x);
  if (!s.active[col]) return;
  R rho2;
  if (split_outcome<R>(s, col, dep2, &rho2) != 0) return;
  const int64_t m = s.m, t0 = int64_t(w) * s.chunk, t1 = t0 + s.chunk < m ? t0 + s.chunk : m;
  const R inv = R(1) / sqrt(rho2);
  const Cx<R>* a = static_cast<const Cx<R>*>(s.acol) + col * m;
  Cx<R>* qk = static_cast<Cx<R>*>(s.q) + col * s.k * m + int64_t(step) * m;
  const Cx<R>* r = static_cast<const Cx<R>*>(s.r) + col * m;
  Cx<R> zk[1] = {{R(0), R(0)}};
  for (int64_t t = t0 + threadIdx.x; t < t1; t += NT) {
    const Cx<R> qv = cscale(a[t], inv);
    qk[t] = qv;
    zk[0] = cadd(zk[0], cmulc(r[t], qv));
  }
  block_sum<R, 1, NT>(zk, red);
  if (threadIdx.x == 0) split_part<R>(s, col, w)[s.k + 2] = zk[0];
}

// r -= q (q^H r) over the chunk; chunk sums of ||r'||^2 (slot k + 3).
template <typename R, int NT>
__global__ __launch_bounds__(NT) void omp_sr_kernel(OmpState s, int step, R dep2) {
  __shared__ R red[2 * (NT / 64)];
  const int64_t col = blockIdx.y;
  const int w = int(blockIdx.x);
  if (!s.active[col]) return;
  R rho2;
  if (split_outcome<R>(s, col, dep2, &rho2) != 0) return;
  const int64_t m = s.m, t0 = int64_t(w) * s.chunk, t1 = t0 + s.chunk < m ? t0 + s.chunk : m;
  const Cx<R> zk = split_total<R>(s, col, s.k + 2);
  const Cx<R>* qk = static_cast<const Cx<R>*>(s.q) + col * s.k * m + int64_t(step) * m;
  Cx<R>* r = static_cast<Cx<R>*>(s.r) + col * m;
  Cx<R> rn[1] = {{R(0), R(0)}};
  for (int64_t t = t0 + threadIdx.x; t < t1; t += NT) {
    const Cx<R> rv = csub(r[t], cmul(qk[t], zk));
    r[t] = rv;
    rn[0].x += rv.x * rv.x + rv.y * rv.y;
  }
  block_sum<R, 1, NT>(rn, red);
  if (threadIdx.x == 0) split_part<R>(s, col, w)[s.k + 3] = rn[0];
}

// The step's outcome; on success the diagonal of R, z, residual norm, atom
// count and the tolerance stop.
template <typename R>
__global__ __launch_bounds__(64) void omp_sfin_kernel(OmpState s, int step, R dep2) {
  const int64_t col = blockIdx.x;
  if (!s.active[col] || threadIdx.x != 0) return;
  R rho2;
  const int outcome = split_outcome<R>(s, col, dep2, &rho2);
  if (outcome != 0) {
    s.active[col] = 0;
    s.status[col] = outcome;
    s.idx[col * s.k + step] = -1;
    return;
  }
  const Cx<R> zk = split_total<R>(s, col, s.k + 2);
  const R rn = split_total<R>(s, col, s.k + 3).x;
  Cx<R>* Rf = static_cast<Cx<R>*>(s.rf) + col * s.k * s.k + int64_t(step) * s.k;
  Rf[step] = {sqrt(rho2), R(0)};
  static_cast<Cx<R>*>(s.z)[col * s.k + step] = zk;
  s.rnorm2[col] = double(rn);
  s.nsel[col] = step + 1;
  if (double(rn) <= s.tol2 * s.bnorm2[col]) s.active[col] = 0;
}

// x_S = R^{-1} z by back substitution, x = 0 elsewhere.
template <typename R>
__global__ __launch_bounds__(256) void omp_finish_kernel(OmpState s, void* xout, int64_t ldx, int* support) {
  __shared__ R red[2 * 4];
  extern __shared__ unsigned char smem[];
  Cx<R>* xs = reinterpret_cast<Cx<R>*>(smem);
  const int64_t col = blockIdx.x;
  const int ns = s.nsel[col];
  const Cx<R>* Rf = static_cast<const Cx<R>*>(s.rf) + col * s.k * s.k;
  const Cx<R>* z = static_cast<const Cx<R>*>(s.z) + col * s.k;
  for (int i = ns - 1; i >= 0; --i) {
    Cx<R> acc[1] = {{R(0), R(0)}};
    for (int j = i + 1 + threadIdx.x; j < ns; j += 256) acc[0] = cadd(acc[0], cmul(Rf[int64_t(j) * s.k + i], xs[j]));
    block_sum<R, 1, 256>(acc, red);
    if (threadIdx.x == 0) {
      const Cx<R> d = Rf[int64_t(i) * s.k + i];  // real, positive
      xs[i] = cscale(csub(z[i], acc[0]), R(1) / d.x);
    }
    __syncthreads();
  }
  Cx<R>* x = static_cast<Cx<R>*>(xout) + col * ldx;
  for (int64_t t = threadIdx.x; t < s.n; t += 256) x[t] = {R(0), R(0)};
  __syncthreads();
  for (int i = threadIdx.x; i < ns; i += 256) x[s.idx[col * s.k + i]] = xs[i];
  if (support)
    for (int64_t i = threadIdx.x; i < s.k; i += 256) support[col * s.k + i] = i < ns ? s.idx[col * s.k + i] : -1;
}

struct OmpPlan {
  size_t r, c, e, acol, q, rf, z, idx, sel, bn, rn, act, nsel, status, part, hbuf, sbest, sidx, exec, total;
  int P, SP;
};

// Work-groups per column of the argmax: with few columns one work-group
// scanning all n indices is a long serial chain; spread it over ~256
// work-groups in all, at least 4096 indices each, at most 16 per column.
int select_split(int64_t ncols, int64_t n) {
  if (ncols <= 0 || ncols >= 128) return 1;
  int64_t p = std::min<int64_t>(256 / ncols, 16);
  p = std::min<int64_t>(p, n / 4096);
  return int(std::max<int64_t>(p, 1));
}

// Work-groups per column of the Gram-Schmidt step: enough to spread few
// columns over the chip (~256 work-groups), at least 256 rows each, at most 16.
int omp_split(int64_t ncols, int64_t m, int64_t k, size_t es) {
  if (ncols <= 0 || ncols >= 128 || size_t(k) * es > 65536) return 1;  // projections staged in LDS
  int64_t p = std::min<int64_t>(256 / ncols, 16);
  p = std::min<int64_t>(p, m / 256);
  return int(std::max<int64_t>(p, 1));
}

fm_status plan_omp(const fm_op_s* a, int64_t ncols, int64_t k, OmpPlan* p) {
  const Elem e = elem_of(a->dt);
  const size_t es = elem_bytes(e);
  const int64_t m = a->m, n = a->n;
  size_t off = 0;
  auto take = [&](size_t* slot, size_t bytes) {
    *slot = off;
    off += up(bytes);
  };
  take(&p->r, size_t(ncols * m) * es);
  take(&p->c, size_t(ncols * n) * es);
  take(&p->e, size_t(ncols * n) * es);
  take(&p->acol, size_t(ncols * m) * es);
  take(&p->q, size_t(ncols) * size_t(k) * size_t(m) * es);
  take(&p->rf, size_t(ncols) * size_t(k * k) * es);
  take(&p->z, size_t(ncols * k) * es);
  take(&p->idx, size_t(ncols * k) * 4);
  take(&p->sel, size_t(ncols * n));
  take(&p->bn, size_t(ncols) * 8);
  take(&p->rn, size_t(ncols) * 8);
  take(&p->act, size_t(ncols) * 4);
  take(&p->nsel, size_t(ncols) * 4);
  take(&p->status, size_t(ncols) * 4);
  p->P = omp_split(ncols, m, k, es);
  take(&p->part, p->P > 1 ? size_t(ncols) * size_t(p->P) * size_t(k + 4) * es : 0);
  take(&p->hbuf, p->P > 1 ? size_t(ncols * k) * es : 0);
  p->SP = select_split(ncols, n);
  take(&p->sbest, p->SP > 1 ? size_t(ncols) * size_t(p->SP) * 8 : 0);
  take(&p->sidx, p->SP > 1 ? size_t(ncols) * size_t(p->SP) * 8 : 0);
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

// Where the columns of A can be read from a stored generator: A = C or
// A = S C, C a circulant or Toeplitz created from its generator.
struct AtomSource {
  const c128* g = nullptr;
  int64_t L = 0;
  const int* rows = nullptr;
};
AtomSource atom_source(const fm_op_s* a) {
  AtomSource src;
  const fm_op_s* C = a;
  const int* rows = nullptr;
  if (a->kind == Kind::Product && a->terms.size() == 2 && a->terms[0]->kind == Kind::Select) {
    rows = static_cast<const int*>(a->terms[0]->idx.p);
    C = a->terms[1];
  }
  if ((C->kind == Kind::Circulant || C->kind == Kind::Toeplitz) && C->gen.p != nullptr && C->L > 0) {
    src.g = static_cast<const c128*>(C->gen.p);
    src.L = C->L;
    src.rows = rows;
  }
  return src;
}

template <typename R>
fm_status run_omp(const fm_op_s* a, int64_t ncols, OmpState st, void* x, int64_t ldx, int* support, Workspace& w,
                  hipStream_t s) {
  const AtomSource atom = atom_source(a);
  const Elem e = elem_of(a->dt);
  const int64_t m = a->m, n = a->n;
  // one work-group per column: 1024 threads keep more loads in flight (the
  // complex128 Gram-Schmidt step needs more registers than 1024 threads allow)
  constexpr int NT = sizeof(R) == 4 ? 1024 : 256;
  const R dep2 = sizeof(R) == 4 ? R(1e-10) : R(1e-24);  // (relative norm left after orthogonalisation)^2
  const size_t orth_lds = size_t(2 * st.k) * sizeof(Cx<R>);
  const size_t fin_lds = size_t(st.k) * sizeof(Cx<R>);
  const dim3 grid{unsigned(ncols)};
  hipLaunchKernelGGL(omp_init_kernel<R>, grid, dim3(256), 0, s, st);
  FM_LAUNCHED();
  const Batch bf{ncols, 1, 1, n, n, m, m}, ba{ncols, 1, 1, m, m, n, n};
  for (int step = 0; step < int(st.k); ++step) {
    FM_TRY(exec(a, true, e, ba, st.r, st.c, false, w, s));      // c = A^H r
    if (st.SP > 1) {
      hipLaunchKernelGGL((omp_select_part_kernel<R, NT>), dim3(unsigned(st.SP), unsigned(ncols)), dim3(NT), 0, s, st);
      hipLaunchKernelGGL(omp_select_fin_kernel<R>, dim3(unsigned(cdiv(ncols, 64))), dim3(64), 0, s, st, ncols, step);
    } else {
      hipLaunchKernelGGL((omp_select_kernel<R, NT>), grid, dim3(NT), 0, s, st, step);
    }
    FM_LAUNCHED();
    if (atom.g) {  // a = A e_j from the generator
      const dim3 ga{unsigned(std::min<int64_t>(cdiv(m, 256), 64)), unsigned(ncols)};
      hipLaunchKernelGGL(omp_atom_kernel<R>, ga, dim3(256), 0, s, st, step, atom.g, atom.L, atom.rows);
      FM_LAUNCHED();
    } else {
      FM_TRY(exec(a, false, e, bf, st.e, st.acol, false, w, s));  // a = A e_j
    }
    if (st.P > 1) {
      const dim3 g2{unsigned(st.P), unsigned(ncols)};
      constexpr int NS = 256;
      for (int pass = 0; pass < 2; ++pass) {
        const dim3 g3{unsigned(st.P), unsigned(ncols), unsigned(std::max(1, (step + kSdotG - 1) / kSdotG))};
        hipLaunchKernelGGL((omp_sdot_kernel<R, NS>), g3, dim3(NS), 0, s, st, step, pass);
        hipLaunchKernelGGL(omp_sred_kernel<R>, grid, dim3(256), 0, s, st, step, pass);
        hipLaunchKernelGGL((omp_supd_kernel<R, NS>), g2, dim3(NS), size_t(st.k) * sizeof(Cx<R>), s, st, step);
      }
      hipLaunchKernelGGL((omp_snorm_kernel<R, NS>), g2, dim3(NS), 0, s, st);
      hipLaunchKernelGGL((omp_sq_kernel<R, NS>), g2, dim3(NS), 0, s, st, step, dep2);
      hipLaunchKernelGGL((omp_sr_kernel<R, NS>), g2, dim3(NS), 0, s, st, step, dep2);
      hipLaunchKernelGGL(omp_sfin_kernel<R>, grid, dim3(64), 0, s, st, step, dep2);
    } else {
      hipLaunchKernelGGL((omp_orth_kernel<R, NT>), grid, dim3(NT), orth_lds, s, st, step, dep2);
    }
    FM_LAUNCHED();
  }
  hipLaunchKernelGGL(omp_finish_kernel<R>, grid, dim3(256), fin_lds, s, st, x, ldx, support);
  FM_LAUNCHED();
  return FM_OK;
}

}  // namespace
}  // namespace fm

using namespace fm;

extern "C" {

fm_status fm_omp_workspace_size(fm_op a, int64_t ncols, int32_t k, size_t* bytes) {
  set_error("");
  FM_CHECK_ARG(a != nullptr, FM_E_INVALID, "operator handle is NULL");
  FM_CHECK_ARG(op_alive(a), FM_E_RELEASED, "operator handle was released");
  FM_CHECK_ARG(bytes != nullptr, FM_E_INVALID, "NULL argument");
  FM_CHECK_ARG(ncols >= 0 && k >= 1, FM_E_INVALID, "need ncols >= 0 and k >= 1");
  OmpPlan p;
  FM_TRY(plan_omp(a, ncols, k, &p));
  *bytes = p.total;
  return FM_OK;
}

fm_status fm_omp(fm_op a, int64_t ncols, const void* b, int64_t ldb, int32_t k, double tol, void* x, int64_t ldx,
                 int32_t* support, fm_omp_stat* stats, void* ws, size_t ws_bytes, void* stream) {
  set_error("");
  FM_CHECK_ARG(a != nullptr, FM_E_INVALID, "operator handle is NULL");
  FM_CHECK_ARG(op_alive(a), FM_E_RELEASED, "operator handle was released");
  FM_CHECK_ARG(is_complex(a->dt), FM_E_DTYPE, "OMP needs a complex operator");
  FM_CHECK_ARG(ncols >= 0, FM_E_INVALID, "negative column count");
  FM_CHECK_ARG(ncols < 65536, FM_E_UNSUPPORTED, "at most 65535 columns per call");
  FM_CHECK_ARG(tol >= 0.0, FM_E_INVALID, "tol must be non-negative");
  const int64_t m = a->m, n = a->n;
  FM_CHECK_ARG(k >= 1 && k <= m && k <= n, FM_E_INVALID, "need 1 <= k <= min(m, n)");
  FM_CHECK_ARG(k <= 1024, FM_E_UNSUPPORTED, "at most 1024 atoms");
  if (ncols == 0) return FM_OK;
  FM_CHECK_ARG(b != nullptr && x != nullptr, FM_E_INVALID, "NULL data pointer");
  FM_CHECK_ARG(ldb >= m && ldx >= n, FM_E_SHAPE, "leading dimensions too small");
  int dev = 0;
  FM_HIP(hipGetDevice(&dev));
  FM_CHECK_ARG(dev == a->device, FM_E_DEVICE, "operator lives on device %d, current is %d", a->device, dev);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  OmpPlan p;
  FM_TRY(plan_omp(a, ncols, k, &p));
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
  OmpState st{};
  st.m = m;
  st.n = n;
  st.k = k;
  st.b = b;
  st.ldb = ldb;
  st.r = B + p.r;
  st.c = B + p.c;
  st.e = B + p.e;
  st.acol = B + p.acol;
  st.q = B + p.q;
  st.rf = B + p.rf;
  st.z = B + p.z;
  st.idx = reinterpret_cast<int*>(B + p.idx);
  st.sel = reinterpret_cast<unsigned char*>(B + p.sel);
  st.bnorm2 = reinterpret_cast<double*>(B + p.bn);
  st.rnorm2 = reinterpret_cast<double*>(B + p.rn);
  st.active = reinterpret_cast<int*>(B + p.act);
  st.nsel = reinterpret_cast<int*>(B + p.nsel);
  st.status = reinterpret_cast<int*>(B + p.status);
  st.tol2 = tol * tol;
  st.P = p.P;
  st.chunk = cdiv(m, p.P);
  st.part = B + p.part;
  st.hbuf = B + p.hbuf;
  st.SP = p.SP;
  st.schunk = cdiv(n, p.SP);
  st.sbest = reinterpret_cast<double*>(B + p.sbest);
  st.sidx = reinterpret_cast<int64_t*>(B + p.sidx);
  Workspace w;
  w.base = B + p.exec;
  w.cap = p.total - p.exec;
  auto body = [&]() -> fm_status {
    if (a->dt == FM_C64)
      FM_TRY(run_omp<float>(a, ncols, st, x, ldx, support, w, s));
    else
      FM_TRY(run_omp<double>(a, ncols, st, x, ldx, support, w, s));
    if (stats) {
      std::vector<int> hn(ncols), hs(ncols);
      std::vector<double> hr(ncols);
      FM_HIP(hipMemcpyAsync(hn.data(), st.nsel, size_t(ncols) * 4, hipMemcpyDeviceToHost, s));
      FM_HIP(hipMemcpyAsync(hs.data(), st.status, size_t(ncols) * 4, hipMemcpyDeviceToHost, s));
      FM_HIP(hipMemcpyAsync(hr.data(), st.rnorm2, size_t(ncols) * 8, hipMemcpyDeviceToHost, s));
      FM_HIP(hipStreamSynchronize(s));
      for (int64_t j = 0; j < ncols; ++j) stats[j] = fm_omp_stat{hn[j], hs[j], std::sqrt(hr[j])};
    }
    return FM_OK;
  };
  fm_status res = body();
  if (own) (void)hipFreeAsync(base, s);
  return res;
}

}  // extern "C"
