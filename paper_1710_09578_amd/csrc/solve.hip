// Kernels of the proximal-gradient solver (the ISTA iteration of the section
// on ultrasonic nondestructive testing and its accelerated FISTA form, for the
// l1-regularised least-squares problem of eq. (8)) and of the FP64 power
// iteration for the step constant.
//
// Per column j (one problem each), with z = y - g/L:
//   x_new = soft(z, lambda_j/L)  (complex modulus shrinkage, |z| <= s -> 0)
//   y_new = x_new + beta (x_new - x_old)
// plus deterministic per-block partial sums of ||x_new - x_old||^2 and
// ||x_new||^2 for the stopping rule, reduced afterwards in a fixed order.
#include "solve.h"

namespace fm {
namespace {

template <typename R>
__device__ __forceinline__ Cx<R> soft(Cx<R> z, R s) {
  const R mag = sqrt(z.x * z.x + z.y * z.y);
  if (!(mag > s)) return {R(0), R(0)};
  const R f = (mag - s) / mag;
  return {z.x * f, z.y * f};
}

constexpr int kTPB = 256;

template <typename R>
__global__ __launch_bounds__(kTPB) void update_kernel(UpdateArgs a) {
  const int64_t c = blockIdx.y;
  const int64_t tile = blockIdx.x;
  __shared__ double sdx[kTPB], snx[kTPB];
  __shared__ int s_active;
  if (threadIdx.x == 0) s_active = a.active ? a.active[c] : 1;
  __syncthreads();
  if (!s_active) return;  // frozen problem: its iterate stays as it is
  const Cx<R>* G = reinterpret_cast<const Cx<R>*>(a.g) + c * a.ldg;
  Cx<R>* Y = reinterpret_cast<Cx<R>*>(a.y) + c * a.ldy;
  Cx<R>* X = reinterpret_cast<Cx<R>*>(a.x) + c * a.ldx;
  const R invL = R(a.invL);
  const R s = R(a.lam[c] * a.invL);
  const R beta = R(a.beta);
  double dx = 0.0, nx = 0.0;
  bool bad = false;
  const int64_t i0 = tile * int64_t(kTPB) * a.per_thread;
  for (int k = 0; k < a.per_thread; ++k) {
    const int64_t i = i0 + int64_t(k) * kTPB + threadIdx.x;
    if (i >= a.rows) break;
    const Cx<R> yv = Y[i], gv = G[i], xo = X[i];
    const Cx<R> z = {yv.x - gv.x * invL, yv.y - gv.y * invL};
    const Cx<R> xn = soft(z, s);
    const Cx<R> d = {xn.x - xo.x, xn.y - xo.y};
    Cx<R> yn = xn;
    if (a.momentum) yn = {xn.x + beta * d.x, xn.y + beta * d.y};
    X[i] = xn;
    Y[i] = yn;
    dx += double(d.x) * double(d.x) + double(d.y) * double(d.y);
    nx += double(xn.x) * double(xn.x) + double(xn.y) * double(xn.y);
    bad |= !(isfinite(z.x) && isfinite(z.y));
  }
  if (bad && a.status) atomicOr(a.status + c, 1);
  if (!a.partial) return;
  sdx[threadIdx.x] = dx;
  snx[threadIdx.x] = nx;
  __syncthreads();
  for (int w = kTPB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sdx[threadIdx.x] += sdx[threadIdx.x + w];
      snx[threadIdx.x] += snx[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.partial[2 * (c * a.ntiles + tile)] = sdx[0];
    a.partial[2 * (c * a.ntiles + tile) + 1] = snx[0];
  }
}

// Freezes column c when ||dx|| <= tol * max(||x||, 1e-30) or when it met a
// non-finite value; records the iteration count.
__global__ __launch_bounds__(256) void stop_kernel(const double* partial, int64_t ntiles, int64_t ncols, double tol,
                                                   int k, int* active, int* iters, const int* status) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= ncols || !active[c]) return;
  if (status && status[c]) {
    active[c] = 0;
    iters[c] = k + 1;
    return;
  }
  if (tol <= 0.0) return;
  double dx = 0.0, nx = 0.0;
  for (int64_t t = 0; t < ntiles; ++t) {
    dx += partial[2 * (c * ntiles + t)];
    nx += partial[2 * (c * ntiles + t) + 1];
  }
  const double nrm = sqrt(nx);
  if (sqrt(dx) <= tol * (nrm > 1e-30 ? nrm : 1e-30)) {
    active[c] = 0;
    iters[c] = k + 1;
  }
}

template <typename R>
__global__ __launch_bounds__(kTPB) void sub_kernel(int64_t rows, const void* b, int64_t ldb, void* r, int64_t ldr,
                                                   const int* active) {
  const int64_t c = blockIdx.y;
  if (active && !active[c]) return;
  const int64_t i = int64_t(blockIdx.x) * kTPB + threadIdx.x;
  if (i >= rows) return;
  const Cx<R> bv = reinterpret_cast<const Cx<R>*>(b)[c * ldb + i];
  Cx<R>* rp = reinterpret_cast<Cx<R>*>(r) + c * ldr + i;
  *rp = csub(*rp, bv);
}

// max_i |g[c, i]| per column (one work-group per column), times rel. The
// maximum does not depend on the order, so a column's 1024 threads keep 8
// independent loads in flight each: a single work-group on a long column is
// bound by the loads it has in flight.
constexpr int kColmaxTPB = 1024;
template <typename R>
__global__ __launch_bounds__(kColmaxTPB) void colmax_kernel(int64_t rows, const void* g, int64_t ldg, double rel,
                                                            double* out) {
  __shared__ double sm[kColmaxTPB];
  const int64_t c = blockIdx.x;
  const Cx<R>* G = reinterpret_cast<const Cx<R>*>(g) + c * ldg;
  double m = 0.0;
  constexpr int kU = 8;
  for (int64_t i0 = threadIdx.x; i0 < rows; i0 += int64_t(kU) * kColmaxTPB) {
    Cx<R> v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = i0 + int64_t(u) * kColmaxTPB;
      v[u] = i < rows ? G[i] : Cx<R>{R(0), R(0)};
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const double re = v[u].x, im = v[u].y;
      const double a = sqrt(re * re + im * im);
      m = a > m ? a : m;
    }
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = kColmaxTPB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] = sm[threadIdx.x] > sm[threadIdx.x + w] ? sm[threadIdx.x] : sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = rel * sm[0];
}

// sum |v_i|^2 of one complex128 vector: per-block partials (fixed order)
__global__ __launch_bounds__(kTPB) void norm2_partial_kernel(int64_t n, const c128* v, double* partial) {
  __shared__ double sm[kTPB];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kTPB + threadIdx.x; i < n; i += int64_t(gridDim.x) * kTPB)
    s += v[i].x * v[i].x + v[i].y * v[i].y;
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int w = kTPB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(kTPB) void norm2_final_kernel(int nparts, const double* partial, double* out) {
  __shared__ double sm[kTPB];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kTPB) s += partial[i];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int w = kTPB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}

// The final sum of norm2_final_kernel, taken by a whole work-group (same
// order, so the same value in every work-group that takes it).
__device__ __forceinline__ double final_sum(int nparts, const double* partial, double* sm) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kTPB) s += partial[i];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int w = kTPB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sm[0];
  __syncthreads();  // sm is reused by the caller
  return r;
}

// Power-iteration step end: ||w||^2 from its partial sums, w *= 1/||w||, and
// (work-group 0) both squared norms of the step stored: out_w = ||w||^2,
// out_a = ||A v||^2 from its own partial sums. One launch in place of two
// final reductions and the scaling; the values are those of
// norm2_final_kernel and normalize_kernel.
__global__ __launch_bounds__(kTPB) void normalize_final_kernel(int64_t n, c128* w, int nparts, const double* part_w,
                                                               const double* part_a, double* out_w, double* out_a) {
  __shared__ double sm[kTPB];
  const double nw = final_sum(nparts, part_w, sm);
  if (blockIdx.x == 0) {
    const double na = final_sum(nparts, part_a, sm);
    if (threadIdx.x == 0) {
      *out_w = nw;
      *out_a = na;
    }
  }
  const int64_t i = int64_t(blockIdx.x) * kTPB + threadIdx.x;
  if (i >= n) return;
  const double f = 1.0 / sqrt(nw);
  w[i].x *= f;
  w[i].y *= f;
}

// v *= 1/sqrt(*nrm2)
__global__ __launch_bounds__(kTPB) void normalize_kernel(int64_t n, c128* v, const double* nrm2) {
  const int64_t i = int64_t(blockIdx.x) * kTPB + threadIdx.x;
  if (i >= n) return;
  const double f = 1.0 / sqrt(*nrm2);
  v[i].x *= f;
  v[i].y *= f;
}

// SplitMix64 output k for a seed: z = seed + (k+1) * golden gamma, then the
// published finaliser.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(kTPB) void start_vector_kernel(int64_t n, uint64_t seed, c128* v) {
  const int64_t i = int64_t(blockIdx.x) * kTPB + threadIdx.x;
  if (i >= n) return;
  const double u0 = double(splitmix64(seed, 2 * uint64_t(i)) >> 11) * 0x1.0p-53;
  const double u1 = double(splitmix64(seed, 2 * uint64_t(i) + 1) >> 11) * 0x1.0p-53;
  v[i] = {u0 - 0.5, u1 - 0.5};
}

template <typename V>
__global__ __launch_bounds__(kTPB) void fill_kernel(int64_t n, V* p, V v) {
  const int64_t i = int64_t(blockIdx.x) * kTPB + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename R>
__global__ __launch_bounds__(kTPB) void zero2d_kernel(int64_t rows, void* p, int64_t ld) {
  const int64_t i = int64_t(blockIdx.x) * kTPB + threadIdx.x;
  if (i < rows) reinterpret_cast<Cx<R>*>(p)[int64_t(blockIdx.y) * ld + i] = {R(0), R(0)};
}

template <typename R>
__global__ __launch_bounds__(kTPB) void copy2d_kernel(int64_t rows, const void* s, int64_t lds, void* d, int64_t ldd) {
  const int64_t i = int64_t(blockIdx.x) * kTPB + threadIdx.x;
  if (i < rows)
    reinterpret_cast<Cx<R>*>(d)[int64_t(blockIdx.y) * ldd + i] =
        reinterpret_cast<const Cx<R>*>(s)[int64_t(blockIdx.y) * lds + i];
}

}  // namespace

int64_t update_tiles(int64_t rows, int* per_thread) {
  int pt = 4;
  *per_thread = pt;
  return cdiv(rows, int64_t(kTPB) * pt);
}

fm_status launch_update(Elem e, const UpdateArgs& a, int64_t ncols, hipStream_t s) {
  if (ncols == 0 || a.rows == 0) return FM_OK;
  FM_CHECK_ARG(ncols < 65536, FM_E_UNSUPPORTED, "solver: at most 65535 columns per call");
  dim3 g(unsigned(a.ntiles), unsigned(ncols));
  if (e == Elem::C64)
    hipLaunchKernelGGL(update_kernel<float>, g, dim3(kTPB), 0, s, a);
  else
    hipLaunchKernelGGL(update_kernel<double>, g, dim3(kTPB), 0, s, a);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_stop(const double* partial, int64_t ntiles, int64_t ncols, double tol, int k, int* active,
                      int* iters, const int* status, hipStream_t s) {
  if (ncols == 0) return FM_OK;
  hipLaunchKernelGGL(stop_kernel, dim3(unsigned(cdiv(ncols, 256))), dim3(256), 0, s, partial, ntiles, ncols, tol, k,
                     active, iters, status);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_sub(Elem e, int64_t rows, int64_t ncols, const void* b, int64_t ldb, void* r, int64_t ldr,
                     const int* active, hipStream_t s) {
  if (ncols == 0 || rows == 0) return FM_OK;
  FM_CHECK_ARG(ncols < 65536, FM_E_UNSUPPORTED, "solver: at most 65535 columns per call");
  dim3 g(unsigned(cdiv(rows, kTPB)), unsigned(ncols));
  if (e == Elem::C64)
    hipLaunchKernelGGL(sub_kernel<float>, g, dim3(kTPB), 0, s, rows, b, ldb, r, ldr, active);
  else
    hipLaunchKernelGGL(sub_kernel<double>, g, dim3(kTPB), 0, s, rows, b, ldb, r, ldr, active);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_colmax(Elem e, int64_t rows, int64_t ncols, const void* g, int64_t ldg, double rel, double* out,
                        hipStream_t s) {
  if (ncols == 0) return FM_OK;
  if (e == Elem::C64)
    hipLaunchKernelGGL(colmax_kernel<float>, dim3(unsigned(ncols)), dim3(kColmaxTPB), 0, s, rows, g, ldg, rel, out);
  else
    hipLaunchKernelGGL(colmax_kernel<double>, dim3(unsigned(ncols)), dim3(kColmaxTPB), 0, s, rows, g, ldg, rel, out);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_norm2(int64_t n, const void* v, double* partial, int nparts, double* out, hipStream_t s) {
  hipLaunchKernelGGL(norm2_partial_kernel, dim3(unsigned(nparts)), dim3(kTPB), 0, s, n, (const c128*)v, partial);
  FM_LAUNCHED();
  hipLaunchKernelGGL(norm2_final_kernel, dim3(1), dim3(kTPB), 0, s, nparts, partial, out);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_norm2_partial(int64_t n, const void* v, double* partial, int nparts, hipStream_t s) {
  FM_CHECK_ARG(nparts > 0 && nparts <= 65535, FM_E_INVALID, "norm2: %d partial sums", nparts);
  hipLaunchKernelGGL(norm2_partial_kernel, dim3(unsigned(nparts)), dim3(kTPB), 0, s, n, (const c128*)v, partial);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_normalize_final(int64_t n, void* w, int nparts, const double* part_w, const double* part_a,
                                 double* out_w, double* out_a, hipStream_t s) {
  hipLaunchKernelGGL(normalize_final_kernel, dim3(unsigned(cdiv(n, kTPB))), dim3(kTPB), 0, s, n, (c128*)w, nparts,
                     part_w, part_a, out_w, out_a);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_normalize(int64_t n, void* v, const double* nrm2, hipStream_t s) {
  hipLaunchKernelGGL(normalize_kernel, dim3(unsigned(cdiv(n, kTPB))), dim3(kTPB), 0, s, n, (c128*)v, nrm2);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_start_vector(int64_t n, uint64_t seed, void* v, hipStream_t s) {
  hipLaunchKernelGGL(start_vector_kernel, dim3(unsigned(cdiv(n, kTPB))), dim3(kTPB), 0, s, n, seed, (c128*)v);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_fill_int(int64_t n, int* p, int v, hipStream_t s) {
  if (n == 0) return FM_OK;
  hipLaunchKernelGGL(fill_kernel<int>, dim3(unsigned(cdiv(n, kTPB))), dim3(kTPB), 0, s, n, p, v);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_fill_double(int64_t n, double* p, double v, hipStream_t s) {
  if (n == 0) return FM_OK;
  hipLaunchKernelGGL(fill_kernel<double>, dim3(unsigned(cdiv(n, kTPB))), dim3(kTPB), 0, s, n, p, v);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_zero2d(Elem e, int64_t rows, int64_t ncols, void* p, int64_t ld, hipStream_t s) {
  if (rows == 0 || ncols == 0) return FM_OK;
  FM_CHECK_ARG(ncols < 65536, FM_E_UNSUPPORTED, "solver: at most 65535 columns per call");
  dim3 g(unsigned(cdiv(rows, kTPB)), unsigned(ncols));
  if (e == Elem::C64)
    hipLaunchKernelGGL(zero2d_kernel<float>, g, dim3(kTPB), 0, s, rows, p, ld);
  else
    hipLaunchKernelGGL(zero2d_kernel<double>, g, dim3(kTPB), 0, s, rows, p, ld);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_copy2d(Elem e, int64_t rows, int64_t ncols, const void* src, int64_t lds, void* dst, int64_t ldd,
                        hipStream_t s) {
  if (rows == 0 || ncols == 0) return FM_OK;
  FM_CHECK_ARG(ncols < 65536, FM_E_UNSUPPORTED, "solver: at most 65535 columns per call");
  dim3 g(unsigned(cdiv(rows, kTPB)), unsigned(ncols));
  if (e == Elem::C64)
    hipLaunchKernelGGL(copy2d_kernel<float>, g, dim3(kTPB), 0, s, rows, src, lds, dst, ldd);
  else
    hipLaunchKernelGGL(copy2d_kernel<double>, g, dim3(kTPB), 0, s, rows, src, lds, dst, ldd);
  FM_LAUNCHED();
  return FM_OK;
}

}  // namespace fm
