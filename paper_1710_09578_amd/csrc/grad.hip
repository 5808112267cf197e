// Differentiation support: the generator gradient of a circulant operator,
// one proximal-gradient (FISTA) step and its vector-Jacobian product, a block
// axpby, and an upper bound of ||A||_2^2 from an operator's structure.
//
// Gradients follow PyTorch's convention for complex tensors: for a real loss
// f and an upstream gradient G of an output s, the gradient of an input z is
// G conj(ds/dz) + conj(G) ds/dz* (Wirtinger derivatives).
//
// Circulant generator (the cyclic convolution y = c (*) x of eq. (5)): y is
// linear in c with matrix C(x), so dL/dc = C(x)^H G, a circular
// cross-correlation, computed as IDFT(DFT(G) . conj(DFT(x))) / n and summed
// over the columns in the frequency domain. For w = C(c)^H u, w is linear in
// conj(c), and the gradient is the cross-correlation of u with G.
#include <algorithm>
#include <cmath>

#include "kernels.h"
#include "runtime.h"
#include "solve.h"

namespace fm {
namespace {

constexpr int kTPB = 256;

template <typename R>
__device__ __forceinline__ Cx<R> soft(Cx<R> z, R s) {
  const R mag = sqrt(z.x * z.x + z.y * z.y);
  if (!(mag > s)) return {R(0), R(0)};
  const R f = (mag - s) / mag;
  return {z.x * f, z.y * f};
}

// Column-summed spectral products of one chunk in two deterministic passes:
// group g = blockIdx.y of the columns [g cpg, (g + 1) cpg) gives
// part[g][f] = sum_j A_j[f] conj(B_j[f]) in column order; then
// P[f] (+)= scale * sum_g part[g][f] in group order. The groups spread the
// chunk over the chip (one thread per frequency alone leaves most CUs idle).
template <typename R>
__global__ __launch_bounds__(kTPB) void corr_part_kernel(int64_t n, int64_t ncols, int64_t cpg,
                                                         const Cx<R>* __restrict__ A, const Cx<R>* __restrict__ B,
                                                         Cx<R>* __restrict__ part) {
  const int64_t f = int64_t(blockIdx.x) * kTPB + threadIdx.x;
  if (f >= n) return;
  const int64_t j0 = int64_t(blockIdx.y) * cpg;
  const int64_t j1 = j0 + cpg < ncols ? j0 + cpg : ncols;
  Cx<R> acc = {R(0), R(0)};
  for (int64_t j = j0; j < j1; ++j) acc = cadd(acc, cmulc(A[j * n + f], B[j * n + f]));
  part[int64_t(blockIdx.y) * n + f] = acc;
}

template <typename R>
__global__ __launch_bounds__(kTPB) void corr_sum_kernel(int64_t n, int64_t ngroups, const Cx<R>* __restrict__ part,
                                                        R scale, Cx<R>* P, int accumulate) {
  const int64_t f = int64_t(blockIdx.x) * kTPB + threadIdx.x;
  if (f >= n) return;
  Cx<R> acc = {R(0), R(0)};
  for (int64_t g = 0; g < ngroups; ++g) acc = cadd(acc, part[g * n + f]);
  acc = cscale(acc, scale);
  P[f] = accumulate ? cadd(P[f], acc) : acc;
}

// Column groups for n frequencies and nc columns: about 2048 work-groups
// in the first pass, at least 4 columns per group.
int64_t corr_groups(int64_t n, int64_t nc) {
  const int64_t tiles = cdiv(n, kTPB);
  const int64_t want = std::max<int64_t>(1, 2048 / tiles);
  return std::max<int64_t>(1, std::min<int64_t>(want, cdiv(nc, 4)));
}

// Four-step lengths (L = n1 n2 above one work-group): the correlation only
// needs the column-summed products of two spectra, so both spectra stay in
// the split's own order, X[k2 + n2 k1] at k1 + n1 k2, and the sum returns to
// natural order through the inverse passes, with no transposes.
// Forward DFT of nc columns of x (leading dimension ldx) into w (ld L).
fm_status dft_split_order(Elem e, const Split& sp, int64_t nc, const void* x, int64_t ldx, void* w,
                          hipStream_t s) {
  const int64_t L = int64_t(1) << sp.logL, n1 = int64_t(1) << sp.log1, n2 = int64_t(1) << sp.log2;
  FftLaunch f1;  // length-n2 transforms at stride n1, then W_L^(k2 n1)
  f1.elem = e;
  f1.logn = sp.log2;
  f1.mode = FFT_FWD;
  f1.b = Batch{nc, 1, n1, ldx, 0, L, 0};
  f1.x = x;
  f1.y = w;
  f1.in_limit = f1.out_limit = L;
  f1.tw_log = sp.logL;
  FM_TRY(launch_fft(f1, s));
  FftLaunch f2;  // contiguous length-n1 transforms of the rows, in place
  f2.elem = e;
  f2.logn = sp.log1;
  f2.mode = FFT_FWD;
  f2.b = Batch{nc, n2, 1, L, n1, L, n1};
  f2.x = w;
  f2.y = w;
  f2.in_limit = f2.out_limit = n1;
  return launch_fft(f2, s);
}

// Unnormalised inverse DFT of one vector p held in the split's order (p is
// overwritten) into y in natural order, y = result or y += result.
fm_status idft_from_split_order(Elem e, const Split& sp, void* p, void* y, int acc, hipStream_t s) {
  const int64_t L = int64_t(1) << sp.logL, n1 = int64_t(1) << sp.log1, n2 = int64_t(1) << sp.log2;
  FftLaunch f2;  // inverse row transforms (k1 -> n1), then W_L^-(n1 k2)
  f2.elem = e;
  f2.logn = sp.log1;
  f2.mode = FFT_INV;
  f2.b = Batch{1, n2, 1, L, n1, L, n1};
  f2.x = p;
  f2.y = p;
  f2.in_limit = f2.out_limit = n1;
  f2.tw_log = sp.logL;
  f2.tw_inv = 1;
  FM_TRY(launch_fft(f2, s));
  FftLaunch f3;  // inverse length-n2 transforms at stride n1 (k2 -> n2), natural order
  f3.elem = e;
  f3.logn = sp.log2;
  f3.mode = FFT_INV;
  f3.b = Batch{1, 1, n1, L, L, L, L};
  f3.x = p;
  f3.y = y;
  f3.in_limit = f3.out_limit = L;
  f3.accumulate = acc;
  return launch_fft(f3, s);
}

struct StepArgs {
  int64_t n, ncols, ld;
  const void* y;
  const void* g;
  const void* xo;
  void* xn;
  void* yn;
  void* z;
  const double* lam;
  double invL, beta;
};

// z = y - g/L; x_new = soft(z, lam_c/L); y_new = x_new + beta (x_new - x_old).
// The arithmetic is the solver's update, so a recomputed step reproduces the
// forward step bit for bit.
template <typename R>
__global__ __launch_bounds__(kTPB) void step_kernel(StepArgs a) {
  const R invL = R(a.invL);
  const R beta = R(a.beta);
  for (int64_t c = blockIdx.y; c < a.ncols; c += gridDim.y) {
    const int64_t i = int64_t(blockIdx.x) * kTPB + threadIdx.x;
    if (i >= a.n) continue;
    const int64_t o = c * a.ld + i;
    const R s = R(a.lam[c] * a.invL);
    const Cx<R> yv = static_cast<const Cx<R>*>(a.y)[o];
    const Cx<R> gv = static_cast<const Cx<R>*>(a.g)[o];
    const Cx<R> xo = static_cast<const Cx<R>*>(a.xo)[o];
    const Cx<R> z = {yv.x - gv.x * invL, yv.y - gv.y * invL};
    const Cx<R> xn = soft(z, s);
    const Cx<R> d = {xn.x - xo.x, xn.y - xo.y};
    static_cast<Cx<R>*>(a.xn)[o] = xn;
    static_cast<Cx<R>*>(a.yn)[o] = {xn.x + beta * d.x, xn.y + beta * d.y};
    if (a.z) static_cast<Cx<R>*>(a.z)[o] = z;
  }
}

struct VjpArgs {
  int64_t n, ncols, ld;
  const void* z;
  const void* gxn;
  const void* gyn;
  void* gz;
  void* gg;
  void* gxo;
  const double* lam;
  double invL, beta;
};

// Reverse of step_kernel. With xt = gx_new + (1 + beta) gy_new (the whole
// gradient reaching x_new) and s = lam_c/L:
//   |z| > s: gz = xt (1 - s/(2|z|)) + conj(xt) s z^2 / (2|z|^3);  else 0
//   gg = -gz/L,  gx_old = -beta gy_new.
template <typename R>
__global__ __launch_bounds__(kTPB) void step_vjp_kernel(VjpArgs a) {
  const R invL = R(a.invL);
  const R beta = R(a.beta);
  for (int64_t c = blockIdx.y; c < a.ncols; c += gridDim.y) {
    const int64_t i = int64_t(blockIdx.x) * kTPB + threadIdx.x;
    if (i >= a.n) continue;
    const int64_t o = c * a.ld + i;
    const R s = R(a.lam[c] * a.invL);
    const Cx<R> z = static_cast<const Cx<R>*>(a.z)[o];
    const Cx<R> gx = static_cast<const Cx<R>*>(a.gxn)[o];
    const Cx<R> gy = static_cast<const Cx<R>*>(a.gyn)[o];
    const Cx<R> xt = {gx.x + (R(1) + beta) * gy.x, gx.y + (R(1) + beta) * gy.y};
    Cx<R> gz = {R(0), R(0)};
    const R m2 = z.x * z.x + z.y * z.y;
    const R m = sqrt(m2);
    if (m > s) {
      const R a1 = R(1) - s / (R(2) * m);
      const R a2 = s / (R(2) * m * m2);
      const Cx<R> z2 = {z.x * z.x - z.y * z.y, R(2) * z.x * z.y};
      const Cx<R> cz = cmul(cconj(xt), z2);
      gz = {a1 * xt.x + a2 * cz.x, a1 * xt.y + a2 * cz.y};
    }
    if (a.gxo) static_cast<Cx<R>*>(a.gxo)[o] = {-beta * gy.x, -beta * gy.y};
    static_cast<Cx<R>*>(a.gz)[o] = gz;
    if (a.gg) static_cast<Cx<R>*>(a.gg)[o] = {-gz.x * invL, -gz.y * invL};
  }
}

template <typename R>
__global__ __launch_bounds__(kTPB) void axpby_kernel(int64_t n, int64_t ncols, R alpha, const Cx<R>* x, int64_t ldx,
                                                     R beta, const Cx<R>* y, int64_t ldy, Cx<R>* out, int64_t ldo) {
  for (int64_t c = blockIdx.y; c < ncols; c += gridDim.y) {
    const int64_t i = int64_t(blockIdx.x) * kTPB + threadIdx.x;
    if (i >= n) continue;
    const Cx<R> xv = x[c * ldx + i], yv = y[c * ldy + i];
    out[c * ldo + i] = {alpha * xv.x + beta * yv.x, alpha * xv.y + beta * yv.y};
  }
}

// Per-block maximum of |v|^2 (mode 0) or sum of |v|^2 (mode 1) over a
// complex128 array, then one work-group reduces the partials in a fixed order.
__device__ __forceinline__ double combine(double a, double b, int mode) {
  return mode == 0 ? (a > b ? a : b) : a + b;
}

__device__ __forceinline__ double block_reduce(double acc, int mode, double* sm) {
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kTPB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] = combine(sm[threadIdx.x], sm[threadIdx.x + w], mode);
    __syncthreads();
  }
  return sm[0];
}

__global__ __launch_bounds__(kTPB) void mag2_partial_kernel(int64_t count, const c128* __restrict__ v, int mode,
                                                            double* part) {
  __shared__ double sm[kTPB];
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kTPB + threadIdx.x; i < count; i += int64_t(gridDim.x) * kTPB)
    acc = combine(acc, v[i].x * v[i].x + v[i].y * v[i].y, mode);
  const double r = block_reduce(acc, mode, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ __launch_bounds__(kTPB) void mag2_final_kernel(int nparts, const double* __restrict__ part, int mode,
                                                          double* out) {
  __shared__ double sm[kTPB];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kTPB) acc = combine(acc, part[i], mode);
  const double r = block_reduce(acc, mode, sm);
  if (threadIdx.x == 0) *out = r;
}

dim3 grid2(int64_t n, int64_t ncols) {
  return dim3(unsigned(cdiv(n, kTPB)), unsigned(std::min<int64_t>(ncols, 65535)));
}

// max (mode 0) or sum (mode 1) of |v_i|^2 over count complex128 values;
// synchronises the stream.
fm_status mag2(const void* v, int64_t count, int mode, double* out, hipStream_t s) {
  const int nb = int(std::min<int64_t>(256, std::max<int64_t>(1, cdiv(count, kTPB))));
  DevBuf part;
  FM_TRY(part.alloc(size_t(nb + 1) * sizeof(double)));
  double* pp = static_cast<double*>(part.p);
  hipLaunchKernelGGL(mag2_partial_kernel, dim3(nb), dim3(kTPB), 0, s, count, static_cast<const c128*>(v), mode, pp);
  FM_LAUNCHED();
  hipLaunchKernelGGL(mag2_final_kernel, dim3(1), dim3(kTPB), 0, s, nb, pp, mode, pp + nb);
  FM_LAUNCHED();
  double h = 0.0;
  FM_HIP(hipMemcpyAsync(&h, pp + nb, sizeof(double), hipMemcpyDeviceToHost, s));
  FM_HIP(hipStreamSynchronize(s));
  *out = h;
  return FM_OK;
}

// Upper bound of ||op||_2^2 from the operator's structure.
fm_status norm_bound(const fm_op_s* op, hipStream_t s, double* out) {
  double v = 0.0;
  switch (op->kind) {
    case Kind::Fourier:
    case Kind::Hadamard:
      *out = double(op->n);  // F^H F = n I, H^T H = n I
      return FM_OK;
    case Kind::Select:
      *out = 1.0;
      return FM_OK;
    case Kind::Diag:
      FM_TRY(mag2(op->p64.p, op->n, 0, &v, s));
      *out = v;
      return FM_OK;
    case Kind::Dense:  // Frobenius norm squared
      FM_TRY(mag2(op->p64.p, op->lda * op->n, 1, &v, s));
      *out = v;
      return FM_OK;
    case Kind::Circulant:
    case Kind::Toeplitz: {  // stored spectrum carries 1/L: ||T|| <= ||C_L|| = max |DFT_L(g)|
      FM_TRY(mag2(op->p64.p, op->L, 0, &v, s));
      *out = v * double(op->L) * double(op->L);
      return FM_OK;
    }
    case Kind::MLToeplitz: {
      int64_t total = 1;
      for (int64_t l : op->lL) total *= l;
      FM_TRY(mag2(op->p64.p, total, 0, &v, s));
      *out = v * double(total) * double(total);
      return FM_OK;
    }
    case Kind::Adjoint:
    case Kind::Conj:
      return norm_bound(op->terms[0], s, out);
    case Kind::Product:
    case Kind::Kron: {
      double p = 1.0;
      for (fm_op t : op->terms) {
        FM_TRY(norm_bound(t, s, &v));
        p *= v;
      }
      *out = p;
      return FM_OK;
    }
    case Kind::Sum: {
      double r = 0.0;
      for (fm_op t : op->terms) {
        FM_TRY(norm_bound(t, s, &v));
        r += std::sqrt(v);
      }
      *out = r * r;
      return FM_OK;
    }
    case Kind::BlkDiag: {
      double m = 0.0;
      for (fm_op t : op->terms) {
        FM_TRY(norm_bound(t, s, &v));
        m = std::max(m, v);
      }
      *out = m;
      return FM_OK;
    }
    case Kind::ToeplitzInv:
      set_error("norm bound: no structural bound for a Toeplitz inverse (use the power iteration)");
      return FM_E_UNSUPPORTED;
    case Kind::Blocks: {  // Schur test on the block norms: ||H||^2 <= max row sum * max column sum
      std::vector<double> rs(op->nbr, 0.0), cs(op->nbc, 0.0);
      for (int i = 0; i < op->nbr; ++i)
        for (int j = 0; j < op->nbc; ++j) {
          FM_TRY(norm_bound(op->terms[size_t(i) * op->nbc + j], s, &v));
          rs[i] += std::sqrt(v);
          cs[j] += std::sqrt(v);
        }
      *out = *std::max_element(rs.begin(), rs.end()) * *std::max_element(cs.begin(), cs.end());
      return FM_OK;
    }
  }
  set_error("norm bound: unknown operator kind");
  return FM_E_INVALID;
}

bool overlaps(const void* a, size_t alen, const void* b, size_t blen) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return !(x + alen <= y || y + blen <= x);
}

size_t block_bytes(int64_t rows, int64_t ncols, int64_t ld, size_t es) {
  return ncols > 0 ? size_t((ncols - 1) * ld + rows) * es : 0;
}

}  // namespace
}  // namespace fm

using namespace fm;

extern "C" {

fm_status fm_circulant_grad_generator(int64_t n, int64_t ncols, fm_dir use, const void* in, int64_t ld_in,
                                      const void* g, int64_t ld_g, void* grad_c, int32_t accumulate, fm_dtype dt,
                                      void* stream) {
  set_error("");
  FM_CHECK_ARG(dt == FM_C64 || dt == FM_C128, FM_E_DTYPE, "generator gradient needs a complex dtype");
  FM_CHECK_ARG(use == FM_FWD || use == FM_ADJ, FM_E_INVALID, "unknown direction");
  FM_CHECK_ARG(is_pow2(n) && ilog2(n) <= 20, FM_E_UNSUPPORTED, "circulant size %lld: powers of two up to 2^20",
               (long long)n);
  FM_CHECK_ARG(ncols >= 0, FM_E_INVALID, "negative column count");
  FM_CHECK_ARG(grad_c != nullptr, FM_E_INVALID, "NULL gradient pointer");
  const size_t es = elem_size(dt);
  const Elem e = elem_of(dt);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (ncols == 0) {
    if (!accumulate) FM_TRY(launch_zero2d(e, n, 1, grad_c, n, s));
    return FM_OK;
  }
  FM_CHECK_ARG(in != nullptr && g != nullptr, FM_E_INVALID, "NULL data pointer");
  FM_CHECK_ARG(ld_in >= n && ld_g >= n, FM_E_SHAPE, "leading dimensions below n");
  FM_CHECK_ARG(!overlaps(grad_c, size_t(n) * es, in, block_bytes(n, ncols, ld_in, es)) &&
                   !overlaps(grad_c, size_t(n) * es, g, block_bytes(n, ncols, ld_g, es)),
               FM_E_ALIAS, "gradient overlaps an input block");
  // correlation r[k] = sum_i a[i] conj(b[i-k]):  FWD: a = g, b = in;  ADJ: a = in, b = g
  const void* pa = use == FM_FWD ? g : in;
  const void* pb = use == FM_FWD ? in : g;
  const int64_t lda = use == FM_FWD ? ld_g : ld_in, ldb = use == FM_FWD ? ld_in : ld_g;
  fm_op F = nullptr;
  FM_TRY(fm_op_create_fourier(&F, n, dt));
  struct Release {
    fm_op f;
    ~Release() { fm_op_release(f); }
  } rel{F};
  // columns per chunk: two spectra blocks of at most 256 MiB together
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(ncols, (int64_t(256) << 20) / (2 * n * int64_t(es))));
  const int64_t maxg = corr_groups(n, chunk);
  const Split sp = split_for(e, ilog2(n));
  const bool split_order = sp.four_step();
  Workspace sz;
  sz.sizing = true;
  {
    size_t fft_ws = 0;
    if (!split_order) {
      Batch b{chunk, 1, 1, n, n, n, n};
      FM_TRY(exec(F, false, e, b, nullptr, nullptr, false, sz, s));
      fft_ws = sz.peak;
    }
    sz = Workspace{};
    sz.sizing = true;
    sz.take(size_t(2 * chunk * n) * es);
    sz.take(size_t(n) * es);
    sz.take(size_t(maxg * n) * es);
    sz.take(fft_ws);
  }
  // stream-ordered workspace: released after the last kernel that reads it,
  // without a host wait
  void* base = nullptr;
  FM_HIP(hipMallocAsync(&base, sz.peak, s));
  struct FreeAsync {
    void* p;
    hipStream_t s;
    ~FreeAsync() { (void)hipFreeAsync(p, s); }
  } fr{base, s};
  Workspace w;
  w.base = static_cast<char*>(base);
  w.cap = sz.peak;
  void* A = w.take(size_t(chunk * n) * es);
  void* B = w.take(size_t(chunk * n) * es);
  void* P = w.take(size_t(n) * es);
  void* part = w.take(size_t(maxg * n) * es);
  for (int64_t c0 = 0; c0 < ncols; c0 += chunk) {
    const int64_t nc = std::min(chunk, ncols - c0);
    Batch ba{nc, 1, 1, lda, n, n, n};
    Batch bb{nc, 1, 1, ldb, n, n, n};
    const void* xa = static_cast<const char*>(pa) + size_t(c0 * lda) * es;
    const void* xb = static_cast<const char*>(pb) + size_t(c0 * ldb) * es;
    if (split_order) {
      FM_TRY(dft_split_order(e, sp, nc, xa, lda, A, s));
      FM_TRY(dft_split_order(e, sp, nc, xb, ldb, B, s));
    } else {
      FM_TRY(exec(F, false, e, ba, xa, A, false, w, s));
      FM_TRY(exec(F, false, e, bb, xb, B, false, w, s));
    }
    const int64_t ng = corr_groups(n, nc);
    const int64_t cpg = cdiv(nc, ng);
    const int64_t ngu = cdiv(nc, cpg);  // groups that hold columns
    const dim3 g1(unsigned(cdiv(n, kTPB)), unsigned(ngu)), g2(unsigned(cdiv(n, kTPB)));
    if (dt == FM_C64) {
      hipLaunchKernelGGL(corr_part_kernel<float>, g1, dim3(kTPB), 0, s, n, nc, cpg, static_cast<const c64*>(A),
                         static_cast<const c64*>(B), static_cast<c64*>(part));
      hipLaunchKernelGGL(corr_sum_kernel<float>, g2, dim3(kTPB), 0, s, n, ngu, static_cast<const c64*>(part),
                         float(1.0 / double(n)), static_cast<c64*>(P), int(c0 > 0));
    } else {
      hipLaunchKernelGGL(corr_part_kernel<double>, g1, dim3(kTPB), 0, s, n, nc, cpg, static_cast<const c128*>(A),
                         static_cast<const c128*>(B), static_cast<c128*>(part));
      hipLaunchKernelGGL(corr_sum_kernel<double>, g2, dim3(kTPB), 0, s, n, ngu, static_cast<const c128*>(part),
                         1.0 / double(n), static_cast<c128*>(P), int(c0 > 0));
    }
    FM_LAUNCHED();
  }
  // grad_c (+)= unnormalised inverse DFT of P (the 1/n is already in P)
  if (split_order) return idft_from_split_order(e, sp, P, grad_c, accumulate != 0, s);
  Batch b1{1, 1, 1, n, n, n, n};
  FM_TRY(exec(F, true, e, b1, P, grad_c, accumulate != 0, w, s));
  return FM_OK;
}

fm_status fm_fista_step(int64_t n, int64_t ncols, const void* y, const void* g, const void* x_old, void* x_new,
                        void* y_new, void* z_out, int64_t ld, const double* lam, double L, int32_t iter,
                        int32_t momentum, fm_dtype dt, void* stream) {
  set_error("");
  FM_CHECK_ARG(dt == FM_C64 || dt == FM_C128, FM_E_DTYPE, "FISTA step needs a complex dtype");
  FM_CHECK_ARG(n >= 0 && ncols >= 0 && ld >= n, FM_E_SHAPE, "bad block shape");
  FM_CHECK_ARG(L > 0.0 && std::isfinite(L), FM_E_INVALID, "step constant L must be positive");
  FM_CHECK_ARG(iter >= 0, FM_E_INVALID, "iteration index must be non-negative");
  const double beta = fista_momentum(iter, momentum != 0);
  if (n == 0 || ncols == 0) return FM_OK;
  FM_CHECK_ARG(y && g && x_old && x_new && y_new && lam, FM_E_INVALID, "NULL pointer");
  const size_t bytes = block_bytes(n, ncols, ld, elem_size(dt));
  FM_CHECK_ARG(!overlaps(x_new, bytes, y_new, bytes), FM_E_ALIAS, "x_new and y_new overlap");
  FM_CHECK_ARG(!z_out || (!overlaps(z_out, bytes, x_new, bytes) && !overlaps(z_out, bytes, y_new, bytes)),
               FM_E_ALIAS, "z overlaps an output");
  StepArgs a{n, ncols, ld, y, g, x_old, x_new, y_new, z_out, lam, 1.0 / L, beta};
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (dt == FM_C64)
    hipLaunchKernelGGL(step_kernel<float>, grid2(n, ncols), dim3(kTPB), 0, s, a);
  else
    hipLaunchKernelGGL(step_kernel<double>, grid2(n, ncols), dim3(kTPB), 0, s, a);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status fm_fista_step_vjp(int64_t n, int64_t ncols, const void* z, const void* gx_new, const void* gy_new,
                            void* gz, void* gg, void* gx_old, int64_t ld, const double* lam, double L, int32_t iter,
                            int32_t momentum, fm_dtype dt, void* stream) {
  set_error("");
  FM_CHECK_ARG(dt == FM_C64 || dt == FM_C128, FM_E_DTYPE, "FISTA step needs a complex dtype");
  FM_CHECK_ARG(n >= 0 && ncols >= 0 && ld >= n, FM_E_SHAPE, "bad block shape");
  FM_CHECK_ARG(L > 0.0 && std::isfinite(L), FM_E_INVALID, "step constant L must be positive");
  FM_CHECK_ARG(iter >= 0, FM_E_INVALID, "iteration index must be non-negative");
  const double beta = fista_momentum(iter, momentum != 0);
  if (n == 0 || ncols == 0) return FM_OK;
  FM_CHECK_ARG(z && gx_new && gy_new && gz && lam, FM_E_INVALID, "NULL pointer");
  const size_t bytes = block_bytes(n, ncols, ld, elem_size(dt));
  FM_CHECK_ARG(!overlaps(gz, bytes, z, bytes), FM_E_ALIAS, "gz overlaps z");
  FM_CHECK_ARG(!gg || (!overlaps(gg, bytes, gz, bytes) && (gg == gx_new || !overlaps(gg, bytes, gx_new, bytes)) &&
                       (gg == gy_new || !overlaps(gg, bytes, gy_new, bytes))),
               FM_E_ALIAS, "gg overlaps another block");
  FM_CHECK_ARG(!gx_old || (!overlaps(gx_old, bytes, gz, bytes) && (!gg || !overlaps(gx_old, bytes, gg, bytes)) &&
                           (gx_old == gx_new || !overlaps(gx_old, bytes, gx_new, bytes)) &&
                           (gx_old == gy_new || !overlaps(gx_old, bytes, gy_new, bytes))),
               FM_E_ALIAS, "gx_old overlaps another block");
  FM_CHECK_ARG((gz == gx_new || !overlaps(gz, bytes, gx_new, bytes)) &&
                   (gz == gy_new || !overlaps(gz, bytes, gy_new, bytes)),
               FM_E_ALIAS, "gz partially overlaps an upstream gradient");
  VjpArgs a{n, ncols, ld, z, gx_new, gy_new, gz, gg, gx_old, lam, 1.0 / L, beta};
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (dt == FM_C64)
    hipLaunchKernelGGL(step_vjp_kernel<float>, grid2(n, ncols), dim3(kTPB), 0, s, a);
  else
    hipLaunchKernelGGL(step_vjp_kernel<double>, grid2(n, ncols), dim3(kTPB), 0, s, a);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status fm_fista_momentum(int32_t iter, int32_t momentum, double* beta) {
  set_error("");
  FM_CHECK_ARG(beta != nullptr, FM_E_INVALID, "NULL output");
  FM_CHECK_ARG(iter >= 0, FM_E_INVALID, "iteration index must be non-negative");
  *beta = fista_momentum(iter, momentum != 0);
  return FM_OK;
}

fm_status fm_axpby(int64_t n, int64_t ncols, double alpha, const void* x, int64_t ldx, double beta, const void* y,
                   int64_t ldy, void* out, int64_t ldo, fm_dtype dt, void* stream) {
  set_error("");
  FM_CHECK_ARG(dt == FM_C64 || dt == FM_C128, FM_E_DTYPE, "axpby needs a complex dtype");
  FM_CHECK_ARG(n >= 0 && ncols >= 0 && ldx >= n && ldy >= n && ldo >= n, FM_E_SHAPE, "bad block shape");
  if (n == 0 || ncols == 0) return FM_OK;
  FM_CHECK_ARG(x && y && out, FM_E_INVALID, "NULL pointer");
  const size_t es = elem_size(dt);
  const size_t ob = block_bytes(n, ncols, ldo, es);
  FM_CHECK_ARG((out == x && ldo == ldx) || !overlaps(out, ob, x, block_bytes(n, ncols, ldx, es)), FM_E_ALIAS,
               "out partially overlaps x");
  FM_CHECK_ARG((out == y && ldo == ldy) || !overlaps(out, ob, y, block_bytes(n, ncols, ldy, es)), FM_E_ALIAS,
               "out partially overlaps y");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (dt == FM_C64)
    hipLaunchKernelGGL(axpby_kernel<float>, grid2(n, ncols), dim3(kTPB), 0, s, n, ncols, float(alpha),
                       static_cast<const c64*>(x), ldx, float(beta), static_cast<const c64*>(y), ldy,
                       static_cast<c64*>(out), ldo);
  else
    hipLaunchKernelGGL(axpby_kernel<double>, grid2(n, ncols), dim3(kTPB), 0, s, n, ncols, alpha,
                       static_cast<const c128*>(x), ldx, beta, static_cast<const c128*>(y), ldy,
                       static_cast<c128*>(out), ldo);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status fm_op_norm_bound(fm_op a, double* bound, void* stream) {
  set_error("");
  FM_CHECK_ARG(a != nullptr, FM_E_INVALID, "operator handle is NULL");
  FM_CHECK_ARG(op_alive(a), FM_E_RELEASED, "operator handle was released");
  FM_CHECK_ARG(bound != nullptr, FM_E_INVALID, "NULL output");
  int dev = 0;
  FM_HIP(hipGetDevice(&dev));
  FM_CHECK_ARG(dev == a->device, FM_E_DEVICE, "operator lives on device %d, current is %d", a->device, dev);
  return norm_bound(a, reinterpret_cast<hipStream_t>(stream), bound);
}

}  // extern "C"
