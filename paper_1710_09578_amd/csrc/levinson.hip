// Levinson recursion for a general (not necessarily Hermitian) n x n
// Toeplitz system T x = b: the inverse of the Toeplitz operator (section
// "General Matrix-free Representations", the inverse of the base-class
// feature table), applied in O(n^2) per right-hand side without forming T.
//
// With T_k the leading k x k block, the recursion keeps the forward vector
// f (T_k f = e_1), the backward vector g (T_k g = e_k) and the partial
// solution x (T_k x = b_0..k-1). Extending each by a zero, the row below
// (resp. the row above) meets the errors
//   ef = sum_j t_{k-j} f_j,   eg = sum_j t_{-(j+1)} g_j,   ex = sum_j t_{k-j} x_j,
// so that with s = 1 / (1 - ef eg)
//   f' = s ([f; 0] - ef [0; g]),   g' = s ([0; g] - eg [f; 0]),
//   x' = [x; 0] + (b_k - ex) g'
// solve the (k+1) x (k+1) problems. One work-group per right-hand side; the
// three dot products of a step share one reduction.
#include "kernels.h"

namespace fm {
namespace {

template <typename R>
__device__ __forceinline__ R wsum(R v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

struct LevArgs {
  int64_t n, L;
  const c128* gen;
  int adjoint;
  const void* b;
  int64_t ldb;
  void* x;
  int64_t ldx;
  void* work;  // per column: f, g (two buffers)
};

template <typename R, int NT>
__global__ __launch_bounds__(NT) void levinson_kernel(LevArgs a) {
  constexpr int NW = NT / 64;
  __shared__ R red[6 * NW];
  const int64_t col = blockIdx.x;
  const int64_t n = a.n;
  Cx<R>* f = static_cast<Cx<R>*>(a.work) + col * 3 * n;
  Cx<R>* gbuf[2] = {f + n, f + 2 * n};
  const Cx<R>* B = static_cast<const Cx<R>*>(a.b) + col * a.ldb;
  Cx<R>* X = static_cast<Cx<R>*>(a.x) + col * a.ldx;
  // generator entry t_k (adjoint: conj(t_{-k}))
  auto t = [&](int64_t k) -> Cx<R> {
    const int64_t kk = a.adjoint ? -k : k;
    const c128 v = a.gen[kk >= 0 ? kk : a.L + kk];
    return {R(v.x), R(a.adjoint ? -v.y : v.y)};
  };
  const Cx<R> t0 = t(0);
  const R d0 = t0.x * t0.x + t0.y * t0.y;
  bool bad = !(d0 > R(0));
  if (threadIdx.x == 0 && !bad) {
    const Cx<R> inv = {t0.x / d0, -t0.y / d0};
    f[0] = inv;
    gbuf[0][0] = inv;
    X[0] = cmul(B[0], inv);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t k = 1; k < n && !bad; ++k) {
    const Cx<R>* g = gbuf[cur];
    Cx<R>* gn = gbuf[cur ^ 1];
    Cx<R> ef = {R(0), R(0)}, eg = {R(0), R(0)}, ex = {R(0), R(0)};
    for (int64_t j = threadIdx.x; j < k; j += NT) {
      const Cx<R> tk = t(k - j);
      ef = cadd(ef, cmul(tk, f[j]));
      ex = cadd(ex, cmul(tk, X[j]));
      eg = cadd(eg, cmul(t(-(j + 1)), g[j]));
    }
    R v[6] = {wsum(ef.x), wsum(ef.y), wsum(eg.x), wsum(eg.y), wsum(ex.x), wsum(ex.y)};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
      for (int q = 0; q < 6; ++q) red[q * NW + wave] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      R sacc = R(0);
      for (int w = 0; w < NW; ++w) sacc += red[q * NW + w];
      v[q] = sacc;
    }
    __syncthreads();
    ef = {v[0], v[1]};
    eg = {v[2], v[3]};
    ex = {v[4], v[5]};
    const Cx<R> den = csub(Cx<R>{R(1), R(0)}, cmul(ef, eg));
    const R dd = den.x * den.x + den.y * den.y;
    if (!(dd > R(0)) || !(dd < R(1e30))) {
      bad = true;
      break;
    }
    const Cx<R> s = {den.x / dd, -den.y / dd};
    const Cx<R> coef = csub(B[k], ex);
    for (int64_t i = threadIdx.x; i <= k; i += NT) {
      const Cx<R> fo = i < k ? f[i] : Cx<R>{R(0), R(0)};
      const Cx<R> go = i > 0 ? g[i - 1] : Cx<R>{R(0), R(0)};
      const Cx<R> fnew = cmul(csub(fo, cmul(ef, go)), s);
      const Cx<R> gnew = cmul(csub(go, cmul(eg, fo)), s);
      f[i] = fnew;
      gn[i] = gnew;
      const Cx<R> xo = i < k ? X[i] : Cx<R>{R(0), R(0)};
      X[i] = cadd(xo, cmul(coef, gnew));
    }
    __syncthreads();
    cur ^= 1;
  }
  if (bad) {  // singular leading minor: the column gets NaN
    const R nan = R(0) / R(0);
    for (int64_t i = threadIdx.x; i < n; i += NT) X[i] = {nan, nan};
  }
}

}  // namespace

fm_status launch_levinson(Elem e, int64_t n, int64_t L, const void* gen, int adjoint, int64_t ncols, const void* b,
                          int64_t ldb, void* x, int64_t ldx, void* work, hipStream_t s) {
  if (ncols == 0 || n == 0) return FM_OK;
  FM_CHECK_ARG(ncols < 65536, FM_E_UNSUPPORTED, "Levinson: at most 65535 columns per call");
  LevArgs a{n, L, static_cast<const c128*>(gen), adjoint, b, ldb, x, ldx, work};
  constexpr int NT = 256;
  if (e == Elem::C64)
    hipLaunchKernelGGL((levinson_kernel<float, NT>), dim3(unsigned(ncols)), dim3(NT), 0, s, a);
  else if (e == Elem::C128)
    hipLaunchKernelGGL((levinson_kernel<double, NT>), dim3(unsigned(ncols)), dim3(NT), 0, s, a);
  else {
    set_error("Levinson: integer element type");
    return FM_E_DTYPE;
  }
  FM_LAUNCHED();
  return FM_OK;
}

}  // namespace fm
