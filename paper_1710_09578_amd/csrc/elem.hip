// Elementwise and data-movement kernels: Diag, row selection (gather /
// scatter), the generic dense mode product, zero-pad / crop boxes, precision
// conversions, spectrum permutation, Toeplitz embedding and index checks.
#include <cstdlib>

#include "kernels.h"

namespace fm {
namespace {

template <typename V>
struct Ops;
template <>
struct Ops<c64> {
  using R = float;
  static __device__ __forceinline__ c64 add(c64 a, c64 b) { return cadd(a, b); }
  static __device__ __forceinline__ c64 zero() { return {0.f, 0.f}; }
};
template <>
struct Ops<c128> {
  using R = double;
  static __device__ __forceinline__ c128 add(c128 a, c128 b) { return cadd(a, b); }
  static __device__ __forceinline__ c128 zero() { return {0.0, 0.0}; }
};
template <>
struct Ops<int32_t> {
  static __device__ __forceinline__ int32_t add(int32_t a, int32_t b) {
    return int32_t(uint32_t(a) + uint32_t(b));
  }
  static __device__ __forceinline__ int32_t zero() { return 0; }
};
template <>
struct Ops<int64_t> {
  static __device__ __forceinline__ int64_t add(int64_t a, int64_t b) {
    return int64_t(uint64_t(a) + uint64_t(b));
  }
  static __device__ __forceinline__ int64_t zero() { return 0; }
};

template <typename V>
__device__ __forceinline__ void store(V* p, V v, int acc) {
  *p = acc ? Ops<V>::add(*p, v) : v;
}

// Grid: x over the flat (row, inner) positions of one vector, y over
// (column, outer) pairs (grid-strided).
struct VecGrid {
  int64_t pairs;   // ncols * outer
  int64_t flat;    // positions per output vector
};

inline dim3 vec_grid(int64_t pairs, int64_t flat, int threads) {
  const int64_t gx = cdiv(flat, threads);
  const int64_t gy = pairs < 65535 ? pairs : 65535;
  return dim3(unsigned(gx), unsigned(gy));
}

template <typename V>
__global__ __launch_bounds__(256) void diag_kernel(int64_t n, Batch b, const V* __restrict__ d,
                                                   int conj, const V* __restrict__ x, V* y, int acc) {
  const int64_t flat_n = n * b.inner;
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= flat_n) return;
  const int64_t r = b.inner == 1 ? f : f / b.inner;
  const V dv = d[r];
  for (int64_t p = blockIdx.y; p < b.ncols * b.outer; p += gridDim.y) {
    const int64_t c = p / b.outer, o = p - c * b.outer;
    const V xv = x[c * b.ldx + o * b.xvs + f];
    store(y + c * b.ldy + o * b.yvs + f, conj ? cmulc(xv, dv) : cmul(xv, dv), acc);
  }
}

// Spectral mixing of a block matrix. The spectra are packed bin-tiled:
// S[((f / TW) nb + o ld + p) TW + f % TW] for block (o, p) (nb blocks, TW
// bins per tile), so the 64 lanes of a wave (64 consecutive bins, TW = 64)
// read 512 contiguous bytes per block and a work-group's reads stay inside one
// compact region. One thread per bin and column, OB outputs per work-group
// row; the inputs of PC blocks are held in registers while the OB x PC
// spectrum values of a chunk stream in, all loads of a chunk in flight
// together; the OB sums stay in registers over the chunks.
struct MixArgs {
  int nout, nin, ld, adjoint, logtw;
  int64_t total, ncols, nb;
  const void* spec;
  const void* x;
  void* y;
};

template <typename R, int OB, int PC>
__global__ __launch_bounds__(256) void block_mix_kernel(MixArgs a) {
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= a.total) return;
  const Cx<R>* X = static_cast<const Cx<R>*>(a.x);
  Cx<R>* Y = static_cast<Cx<R>*>(a.y);
  const int tw = 1 << a.logtw;
  const Cx<R>* S = static_cast<const Cx<R>*>(a.spec) + (f >> a.logtw) * a.nb * tw + (f & (tw - 1));
  const int o0 = int(blockIdx.z) * OB;
  const int no = a.nout - o0 < OB ? a.nout - o0 : OB;
  for (int64_t c = blockIdx.y; c < a.ncols; c += gridDim.y) {
    Cx<R> acc[OB];
#pragma unroll
    for (int k = 0; k < OB; ++k) acc[k] = {R(0), R(0)};
    for (int p0 = 0; p0 < a.nin; p0 += PC) {
      Cx<R> xr[PC];
#pragma unroll
      for (int q = 0; q < PC; ++q)
        xr[q] = p0 + q < a.nin ? X[(int64_t(p0 + q) * a.ncols + c) * a.total + f] : Cx<R>{R(0), R(0)};
#pragma unroll
      for (int k = 0; k < OB; ++k) {
        if (k < no) {
          const int o = o0 + k;
          Cx<R> sv[PC];
#pragma unroll
          for (int q = 0; q < PC; ++q) {
            const int p = p0 + q;
            const int64_t blk = a.adjoint ? int64_t(p) * a.ld + o : int64_t(o) * a.ld + p;
            sv[q] = p < a.nin ? S[blk * tw] : Cx<R>{R(0), R(0)};
          }
#pragma unroll
          for (int q = 0; q < PC; ++q)
            acc[k] = cadd(acc[k], a.adjoint ? cmulc(xr[q], sv[q]) : cmul(xr[q], sv[q]));
        }
      }
    }
#pragma unroll
    for (int k = 0; k < OB; ++k)
      if (k < no) Y[(int64_t(o0 + k) * a.ncols + c) * a.total + f] = acc[k];
  }
}

// Packs nb spectra (table of device pointers, total bins each) bin-tiled as
// read by block_mix_kernel.
template <typename R>
__global__ __launch_bounds__(256) void block_pack_kernel(int64_t nb, int64_t total, int logtw,
                                                         const void* const* table, Cx<R>* out) {
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= total) return;
  const int tw = 1 << logtw;
  for (int64_t k = blockIdx.y; k < nb; k += gridDim.y) {
    const Cx<R>* src = static_cast<const Cx<R>*>(table[k]);
    out[((f >> logtw) * nb + k) * tw + (f & (tw - 1))] = src[f];
  }
}

template <typename V>
__global__ __launch_bounds__(256) void gather_kernel(int64_t m, Batch b, const int32_t* __restrict__ idx,
                                                     const V* __restrict__ x, V* y, int acc) {
  const int64_t flat_m = m * b.inner;
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= flat_m) return;
  const int64_t r = b.inner == 1 ? f : f / b.inner;
  const int64_t i = f - r * b.inner;
  const int64_t src = int64_t(idx[r]) * b.inner + i;
  for (int64_t p = blockIdx.y; p < b.ncols * b.outer; p += gridDim.y) {
    const int64_t c = p / b.outer, o = p - c * b.outer;
    store(y + c * b.ldy + o * b.yvs + f, x[c * b.ldx + o * b.xvs + src], acc);
  }
}

template <typename V>
__global__ __launch_bounds__(256) void scatter_kernel(int64_t m, Batch b, const int32_t* __restrict__ idx,
                                                      const V* __restrict__ x, V* y, int acc) {
  const int64_t flat_m = m * b.inner;
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= flat_m) return;
  const int64_t r = b.inner == 1 ? f : f / b.inner;
  const int64_t i = f - r * b.inner;
  const int64_t dst = int64_t(idx[r]) * b.inner + i;
  for (int64_t p = blockIdx.y; p < b.ncols * b.outer; p += gridDim.y) {
    const int64_t c = p / b.outer, o = p - c * b.outer;
    store(y + c * b.ldy + o * b.yvs + dst, x[c * b.ldx + o * b.xvs + f], acc);
  }
}

// Adjoint of a row selection in one pass over the output: y[r] = x[inv[r]]
// where row r is selected (inv[r] >= 0), 0 elsewhere (nothing added with acc).
template <typename V>
__global__ __launch_bounds__(256) void expand_kernel(int64_t n_in, Batch b, const int32_t* __restrict__ inv,
                                                     const V* __restrict__ x, V* y, int acc) {
  const int64_t flat_n = n_in * b.inner;
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= flat_n) return;
  const int64_t r = b.inner == 1 ? f : f / b.inner;
  const int64_t i = f - r * b.inner;
  const int32_t k = inv[r];
  if (acc && k < 0) return;
  for (int64_t p = blockIdx.y; p < b.ncols * b.outer; p += gridDim.y) {
    const int64_t c = p / b.outer, o = p - c * b.outer;
    const V v = k >= 0 ? x[c * b.ldx + o * b.xvs + int64_t(k) * b.inner + i] : V{};
    store(y + c * b.ldy + o * b.yvs + f, v, acc);
  }
}

// expand_kernel for complex64 contiguous vectors without accumulation, two
// positions per thread and one 16-byte store (y 16-byte aligned, ldy even).
__global__ __launch_bounds__(256) void expand_pair_kernel(int64_t n_in, Batch b, const int32_t* __restrict__ inv,
                                                          const c64* __restrict__ x, c64* y) {
  const int64_t f = 2 * (int64_t(blockIdx.x) * blockDim.x + threadIdx.x);
  if (f >= n_in) return;
  const bool two = f + 1 < n_in;
  const int32_t k0 = inv[f];
  const int32_t k1 = two ? inv[f + 1] : -1;
  for (int64_t p = blockIdx.y; p < b.ncols; p += gridDim.y) {
    const c64* xc = x + p * b.ldx;
    c64* yc = y + p * b.ldy;
    const c64 v0 = k0 >= 0 ? xc[k0] : c64{0.f, 0.f};
    const c64 v1 = k1 >= 0 ? xc[k1] : c64{0.f, 0.f};
    if (two)
      *reinterpret_cast<float4*>(yc + f) = float4{v0.x, v0.y, v1.x, v1.y};
    else
      yc[f] = v0;
  }
}

template <typename V>
__global__ __launch_bounds__(256) void copy_kernel(int64_t flat_n, Batch b, const V* __restrict__ x, V* y,
                                                   int acc) {
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= flat_n) return;
  for (int64_t p = blockIdx.y; p < b.ncols * b.outer; p += gridDim.y) {
    const int64_t c = p / b.outer, o = p - c * b.outer;
    store(y + c * b.ldy + o * b.yvs + f, x[c * b.ldx + o * b.xvs + f], acc);
  }
}

template <typename R>
__global__ __launch_bounds__(256) void conj_kernel(int64_t flat_n, Batch b, const Cx<R>* x, Cx<R>* y,
                                                   int acc) {
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= flat_n) return;
  for (int64_t p = blockIdx.y; p < b.ncols * b.outer; p += gridDim.y) {
    const int64_t c = p / b.outer, o = p - c * b.outer;
    const Cx<R> v = cconj(x[c * b.ldx + o * b.xvs + f]);
    Cx<R>* d = y + c * b.ldy + o * b.yvs + f;
    *d = acc ? cadd(*d, v) : v;
  }
}

// Elementwise map of complex128 parameters: mode 0 out = scale |in|^2,
// mode 1 out = scale / in (flag[0] set when an entry is zero or not finite).
__global__ __launch_bounds__(256) void param_map_kernel(int64_t count, int mode, double scale,
                                                        const c128* __restrict__ in, c128* out, int* flag) {
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= count) return;
  const c128 v = in[f];
  const double m2 = v.x * v.x + v.y * v.y;
  if (mode == 0) {
    out[f] = {scale * m2, 0.0};
  } else {
    if (!(m2 > 0.0) || !(m2 < 1e300)) {
      flag[0] = 1;
      out[f] = {0.0, 0.0};
    } else {
      out[f] = {scale * v.x / m2, -scale * v.y / m2};
    }
  }
}

template <typename V>
__global__ __launch_bounds__(256) void zero_kernel(int64_t flat_n, Batch b, V* y) {
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= flat_n) return;
  for (int64_t p = blockIdx.y; p < b.ncols * b.outer; p += gridDim.y) {
    const int64_t c = p / b.outer, o = p - c * b.outer;
    y[c * b.ldy + o * b.yvs + f] = Ops<V>::zero();
  }
}

// y[c,o,r,i] (+)= sum_k A[r,k] x[c,o,k,i]      (forward, r < m, k < n)
// y[c,o,r,i] (+)= sum_k conj(A[k,r]) x[c,o,k,i] (adjoint, r < n, k < m)
template <typename V>
__global__ __launch_bounds__(256) void dense_kernel(int64_t m, int64_t n, const V* __restrict__ a,
                                                    int64_t lda, int adj, Batch b,
                                                    const V* __restrict__ x, V* y, int acc) {
  const int64_t rows_out = adj ? n : m, rows_in = adj ? m : n;
  const int64_t flat_n = rows_out * b.inner;
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= flat_n) return;
  const int64_t r = b.inner == 1 ? f : f / b.inner;
  const int64_t i = f - r * b.inner;
  for (int64_t p = blockIdx.y; p < b.ncols * b.outer; p += gridDim.y) {
    const int64_t c = p / b.outer, o = p - c * b.outer;
    const V* X = x + c * b.ldx + o * b.xvs + i;
    V s = Ops<V>::zero();
    for (int64_t k = 0; k < rows_in; ++k) {
      const V xv = X[k * b.inner];
      s = adj ? cadd(s, cmulc(xv, a[k + r * lda])) : cadd(s, cmul(a[r + k * lda], xv));
    }
    store(y + c * b.ldy + o * b.yvs + f, s, acc);
  }
}

// Dense mode product along the contiguous axis (inner == 1) for small
// factors: one vector per thread. A work-group copies op(A) into LDS (zero-
// padded to NMAX columns, conjugate-transposed for the adjoint, real parts
// only when A is real), stages 256 input vectors through LDS (coalesced
// loads), keeps each thread's vector in registers and forms every output row
// from broadcast LDS reads of the matrix; the outputs leave through LDS again
// (coalesced stores).
constexpr int kDV = 256;  // vectors per work-group

template <typename V, int NMAX, bool REAL>
constexpr size_t dense_vec_abytes(int nout) {
  return (size_t(nout) * NMAX * (REAL ? 1 : 2) * sizeof(typename Ops<V>::R) + 15) & ~size_t(15);
}

template <typename V, int NMAX, bool REAL, bool ADJ>
__global__ __launch_bounds__(kDV) void dense_vec_kernel(int64_t m, int64_t n, const V* __restrict__ a, int64_t lda,
                                                        Batch b, const V* __restrict__ x, V* y, int acc) {
  using R = typename Ops<V>::R;
  constexpr int C = REAL ? 1 : 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nin = int(ADJ ? m : n), nout = int(ADJ ? n : m);
  R* amat = reinterpret_cast<R*>(smem_raw);
  V* lds = reinterpret_cast<V*>(smem_raw + dense_vec_abytes<V, NMAX, REAL>(nout));
  const int stride = (nin > nout ? nin : nout) + 1;  // odd padding spreads the banks
  const int64_t P = b.ncols * b.outer;
  const int64_t p0 = int64_t(blockIdx.x) * kDV;
  const int nv = int(P - p0 < kDV ? P - p0 : kDV);
  const int t = threadIdx.x;
  // ---- op(A) row by row: amat[(r*NMAX + k)*C + {0,1}]
  for (int idx = t; idx < nout * NMAX; idx += kDV) {
    const int r = idx / NMAX, k = idx - r * NMAX;
    V v = Ops<V>::zero();
    if (k < nin) {
      v = ADJ ? a[k + int64_t(r) * lda] : a[r + int64_t(k) * lda];
      if (ADJ) v.y = -v.y;
    }
    amat[idx * C] = v.x;
    if constexpr (!REAL) amat[idx * C + 1] = v.y;
  }
  const bool packed = b.outer == 1 || b.ldx == b.outer * b.xvs;
  const bool packed_y = b.outer == 1 || b.ldy == b.outer * b.yvs;
  // ---- stage the inputs: element e = v*nin + k of the tile (at most NMAX per
  // thread). When the vectors are adjacent the tile is one contiguous array
  // and all its loads are issued before the first LDS store.
  const int64_t vstride = b.outer == 1 ? b.ldx : b.xvs;
  if (packed && vstride == nin) {
    const V* src = x + p0 * nin;
    V ld[NMAX];
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
      const int e = t + kDV * i;
      ld[i] = e < nv * nin ? src[e] : Ops<V>::zero();
    }
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
      const int e = t + kDV * i;
      if (e < nv * nin) {
        const int v = e / nin, k = e - v * nin;
        lds[v * stride + k] = ld[i];
      }
    }
  } else {
    int v = t / nin, k = t % nin;
    const int dv = kDV / nin, dk = kDV % nin;
    for (int e = t; e < nv * nin; e += kDV) {
      const int64_t p = p0 + v;
      const int64_t off = packed ? p * vstride : (p / b.outer) * b.ldx + (p % b.outer) * b.xvs;
      lds[v * stride + k] = x[off + k];
      v += dv;
      k += dk;
      if (k >= nin) {
        k -= nin;
        ++v;
      }
    }
  }
  __syncthreads();
  V xv[NMAX];
#pragma unroll
  for (int k = 0; k < NMAX; ++k) xv[k] = (k < nin && t < nv) ? lds[t * stride + k] : Ops<V>::zero();
  __syncthreads();
  for (int r = 0; r < nout; ++r) {
    const R* ar = amat + r * NMAX * C;
    R sr = R(0), si = R(0);
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
      if constexpr (REAL) {
        sr += ar[k] * xv[k].x;
        si += ar[k] * xv[k].y;
      } else {
        sr += ar[2 * k] * xv[k].x - ar[2 * k + 1] * xv[k].y;
        si += ar[2 * k] * xv[k].y + ar[2 * k + 1] * xv[k].x;
      }
    }
    lds[t * stride + r] = V{sr, si};
  }
  __syncthreads();
  // ---- coalesced stores of the outputs
  {
    int v = t / nout, k = t % nout;
    const int dv = kDV / nout, dk = kDV % nout;
    for (int e = t; e < nv * nout; e += kDV) {
      const int64_t p = p0 + v;
      const int64_t off = packed_y ? (b.outer == 1 ? p * b.ldy : p * b.yvs)
                                   : (p / b.outer) * b.ldy + (p % b.outer) * b.yvs;
      store(y + off + k, lds[v * stride + k], acc);
      v += dv;
      k += dk;
      if (k >= nout) {
        k -= nout;
        ++v;
      }
    }
  }
}

struct Box {
  int ndim;
  int64_t box[3], src[3], dst[3];
  int64_t outer, xos, yos;  // vector q = (c, o): x + c ldx + o xos, y + c ldy + o yos
};

template <typename V>
__global__ __launch_bounds__(256) void box_kernel(Box bx, int64_t ncols, const V* __restrict__ x,
                                                  int64_t ldx, V* y, int64_t ldy, int acc) {
  int64_t total = 1;
  for (int d = 0; d < bx.ndim; ++d) total *= bx.dst[d];
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= total) return;
  int64_t rem = f, src = 0, stride = 1;
  bool inside = true;
  int64_t idx[3];
  for (int d = bx.ndim - 1; d >= 0; --d) {
    idx[d] = rem % bx.dst[d];
    rem /= bx.dst[d];
  }
  for (int d = bx.ndim - 1; d >= 0; --d) {
    if (idx[d] >= bx.box[d]) inside = false;
    src += idx[d] * stride;
    stride *= bx.src[d];
  }
  for (int64_t q = blockIdx.y; q < ncols * bx.outer; q += gridDim.y) {
    const int64_t c = q / bx.outer, o = q - c * bx.outer;
    const V v = inside ? x[c * ldx + o * bx.xos + src] : Ops<V>::zero();
    V* dst = y + c * ldy + o * bx.yos + f;
    if (acc) {
      if (inside) store(dst, v, 1);
    } else {
      *dst = v;
    }
  }
}

template <typename V, typename R>
__global__ __launch_bounds__(256) void scale_kernel(int64_t count, R alpha, const V* __restrict__ x, V* y) {
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f < count) y[f] = cscale(x[f], alpha);
}

__global__ __launch_bounds__(256) void up_kernel(int64_t count, const c64* __restrict__ x, c128* y) {
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f < count) y[f] = {double(x[f].x), double(x[f].y)};
}
__global__ __launch_bounds__(256) void down_kernel(int64_t count, const c128* __restrict__ x, c64* y) {
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f < count) y[f] = {float(x[f].x), float(x[f].y)};
}

// Rounds a convolution spectrum to complex64 in the pair order read by the
// transform engine: within each row of lr = 16 T values, natural entry
// t + T k goes to 2 (t + T (k / 2)) + k % 2, so that a thread's values k and
// k + 1 are adjacent (one 16-byte load per pair).
__global__ __launch_bounds__(256) void down_paired_kernel(int64_t count, int64_t lr, const c128* __restrict__ x,
                                                          c64* y) {
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= count) return;
  const int64_t T = lr >> 4;
  const int64_t row = f / lr, r = f - row * lr;
  const int64_t t = r % T, k = r / T;
  y[row * lr + 2 * (t + T * (k >> 1)) + (k & 1)] = {float(x[f].x), float(x[f].y)};
}

__global__ __launch_bounds__(256) void permute_kernel(int64_t n1, int64_t n2, const c128* __restrict__ x,
                                                      c128* y) {
  const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;  // f = k1 + n1 * k2
  if (f >= n1 * n2) return;
  const int64_t k1 = f % n1, k2 = f / n1;
  y[f] = x[k2 + n2 * k1];
}

template <typename V>
__global__ __launch_bounds__(256) void embed_kernel(int64_t m, int64_t n, int64_t L, const V* __restrict__ col,
                                                    const V* __restrict__ row, c128* g) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= L) return;
  c128 v = {0.0, 0.0};
  if (k < m) {
    v = {double(col[k].x), double(col[k].y)};
  } else if (k > L - n) {
    const V r = row[L - k];
    v = {double(r.x), double(r.y)};
  }
  g[k] = v;
}

__global__ __launch_bounds__(256) void fill_i32_kernel(int64_t n, int32_t v, int32_t* __restrict__ a) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r < n) a[r] = v;
}

// inv[idx[r]] = r for distinct, in-range indices (checked before).
__global__ __launch_bounds__(256) void invert_idx_kernel(int64_t m, const int32_t* __restrict__ idx,
                                                         int32_t* __restrict__ inv) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r < m) inv[idx[r]] = int32_t(r);
}

__global__ __launch_bounds__(256) void check_idx_kernel(int64_t n, int64_t m, const int32_t* __restrict__ idx,
                                                        int* flags, int* bad) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= m) return;
  const int32_t v = idx[r];
  if (v < 0 || int64_t(v) >= n) {
    atomicOr(bad, 1);
    return;
  }
  if (atomicAdd(flags + v, 1) != 0) atomicOr(bad, 1);
}

}  // namespace

#define FM_ELEM_SWITCH(e, V, ...)        \
  switch (e) {                           \
    case Elem::C64: {                    \
      using V = c64;                     \
      __VA_ARGS__;                       \
      break;                             \
    }                                    \
    case Elem::C128: {                   \
      using V = c128;                    \
      __VA_ARGS__;                       \
      break;                             \
    }                                    \
    case Elem::I32: {                    \
      using V = int32_t;                 \
      __VA_ARGS__;                       \
      break;                             \
    }                                    \
    case Elem::I64: {                    \
      using V = int64_t;                 \
      __VA_ARGS__;                       \
      break;                             \
    }                                    \
  }

fm_status launch_diag(Elem e, int64_t n, const Batch& b, const void* d, int conj, const void* x,
                      void* y, int acc, hipStream_t s) {
  if (b.ncols == 0 || n == 0) return FM_OK;
  dim3 g = vec_grid(b.ncols * b.outer, n * b.inner, 256);
  if (e == Elem::C64)
    hipLaunchKernelGGL(diag_kernel<c64>, g, dim3(256), 0, s, n, b, (const c64*)d, conj, (const c64*)x,
                       (c64*)y, acc);
  else if (e == Elem::C128)
    hipLaunchKernelGGL(diag_kernel<c128>, g, dim3(256), 0, s, n, b, (const c128*)d, conj,
                       (const c128*)x, (c128*)y, acc);
  else {
    set_error("diag: integer element type");
    return FM_E_DTYPE;
  }
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_select(Elem e, int64_t n_in, int64_t m, const int32_t* idx, const int32_t* inv, int adjoint,
                        const Batch& b, const void* x, void* y, int acc, hipStream_t s) {
  if (b.ncols == 0) return FM_OK;
  if (!adjoint) {
    if (m == 0) return FM_OK;
    dim3 g = vec_grid(b.ncols * b.outer, m * b.inner, 256);
    FM_ELEM_SWITCH(e, V, hipLaunchKernelGGL(gather_kernel<V>, g, dim3(256), 0, s, m, b, idx,
                                            (const V*)x, (V*)y, acc));
  } else if (inv != nullptr && m > 0 && e == Elem::C64 && !acc && b.inner == 1 && b.outer == 1 &&
             (reinterpret_cast<uintptr_t>(y) & 15) == 0 && (b.ldy & 1) == 0) {
    dim3 g = vec_grid(b.ncols, cdiv(n_in, 2), 256);
    hipLaunchKernelGGL(expand_pair_kernel, g, dim3(256), 0, s, n_in, b, inv, (const c64*)x, (c64*)y);
  } else if (inv != nullptr && m > 0) {
    dim3 g = vec_grid(b.ncols * b.outer, n_in * b.inner, 256);
    FM_ELEM_SWITCH(e, V, hipLaunchKernelGGL(expand_kernel<V>, g, dim3(256), 0, s, n_in, b, inv,
                                            (const V*)x, (V*)y, acc));
  } else {
    if (!acc && n_in > 0) {
      dim3 gz = vec_grid(b.ncols * b.outer, n_in * b.inner, 256);
      FM_ELEM_SWITCH(e, V, hipLaunchKernelGGL(zero_kernel<V>, gz, dim3(256), 0, s, n_in * b.inner, b,
                                              (V*)y));
      FM_LAUNCHED();
    }
    if (m == 0) return FM_OK;
    dim3 g = vec_grid(b.ncols * b.outer, m * b.inner, 256);
    FM_ELEM_SWITCH(e, V, hipLaunchKernelGGL(scatter_kernel<V>, g, dim3(256), 0, s, m, b, idx,
                                            (const V*)x, (V*)y, 1));
  }
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_copy(Elem e, int64_t n, const Batch& b, const void* x, void* y, int acc,
                      hipStream_t s) {
  if (b.ncols == 0 || n == 0) return FM_OK;
  dim3 g = vec_grid(b.ncols * b.outer, n * b.inner, 256);
  FM_ELEM_SWITCH(e, V, hipLaunchKernelGGL(copy_kernel<V>, g, dim3(256), 0, s, n * b.inner, b,
                                          (const V*)x, (V*)y, acc));
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_conj(Elem e, int64_t n, const Batch& b, const void* x, void* y, int acc, hipStream_t s) {
  if (b.ncols == 0 || n == 0) return FM_OK;
  dim3 g = vec_grid(b.ncols * b.outer, n * b.inner, 256);
  if (e == Elem::C64)
    hipLaunchKernelGGL(conj_kernel<float>, g, dim3(256), 0, s, n * b.inner, b, (const c64*)x, (c64*)y, acc);
  else if (e == Elem::C128)
    hipLaunchKernelGGL(conj_kernel<double>, g, dim3(256), 0, s, n * b.inner, b, (const c128*)x, (c128*)y, acc);
  else
    return launch_copy(e, n, b, x, y, acc, s);  // integers are their own conjugates
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_param_map(int64_t count, int mode, double scale, const void* in, void* out, int* flag,
                           hipStream_t s) {
  if (count == 0) return FM_OK;
  hipLaunchKernelGGL(param_map_kernel, dim3(unsigned(cdiv(count, 256))), dim3(256), 0, s, count, mode, scale,
                     (const c128*)in, (c128*)out, flag);
  FM_LAUNCHED();
  return FM_OK;
}

// LDS bytes one work-group may allocate on the current device (cached).
size_t max_lds_per_block() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
  if (cached[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) v = 65536;
    cached[dev] = v;
  }
  return size_t(cached[dev]);
}

// FM_DENSE_MFMA=0 keeps complex64 dense products on the vector units.
static bool dense_mfma_enabled() {
  static const bool v = [] {
    const char* e = std::getenv("FM_DENSE_MFMA");
    return !(e && e[0] == '0');
  }();
  return v;
}

fm_status launch_dense(Elem e, int64_t m, int64_t n, const void* a, int64_t lda, int adjoint, int real_a,
                       const Batch& b, const void* x, void* y, int acc, hipStream_t s) {
  if (b.ncols == 0) return FM_OK;
  // complex64 on the matrix cores when a work-group's 64 vectors are there
  if (dense_mfma_enabled() && dense_mfma_supported(e, m, n, b) && b.ncols * b.outer >= 64)
    return launch_dense_mfma(m, n, a, lda, adjoint, b, x, y, acc, s);
  const int64_t rows_out = adjoint ? n : m;
  if (rows_out == 0) return FM_OK;
  const int64_t rows_in = adjoint ? m : n;
  const int64_t P = b.ncols * b.outer;
  const int nmax = rows_in <= 8 ? 8 : rows_in <= 16 ? 16 : rows_in <= 32 ? 32 : 64;
  const size_t abytes = (size_t(rows_out) * nmax * (real_a ? 1 : 2) * (e == Elem::C64 ? 4 : 8) + 15) & ~size_t(15);
  const size_t lds = abytes + size_t(kDV) * size_t((rows_in > rows_out ? rows_in : rows_out) + 1) * elem_bytes(e);
  if (b.inner == 1 && rows_in <= 64 && rows_out <= 64 && (e == Elem::C64 || (e == Elem::C128 && rows_in <= 32)) &&
      P >= 4 * kDV && lds <= max_lds_per_block()) {
    const dim3 g(unsigned(cdiv(P, kDV)));
#define FM_DV(V, N)                                                                                        \
  do {                                                                                                     \
    if (real_a) {                                                                                          \
      if (adjoint)                                                                                         \
        hipLaunchKernelGGL((dense_vec_kernel<V, N, true, true>), g, dim3(kDV), lds, s, m, n, (const V*)a, \
                           lda, b, (const V*)x, (V*)y, acc);                                               \
      else                                                                                                 \
        hipLaunchKernelGGL((dense_vec_kernel<V, N, true, false>), g, dim3(kDV), lds, s, m, n, (const V*)a, \
                           lda, b, (const V*)x, (V*)y, acc);                                               \
    } else {                                                                                               \
      if (adjoint)                                                                                         \
        hipLaunchKernelGGL((dense_vec_kernel<V, N, false, true>), g, dim3(kDV), lds, s, m, n, (const V*)a, \
                           lda, b, (const V*)x, (V*)y, acc);                                               \
      else                                                                                                 \
        hipLaunchKernelGGL((dense_vec_kernel<V, N, false, false>), g, dim3(kDV), lds, s, m, n,            \
                           (const V*)a, lda, b, (const V*)x, (V*)y, acc);                                  \
    }                                                                                                      \
  } while (0)
    if (e == Elem::C64) {
      if (nmax == 8) FM_DV(c64, 8);
      else if (nmax == 16) FM_DV(c64, 16);
      else if (nmax == 32) FM_DV(c64, 32);
      else FM_DV(c64, 64);
    } else {
      if (nmax == 8) FM_DV(c128, 8);
      else if (nmax == 16) FM_DV(c128, 16);
      else FM_DV(c128, 32);
    }
#undef FM_DV
    FM_LAUNCHED();
    return FM_OK;
  }
  dim3 g = vec_grid(b.ncols * b.outer, rows_out * b.inner, 256);
  if (e == Elem::C64)
    hipLaunchKernelGGL(dense_kernel<c64>, g, dim3(256), 0, s, m, n, (const c64*)a, lda, adjoint, b,
                       (const c64*)x, (c64*)y, acc);
  else if (e == Elem::C128)
    hipLaunchKernelGGL(dense_kernel<c128>, g, dim3(256), 0, s, m, n, (const c128*)a, lda, adjoint, b,
                       (const c128*)x, (c128*)y, acc);
  else {
    set_error("dense: integer element type");
    return FM_E_DTYPE;
  }
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_box_copy(Elem e, int ndim, const int64_t* box, const int64_t* src_dims,
                          const int64_t* dst_dims, int64_t ncols, const void* x, int64_t ldx,
                          void* y, int64_t ldy, int acc, hipStream_t s, int64_t outer, int64_t xos, int64_t yos) {
  if (ncols == 0 || outer == 0) return FM_OK;
  FM_CHECK_ARG(ndim >= 1 && ndim <= 3, FM_E_UNSUPPORTED, "box copy: 1..3 dimensions");
  Box bx{};
  bx.ndim = ndim;
  bx.outer = outer;
  bx.xos = xos;
  bx.yos = yos;
  int64_t total = 1;
  for (int d = 0; d < ndim; ++d) {
    bx.box[d] = box[d];
    bx.src[d] = src_dims[d];
    bx.dst[d] = dst_dims[d];
    total *= dst_dims[d];
  }
  const int64_t nv = ncols * outer;
  dim3 g(unsigned(cdiv(total, 256)), unsigned(nv < 65535 ? nv : 65535));
  FM_ELEM_SWITCH(e, V, hipLaunchKernelGGL(box_kernel<V>, g, dim3(256), 0, s, bx, ncols, (const V*)x,
                                          ldx, (V*)y, ldy, acc));
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_block_mix(Elem e, int nout, int nin, int ld, int64_t nb, int64_t total, int logtw, int64_t ncols,
                           const void* spec, int adjoint, const void* x, void* y, hipStream_t s) {
  if (ncols == 0 || total == 0 || nout == 0) return FM_OK;
  MixArgs a{nout, nin, ld, adjoint, logtw, total, ncols, nb, spec, x, y};
  const unsigned gy = unsigned(ncols < 65535 ? ncols : 65535);
  if (e == Elem::C64) {
    constexpr int OB = 8;
    const dim3 g(unsigned(cdiv(total, 256)), gy, unsigned(cdiv(nout, OB)));
    hipLaunchKernelGGL((block_mix_kernel<float, OB, 16>), g, dim3(256), 0, s, a);
  } else if (e == Elem::C128) {
    constexpr int OB = 4;
    const dim3 g(unsigned(cdiv(total, 256)), gy, unsigned(cdiv(nout, OB)));
    hipLaunchKernelGGL((block_mix_kernel<double, OB, 16>), g, dim3(256), 0, s, a);
  } else {
    set_error("block mix: integer element type");
    return FM_E_DTYPE;
  }
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_block_pack(Elem e, int64_t nb, int64_t total, int logtw, const void* table, void* out,
                            hipStream_t s) {
  if (nb == 0 || total == 0) return FM_OK;
  const dim3 g(unsigned(cdiv(total, 256)), unsigned(nb < 65535 ? nb : 65535));
  const auto* tab = static_cast<const void* const*>(table);
  if (e == Elem::C64)
    hipLaunchKernelGGL(block_pack_kernel<float>, g, dim3(256), 0, s, nb, total, logtw, tab, (c64*)out);
  else if (e == Elem::C128)
    hipLaunchKernelGGL(block_pack_kernel<double>, g, dim3(256), 0, s, nb, total, logtw, tab, (c128*)out);
  else {
    set_error("block pack: integer element type");
    return FM_E_DTYPE;
  }
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_scale_copy(Elem e, int64_t count, double alpha, const void* x, void* y,
                            hipStream_t s) {
  if (count == 0) return FM_OK;
  dim3 g(unsigned(cdiv(count, 256)));
  if (e == Elem::C64)
    hipLaunchKernelGGL((scale_kernel<c64, float>), g, dim3(256), 0, s, count, float(alpha),
                       (const c64*)x, (c64*)y);
  else if (e == Elem::C128)
    hipLaunchKernelGGL((scale_kernel<c128, double>), g, dim3(256), 0, s, count, alpha,
                       (const c128*)x, (c128*)y);
  else {
    set_error("scale: integer element type");
    return FM_E_DTYPE;
  }
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_c64_to_c128(int64_t count, const void* x, void* y, hipStream_t s) {
  if (count == 0) return FM_OK;
  hipLaunchKernelGGL(up_kernel, dim3(unsigned(cdiv(count, 256))), dim3(256), 0, s, count,
                     (const c64*)x, (c128*)y);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_spectrum_c64(int64_t count, const void* x, void* y, hipStream_t s) {
  if (count == 0) return FM_OK;
  if (count < 16) return launch_c128_to_c64(count, x, y, s);
  const int64_t lr = count < 4096 ? count : 4096;
  hipLaunchKernelGGL(down_paired_kernel, dim3(unsigned(cdiv(count, 256))), dim3(256), 0, s, count, lr,
                     (const c128*)x, (c64*)y);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_c128_to_c64(int64_t count, const void* x, void* y, hipStream_t s) {
  if (count == 0) return FM_OK;
  hipLaunchKernelGGL(down_kernel, dim3(unsigned(cdiv(count, 256))), dim3(256), 0, s, count,
                     (const c128*)x, (c64*)y);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_fourstep_permute(int64_t n1, int64_t n2, const void* x, void* y, hipStream_t s) {
  hipLaunchKernelGGL(permute_kernel, dim3(unsigned(cdiv(n1 * n2, 256))), dim3(256), 0, s, n1, n2,
                     (const c128*)x, (c128*)y);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_toeplitz_embed(int64_t m, int64_t n, int64_t L, const void* col, const void* row,
                                int elem_c64, void* g, hipStream_t s) {
  dim3 gr(unsigned(cdiv(L, 256)));
  if (elem_c64)
    hipLaunchKernelGGL(embed_kernel<c64>, gr, dim3(256), 0, s, m, n, L, (const c64*)col,
                       (const c64*)row, (c128*)g);
  else
    hipLaunchKernelGGL(embed_kernel<c128>, gr, dim3(256), 0, s, m, n, L, (const c128*)col,
                       (const c128*)row, (c128*)g);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_invert_indices(int64_t n, int64_t m, const int32_t* idx, int32_t* inv, hipStream_t s) {
  if (n == 0) return FM_OK;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(unsigned(cdiv(n, 256))), dim3(256), 0, s, n, int32_t(-1), inv);
  FM_LAUNCHED();
  if (m == 0) return FM_OK;
  hipLaunchKernelGGL(invert_idx_kernel, dim3(unsigned(cdiv(m, 256))), dim3(256), 0, s, m, idx, inv);
  FM_LAUNCHED();
  return FM_OK;
}

fm_status launch_check_indices(int64_t n, int64_t m, const int32_t* idx, int* flags_and_bad,
                               hipStream_t s) {
  // flags_and_bad: n + 1 zeroed ints; the last one receives the verdict
  if (m == 0) return FM_OK;
  hipLaunchKernelGGL(check_idx_kernel, dim3(unsigned(cdiv(m, 256))), dim3(256), 0, s, n, m, idx,
                     flags_and_bad, flags_and_bad + n);
  FM_LAUNCHED();
  return FM_OK;
}

}  // namespace fm
