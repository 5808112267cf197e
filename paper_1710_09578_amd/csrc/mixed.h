// Strided passes of a four-step convolution whose length L = 4096 * N2 has a
// strided factor N2 that is not a power of two (3, 5, 6, 9, 10, 12, 20, 24
// or 30): the
// embedding of a Toeplitz operator only needs L >= M + N - 1, and a length of
// this form wastes far less than the next power of two.
//
// One thread owns one column position n1 and its N2 points (stride 4096,
// coalesced across the threads of a work-group). The N2-point DFT is a
// mixed-radix Cooley-Tukey split on the smallest prime factor down to
// radix-2/3/4/5/8/16 codelets; its twiddles W_N^e are entries of the operator's
// W_L table (W_N^e = W_L^(L e / N)), at indices that are the same for every
// thread.
#pragma once

#include "xform.h"

namespace fm {
namespace xf {

// 3-point DFT: X1 = a0 - (a1 + a2)/2 - j (sqrt 3 / 2)(a1 - a2), X2 its mirror.
template <typename R>
__device__ __forceinline__ void dft3(Cx<R>* a) {
  const R h = R(0.86602540378443864676);  // sqrt(3) / 2
  const Cx<R> t1 = cadd(a[1], a[2]), t2 = csub(a[1], a[2]);
  const Cx<R> m = {a[0].x - R(0.5) * t1.x, a[0].y - R(0.5) * t1.y};
  const Cx<R> s = {h * t2.y, -h * t2.x};  // -j h t2
  a[0] = cadd(a[0], t1);
  a[1] = cadd(m, s);
  a[2] = csub(m, s);
}

// 5-point DFT from the pairs a1 +- a4, a2 +- a3 with c_k = cos(2 pi k / 5),
// s_k = sin(2 pi k / 5).
template <typename R>
__device__ __forceinline__ void dft5(Cx<R>* a) {
  const R c1 = R(0.30901699437494742410), c2 = R(-0.80901699437494742410);
  const R s1 = R(0.95105651629515357212), s2 = R(0.58778525229247312917);
  const Cx<R> t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
  const Cx<R> t3 = csub(a[1], a[4]), t4 = csub(a[2], a[3]);
  const Cx<R> b1 = {a[0].x + c1 * t1.x + c2 * t2.x, a[0].y + c1 * t1.y + c2 * t2.y};
  const Cx<R> b2 = {a[0].x + c2 * t1.x + c1 * t2.x, a[0].y + c2 * t1.y + c1 * t2.y};
  const Cx<R> u1 = {s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y};
  const Cx<R> u2 = {s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y};
  a[0] = cadd(a[0], cadd(t1, t2));
  a[1] = {b1.x + u1.y, b1.y - u1.x};  // b1 - j u1
  a[4] = {b1.x - u1.y, b1.y + u1.x};  // b1 + j u1
  a[2] = {b2.x + u2.y, b2.y - u2.x};
  a[3] = {b2.x - u2.y, b2.y + u2.x};
}

template <int N>
struct SmallestFactor {
  static constexpr int v = N % 2 == 0 ? 2 : N % 3 == 0 ? 3 : 5;
};

// Forward DFT of N points (natural order in and out), N a 5-smooth divisor
// of the strided factor N2 of L = 4096 N2. With n = P m + r and
// k = k1 + Q k2 (N = P Q, P the smallest prime factor):
// X[k1 + Q k2] = sum_r W_P^(r k2) W_N^(r k1) A_r[k1], A_r the Q-point DFT of
// x[P m + r]. W_N^e = twl[4096 (N2 / N) e] (a compile-time index).
template <int N, int N2, typename R>
__device__ __forceinline__ void dft_mixed(Cx<R>* v, const Cx<R>* twl) {
  if constexpr (N == 1) {
    return;
  } else if constexpr (N == 2 || N == 4 || N == 8 || N == 16) {
    dft<N>(v);
  } else if constexpr (N == 3) {
    dft3(v);
  } else if constexpr (N == 5) {
    dft5(v);
  } else {
    constexpr int P = SmallestFactor<N>::v;
    constexpr int Q = N / P;
    Cx<R> a[P][Q];
#pragma unroll
    for (int r = 0; r < P; ++r)
#pragma unroll
      for (int m = 0; m < Q; ++m) a[r][m] = v[P * m + r];
#pragma unroll
    for (int r = 0; r < P; ++r) dft_mixed<Q, N2>(a[r], twl);
    constexpr int step = 4096 * (N2 / N);
#pragma unroll
    for (int k1 = 0; k1 < Q; ++k1) {
      Cx<R> b[P];
#pragma unroll
      for (int r = 0; r < P; ++r)
        b[r] = (r == 0 || k1 == 0) ? a[r][k1] : cmul(a[r][k1], twl[step * ((r * k1) % N)]);
      dft_mixed<P, N2>(b, twl);
#pragma unroll
      for (int k2 = 0; k2 < P; ++k2) v[k1 + Q * k2] = b[k2];
    }
  }
}

// Column position n1 of a mixed four-step convolution (one thread).
// Forward (first pass): the N2 points x[n1 + 4096 j] (zero at or beyond
// in_limit), their DFT, times W_L^(n1 k2), into y[n1 + 4096 k2].
// Inverse (last pass): the N2 points of the slot x, their inverse DFT (conj
// trick), stored where n1 + 4096 k < out_limit (added with acc, or handed to
// the epilogue in chunks of 8 with all of a chunk's operand loads first).
// IMAP: point r is read at x[imap[r]] (zero where imap[r] < 0), the adjoint
// of a row selection applied at the load.
template <int N2, typename R, class EP, bool IMAP = false>
__device__ __forceinline__ void mixed_column(const Cx<R>* x, int64_t in_limit, Cx<R>* y, int64_t out_limit, int n1,
                                             bool inverse, const Cx<R>* twl, int64_t L, int acc, EP* ep,
                                             const int* imap = nullptr) {
  Cx<R> v[N2];
#pragma unroll
  for (int j = 0; j < N2; ++j) {
    const int64_t r = n1 + 4096 * int64_t(j);
    if constexpr (IMAP) {
      const int m = r < in_limit ? imap[r] : -1;
      v[j] = m >= 0 ? x[m] : Cx<R>{R(0), R(0)};
    } else {
      v[j] = r < in_limit ? x[r] : Cx<R>{R(0), R(0)};
    }
  }
  if (inverse) {
#pragma unroll
    for (int j = 0; j < N2; ++j) v[j].y = -v[j].y;
  }
  dft_mixed<N2, N2>(v, twl);
  if (inverse) {
#pragma unroll
    for (int j = 0; j < N2; ++j) v[j].y = -v[j].y;
  } else {  // W_L^(n1 k) = (W_L^n1)^k: one coalesced load, then products
    const Cx<R> w1 = twl[n1];
    Cx<R> w = w1;
#pragma unroll
    for (int k = 1; k < N2; ++k) {
      v[k] = cmul(v[k], w);
      w = cmul(w, w1);
    }
  }
  if constexpr (EP::kOn) {
#pragma unroll
    for (int h = 0; h < N2; h += 8) {
#pragma unroll
      for (int k = h; k < h + 8 && k < N2; ++k) {
        const int64_t r = n1 + 4096 * int64_t(k);
        if (r < out_limit) ep->pre(k & 7, 0, int(r), y + r);
      }
#pragma unroll
      for (int k = h; k < h + 8 && k < N2; ++k) {
        const int64_t r = n1 + 4096 * int64_t(k);
        if (r < out_limit) ep->put(k & 7, 0, 0, int(r), y + r, v[k]);
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < N2; ++k) {
      const int64_t r = n1 + 4096 * int64_t(k);
      if (r < out_limit) y[r] = acc ? cadd(y[r], v[k]) : v[k];
    }
  }
}

// Strided factors N2 = 2M of 20, 24 and 30 take two threads per column
// position (a single thread would need 140-190 registers, more than the stage
// kernel's 128 at four work-groups per CU): thread h loads the
// points 2m + h, forms their M-point DFT A_h (times W_N2^k1 for h = 1), the
// pair exchanges A_0, A_1 through LDS and thread h keeps
// X[k1 + h M] = A_0[k1] + (-1)^h A_1[k1]. lds: 2 M + 1 values per column
// position of the work-group (an odd stride: the 64 positions of a wave fall
// in distinct banks). Every thread of the work-group calls it (one barrier).
template <int M, typename R, class EP, bool IMAP = false>
__device__ __forceinline__ void mixed_column_pair(const Cx<R>* x, int64_t in_limit, Cx<R>* y, int64_t out_limit,
                                                  int n1, int h, int slot, bool inverse, const Cx<R>* twl, int64_t L,
                                                  int acc, EP* ep, Cx<R>* lds, const int* imap = nullptr) {
  constexpr int N2 = 2 * M;
  Cx<R> v[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int64_t r = n1 + 4096 * int64_t(2 * m + h);
    if constexpr (IMAP) {
      const int mi = r < in_limit ? imap[r] : -1;
      v[m] = mi >= 0 ? x[mi] : Cx<R>{R(0), R(0)};
    } else {
      v[m] = r < in_limit ? x[r] : Cx<R>{R(0), R(0)};
    }
  }
  if (inverse) {
#pragma unroll
    for (int m = 0; m < M; ++m) v[m].y = -v[m].y;
  }
  dft_mixed<M, N2>(v, twl);
  if (h == 1) {
    constexpr int step = 4096;  // W_N2 = W_L^(L / N2)
#pragma unroll
    for (int k1 = 1; k1 < M; ++k1) v[k1] = cmul(v[k1], twl[step * k1]);
  }
  Cx<R>* mine = lds + int64_t(slot) * (N2 + 1);
#pragma unroll
  for (int k1 = 0; k1 < M; ++k1) mine[h * M + k1] = v[k1];
  __syncthreads();
#pragma unroll
  for (int k1 = 0; k1 < M; ++k1) {
    const Cx<R> a0 = mine[k1], a1 = mine[M + k1];
    v[k1] = h ? csub(a0, a1) : cadd(a0, a1);
  }
  if (inverse) {
#pragma unroll
    for (int m = 0; m < M; ++m) v[m].y = -v[m].y;
  } else {  // W_L^(n1 (k1 + h M)) = W_L^(n1 h M) (W_L^n1)^k1
    const Cx<R> w1 = twl[n1];
    Cx<R> w = h ? twl[int64_t(n1) * M] : Cx<R>{R(1), R(0)};
#pragma unroll
    for (int k1 = 0; k1 < M; ++k1) {
      v[k1] = cmul(v[k1], w);
      w = cmul(w, w1);
    }
  }
  if constexpr (EP::kOn) {
#pragma unroll
    for (int c = 0; c < M; c += 8) {
#pragma unroll
      for (int k1 = c; k1 < c + 8 && k1 < M; ++k1) {
        const int64_t r = n1 + 4096 * int64_t(k1 + h * M);
        if (r < out_limit) ep->pre(k1 & 7, 0, int(r), y + r);
      }
#pragma unroll
      for (int k1 = c; k1 < c + 8 && k1 < M; ++k1) {
        const int64_t r = n1 + 4096 * int64_t(k1 + h * M);
        if (r < out_limit) ep->put(k1 & 7, 0, 0, int(r), y + r, v[k1]);
      }
    }
  } else {
#pragma unroll
    for (int k1 = 0; k1 < M; ++k1) {
      const int64_t r = n1 + 4096 * int64_t(k1 + h * M);
      if (r < out_limit) y[r] = acc ? cadd(y[r], v[k1]) : v[k1];
    }
  }
}

// Threads per column position and work-group tiles per column (256 threads
// per work-group, one column position per thread or thread pair). Several
// positions per thread (fewer, fuller work-groups) measured slower: the
// rounds serialise their load latencies.
__host__ __device__ inline int mixed_threads(int n2) { return n2 > 12 ? 2 : 1; }
__host__ __device__ inline int mixed_tiles(int n2) { return 16 * mixed_threads(n2); }

// Tile `tile` of one column for the strided factor N2: 256 / mixed_threads(N2)
// consecutive column positions. Every thread of the work-group calls it; lds
// holds 256 / threads * (N2 + 1) values (pairs only).
template <int N2, typename R, class EP, bool IMAP = false>
__device__ __forceinline__ void mixed_tile_n(int tile, const Cx<R>* x, int64_t in_limit, Cx<R>* y, int64_t out_limit,
                                             bool inverse, const Cx<R>* twl, int64_t L, int acc, EP* ep,
                                             Cx<R>* lds, const int* imap = nullptr) {
  const int tid = int(threadIdx.x);
  if constexpr (N2 > 12)
    mixed_column_pair<N2 / 2, R, EP, IMAP>(x, in_limit, y, out_limit, tile * 128 + (tid & 127), tid >> 7, tid & 127,
                                           inverse, twl, L, acc, ep, lds, imap);
  else
    mixed_column<N2, R, EP, IMAP>(x, in_limit, y, out_limit, tile * 256 + tid, inverse, twl, L, acc, ep, imap);
}

// The same with the factor chosen at run time (the stage kernel's items).
template <typename R, class EP, bool IMAP = false>
__device__ __forceinline__ void mixed_tile(int n2, int tile, const Cx<R>* x, int64_t in_limit, Cx<R>* y,
                                           int64_t out_limit, bool inverse, const Cx<R>* twl, int64_t L, int acc,
                                           EP* ep, Cx<R>* lds, const int* imap = nullptr) {
#define FM_MIXED_CASE(N)                                                                               \
  case N:                                                                                              \
    mixed_tile_n<N, R, EP, IMAP>(tile, x, in_limit, y, out_limit, inverse, twl, L, acc, ep, lds, imap); \
    break;
  switch (n2) {
    FM_MIXED_CASE(3)
    FM_MIXED_CASE(5)
    FM_MIXED_CASE(6)
    FM_MIXED_CASE(9)
    FM_MIXED_CASE(10)
    FM_MIXED_CASE(12)
    FM_MIXED_CASE(20)
    FM_MIXED_CASE(24)
    FM_MIXED_CASE(30)
    default:
      break;
  }
#undef FM_MIXED_CASE
}

}  // namespace xf
}  // namespace fm
