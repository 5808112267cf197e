// Device-side FFT engine shared by the per-operator kernels and the batched
// stage kernel (the fast transform behind the DFT of eq. (1) and the
// cyclic convolution of eq. (5)).
//
// A work-group holds 2^LOGW complex values, 16 per thread in registers
// (256 threads for LOGW = 12).
//
// Transforms of N = 2^n >= 16 points (n <= LOGW) are held by T = N/16
// threads, thread t holding positions t + T*k (k = 0..15), and the
// work-group holds 2^LOGW/N of them. The arithmetic of one transform does not
// depend on LOGW, so both engines give the same bits. The transform is a sequence of Stockham steps: one short
// radix-2/4/8 step first when n is not a multiple of 4, then radix-16 steps.
// Butterfly j of a step with radix R and span Ns reads positions j + r*N/R --
// in the thread's own registers -- multiplies by W_{Ns R}^{(j mod Ns) r}, runs
// a radix-R DFT in registers and writes result q to position
// (j div Ns)*Ns*R + (j mod Ns) + q*Ns. Between steps the values go through LDS
// (one padding slot every 32 spreads the banks); after the last step they are
// back in the natural layout, so global loads and stores are coalesced and the
// spectral product between a forward and an inverse transform needs no
// exchange. The number of steps is a run-time value, so one code path serves
// every length.
//
// Shorter transforms (N < 16) run without LDS: each thread holds 16/N of them.
//
// The inverse (unnormalised) transform is conj(F(conj(x))), so only forward
// butterflies exist.
#pragma once

#include "kernels.h"

namespace fm {
namespace xf {

constexpr int kE = 16;  // values per thread
template <int LOGW>
struct Geo {
  static constexpr int kThreads = 1 << (LOGW - 4);
  static constexpr int kVals = 1 << LOGW;
};

// cos of 2 pi m / 16, m = 0..4 (sin by symmetry)
__device__ constexpr double kCos16[5] = {1.0, 0.92387953251128675613, 0.70710678118654752440,
                                         0.38268343236508977173, 0.0};

// a * exp(-2 pi j e / 16)
template <typename R>
__device__ __forceinline__ Cx<R> rot16(Cx<R> a, int e) {
  e &= 15;
  if (e == 0) return a;
  if (e == 8) return {-a.x, -a.y};
  if (e == 4) return {a.y, -a.x};
  if (e == 12) return {-a.y, a.x};
  const int q = e >> 2, r = e & 3;
  R c = R(kCos16[r]), sn = R(kCos16[4 - r]);
  for (int k = 0; k < q; ++k) {  // a quarter turn: (c, s) -> (-s, c)
    R t = c;
    c = -sn;
    sn = t;
  }
  sn = -sn;
  return {a.x * c - a.y * sn, a.x * sn + a.y * c};
}

// In-register forward DFT of RAD points (natural order in and out).
template <int RAD, typename R>
__device__ __forceinline__ void dft(Cx<R>* a) {
  if constexpr (RAD == 2) {
    Cx<R> t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  } else if constexpr (RAD == 4) {
    Cx<R> t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    Cx<R> t2 = cadd(a[1], a[3]), d = csub(a[1], a[3]);
    Cx<R> t3 = {d.y, -d.x};  // d * (-j)
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
  } else if constexpr (RAD == 8 || RAD == 16) {
    // RAD = P*Q, n = Q*n1 + n2, k = k1 + P*k2:
    // X[k1 + P k2] = sum_n2 W_Q^{n2 k2} W_RAD^{n2 k1} sum_n1 x[Q n1 + n2] W_P^{n1 k1}
    constexpr int P = RAD == 8 ? 2 : 4;
    constexpr int Q = RAD / P;
    Cx<R> b[RAD];
#pragma unroll
    for (int n2 = 0; n2 < Q; ++n2) {
      Cx<R> t[P];
#pragma unroll
      for (int n1 = 0; n1 < P; ++n1) t[n1] = a[Q * n1 + n2];
      dft<P>(t);
#pragma unroll
      for (int k1 = 0; k1 < P; ++k1) b[n2 * P + k1] = rot16(t[k1], n2 * k1 * (16 / RAD));
    }
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) {
      Cx<R> t[Q];
#pragma unroll
      for (int n2 = 0; n2 < Q; ++n2) t[n2] = b[n2 * P + k1];
      dft<Q>(t);
#pragma unroll
      for (int k2 = 0; k2 < Q; ++k2) a[k1 + P * k2] = t[k2];
    }
  }
}

__device__ __forceinline__ int pad32(int pos) { return pos + (pos >> 5); }

// Twiddles W^(jj r), r = 1..15, from the single table entry W^(jj): W^(2jj),
// W^(4jj), W^(8jj) by squaring, the others as products of at most three of
// them. The transform is bound by its loads, so one load and 14 complex
// products beat four loads and 11 products.
template <typename R>
__device__ __forceinline__ void twiddles16_from(Cx<R> w1, Cx<R>* w) {
  w[1] = w1;
  w[2] = cmul(w[1], w[1]);
  w[3] = cmul(w[1], w[2]);
  w[4] = cmul(w[2], w[2]);
  w[5] = cmul(w[1], w[4]);
  w[6] = cmul(w[2], w[4]);
  w[7] = cmul(w[3], w[4]);
  w[8] = cmul(w[4], w[4]);
#pragma unroll
  for (int r = 9; r < 16; ++r) w[r] = cmul(w[r - 8], w[8]);
}
template <typename R>
__device__ __forceinline__ void twiddles16(const Cx<R>* __restrict__ tab, int jj, Cx<R>* w) {
  twiddles16_from(tab[jj], w);
}

// The table entries W_{16 Ns}^(t mod Ns) of the (at most two) twiddled steps
// of a 2^logn-point transform (4 <= logn <= 12), in step order: loaded once,
// ahead of the transform, instead of on the critical path of every step.
template <typename R>
__device__ __forceinline__ void twiddle_seeds(int logn, int t, const Cx<R>* __restrict__ tw, Cx<R>* seeds) {
  const int first = logn & 3;
  const int nsteps = (logn >> 2) + (first ? 1 : 0);
  int lns = first;
  int ti = 0;
  for (int step = first ? 1 : 0; step < nsteps; ++step) {
    if (lns > 0) {  // constant indices only (the step count may be a run-time value)
      const Cx<R> w1 = tw[((1 << lns) << 4) + (t & ((1 << lns) - 1))];
      if (ti == 0)
        seeds[0] = w1;
      else
        seeds[1] = w1;
      ++ti;
    }
    lns += 4;
  }
}

// Short first step (radix RR = 2, 4, 8, span 1, no twiddles) into LDS.
template <int RR, typename R>
__device__ __forceinline__ void first_step(Cx<R>* v, Cx<R>* lds, int t, int T) {
  constexpr int M = kE / RR;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int j = t + T * m;
    Cx<R> a[RR];
#pragma unroll
    for (int r = 0; r < RR; ++r) a[r] = v[m + r * M];
    dft<RR>(a);
#pragma unroll
    for (int q = 0; q < RR; ++q) lds[pad32(j * RR + q)] = a[q];
  }
}

// Forward transform of 2^logn points (4 <= logn <= 12) held as described
// above. seeds: the twiddle_seeds of this length (NULL: loaded per step).
template <typename R>
__device__ __forceinline__ void forward(Cx<R>* v, int logn, int t, Cx<R>* lds, const Cx<R>* __restrict__ tw,
                                        const Cx<R>* seeds = nullptr) {
  const int T = 1 << (logn - 4);
  const int first = logn & 3;
  const int nsteps = (logn >> 2) + (first ? 1 : 0);
  int lns = 0;
  int step = 0;
  if (first) {
    if (first == 1)
      first_step<2>(v, lds, t, T);
    else if (first == 2)
      first_step<4>(v, lds, t, T);
    else
      first_step<8>(v, lds, t, T);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kE; ++k) v[k] = lds[pad32(t + T * k)];
    __syncthreads();
    lns = first;
    step = 1;
  }
  int ti = 0;
  for (; step < nsteps; ++step) {
    const int ns = 1 << lns;
    if (lns > 0) {
      Cx<R> w[16];
      if (seeds)
        twiddles16_from(ti++ == 0 ? seeds[0] : seeds[1], w);
      else
        twiddles16(tw + (ns << 4), t & (ns - 1), w);  // table of W_{16 Ns}
#pragma unroll
      for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], w[r]);
    }
    dft<16>(v);
    if (step == nsteps - 1) break;
    const int idxd = ((t >> lns) << (lns + 4)) | (t & (ns - 1));
#pragma unroll
    for (int q = 0; q < 16; ++q) lds[pad32(idxd + q * ns)] = v[q];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kE; ++k) v[k] = lds[pad32(t + T * k)];
    __syncthreads();
    lns += 4;
  }
}

template <typename R>
__device__ __forceinline__ void conj_all(Cx<R>* v) {
#pragma unroll
  for (int k = 0; k < kE; ++k) v[k].y = -v[k].y;
}

// Forward DFT of G = 16/N independent transforms of N = 2^logn < 16 points
// held by one thread (transform g at v[g*N .. g*N + N)).
template <typename R>
__device__ __forceinline__ void forward_tiny(Cx<R>* v, int logn) {
  if (logn == 1) {
#pragma unroll
    for (int g = 0; g < 8; ++g) dft<2>(v + 2 * g);
  } else if (logn == 2) {
#pragma unroll
    for (int g = 0; g < 4; ++g) dft<4>(v + 4 * g);
  } else if (logn == 3) {
#pragma unroll
    for (int g = 0; g < 2; ++g) dft<8>(v + 8 * g);
  }
}

// ---------------------------------------------------------------- one work-group's job
// A work-group's 2^LOGW values are 2^LOGW/N transforms. Transform b starts at
// base + b*bstride (contiguous vectors) or at base + b (strided vectors,
// element r at r*inner); its spectrum row starts at S + b*sbstride; its
// twiddle-epilogue index is q0 + b. Transforms with b >= nvalid are computed
// on zeros and not stored.
//
// Fused input (fuse_n2 > 0, contiguous, one transform per work-group): the
// row k2 = q0 of a four-step convolution with L = N * N2 (N2 = fuse_n2 <= 32,
// any integer) is formed while loading: point p is
// sum_n2 x[p + N n2] W_N2^(n2 k2) (zero beyond in_limit), times W_L^(p k2);
// x is the column base. twl is the table of W_L^m, 0 <= m < L, of the
// four-step length L (row twiddles, the fold's W_N2 = W_L^(N .), and the
// twiddle epilogue); every index formed from it is below L.
template <typename R>
struct Job {
  const Cx<R>* x;
  Cx<R>* y;
  int64_t xbstride, ybstride;  // contiguous: element offset between transforms
  int inner;                   // strided: element stride of the points (1: contiguous)
  int nvalid;
  int in_limit, out_limit;     // point r of transform b is read if r*inner + i_b < in_limit,
                               // stored if < out_limit (i_b = i0 + b when strided, else 0)
  int i0;
  const Cx<R>* S;
  int64_t sbstride;
  int q0;
  int fuse_n2 = 0;
  const Cx<R>* twl = nullptr;
  // IMAP (run_job template flag): input position p of a vector is read at
  // xcol[imap[p]] (strided items; contiguous items: at x + b*xbstride +
  // imap[p]), and is zero where imap[p] < 0: the adjoint of a row selection
  // applied at the load (p is the position inside the vector)
  const int* imap = nullptr;
  const Cx<R>* xcol = nullptr;
  // RIN (run_job template flag): the input values are already in the
  // caller's registers, rin[k] for value k of the thread (the layout of the
  // job's transform), instead of being loaded
  const Cx<R>* rin = nullptr;
};
struct Mode {
  int mode, spec_conj, tw_log, tw_inv, accumulate;
};

// Store epilogue: the default stores (or adds) each result at its
// destination. An epilogue type with kOn = true receives every result
// instead, in two passes over the thread's values so that all of its loads
// are in flight before the first store: pre(k, b, e, dst) for every value
// (load operands), then put(k, slot, b, e, dst, v). k is the value's register
// index, b the transform inside the work-group, e the element index inside
// the output vector and slot the thread's accumulator for that transform (g
// for contiguous transforms of fewer than 16 points, 0 otherwise).
struct NoEp {
  static constexpr bool kOn = false;
};

// Offset (in values) between the LDS regions of the transforms of one
// work-group of B transforms of 2^logn points. A region holds 33/32 of its
// points (pad32). Contiguous layout: the lanes of a wave are consecutive t of
// 64/T transforms, and the plain 33 T / 2 keeps their accesses apart. Strided
// layout: the lanes are min(B, 64) transforms times 64 / min(B, 64)
// consecutive t, all at the same in-region offset; the plain spacing (an even
// multiple of that count) puts many of them in the same banks. The smallest
// odd stride of at least base + 2 was chosen by timing the exchanges alone
// (64..2048-point transforms, strides base + 0..32): within 8 % of the
// fastest stride at every length, against up to 3x slower for the plain one.
__host__ __device__ constexpr int region_stride(int logn, int B, bool strided) {
  const int base = (1 << logn) + ((1 << logn) >> 5);
  return strided && B > 1 ? (base + 2) | 1 : base;
}

// Loads, transforms and stores one job. Every thread of the work-group calls it.
// SPLIT_SPEC: complex64 spectra are loaded and applied in two halves of 8
// values, which keeps 16 fewer registers live at the spectral product (the
// batched stage kernel then fits 128 VGPRs, four work-groups per CU) at the
// cost of a second round of spectrum loads.
// PRETW: the twiddle seeds of the transforms and of the twiddle epilogue, and
// a convolution's spectrum, are loaded with the input, ahead of the
// arithmetic (for latency-bound launches of few work-groups; more registers
// live through the transforms).
// EARLY_EP: the store epilogue's operand loads (EP::pre) are issued before
// the input loads, so their latency overlaps the transform (registers held
// through it).
template <typename R, bool STRIDED, int LOGW, bool SPLIT_SPEC = false, class EP = NoEp, bool IMAP = false,
          bool RIN = false, bool PRETW = false, bool EARLY_EP = false>
__device__ __forceinline__ void run_job(const Job<R>& jb, const Mode& md, int logn, Cx<R>* lds,
                                        const Cx<R>* __restrict__ tw, EP* ep = nullptr) {
  constexpr int kWG = Geo<LOGW>::kThreads;
  const int tid = threadIdx.x;
  Cx<R> v[kE];
  if (logn >= 4) {
    const int T = 1 << (logn - 4);
    const int B = kWG / T;
    const int b = STRIDED ? (tid % B) : (tid / T);
    const int t = STRIDED ? (tid / B) : (tid % T);
    const bool valid = b < jb.nvalid;
    const int inner = STRIDED ? jb.inner : 1;
    const int ii = STRIDED ? jb.i0 + b : 0;
    const Cx<R>* X = STRIDED ? jb.x + b : jb.x + b * jb.xbstride;
    Cx<R>* Y = STRIDED ? jb.y + b : jb.y + b * jb.ybstride;
    Cx<R> seeds[2], ew0, ews, spre[PRETW ? kE : 1];
    if constexpr (PRETW) {
      twiddle_seeds(logn, t, tw, seeds);
      if (md.tw_log > 0) {
        ew0 = jb.twl[t * (jb.q0 + b)];
        ews = jb.twl[T * (jb.q0 + b)];
      }
      if (md.mode == FFT_CONV) {  // the whole spectrum, in one round
        const Cx<R>* S = jb.S + b * jb.sbstride;
        if constexpr (sizeof(R) == 4) {
          const float4* S4 = reinterpret_cast<const float4*>(S);
#pragma unroll
          for (int j = 0; j < kE / 2; ++j) {
            const float4 q = S4[t + T * j];
            spre[2 * j] = {q.x, q.y};
            spre[2 * j + 1] = {q.z, q.w};
          }
        } else {
#pragma unroll
          for (int k = 0; k < kE; ++k) spre[k] = S[t + T * k];
        }
      }
    }
    const Cx<R>* sd = PRETW ? seeds : nullptr;
    if constexpr (EARLY_EP && EP::kOn) {
      if (valid) {
#pragma unroll
        for (int k = 0; k < kE; ++k) {
          const int p = t + T * k;
          if (p * inner + ii < jb.out_limit) ep->pre(k, b, p * inner + ii, Y + p * inner);
        }
      }
    }
    if constexpr (RIN) {
#pragma unroll
      for (int k = 0; k < kE; ++k) v[k] = valid ? jb.rin[k] : Cx<R>{R(0), R(0)};
    } else if (!STRIDED && jb.fuse_n2 > 0) {
      // n2-outer order: the 16 loads of one n2 are in flight together and
      // consumed only after all of them were issued
      const int n2s = jb.fuse_n2;
      const int k2 = jb.q0;
      const int N = 1 << logn;
#pragma unroll
      for (int k = 0; k < kE; ++k) v[k] = Cx<R>{R(0), R(0)};
      const int n2e = (jb.in_limit + N - 1) / N < n2s ? (jb.in_limit + N - 1) / N : n2s;  // rows holding data
      for (int n2 = 0; n2 < n2e; ++n2) {
        Cx<R> val[kE];
        if (!IMAP && N * (n2 + 1) <= jb.in_limit) {  // a full row of the input: unpredicated loads
#pragma unroll
          for (int k = 0; k < kE; ++k) val[k] = X[t + T * k + N * n2];
        } else {
#pragma unroll
          for (int k = 0; k < kE; ++k) {
            const int q = t + T * k + N * n2;
            if constexpr (IMAP) {
              const int m = q < jb.in_limit ? jb.imap[q] : -1;
              val[k] = m >= 0 ? X[m] : Cx<R>{R(0), R(0)};
            } else {
              val[k] = q < jb.in_limit ? X[q] : Cx<R>{R(0), R(0)};
            }
          }
        }
        const Cx<R> w = jb.twl[N * ((n2 * k2) % n2s)];  // W_N2^(n2 k2)
#pragma unroll
        for (int k = 0; k < kE; ++k) v[k] = cadd(v[k], cmul(val[k], w));
      }
      {  // W_L^((t + T k) k2) = W_L^(t k2) (W_L^(T k2))^k: two loads, the rest by products
        Cx<R> w = jb.twl[t * k2];
        const Cx<R> ws = jb.twl[T * k2];
#pragma unroll
        for (int k = 0; k < kE; ++k) {
          v[k] = cmul(v[k], w);
          w = cmul(w, ws);
        }
      }
    } else if (!IMAP && valid && ((1 << logn) - 1) * inner + ii < jb.in_limit) {
      // the whole transform lies inside the input: unpredicated loads
#pragma unroll
      for (int k = 0; k < kE; ++k) v[k] = X[(t + T * k) * inner];
    } else {
#pragma unroll
      for (int k = 0; k < kE; ++k) {
        const int p = t + T * k;
        const bool in = valid && p * inner + ii < jb.in_limit;
        if constexpr (IMAP) {
          const int m = in ? jb.imap[p * inner + ii] : -1;
          v[k] = m >= 0 ? (STRIDED ? jb.xcol[m] : X[m]) : Cx<R>{R(0), R(0)};
        } else {
          v[k] = in ? X[p * inner] : Cx<R>{R(0), R(0)};
        }
      }
    }
    Cx<R>* my = lds + b * region_stride(logn, kWG >> (logn - 4), STRIDED);
    if (md.mode == FFT_INV) conj_all(v);
    forward(v, logn, t, my, tw, sd);
    if (md.mode == FFT_CONV) {
      const Cx<R>* S = jb.S + b * jb.sbstride;
      constexpr int kPart = (SPLIT_SPEC && sizeof(R) == 4 && !PRETW) ? kE / 2 : kE;
#pragma unroll
      for (int h = 0; h < kE; h += kPart) {
        Cx<R> sv[kPart];
        if constexpr (PRETW) {
#pragma unroll
          for (int k = 0; k < kPart; ++k) sv[k] = spre[h + k];
        } else if constexpr (sizeof(R) == 4) {
          // complex64 spectra are stored in pair order: values k and k + 1 of
          // a thread are adjacent, one 16-byte load per pair
          const float4* S4 = reinterpret_cast<const float4*>(S);
#pragma unroll
          for (int j = 0; j < kPart / 2; ++j) {
            const float4 q = S4[t + T * (h / 2 + j)];
            sv[2 * j] = {q.x, q.y};
            sv[2 * j + 1] = {q.z, q.w};
          }
        } else {
#pragma unroll
          for (int k = 0; k < kPart; ++k) sv[k] = S[t + T * (h + k)];
        }
#pragma unroll
        for (int k = 0; k < kPart; ++k) {
          // inverse follows: keep conj(X s) (or conj(X conj s)) for the conj trick
          const Cx<R> p = md.spec_conj ? cmulc(v[h + k], sv[k]) : cmul(v[h + k], sv[k]);
          v[h + k] = {p.x, -p.y};
        }
      }
      forward(v, logn, t, my, tw, sd);
      conj_all(v);
    } else if (md.mode == FFT_INV) {
      conj_all(v);
    }
    if (md.tw_log > 0) {
      const Cx<R>* tab = jb.twl;
      const int qq = jb.q0 + b;
      // W^((t + T k) q) = W^(t q) (W^(T q))^k: two loads, the rest by products
      Cx<R> w = PRETW ? ew0 : tab[t * qq];
      const Cx<R> ws = PRETW ? ews : tab[T * qq];
#pragma unroll
      for (int k = 0; k < kE; ++k) {
        v[k] = md.tw_inv ? cmulc(v[k], w) : cmul(v[k], w);
        w = cmul(w, ws);
      }
    }
    if (valid) {
      if constexpr (EP::kOn) {  // two halves of 8 values: loads of a half in flight together
#pragma unroll
        for (int h = 0; h < kE; h += 8) {
#pragma unroll
          for (int k = h; k < h + 8; ++k) {
            const int p = t + T * k;
            if (!EARLY_EP && p * inner + ii < jb.out_limit) ep->pre(k, b, p * inner + ii, Y + p * inner);
          }
#pragma unroll
          for (int k = h; k < h + 8; ++k) {
            const int p = t + T * k;
            if (p * inner + ii < jb.out_limit) ep->put(k, 0, b, p * inner + ii, Y + p * inner, v[k]);
          }
        }
        return;
      }
      if (!md.accumulate && ((1 << logn) - 1) * inner + ii < jb.out_limit) {
        // the whole transform lies inside the output: unpredicated stores
#pragma unroll
        for (int k = 0; k < kE; ++k) Y[(t + T * k) * inner] = v[k];
        return;
      }
#pragma unroll
      for (int k = 0; k < kE; ++k) {
        const int p = t + T * k;
        if (p * inner + ii < jb.out_limit) {
          Cx<R>* dst = Y + p * inner;
          if (md.accumulate) {
            const Cx<R> old = *dst;
            *dst = cadd(old, v[k]);
          } else {
            *dst = v[k];
          }
        }
      }
    }
    return;
  }
  // ---- N < 16: G = 16/N transforms per thread, no LDS
  const int N = 1 << logn;
  const int G = kE >> logn;
  // transform of (thread, g): contiguous b = tid*G + g; strided b = tid + 256*g
#pragma unroll
  for (int k = 0; k < kE; ++k) {
    const int g = k >> logn, r = k & (N - 1);
    const int b = STRIDED ? tid + kWG * g : tid * G + g;
    const int inner = STRIDED ? jb.inner : 1;
    const int ii = STRIDED ? jb.i0 + b : 0;
    const bool in = b < jb.nvalid && r * inner + ii < jb.in_limit;
    if constexpr (IMAP) {
      const int m = in ? jb.imap[r * inner + ii] : -1;
      v[k] = m >= 0 ? (STRIDED ? jb.xcol[m] : jb.x[b * jb.xbstride + m]) : Cx<R>{R(0), R(0)};
    } else {
      const Cx<R>* src = STRIDED ? jb.x + b + r * inner : jb.x + b * jb.xbstride + r;
      v[k] = in ? *src : Cx<R>{R(0), R(0)};
    }
  }
  if (md.mode == FFT_INV) conj_all(v);
  forward_tiny(v, logn);
  if (md.mode == FFT_CONV) {
#pragma unroll
    for (int k = 0; k < kE; ++k) {
      const int g = k >> logn, r = k & (N - 1);
      const int b = STRIDED ? tid + kWG * g : tid * G + g;
      const Cx<R> s = jb.S[b * jb.sbstride + r];
      const Cx<R> p = md.spec_conj ? cmulc(v[k], s) : cmul(v[k], s);
      v[k] = {p.x, -p.y};
    }
    forward_tiny(v, logn);
    conj_all(v);
  } else if (md.mode == FFT_INV) {
    conj_all(v);
  }
  if (md.tw_log > 0) {
    const Cx<R>* tab = jb.twl;
#pragma unroll
    for (int k = 0; k < kE; ++k) {
      const int g = k >> logn, r = k & (N - 1);
      const int b = STRIDED ? tid + kWG * g : tid * G + g;
      const Cx<R> w = tab[r * (jb.q0 + b)];
      v[k] = md.tw_inv ? cmulc(v[k], w) : cmul(v[k], w);
    }
  }
  if constexpr (EP::kOn) {  // two halves of 8 values, as above
#pragma unroll
    for (int h = 0; h < kE; h += 8) {
#pragma unroll
      for (int k = h; k < h + 8; ++k) {
        const int g = k >> logn, r = k & (N - 1);
        const int b = STRIDED ? tid + kWG * g : tid * G + g;
        const int inner = STRIDED ? jb.inner : 1;
        const int ii = STRIDED ? jb.i0 + b : 0;
        if (b < jb.nvalid && r * inner + ii < jb.out_limit)
          ep->pre(k, b, r * inner + ii, STRIDED ? jb.y + b + r * inner : jb.y + b * jb.ybstride + r);
      }
#pragma unroll
      for (int k = h; k < h + 8; ++k) {
        const int g = k >> logn, r = k & (N - 1);
        const int b = STRIDED ? tid + kWG * g : tid * G + g;
        const int inner = STRIDED ? jb.inner : 1;
        const int ii = STRIDED ? jb.i0 + b : 0;
        if (b < jb.nvalid && r * inner + ii < jb.out_limit)
          ep->put(k, STRIDED ? 0 : g, b, r * inner + ii,
                  STRIDED ? jb.y + b + r * inner : jb.y + b * jb.ybstride + r, v[k]);
      }
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < kE; ++k) {
    const int g = k >> logn, r = k & (N - 1);
    const int b = STRIDED ? tid + kWG * g : tid * G + g;
    const int inner = STRIDED ? jb.inner : 1;
    const int ii = STRIDED ? jb.i0 + b : 0;
    if (b < jb.nvalid && r * inner + ii < jb.out_limit) {
      Cx<R>* dst = STRIDED ? jb.y + b + r * inner : jb.y + b * jb.ybstride + r;
      if (md.accumulate) {
        const Cx<R> old = *dst;
        *dst = cadd(old, v[k]);
      } else {
        *dst = v[k];
      }
    }
  }
}

// LDS bytes of one work-group: the largest region set over the lengths that
// use LDS (2^5 .. 2^LOGW points), strided or contiguous.
template <int LOGW>
constexpr int job_lds_values() {
  int v = Geo<LOGW>::kVals + Geo<LOGW>::kVals / 16;
  for (int lg = 5; lg <= LOGW; ++lg) {
    const int B = 1 << (LOGW - lg);
    const int need = B * region_stride(lg, B, true);
    v = need > v ? need : v;
  }
  return v;
}
template <typename R, int LOGW>
constexpr size_t job_lds_bytes() {
  return size_t(job_lds_values<LOGW>()) * sizeof(Cx<R>);
}

}  // namespace xf
}  // namespace fm
