// C ABI: operator creation (with the one-time precomputation of spectra),
// composition, validation at every entry point, and fm_apply.
#include <complex>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "runtime.h"

namespace fm {
void register_op(const fm_op_s* op);
void unregister_op(const fm_op_s* op);
}  // namespace fm

using namespace fm;

namespace {

constexpr int kMaxLog = 20;

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

fm_status current_device(int* dev) {
  FM_HIP(hipGetDevice(dev));
  return FM_OK;
}

fm_status new_op(Kind k, fm_dtype dt, int64_t m, int64_t n, fm_op_s** out) {
  fm_op_s* op = new (std::nothrow) fm_op_s();
  FM_CHECK_ARG(op != nullptr, FM_E_NOMEM, "out of host memory");
  op->kind = k;
  op->dt = dt;
  op->m = m;
  op->n = n;
  fm_status st = current_device(&op->device);
  if (st != FM_OK) {
    delete op;
    return st;
  }
  *out = op;
  return FM_OK;
}

void destroy(fm_op_s* op);

void drop(fm_op_s* op) {
  if (op->refs.fetch_sub(1) == 1) destroy(op);
}

void destroy(fm_op_s* op) {
  unregister_op(op);
  for (fm_op t : op->terms) drop(t);
  op->magic = 0;
  delete op;
}

// The twiddle tables an operator's transforms read, created with the
// operator so that applying it never allocates (both precisions: the power
// iteration runs in complex128 whatever the operator's dtype).
fm_status ensure_tables(const fm_op_s* op) {
  if (op->dt != FM_C64 && op->dt != FM_C128) return FM_OK;
  if (!twiddle_table(Elem::C64, kMaxLog) || !twiddle_table(Elem::C128, kMaxLog)) return FM_E_NOMEM;
  for (Elem e : {Elem::C64, Elem::C128}) {
    const Split& sp = e == Elem::C64 ? op->s32 : op->s64;
    if (op->L > 0 && sp.mixed() && !twiddle_table_L(e, op->L)) return FM_E_NOMEM;
  }
  return FM_OK;
}

fm_status publish(fm_op_s* op, fm_op* out) {
  fm_status st = ensure_tables(op);
  if (st != FM_OK) {
    destroy(op);
    return st;
  }
  register_op(op);
  *out = op;
  return FM_OK;
}

// Guard that deletes a half-built operator on an error path.
struct Building {
  fm_op_s* op;
  ~Building() {
    if (op) {
      for (fm_op t : op->terms) drop(t);
      delete op;
    }
  }
  fm_op_s* release() {
    fm_op_s* o = op;
    op = nullptr;
    return o;
  }
};

bool valid_dtype(fm_dtype dt) { return dt == FM_C64 || dt == FM_C128 || dt == FM_I32 || dt == FM_I64; }

// Copies n complex values of dtype dt from src into the operator's complex128
// store (exact upcast) and, for FM_C64, its complex64 store.
fm_status store_params(fm_op_s* op, const void* src, int64_t count, hipStream_t s) {
  FM_TRY(op->p64.alloc(size_t(count) * 16));
  if (op->dt == FM_C64) {
    FM_TRY(op->p32.alloc(size_t(count) * 8));
    FM_HIP(hipMemcpyAsync(op->p32.p, src, size_t(count) * 8, hipMemcpyDeviceToDevice, s));
    FM_TRY(launch_c64_to_c128(count, src, op->p64.p, s));
  } else {
    FM_HIP(hipMemcpyAsync(op->p64.p, src, size_t(count) * 16, hipMemcpyDeviceToDevice, s));
  }
  return FM_OK;
}

// Turns a natural-order complex128 spectrum g_hat (length L, already scaled)
// into the operator's stores, in the order each precision's split expects.
fm_status store_spectrum(fm_op_s* op, const void* ghat, hipStream_t s) {
  const int64_t L = op->L;
  FM_TRY(op->p64.alloc(size_t(L) * 16));
  if (op->s64.four_step())
    FM_TRY(launch_fourstep_permute(int64_t(1) << op->s64.log1, int64_t(1) << op->s64.log2, ghat,
                                   op->p64.p, s));
  else
    FM_HIP(hipMemcpyAsync(op->p64.p, ghat, size_t(L) * 16, hipMemcpyDeviceToDevice, s));
  if (op->dt == FM_C64) {
    FM_TRY(op->p32.alloc(size_t(L) * 8));
    DevBuf tmp;
    const void* src = ghat;
    if (op->s32.four_step()) {
      FM_TRY(tmp.alloc(size_t(L) * 16));
      FM_TRY(launch_fourstep_permute(int64_t(1) << op->s32.log1, int64_t(1) << op->s32.log2, ghat,
                                     tmp.p, s));
      src = tmp.p;
    }
    FM_TRY(launch_spectrum_c64(L, src, op->p32.p, s));
    FM_HIP(hipStreamSynchronize(s));  // tmp is freed on return
  }
  return FM_OK;
}

// DFT in complex128 of `count` contiguous vectors of length L (natural order),
// scaled by `scale`, through the library's own transform.
fm_status dft128(int64_t L, const void* in, void* out, double scale, hipStream_t s) {
  fm_op_s f;
  f.kind = Kind::Fourier;
  f.dt = FM_C128;
  f.m = f.n = f.L = L;
  f.s32 = split_for(Elem::C64, ilog2(L));
  f.s64 = split_for(Elem::C128, ilog2(L));
  Batch b{1, 1, 1, L, L, L, L};
  Workspace ws;
  ws.sizing = true;
  FM_TRY(exec(&f, false, Elem::C128, b, in, out, false, ws, s));
  DevBuf wbuf;
  FM_TRY(wbuf.alloc(ws.peak));
  Workspace run;
  run.base = static_cast<char*>(wbuf.p);
  run.cap = wbuf.bytes;
  FM_TRY(exec(&f, false, Elem::C128, b, in, out, false, run, s));
  if (scale != 1.0) FM_TRY(launch_scale_copy(Elem::C128, L, scale, out, out, s));
  FM_HIP(hipStreamSynchronize(s));
  return FM_OK;
}

// Largest workspace fm_apply needs (contiguous blocks).
fm_status size_of(const fm_op_s* op, bool adj, int64_t ncols, size_t* bytes) {
  Batch b{ncols, 1, 1, in_rows(op, adj), in_rows(op, adj), out_rows(op, adj), out_rows(op, adj)};
  Workspace ws;
  ws.sizing = true;
  FM_TRY(exec(op, adj, elem_of(op->dt), b, nullptr, nullptr, false, ws, nullptr));
  *bytes = ws.peak;
  return FM_OK;
}

#define CHECK_OUT(out) FM_CHECK_ARG((out) != nullptr, FM_E_INVALID, "output handle pointer is NULL")
#define CHECK_LIVE(a)                                                                  \
  do {                                                                                 \
    FM_CHECK_ARG((a) != nullptr, FM_E_INVALID, "operator handle is NULL");             \
    FM_CHECK_ARG(op_alive(a), FM_E_RELEASED, "operator handle was released");          \
  } while (0)

}  // namespace

// fm_apply with its checks; with may_allocate = false a missing or short
// workspace is an error instead of a stream-ordered allocation.
fm_status fm::apply_op(const fm_op_s* a, fm_dir dir, int64_t ncols, const void* x, int64_t ldx, void* y, int64_t ldy,
                   void* ws, size_t ws_bytes, bool may_allocate, void* stream) {
  set_error("");
  CHECK_LIVE(a);
  FM_CHECK_ARG(dir == FM_FWD || dir == FM_ADJ, FM_E_INVALID, "unknown direction");
  FM_CHECK_ARG(ncols >= 0, FM_E_INVALID, "negative column count");
  if (ncols == 0) return FM_OK;
  const bool adj = dir == FM_ADJ;
  const int64_t rin = in_rows(a, adj), rout = out_rows(a, adj);
  FM_CHECK_ARG(x != nullptr && y != nullptr, FM_E_INVALID, "NULL data pointer");
  FM_CHECK_ARG(ldx >= rin && ldy >= rout, FM_E_SHAPE,
               "leading dimensions too small: ldx %lld (need %lld), ldy %lld (need %lld)",
               (long long)ldx, (long long)rin, (long long)ldy, (long long)rout);
  const size_t es = elem_size(a->dt);
  const char* xb = static_cast<const char*>(x);
  const char* yb = static_cast<const char*>(y);
  const size_t xlen = size_t((ncols - 1) * ldx + rin) * es, ylen = size_t((ncols - 1) * ldy + rout) * es;
  FM_CHECK_ARG(xb + xlen <= yb || yb + ylen <= xb, FM_E_ALIAS, "x and y overlap");
  int dev = 0;
  FM_TRY(current_device(&dev));
  FM_CHECK_ARG(dev == a->device, FM_E_DEVICE, "operator lives on device %d, current is %d", a->device, dev);
  size_t need = 0;
  FM_TRY(size_of(a, adj, ncols, &need));
  hipStream_t s = as_stream(stream);
  void* wsp = ws;
  bool own = false;
  if (need > 0) {
    if (may_allocate && ws == nullptr && ws_bytes == 0) {
      FM_HIP(hipMallocAsync(&wsp, need, s));
      own = true;
    } else {
      FM_CHECK_ARG(ws != nullptr && ws_bytes >= need, FM_E_WORKSPACE,
                   "workspace of %zu bytes given, %zu needed", ws_bytes, need);
    }
  }
  Batch b{ncols, 1, 1, ldx, rin, ldy, rout};
  Workspace w;
  w.base = static_cast<char*>(wsp);
  w.cap = own ? need : ws_bytes;
  fm_status st = exec(a, adj, elem_of(a->dt), b, x, y, false, w, s);
  if (own) (void)hipFreeAsync(wsp, s);
  return st;
}

extern "C" {

const char* fm_last_error(void) { return last_error(); }
const char* fm_version(void) { return "0.1.0"; }

fm_status fm_op_create_fourier(fm_op* out, int64_t n, fm_dtype dt) {
  set_error("");
  CHECK_OUT(out);
  FM_CHECK_ARG(valid_dtype(dt), FM_E_INVALID, "unknown dtype %d", int(dt));
  FM_CHECK_ARG(is_complex(dt), FM_E_DTYPE, "Fourier needs a complex dtype");
  FM_CHECK_ARG(n >= 1 && n <= (int64_t(1) << kMaxLog), FM_E_UNSUPPORTED,
               "Fourier size %lld: 1 .. 2^20 are supported", (long long)n);
  FM_CHECK_ARG(is_pow2(n) || n <= (int64_t(1) << (kMaxLog - 1)), FM_E_UNSUPPORTED,
               "Fourier size %lld: sizes that are not powers of two go up to 2^19", (long long)n);
  fm_op_s* op;
  FM_TRY(new_op(Kind::Fourier, dt, n, n, &op));
  Building g{op};
  op->L = n;
  if (is_pow2(n)) {
    op->s32 = split_for(Elem::C64, ilog2(n));
    op->s64 = split_for(Elem::C128, ilog2(n));
    return publish(g.release(), out);
  }
  // Bluestein: W^(jk) = W^(j^2/2) W^(k^2/2) W^(-(k-j)^2/2) with W = exp(-2 pi i / n),
  // so F = D T D with D = diag(exp(-pi i j^2 / n)) and the Toeplitz
  // T[j, k] = exp(pi i (j - k)^2 / n). Angles reduced exactly (j^2 mod 2n).
  const size_t es = elem_size(dt);
  std::vector<unsigned char> dh(size_t(n) * es), th(size_t(n) * es);
  const double pi = 3.14159265358979323846;
  for (int64_t j = 0; j < n; ++j) {
    const int64_t q = (j * j) % (2 * n);
    const double ang = pi * double(q) / double(n);
    const double c = std::cos(ang), sn = std::sin(ang);
    if (dt == FM_C64) {
      float* d = reinterpret_cast<float*>(dh.data()) + 2 * j;
      float* t = reinterpret_cast<float*>(th.data()) + 2 * j;
      d[0] = float(c), d[1] = float(-sn), t[0] = float(c), t[1] = float(sn);
    } else {
      double* d = reinterpret_cast<double*>(dh.data()) + 2 * j;
      double* t = reinterpret_cast<double*>(th.data()) + 2 * j;
      d[0] = c, d[1] = -sn, t[0] = c, t[1] = sn;
    }
  }
  DevBuf dd, td;
  FM_TRY(dd.alloc(dh.size()));
  FM_TRY(td.alloc(th.size()));
  FM_HIP(hipMemcpy(dd.p, dh.data(), dh.size(), hipMemcpyHostToDevice));
  FM_HIP(hipMemcpy(td.p, th.data(), th.size(), hipMemcpyHostToDevice));
  fm_op D = nullptr, T = nullptr, P = nullptr;
  fm_status st = fm_op_create_diag(&D, n, dd.p, dt, nullptr);
  if (st == FM_OK) st = fm_op_create_toeplitz(&T, n, n, td.p, td.p, dt, nullptr);
  if (st == FM_OK) {
    fm_op t3[3] = {D, T, D};
    st = fm_op_compose(&P, FM_PRODUCT, 3, t3);
  }
  if (D) fm_op_release(D);
  if (T) fm_op_release(T);
  FM_TRY(st);
  op->terms.push_back(P);
  return publish(g.release(), out);
}

fm_status fm_op_create_hadamard(fm_op* out, int64_t n, fm_dtype dt) {
  set_error("");
  CHECK_OUT(out);
  FM_CHECK_ARG(valid_dtype(dt), FM_E_INVALID, "unknown dtype %d", int(dt));
  FM_CHECK_ARG(n >= 1 && is_pow2(n) && ilog2(n) <= 26, FM_E_UNSUPPORTED,
               "Hadamard size %lld: powers of two up to 2^26 are supported", (long long)n);
  fm_op_s* op;
  FM_TRY(new_op(Kind::Hadamard, dt, n, n, &op));
  return publish(op, out);
}

fm_status fm_op_create_diag(fm_op* out, int64_t n, const void* d, fm_dtype dt, void* stream) {
  set_error("");
  CHECK_OUT(out);
  FM_CHECK_ARG(valid_dtype(dt), FM_E_INVALID, "unknown dtype %d", int(dt));
  FM_CHECK_ARG(is_complex(dt), FM_E_DTYPE, "Diag needs a complex dtype");
  FM_CHECK_ARG(n >= 1, FM_E_INVALID, "Diag size must be positive");
  FM_CHECK_ARG(d != nullptr, FM_E_INVALID, "Diag: NULL diagonal");
  hipStream_t s = as_stream(stream);
  fm_op_s* op;
  FM_TRY(new_op(Kind::Diag, dt, n, n, &op));
  Building g{op};
  FM_TRY(store_params(op, d, n, s));
  FM_HIP(hipStreamSynchronize(s));
  return publish(g.release(), out);
}

fm_status fm_op_create_dense(fm_op* out, int64_t m, int64_t n, const void* a, int64_t lda,
                             fm_dtype dt, void* stream) {
  set_error("");
  CHECK_OUT(out);
  FM_CHECK_ARG(valid_dtype(dt), FM_E_INVALID, "unknown dtype %d", int(dt));
  FM_CHECK_ARG(is_complex(dt), FM_E_DTYPE, "Dense needs a complex dtype");
  FM_CHECK_ARG(m >= 1 && n >= 1, FM_E_INVALID, "Dense shape must be positive");
  FM_CHECK_ARG(lda >= m, FM_E_SHAPE, "Dense: lda %lld < m %lld", (long long)lda, (long long)m);
  FM_CHECK_ARG(a != nullptr, FM_E_INVALID, "Dense: NULL matrix");
  hipStream_t s = as_stream(stream);
  fm_op_s* op;
  FM_TRY(new_op(Kind::Dense, dt, m, n, &op));
  Building g{op};
  const size_t es = elem_size(dt);
  DevBuf packed;
  FM_TRY(packed.alloc(size_t(m * n) * es));
  FM_HIP(hipMemcpy2DAsync(packed.p, size_t(m) * es, a, size_t(lda) * es, size_t(m) * es, size_t(n),
                          hipMemcpyDeviceToDevice, s));
  FM_TRY(store_params(op, packed.p, m * n, s));
  op->lda = m;
  if (m * n <= (int64_t(1) << 22)) {  // record a real matrix (kernels then skip the imaginary parts)
    std::vector<double> h(size_t(m * n) * 2);
    FM_HIP(hipMemcpyAsync(h.data(), op->p64.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    FM_HIP(hipStreamSynchronize(s));
    bool real = true;
    for (size_t i = 1; i < h.size() && real; i += 2) real = h[i] == 0.0;
    op->real_entries = real;
  }
  FM_HIP(hipStreamSynchronize(s));
  return publish(g.release(), out);
}

fm_status fm_op_create_circulant(fm_op* out, int64_t n, const void* c, fm_dtype dt, void* stream) {
  set_error("");
  CHECK_OUT(out);
  FM_CHECK_ARG(valid_dtype(dt), FM_E_INVALID, "unknown dtype %d", int(dt));
  FM_CHECK_ARG(is_complex(dt), FM_E_DTYPE, "Circulant needs a complex dtype");
  FM_CHECK_ARG(n >= 1 && n <= (int64_t(1) << kMaxLog), FM_E_UNSUPPORTED,
               "Circulant size %lld: 1 .. 2^20 are supported", (long long)n);
  FM_CHECK_ARG(is_pow2(n) || n <= (int64_t(1) << (kMaxLog - 1)), FM_E_UNSUPPORTED,
               "Circulant size %lld: sizes that are not powers of two go up to 2^19", (long long)n);
  FM_CHECK_ARG(c != nullptr, FM_E_INVALID, "Circulant: NULL generator");
  hipStream_t s = as_stream(stream);
  if (!is_pow2(n)) {
    // C(c) is the n x n Toeplitz with first column c and first row
    // (c_0, c_{n-1}, ..., c_1): applied through the power-of-two embedding
    const size_t es = elem_size(dt);
    std::vector<unsigned char> ch(size_t(n) * es), rh(size_t(n) * es);
    FM_HIP(hipMemcpyAsync(ch.data(), c, ch.size(), hipMemcpyDeviceToHost, s));
    FM_HIP(hipStreamSynchronize(s));
    std::memcpy(rh.data(), ch.data(), es);
    for (int64_t k = 1; k < n; ++k) std::memcpy(rh.data() + size_t(k) * es, ch.data() + size_t(n - k) * es, es);
    DevBuf rd;
    FM_TRY(rd.alloc(rh.size()));
    FM_HIP(hipMemcpy(rd.p, rh.data(), rh.size(), hipMemcpyHostToDevice));
    return fm_op_create_toeplitz(out, n, n, c, rd.p, dt, stream);
  }
  fm_op_s* op;
  FM_TRY(new_op(Kind::Circulant, dt, n, n, &op));
  Building g{op};
  op->L = n;
  op->s32 = split_for(Elem::C64, ilog2(n));
  op->s64 = split_for(Elem::C128, ilog2(n));
  DevBuf c128, ghat;
  FM_TRY(c128.alloc(size_t(n) * 16));
  FM_TRY(ghat.alloc(size_t(n) * 16));
  if (dt == FM_C64)
    FM_TRY(launch_c64_to_c128(n, c, c128.p, s));
  else
    FM_HIP(hipMemcpyAsync(c128.p, c, size_t(n) * 16, hipMemcpyDeviceToDevice, s));
  // C = F^-1 diag(F c) F: spectrum F c with the 1/n of the inverse folded in
  FM_TRY(dft128(n, c128.p, ghat.p, 1.0 / double(n), s));
  FM_TRY(store_spectrum(op, ghat.p, s));
  FM_HIP(hipStreamSynchronize(s));
  op->gen = std::move(c128);  // the generator in FP64: columns C e_j for OMP
  return publish(g.release(), out);
}

fm_status fm_op_create_lfsr_circulant(fm_op* out, int32_t order, uint64_t taps, uint64_t state, fm_dtype dt,
                                       void* stream) {
  set_error("");
  CHECK_OUT(out);
  FM_CHECK_ARG(valid_dtype(dt), FM_E_INVALID, "unknown dtype %d", int(dt));
  FM_CHECK_ARG(is_complex(dt), FM_E_DTYPE, "LFSR circulant needs a complex dtype");
  FM_CHECK_ARG(order >= 2 && order <= kMaxLog - 1, FM_E_UNSUPPORTED, "LFSR order %d: 2 .. 19 are supported",
               int(order));
  const uint64_t mask = (uint64_t(1) << order) - 1;
  FM_CHECK_ARG((taps & mask) != 0 && (taps & ~mask) == 0, FM_E_INVALID, "LFSR taps must lie in the low %d bits",
               int(order));
  FM_CHECK_ARG((state & mask) != 0 && (state & ~mask) == 0, FM_E_INVALID,
               "LFSR state must be nonzero and lie in the low %d bits", int(order));
  const int64_t n = int64_t(mask);
  const size_t es = elem_size(dt);
  std::vector<unsigned char> ch(size_t(n) * es, 0);
  uint64_t r = state;
  for (int64_t k = 0; k < n; ++k) {
    const double v = (r & 1) ? -1.0 : 1.0;  // output bit 0 -> +1, 1 -> -1
    if (dt == FM_C64)
      reinterpret_cast<float*>(ch.data())[2 * k] = float(v);
    else
      reinterpret_cast<double*>(ch.data())[2 * k] = v;
    const uint64_t fb = uint64_t(__builtin_popcountll(r & taps) & 1);
    r = (r >> 1) | (fb << (order - 1));
  }
  DevBuf cd;
  FM_TRY(cd.alloc(ch.size()));
  FM_HIP(hipMemcpy(cd.p, ch.data(), ch.size(), hipMemcpyHostToDevice));
  return fm_op_create_circulant(out, n, cd.p, dt, stream);
}

}  // extern "C"

namespace {

// Embedding length of a Toeplitz operator: the smallest L >= need among the
// powers of two and, above 4096, the mixed lengths 4096 * n2 whose strided
// passes exist (FM_EMBED=pow2 keeps powers of two).
int64_t embed_length(int64_t need) {
  int64_t best = next_pow2(need);
  static const bool pow2_only = [] {
    const char* e = std::getenv("FM_EMBED");
    return e != nullptr && std::strcmp(e, "pow2") == 0;
  }();
  if (need <= 4096 || pow2_only) return best;
  for (int n2 : {3, 5, 6, 9, 10, 12, 20, 24, 30}) {
    const int64_t L = int64_t(4096) * n2;
    if (L >= need && L < best) best = L;
  }
  return best;
}

// In-place forward DFT of 4096 points in FP64 (iterative radix 2).
void host_fft4096(std::vector<std::complex<double>>& a, const std::vector<std::complex<double>>& w) {
  const int n = 4096;
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (int len = 2; len <= n; len <<= 1) {
    const int half = len >> 1, stride = n / len;
    for (int i = 0; i < n; i += len)
      for (int k = 0; k < half; ++k) {
        const std::complex<double> u = a[i + k], v = a[i + k + half] * w[size_t(k) * stride];
        a[i + k] = u + v;
        a[i + k + half] = u - v;
      }
  }
}

// Spectrum of a mixed length L = 4096 n2 in the row order the four-step
// convolution reads, in FP64: row k2 holds ghat[k2 + n2 k1] / L at k1, with
// ghat = DFT_L(g); row k2 = DFT_4096 of W_L^(n1 k2) sum_j g[n1 + 4096 j] W_n2^(j k2).
std::vector<std::complex<double>> mixed_spectrum(const std::vector<std::complex<double>>& g, int64_t L) {
  const int n2 = int(L / 4096);
  std::vector<std::complex<double>> w4096(2048);
  std::vector<std::complex<double>> out(static_cast<size_t>(L));
  for (int k = 0; k < 2048; ++k) {
    double re, im;
    root_of_unity(k, 4096, &re, &im);
    w4096[size_t(k)] = {re, im};
  }
  std::vector<std::complex<double>> row(4096);
  for (int k2 = 0; k2 < n2; ++k2) {
    std::vector<std::complex<double>> wn(static_cast<size_t>(n2));
    for (int j = 0; j < n2; ++j) {
      double re, im;
      root_of_unity(int64_t(4096) * ((int64_t(j) * k2) % n2), L, &re, &im);  // W_n2^(j k2)
      wn[size_t(j)] = {re, im};
    }
    for (int n1 = 0; n1 < 4096; ++n1) {
      std::complex<double> acc = 0.0;
      for (int j = 0; j < n2; ++j) acc += g[size_t(n1 + 4096 * j)] * wn[size_t(j)];
      double re, im;
      root_of_unity(int64_t(n1) * k2, L, &re, &im);  // W_L^(n1 k2)
      row[size_t(n1)] = acc * std::complex<double>(re, im);
    }
    host_fft4096(row, w4096);
    for (int k1 = 0; k1 < 4096; ++k1) out[size_t(k1 + 4096 * k2)] = row[size_t(k1)] / double(L);
  }
  return out;
}

}  // namespace

extern "C" {

fm_status fm_op_create_toeplitz(fm_op* out, int64_t m, int64_t n, const void* col, const void* row,
                                fm_dtype dt, void* stream) {
  set_error("");
  CHECK_OUT(out);
  FM_CHECK_ARG(valid_dtype(dt), FM_E_INVALID, "unknown dtype %d", int(dt));
  FM_CHECK_ARG(is_complex(dt), FM_E_DTYPE, "Toeplitz needs a complex dtype");
  FM_CHECK_ARG(m >= 1 && n >= 1, FM_E_INVALID, "Toeplitz shape must be positive");
  FM_CHECK_ARG(col != nullptr && (row != nullptr || n == 1), FM_E_INVALID, "Toeplitz: NULL generator");
  FM_CHECK_ARG(m + n - 1 <= (int64_t(1) << kMaxLog), FM_E_UNSUPPORTED,
               "Toeplitz %lld x %lld: embedding length above 2^20", (long long)m, (long long)n);
  const int64_t L = embed_length(m + n - 1);
  const bool mixed = !is_pow2(L);
  hipStream_t s = as_stream(stream);
  fm_op_s* op;
  FM_TRY(new_op(Kind::Toeplitz, dt, m, n, &op));
  Building g{op};
  op->L = L;
  op->s32 = mixed ? split_mixed(L) : split_for(Elem::C64, ilog2(L));
  op->s64 = mixed ? split_mixed(L) : split_for(Elem::C128, ilog2(L));
  DevBuf emb, ghat;
  FM_TRY(emb.alloc(size_t(L) * 16));
  FM_TRY(launch_toeplitz_embed(m, n, L, col, row != nullptr ? row : col, dt == FM_C64, emb.p, s));
  if (mixed) {  // FP64 on the host, already in the four-step row order
    std::vector<std::complex<double>> gh(static_cast<size_t>(L));
    FM_HIP(hipMemcpyAsync(gh.data(), emb.p, size_t(L) * 16, hipMemcpyDeviceToHost, s));
    FM_HIP(hipStreamSynchronize(s));
    const std::vector<std::complex<double>> P = mixed_spectrum(gh, L);
    FM_TRY(op->p64.alloc(size_t(L) * 16));
    FM_HIP(hipMemcpyAsync(op->p64.p, P.data(), size_t(L) * 16, hipMemcpyHostToDevice, s));
    if (dt == FM_C64) {
      FM_TRY(op->p32.alloc(size_t(L) * 8));
      FM_TRY(launch_spectrum_c64(L, op->p64.p, op->p32.p, s));
    }
    FM_HIP(hipStreamSynchronize(s));
  } else {
    FM_TRY(ghat.alloc(size_t(L) * 16));
    FM_TRY(dft128(L, emb.p, ghat.p, 1.0 / double(L), s));
    FM_TRY(store_spectrum(op, ghat.p, s));
  }
  FM_HIP(hipStreamSynchronize(s));
  op->gen = std::move(emb);  // the embedded generator in FP64: the inverse (Levinson) and columns T e_j (OMP)
  return publish(g.release(), out);
}

fm_status fm_op_create_mltoeplitz(fm_op* out, int32_t levels, const int64_t* n_per_level,
                                  const void* t, fm_dtype dt, void* stream) {
  set_error("");
  CHECK_OUT(out);
  FM_CHECK_ARG(valid_dtype(dt), FM_E_INVALID, "unknown dtype %d", int(dt));
  FM_CHECK_ARG(is_complex(dt), FM_E_DTYPE, "multilevel Toeplitz needs a complex dtype");
  FM_CHECK_ARG(levels >= 1 && levels <= 3, FM_E_UNSUPPORTED, "multilevel Toeplitz: 1..3 levels");
  FM_CHECK_ARG(n_per_level != nullptr && t != nullptr, FM_E_INVALID, "multilevel Toeplitz: NULL argument");
  std::vector<int64_t> lv(levels), lL(levels);
  int64_t size = 1, tsize = 1, total = 1;
  for (int l = 0; l < levels; ++l) {
    FM_CHECK_ARG(n_per_level[l] >= 1, FM_E_INVALID, "multilevel Toeplitz: level sizes must be positive");
    lv[l] = n_per_level[l];
    lL[l] = next_pow2(2 * lv[l] - 1);
    FM_CHECK_ARG(ilog2(lL[l]) <= fft_lds_max_log(Elem::C128), FM_E_UNSUPPORTED,
                 "multilevel Toeplitz: level %d too long", l);
    size *= lv[l];
    tsize *= 2 * lv[l] - 1;
    total *= lL[l];
  }
  hipStream_t s = as_stream(stream);
  fm_op_s* op;
  FM_TRY(new_op(Kind::MLToeplitz, dt, size, size, &op));
  Building g{op};
  op->lv = lv;
  op->lL = lL;
  // Kron of the per-level Fourier matrices: the multi-dimensional DFT
  std::vector<fm_op> fs(levels);
  for (int l = 0; l < levels; ++l) {
    fm_status st = fm_op_create_fourier(&fs[l], lL[l], dt);
    if (st != FM_OK) {
      for (int k = 0; k < l; ++k) fm_op_release(fs[k]);
      return st;
    }
  }
  fm_op kf;
  fm_status st = fm_op_compose(&kf, FM_KRON, levels, fs.data());
  for (int l = 0; l < levels; ++l) fm_op_release(fs[l]);
  FM_TRY(st);
  op->terms.push_back(kf);
  // embed the generator on the host in FP64: offset o_l lands at o_l mod L_l
  const size_t es = elem_size(dt);
  std::vector<unsigned char> th(size_t(tsize) * es);
  FM_HIP(hipMemcpyAsync(th.data(), t, th.size(), hipMemcpyDeviceToHost, s));
  FM_HIP(hipStreamSynchronize(s));
  std::vector<double> gh(size_t(total) * 2, 0.0);
  for (int64_t k = 0; k < tsize; ++k) {
    int64_t rem = k, pos = 0, stride = 1;
    for (int l = levels - 1; l >= 0; --l) {
      const int64_t w = 2 * lv[l] - 1;
      const int64_t idx = rem % w;
      rem /= w;
      const int64_t off = idx - (lv[l] - 1);
      pos += ((off % lL[l] + lL[l]) % lL[l]) * stride;
      stride *= lL[l];
    }
    double re, im;
    if (dt == FM_C64) {
      const float* f = reinterpret_cast<const float*>(th.data()) + 2 * k;
      re = f[0];
      im = f[1];
    } else {
      const double* f = reinterpret_cast<const double*>(th.data()) + 2 * k;
      re = f[0];
      im = f[1];
    }
    gh[2 * pos] = re;
    gh[2 * pos + 1] = im;
  }
  DevBuf gd, ghat, wsb;
  FM_TRY(gd.alloc(size_t(total) * 16));
  FM_TRY(ghat.alloc(size_t(total) * 16));
  FM_HIP(hipMemcpyAsync(gd.p, gh.data(), size_t(total) * 16, hipMemcpyHostToDevice, s));
  {
    Batch b{1, 1, 1, total, total, total, total};
    Workspace ws;
    ws.sizing = true;
    FM_TRY(exec(kf, false, Elem::C128, b, gd.p, ghat.p, false, ws, s));
    FM_TRY(wsb.alloc(ws.peak));
    Workspace run;
    run.base = static_cast<char*>(wsb.p);
    run.cap = wsb.bytes;
    FM_TRY(exec(kf, false, Elem::C128, b, gd.p, ghat.p, false, run, s));
  }
  FM_TRY(op->p64.alloc(size_t(total) * 16));
  FM_TRY(launch_scale_copy(Elem::C128, total, 1.0 / double(total), ghat.p, op->p64.p, s));
  if (dt == FM_C64) {
    FM_TRY(op->p32.alloc(size_t(total) * 8));
    FM_TRY(launch_c128_to_c64(total, op->p64.p, op->p32.p, s));
  }
  FM_HIP(hipStreamSynchronize(s));
  return publish(g.release(), out);
}

fm_status fm_op_create_select_rows(fm_op* out, int64_t n_in, int64_t m, const int32_t* idx,
                                   fm_dtype dt, void* stream) {
  set_error("");
  CHECK_OUT(out);
  FM_CHECK_ARG(valid_dtype(dt), FM_E_INVALID, "unknown dtype %d", int(dt));
  FM_CHECK_ARG(n_in >= 1 && m >= 0 && m <= n_in, FM_E_SHAPE, "selection: need 0 <= m <= n_in");
  FM_CHECK_ARG(n_in < (int64_t(1) << 31), FM_E_UNSUPPORTED, "selection: n_in must fit int32");
  FM_CHECK_ARG(idx != nullptr || m == 0, FM_E_INVALID, "selection: NULL indices");
  hipStream_t s = as_stream(stream);
  fm_op_s* op;
  FM_TRY(new_op(Kind::Select, dt, m, n_in, &op));
  Building g{op};
  FM_TRY(op->idx.alloc(size_t(m > 0 ? m : 1) * 4));
  if (m > 0) {
    FM_HIP(hipMemcpyAsync(op->idx.p, idx, size_t(m) * 4, hipMemcpyDeviceToDevice, s));
    DevBuf flags;
    FM_TRY(flags.alloc(size_t(n_in + 1) * 4));
    FM_HIP(hipMemsetAsync(flags.p, 0, flags.bytes, s));
    FM_TRY(launch_check_indices(n_in, m, static_cast<const int32_t*>(op->idx.p),
                                static_cast<int*>(flags.p), s));
    int bad = 0;
    FM_HIP(hipMemcpyAsync(&bad, static_cast<int*>(flags.p) + n_in, 4, hipMemcpyDeviceToHost, s));
    FM_HIP(hipStreamSynchronize(s));
    FM_CHECK_ARG(bad == 0, FM_E_SHAPE, "selection: indices must be distinct and in [0, n_in)");
    FM_TRY(op->inv.alloc(size_t(n_in) * 4));
    FM_TRY(launch_invert_indices(n_in, m, static_cast<const int32_t*>(op->idx.p), static_cast<int32_t*>(op->inv.p),
                                 s));
    FM_HIP(hipStreamSynchronize(s));
  }
  return publish(g.release(), out);
}

fm_status fm_op_compose(fm_op* out, fm_compose_kind kind, int32_t nterms, const fm_op* terms) {
  set_error("");
  CHECK_OUT(out);
  FM_CHECK_ARG(nterms >= 1 && terms != nullptr, FM_E_INVALID, "compose: need at least one term");
  FM_CHECK_ARG(kind >= FM_PRODUCT && kind <= FM_BLKDIAG, FM_E_INVALID, "compose: unknown kind");
  for (int i = 0; i < nterms; ++i) {
    CHECK_LIVE(terms[i]);
    FM_CHECK_ARG(terms[i]->dt == terms[0]->dt, FM_E_DTYPE, "compose: terms have different dtypes");
  }
  int64_t m = 0, n = 0;
  Kind k = Kind::Product;
  switch (kind) {
    case FM_PRODUCT:
      k = Kind::Product;
      for (int i = 0; i + 1 < nterms; ++i)
        FM_CHECK_ARG(terms[i]->n == terms[i + 1]->m, FM_E_SHAPE,
                     "product: term %d has %lld columns, term %d has %lld rows", i,
                     (long long)terms[i]->n, i + 1, (long long)terms[i + 1]->m);
      m = terms[0]->m;
      n = terms[nterms - 1]->n;
      break;
    case FM_SUM:
      k = Kind::Sum;
      for (int i = 1; i < nterms; ++i)
        FM_CHECK_ARG(terms[i]->m == terms[0]->m && terms[i]->n == terms[0]->n, FM_E_SHAPE,
                     "sum: terms differ in shape");
      m = terms[0]->m;
      n = terms[0]->n;
      break;
    case FM_KRON:
      k = Kind::Kron;
      m = n = 1;
      for (int i = 0; i < nterms; ++i) {
        m *= terms[i]->m;
        n *= terms[i]->n;
      }
      break;
    case FM_BLKDIAG:
      k = Kind::BlkDiag;
      for (int i = 0; i < nterms; ++i) {
        m += terms[i]->m;
        n += terms[i]->n;
      }
      break;
  }
  fm_op_s* op;
  FM_TRY(new_op(k, terms[0]->dt, m, n, &op));
  for (int i = 0; i < nterms; ++i) {
    terms[i]->refs.fetch_add(1);
    op->terms.push_back(terms[i]);
  }
  return publish(op, out);
}

fm_status fm_op_create_blocks(fm_op* out, int32_t nbr, int32_t nbc, const fm_op* terms) {
  set_error("");
  CHECK_OUT(out);
  FM_CHECK_ARG(nbr >= 1 && nbc >= 1 && terms != nullptr, FM_E_INVALID, "blocks: need a non-empty grid");
  FM_CHECK_ARG(int64_t(nbr) * nbc <= (int64_t(1) << 20), FM_E_UNSUPPORTED, "blocks: more than 2^20 blocks");
  const int64_t nb = int64_t(nbr) * nbc;
  for (int64_t k = 0; k < nb; ++k) {
    CHECK_LIVE(terms[k]);
    FM_CHECK_ARG(terms[k]->dt == terms[0]->dt, FM_E_DTYPE, "blocks: blocks have different dtypes");
  }
  std::vector<int64_t> roff(nbr + 1, 0), coff(nbc + 1, 0);
  for (int i = 0; i < nbr; ++i) {
    for (int j = 1; j < nbc; ++j)
      FM_CHECK_ARG(terms[i * nbc + j]->m == terms[i * nbc]->m, FM_E_SHAPE,
                   "blocks: block (%d, %d) has %lld rows, block (%d, 0) has %lld", i, j,
                   (long long)terms[i * nbc + j]->m, i, (long long)terms[i * nbc]->m);
    roff[i + 1] = roff[i] + terms[i * nbc]->m;
  }
  for (int j = 0; j < nbc; ++j) {
    for (int i = 1; i < nbr; ++i)
      FM_CHECK_ARG(terms[i * nbc + j]->n == terms[j]->n, FM_E_SHAPE,
                   "blocks: block (%d, %d) has %lld columns, block (0, %d) has %lld", i, j,
                   (long long)terms[i * nbc + j]->n, j, (long long)terms[j]->n);
    coff[j + 1] = coff[j] + terms[j]->n;
  }
  fm_op_s* op;
  FM_TRY(new_op(Kind::Blocks, terms[0]->dt, roff[nbr], coff[nbc], &op));
  Building g{op};
  for (int64_t k = 0; k < nb; ++k) {
    terms[k]->refs.fetch_add(1);
    op->terms.push_back(terms[k]);
  }
  op->nbr = nbr;
  op->nbc = nbc;
  op->roff = roff;
  op->coff = coff;
  // spectral mixing applies when every block is a multilevel Toeplitz of one geometry
  bool mix = true;
  for (int64_t k = 0; k < nb && mix; ++k)
    mix = terms[k]->kind == Kind::MLToeplitz && terms[k]->lv == terms[0]->lv && terms[k]->lL == terms[0]->lL;
  if (mix) {
    // pack the block spectra bin-tiled (tiles of up to 64 bins) for the mixing kernel
    int64_t total = 1;
    for (int64_t l : terms[0]->lL) total *= l;
    op->mix_logtw = ilog2(total < 64 ? total : 64);
    std::vector<const void*> t32(nb), t64(nb);
    for (int64_t k = 0; k < nb; ++k) {
      t32[k] = terms[k]->p32.p;
      t64[k] = terms[k]->p64.p;
    }
    DevBuf tab;
    FM_TRY(tab.alloc(size_t(nb) * sizeof(void*)));
    FM_HIP(hipMemcpy(tab.p, t64.data(), size_t(nb) * sizeof(void*), hipMemcpyHostToDevice));
    FM_TRY(op->p64.alloc(size_t(nb * total) * 16));
    FM_TRY(launch_block_pack(Elem::C128, nb, total, op->mix_logtw, tab.p, op->p64.p, nullptr));
    if (op->dt == FM_C64) {
      FM_HIP(hipDeviceSynchronize());
      FM_HIP(hipMemcpy(tab.p, t32.data(), size_t(nb) * sizeof(void*), hipMemcpyHostToDevice));
      FM_TRY(op->p32.alloc(size_t(nb * total) * 8));
      FM_TRY(launch_block_pack(Elem::C64, nb, total, op->mix_logtw, tab.p, op->p32.p, nullptr));
    }
    FM_HIP(hipDeviceSynchronize());
    op->lv = terms[0]->lv;
    op->lL = terms[0]->lL;
  }
  op->mix = mix;
  return publish(g.release(), out);
}

fm_status fm_op_adjoint(fm_op* out, fm_op a) {
  set_error("");
  CHECK_OUT(out);
  CHECK_LIVE(a);
  fm_op_s* op;
  FM_TRY(new_op(Kind::Adjoint, a->dt, a->n, a->m, &op));
  a->refs.fetch_add(1);
  op->terms.push_back(a);
  return publish(op, out);
}

fm_status fm_op_conj(fm_op* out, fm_op a) {
  set_error("");
  CHECK_OUT(out);
  CHECK_LIVE(a);
  fm_op_s* op;
  FM_TRY(new_op(Kind::Conj, a->dt, a->m, a->n, &op));
  a->refs.fetch_add(1);
  op->terms.push_back(a);
  return publish(op, out);
}

}  // extern "C"

namespace {

// Owns a handle until it is released or handed out.
struct Held {
  fm_op h = nullptr;
  ~Held() {
    if (h) fm_op_release(h);
  }
  fm_op give() {
    fm_op r = h;
    h = nullptr;
    return r;
  }
};

// Diagonal operator with every entry equal to `value`.
fm_status diag_const(int64_t n, double value, fm_dtype dt, fm_op* out) {
  const size_t es = elem_size(dt);
  std::vector<unsigned char> host(size_t(n) * es, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (dt == FM_C64)
      reinterpret_cast<float*>(host.data())[2 * i] = float(value);
    else
      reinterpret_cast<double*>(host.data())[2 * i] = value;
  }
  DevBuf d;
  FM_TRY(d.alloc(host.size()));
  FM_HIP(hipMemcpy(d.p, host.data(), host.size(), hipMemcpyHostToDevice));
  return fm_op_create_diag(out, n, d.p, dt, nullptr);
}

// New operator of src's kind and geometry whose parameters are an
// elementwise map of src's FP64 parameters (mode / scale as launch_param_map),
// rounded once for complex64.
fm_status derive_params(const fm_op_s* src, int64_t count, int mode, double scale, fm_op* out) {
  FM_CHECK_ARG(src->s32.log1 == src->s64.log1 && src->s32.log2 == src->s64.log2, FM_E_UNSUPPORTED,
               "parameter orders differ between precisions");
  fm_op_s* op;
  FM_TRY(new_op(src->kind, src->dt, src->m, src->n, &op));
  Building g{op};
  op->L = src->L;
  op->s32 = src->s32;
  op->s64 = src->s64;
  op->lv = src->lv;
  op->lL = src->lL;
  DevBuf flag;
  FM_TRY(flag.alloc(sizeof(int)));
  FM_HIP(hipMemset(flag.p, 0, sizeof(int)));
  FM_TRY(op->p64.alloc(size_t(count) * 16));
  FM_TRY(launch_param_map(count, mode, scale, src->p64.p, op->p64.p, static_cast<int*>(flag.p), nullptr));
  if (op->dt == FM_C64) {
    FM_TRY(op->p32.alloc(size_t(count) * 8));
    if (op->kind == Kind::Circulant || op->kind == Kind::Toeplitz)
      FM_TRY(launch_spectrum_c64(count, op->p64.p, op->p32.p, nullptr));  // convolution spectra: pair order
    else
      FM_TRY(launch_c128_to_c64(count, op->p64.p, op->p32.p, nullptr));
  }
  int bad = 0;
  FM_HIP(hipMemcpy(&bad, flag.p, sizeof(int), hipMemcpyDeviceToHost));
  FM_CHECK_ARG(bad == 0, FM_E_INVALID, "the operator is singular (a zero eigenvalue or diagonal entry)");
  return publish(g.release(), out);
}

fm_status compose_of(fm_compose_kind k, std::vector<Held>& parts, fm_op* out) {
  std::vector<fm_op> hs;
  for (Held& p : parts) hs.push_back(p.h);
  return fm_op_compose(out, k, int32_t(hs.size()), hs.data());
}

fm_status gram_of(const fm_op_s* a, fm_op* out);
fm_status inverse_of(const fm_op_s* a, fm_op* out);

fm_status gram_of(const fm_op_s* a, fm_op* out) {
  switch (a->kind) {
    case Kind::Circulant:  // C^H C = F^-1 diag(|c_hat|^2) F; the stored spectrum carries 1/L
      return derive_params(a, a->L, 0, double(a->L), out);
    case Kind::Diag:
      return derive_params(a, a->n, 0, 1.0, out);
    case Kind::Fourier:
    case Kind::Hadamard:  // F^H F = H^T H = n I
      return diag_const(a->n, double(a->n), a->dt, out);
    case Kind::Select: {  // S^H S = diag(1 at the selected indices)
      std::vector<int32_t> idx(size_t(a->m));
      if (a->m > 0) FM_HIP(hipMemcpy(idx.data(), a->idx.p, size_t(a->m) * 4, hipMemcpyDeviceToHost));
      const size_t es = elem_size(a->dt);
      std::vector<unsigned char> host(size_t(a->n) * es, 0);
      for (int32_t i : idx) {
        if (a->dt == FM_C64)
          reinterpret_cast<float*>(host.data())[2 * size_t(i)] = 1.0f;
        else
          reinterpret_cast<double*>(host.data())[2 * size_t(i)] = 1.0;
      }
      DevBuf d;
      FM_TRY(d.alloc(host.size()));
      FM_HIP(hipMemcpy(d.p, host.data(), host.size(), hipMemcpyHostToDevice));
      return fm_op_create_diag(out, a->n, d.p, a->dt, nullptr);
    }
    case Kind::Kron:
    case Kind::BlkDiag: {  // (A (x) B)^H (A (x) B) = A^H A (x) B^H B; block diagonal likewise
      std::vector<Held> parts(a->terms.size());
      for (size_t i = 0; i < a->terms.size(); ++i) FM_TRY(gram_of(a->terms[i], &parts[i].h));
      return compose_of(a->kind == Kind::Kron ? FM_KRON : FM_BLKDIAG, parts, out);
    }
    case Kind::Conj: {  // conj(A)^H conj(A) = conj(A^H A)
      Held g;
      FM_TRY(gram_of(a->terms[0], &g.h));
      return fm_op_conj(out, g.h);
    }
    default: {
      Held ah;
      FM_TRY(fm_op_adjoint(&ah.h, const_cast<fm_op_s*>(a)));
      std::vector<fm_op> t{ah.h, const_cast<fm_op_s*>(a)};
      return fm_op_compose(out, FM_PRODUCT, 2, t.data());
    }
  }
}

fm_status inverse_of(const fm_op_s* a, fm_op* out) {
  FM_CHECK_ARG(a->m == a->n, FM_E_SHAPE, "inverse of a non-square operator (%lld x %lld)", (long long)a->m,
               (long long)a->n);
  switch (a->kind) {
    case Kind::Circulant:  // spectrum 1/c_hat; stored with 1/L: 1/(s L^2)
      return derive_params(a, a->L, 1, 1.0 / (double(a->L) * double(a->L)), out);
    case Kind::Diag:
      return derive_params(a, a->n, 1, 1.0, out);
    case Kind::Fourier:
    case Kind::Hadamard: {  // F^-1 = F^H / n, H^-1 = H / n
      Held d, t;
      FM_TRY(diag_const(a->n, 1.0 / double(a->n), a->dt, &d.h));
      if (a->kind == Kind::Fourier)
        FM_TRY(fm_op_adjoint(&t.h, const_cast<fm_op_s*>(a)));
      else {
        fm_op_s* self = const_cast<fm_op_s*>(a);
        self->refs.fetch_add(1);
        t.h = self;
      }
      std::vector<fm_op> hs{d.h, t.h};
      return fm_op_compose(out, FM_PRODUCT, 2, hs.data());
    }
    case Kind::Select:  // a square selection is a permutation: S^-1 = S^H
      return fm_op_adjoint(out, const_cast<fm_op_s*>(a));
    case Kind::Toeplitz: {  // applied by Levinson solves
      FM_CHECK_ARG(a->gen.p != nullptr, FM_E_UNSUPPORTED, "Toeplitz without a stored generator");
      fm_op_s* op;
      FM_TRY(new_op(Kind::ToeplitzInv, a->dt, a->n, a->n, &op));
      fm_op_s* self = const_cast<fm_op_s*>(a);
      self->refs.fetch_add(1);
      op->terms.push_back(self);
      return publish(op, out);
    }
    case Kind::ToeplitzInv: {  // (T^-1)^-1 = T
      fm_op_s* t = a->terms[0];
      t->refs.fetch_add(1);
      *out = t;
      return FM_OK;
    }
    case Kind::Adjoint:
    case Kind::Conj: {
      Held i;
      FM_TRY(inverse_of(a->terms[0], &i.h));
      return a->kind == Kind::Adjoint ? fm_op_adjoint(out, i.h) : fm_op_conj(out, i.h);
    }
    case Kind::Kron:
    case Kind::BlkDiag:
    case Kind::Product: {  // (A B)^-1 = B^-1 A^-1 (square factors)
      const size_t k = a->terms.size();
      std::vector<Held> parts(k);
      for (size_t i = 0; i < k; ++i) {
        const fm_op_s* t = a->kind == Kind::Product ? a->terms[k - 1 - i] : a->terms[i];
        FM_TRY(inverse_of(t, &parts[i].h));
      }
      return compose_of(a->kind == Kind::Kron ? FM_KRON : a->kind == Kind::BlkDiag ? FM_BLKDIAG : FM_PRODUCT, parts,
                        out);
    }
    default:
      set_error("no structured inverse for this operator kind");
      return FM_E_UNSUPPORTED;
  }
}

}  // namespace

extern "C" {

fm_status fm_op_gram(fm_op* out, fm_op a) {
  set_error("");
  CHECK_OUT(out);
  CHECK_LIVE(a);
  FM_CHECK_ARG(is_complex(a->dt), FM_E_DTYPE, "Gram operator of an integer operator");
  return gram_of(a, out);
}

fm_status fm_op_inverse(fm_op* out, fm_op a) {
  set_error("");
  CHECK_OUT(out);
  CHECK_LIVE(a);
  FM_CHECK_ARG(is_complex(a->dt), FM_E_DTYPE, "inverse of an integer operator");
  return inverse_of(a, out);
}

fm_status fm_op_shape(fm_op a, int64_t* m, int64_t* n, fm_dtype* dt) {
  set_error("");
  CHECK_LIVE(a);
  if (m) *m = a->m;
  if (n) *n = a->n;
  if (dt) *dt = a->dt;
  return FM_OK;
}

fm_status fm_op_transform_length(fm_op a, int64_t* L) {
  set_error("");
  CHECK_LIVE(a);
  FM_CHECK_ARG(L != nullptr, FM_E_INVALID, "NULL output");
  const fm_op_s* c = a;
  if (c->kind == Kind::Fourier && !c->terms.empty())  // Bluestein: the product D T D
    for (const fm_op_s* t : c->terms[0]->terms)
      if (t->kind == Kind::Toeplitz) c = t;
  const bool cyclic = c->kind == Kind::Fourier || c->kind == Kind::Circulant || c->kind == Kind::Toeplitz;
  *L = cyclic ? c->L : 0;
  return FM_OK;
}

fm_status fm_op_release(fm_op a) {
  set_error("");
  CHECK_LIVE(a);
  drop(a);
  return FM_OK;
}

fm_status fm_workspace_size(fm_op a, fm_dir dir, int64_t ncols, size_t* bytes) {
  set_error("");
  CHECK_LIVE(a);
  FM_CHECK_ARG(bytes != nullptr, FM_E_INVALID, "NULL output");
  FM_CHECK_ARG(dir == FM_FWD || dir == FM_ADJ, FM_E_INVALID, "unknown direction");
  FM_CHECK_ARG(ncols >= 0, FM_E_INVALID, "negative column count");
  return size_of(a, dir == FM_ADJ, ncols, bytes);
}

fm_status fm_apply(fm_op a, fm_dir dir, int64_t ncols, const void* x, int64_t ldx, void* y,
                   int64_t ldy, void* ws, size_t ws_bytes, void* stream) {
  return apply_op(a, dir, ncols, x, ldx, y, ldy, ws, ws_bytes, true, stream);
}

}  // extern "C"
