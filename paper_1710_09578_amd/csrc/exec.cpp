// Executor: applies an operator tree to a strided batch of vectors.
//
// Composite operators are applied only through their terms' transforms
// (section "General Matrix-free Representations"): a Product applies its terms
// right to left (forward) or its term adjoints left to right (adjoint); a Sum
// accumulates its terms; a Kronecker product applies each factor as a mode
// product along its own axis (eq. (7) structure, first factor slowest); a
// block-diagonal operator applies each block to its slice of rows (runs of one
// repeated block in one batched call); a block matrix accumulates its blocks
// into the output slices, or, for multilevel Toeplitz blocks of one geometry,
// transforms each slice once and mixes the blocks per frequency bin. Leaves
// launch the HIP kernels. Temporaries come from a stack over the workspace.
#include <cstring>

#include "runtime.h"

namespace fm {

#define LAUNCH(expr)                     \
  do {                                   \
    if (!ws.sizing) FM_TRY(expr);        \
  } while (0)

namespace {

// (ncols, outer) pairs folded into one column index when the strides allow it.
bool fold_outer(const Batch& b, int64_t rows_in, int64_t rows_out, Batch* out) {
  *out = b;
  if (b.outer == 1) return true;
  if (b.inner != 1) return false;
  if ((b.ncols == 1 || b.ldx == b.outer * b.xvs) && (b.ncols == 1 || b.ldy == b.outer * b.yvs)) {
    out->ncols = b.ncols * b.outer;
    out->outer = 1;
    out->ldx = b.xvs;
    out->ldy = b.yvs;
    out->xvs = rows_in;
    out->yvs = rows_out;
    (void)rows_in;
    return true;
  }
  return false;
}

bool packed(const Batch& b, int64_t rows_in, int64_t rows_out) {
  return b.outer == 1 || (b.xvs == rows_in * b.inner && b.yvs == rows_out * b.inner);
}

const void* param(const fm_op_s* op, Elem e) { return e == Elem::C64 ? op->p32.p : op->p64.p; }
const Split& split(const fm_op_s* op, Elem e) { return e == Elem::C64 ? op->s32 : op->s64; }

// Plain DFT (or its unnormalised inverse) of length L along the vector axis.
fm_status exec_fourier(const fm_op_s* op, bool adj, Elem e, const Batch& b, const void* x, void* y,
                       bool acc, Workspace& ws, hipStream_t s) {
  if (!op->terms.empty()) return exec(op->terms[0], adj, e, b, x, y, acc, ws, s);  // Bluestein (any n)
  const Split& sp = split(op, e);
  const int64_t L = op->L;
  if (!sp.four_step()) {
    FftLaunch f;
    f.elem = e;
    f.logn = sp.logL;
    f.mode = adj ? FFT_INV : FFT_FWD;
    f.b = b;
    f.x = x;
    f.y = y;
    f.in_limit = f.out_limit = L * b.inner;
    f.accumulate = acc;
    LAUNCH(launch_fft(f, s));
    return FM_OK;
  }
  Batch fb;
  FM_CHECK_ARG(b.inner == 1 && fold_outer(b, L, L, &fb), FM_E_UNSUPPORTED,
               "Fourier of length %lld along a strided axis", (long long)L);
  const int64_t n1 = int64_t(1) << sp.log1, n2 = int64_t(1) << sp.log2;
  const size_t mk = ws.mark();
  void* w = ws.take(size_t(fb.ncols * L) * elem_bytes(e));
  // step 1: length-n2 transforms at stride n1, then twiddles W_L^(k2 n1)
  FftLaunch f1;
  f1.elem = e;
  f1.logn = sp.log2;
  f1.mode = adj ? FFT_INV : FFT_FWD;
  f1.b = Batch{fb.ncols, 1, n1, fb.ldx, 0, L, 0};
  f1.x = x;
  f1.y = w;
  f1.in_limit = f1.out_limit = L;
  f1.tw_log = sp.logL;
  f1.tw_inv = adj;
  LAUNCH(launch_fft(f1, s));
  // step 2: contiguous length-n1 transforms in place; result X[k2 + n2 k1] at k1 + n1 k2
  FftLaunch f2;
  f2.elem = e;
  f2.logn = sp.log1;
  f2.mode = adj ? FFT_INV : FFT_FWD;
  f2.b = Batch{fb.ncols, n2, 1, L, n1, L, n1};
  f2.x = w;
  f2.y = w;
  f2.in_limit = f2.out_limit = n1;
  LAUNCH(launch_fft(f2, s));
  // step 3: into natural order
  LAUNCH(launch_transpose(e, fb.ncols, n2, n1, w, L, y, fb.ldy, acc, s));
  ws.release(mk);
  return FM_OK;
}

// Four-step convolution of a mixed length L = 4096 * n2 (n2 5-smooth, not a
// power of two): rows formed from x with the strided n2-point DFT folded in
// (n2 <= 2^conv_max_fuse()) or a separate strided pass, the 4096-point row
// convolutions, then the strided inverse pass with the cropped store.
fm_status exec_conv_mixed(const fm_op_s* op, bool adj, Elem e, const Batch& b, const void* x, void* y, bool acc,
                          Workspace& ws, hipStream_t s) {
  const Split& sp = split(op, e);
  const int64_t L = op->L, n1 = 4096;
  const int n2 = sp.n2;
  const int64_t nin = in_rows(op, adj), nout = out_rows(op, adj);
  Batch fb;
  FM_CHECK_ARG(fold_outer(b, nin, nout, &fb) && fb.outer == 1, FM_E_UNSUPPORTED,
               "convolution of mixed length %lld on an unpacked batch", (long long)L);
  const void* twl = twiddle_table_L(e, L);
  FM_CHECK_ARG(twl != nullptr, FM_E_DEVICE, "twiddle table unavailable: %s", last_error());
  const size_t mk = ws.mark();
  void* w = ws.take(size_t(fb.ncols * L) * elem_bytes(e));
  FftLaunch fr;
  fr.elem = e;
  fr.logn = sp.log1;
  fr.mode = FFT_CONV;
  fr.b = Batch{fb.ncols, n2, 1, fb.ldx, 0, L, n1};
  fr.out_limit = n1;
  fr.spec = param(op, e);
  fr.spec_ostride = n1;
  fr.spec_conj = adj;
  fr.tw_log = 1;  // twiddle epilogue from twl
  fr.tw_inv = 1;
  fr.twl = twl;
  if (n2 <= (1 << conv_max_fuse())) {
    fr.x = x;
    fr.in_limit = nin;
    fr.fuse_n2 = n2;
  } else {
    LAUNCH(launch_mixed(e, n2, 0, fb.ncols, x, fb.ldx, nin, w, L, L, twl, L, 0, s));
    fr.b = Batch{fb.ncols, n2, 1, L, n1, L, n1};
    fr.x = w;
    fr.in_limit = n1;
  }
  fr.y = w;
  LAUNCH(launch_fft(fr, s));
  LAUNCH(launch_mixed(e, n2, 1, fb.ncols, w, L, L, y, fb.ldy, nout, twl, L, acc ? 1 : 0, s));
  ws.release(mk);
  return FM_OK;
}

// Cyclic convolution of length L with pad / crop (Circulant, Toeplitz):
// y = crop(IFFT(spec .* FFT(pad(x)))), spec conj'ed for the adjoint.
// omap (contiguous vectors, power-of-two L): a row selection's inverse map
// applied at the last pass's store (the output is S of the result: position
// p goes to row omap[p] of y, nowhere where -1).
fm_status exec_conv(const fm_op_s* op, bool adj, Elem e, const Batch& b, const void* x, void* y,
                    bool acc, Workspace& ws, hipStream_t s, const int32_t* omap = nullptr) {
  const Split& sp = split(op, e);
  const int64_t L = op->L;
  const int64_t nin = in_rows(op, adj), nout = out_rows(op, adj);
  const void* spec = param(op, e);
  FM_CHECK_ARG(!omap || (b.inner == 1 && b.outer == 1 && !sp.mixed()), FM_E_UNSUPPORTED,
               "convolution: row selection fused only on contiguous vectors");
  if (!sp.four_step()) {
    FftLaunch f;
    f.elem = e;
    f.logn = sp.logL;
    f.mode = FFT_CONV;
    f.b = b;
    f.x = x;
    f.y = y;
    f.in_limit = nin * b.inner;
    f.out_limit = nout * b.inner;
    f.spec = spec;
    f.spec_conj = adj;
    f.accumulate = acc;
    f.omap = omap;
    LAUNCH(launch_fft(f, s));
    return FM_OK;
  }
  FM_CHECK_ARG(b.inner == 1, FM_E_UNSUPPORTED, "convolution of length %lld along a strided axis",
               (long long)L);
  if (sp.mixed()) return exec_conv_mixed(op, adj, e, b, x, y, acc, ws, s);
  const int64_t n1 = int64_t(1) << sp.log1, n2 = int64_t(1) << sp.log2;
  const size_t mk = ws.mark();
  void* w = ws.take(size_t(b.ncols * b.outer * L) * elem_bytes(e));
  Batch fb;
  if (sp.log1 == fft_lds_max_log(e) && sp.log2 <= conv_max_fuse() && fold_outer(b, nin, nout, &fb) &&
      fb.outer == 1) {
    // rows k2 formed from x directly (strided n2-point transform folded into
    // the load), transform, spectral product, inverse, twiddles W_L^-(n1 k2)
    FftLaunch fr;
    fr.elem = e;
    fr.logn = sp.log1;
    fr.mode = FFT_CONV;
    fr.b = Batch{fb.ncols, n2, 1, fb.ldx, 0, L, n1};
    fr.x = x;
    fr.y = w;
    fr.in_limit = nin;
    fr.out_limit = n1;
    fr.spec = spec;
    fr.spec_ostride = n1;
    fr.spec_conj = adj;
    fr.tw_log = sp.logL;
    fr.tw_inv = 1;
    fr.fuse_n2 = int(n2);
    LAUNCH(launch_fft(fr, s));
  } else {
    // step 1: forward length-n2 transforms at stride n1 of the zero-padded
    // input, then twiddles W_L^(k2 n1)
    FftLaunch f1;
  f1.elem = e;
  f1.logn = sp.log2;
  f1.mode = FFT_FWD;
  f1.b = Batch{b.ncols, b.outer, n1, b.ldx, b.xvs, b.outer * L, L};
  f1.x = x;
  f1.y = w;
  f1.in_limit = nin;
  f1.out_limit = L;
  f1.tw_log = sp.logL;
  LAUNCH(launch_fft(f1, s));
  // step 2: contiguous length-n1 forward transform, spectral product (spectrum
  // stored in the same transposed order), inverse transform, twiddles W_L^-(n1 k2)
  FftLaunch f2;
  f2.elem = e;
  f2.logn = sp.log1;
  f2.mode = FFT_CONV;
  f2.b = Batch{b.ncols * b.outer, n2, 1, L, n1, L, n1};
  f2.x = w;
  f2.y = w;
  f2.in_limit = f2.out_limit = n1;
  f2.spec = spec;
  f2.spec_ostride = n1;
  f2.spec_conj = adj;
  f2.tw_log = sp.logL;
  f2.tw_inv = 1;
  LAUNCH(launch_fft(f2, s));
  }
  // step 3: inverse length-n2 transforms at stride n1, cropped store
  FftLaunch f3;
  f3.elem = e;
  f3.logn = sp.log2;
  f3.mode = FFT_INV;
  f3.b = Batch{b.ncols, b.outer, n1, b.outer * L, L, b.ldy, b.yvs};
  f3.x = w;
  f3.y = y;
  f3.in_limit = L;
  f3.out_limit = nout;
  f3.accumulate = acc;
  f3.omap = omap;
  LAUNCH(launch_fft(f3, s));
  ws.release(mk);
  return FM_OK;
}

fm_status exec_hadamard(const fm_op_s* op, Elem e, const Batch& b, const void* x, void* y, bool acc,
                        Workspace& ws, hipStream_t s) {
  const int logn = ilog2(op->n);
  if (logn <= fwht_lds_max_log(e)) {
    LAUNCH(launch_fwht(e, logn, b, x, y, acc, s));
    return FM_OK;
  }
  // H_N = H_N1 (x) H_N2: two mode products, the second in place.
  FM_CHECK_ARG(packed(b, op->n, op->n), FM_E_UNSUPPORTED, "Hadamard: unpacked outer batch");
  const int log2n = logn / 2, log1n = logn - log2n;
  const int64_t n1 = int64_t(1) << log1n, n2 = int64_t(1) << log2n;
  const size_t mk = ws.mark();
  void* dst = y;
  Batch bd = b;
  if (acc) {
    dst = ws.take(size_t(b.ncols * b.outer * op->n * b.inner) * elem_bytes(e));
    bd.ldy = b.outer * op->n * b.inner;
    bd.yvs = op->n * b.inner;
  }
  Batch pa{b.ncols, b.outer * n1, b.inner, b.ldx, n2 * b.inner, bd.ldy, n2 * b.inner};
  LAUNCH(launch_fwht(e, log2n, pa, x, dst, 0, s));
  Batch pb{b.ncols, b.outer, n2 * b.inner, bd.ldy, bd.yvs, bd.ldy, bd.yvs};
  LAUNCH(launch_fwht(e, log1n, pb, dst, dst, 0, s));
  if (acc) {
    Batch cb{b.ncols, b.outer, b.inner, bd.ldy, bd.yvs, b.ldy, b.yvs};
    LAUNCH(launch_copy(e, op->n, cb, dst, y, 1, s));
  }
  ws.release(mk);
  return FM_OK;
}

fm_status exec_mltoeplitz(const fm_op_s* op, bool adj, Elem e, const Batch& b, const void* x, void* y,
                          bool acc, Workspace& ws, hipStream_t s) {
  Batch fb;
  FM_CHECK_ARG(b.inner == 1 && fold_outer(b, op->n, op->m, &fb), FM_E_UNSUPPORTED,
               "multilevel Toeplitz along a strided axis");
  const int d = int(op->lv.size());
  int64_t total = 1;
  for (int l = 0; l < d; ++l) total *= op->lL[l];
  const size_t mk = ws.mark();
  const size_t bytes = size_t(fb.ncols * total) * elem_bytes(e);
  void* w1 = ws.take(bytes);
  void* w2 = ws.take(bytes);
  const fm_op_s* kf = op->terms[0];  // Kron of Fourier(L_l)
  // zero-pad into the embedding grid
  LAUNCH(launch_box_copy(e, d, op->lv.data(), op->lv.data(), op->lL.data(), fb.ncols, x, fb.ldx, w1,
                         total, 0, s));
  Batch kb{fb.ncols, 1, 1, total, total, total, total};
  FM_TRY(exec(kf, false, e, kb, w1, w2, false, ws, s));
  Batch db{fb.ncols, 1, 1, total, total, total, total};
  LAUNCH(launch_diag(e, total, db, param(op, e), adj, w2, w2, 0, s));
  FM_TRY(exec(kf, true, e, kb, w2, w1, false, ws, s));
  LAUNCH(launch_box_copy(e, d, op->lv.data(), op->lL.data(), op->lv.data(), fb.ncols, w1, total, y,
                         fb.ldy, acc, s));
  ws.release(mk);
  return FM_OK;
}

fm_status exec_product(const fm_op_s* op, bool adj, Elem e, const Batch& b, const void* x, void* y,
                       bool acc, Workspace& ws, hipStream_t s) {
  const int k = int(op->terms.size());
  // S C forward (S a row selection, C a circulant or Toeplitz of
  // power-of-two length): S is applied inside C's last pass, at the store,
  // with S's inverse index map; no intermediate and no gather launch, the
  // same values as the two steps. (Reading S^H x through the map in C^H's
  // first pass measured slower than the expand launch it saves: two
  // dependent loads per value.)
  if (k == 2 && !adj && b.inner == 1 && b.outer == 1 && (e == Elem::C64 || e == Elem::C128)) {
    const fm_op_s* S = op->terms[0];
    const fm_op_s* C = op->terms[1];
    if (S->kind == Kind::Select && (C->kind == Kind::Circulant || C->kind == Kind::Toeplitz) &&
        S->path.load(std::memory_order_acquire) == 0 && C->path.load(std::memory_order_acquire) == 0 &&
        !split(C, e).mixed() && S->inv.p != nullptr) {
      const int32_t* inv = static_cast<const int32_t*>(S->inv.p);
      return exec_conv(C, false, e, b, x, y, acc, ws, s, inv);
    }
  }
  // application order
  std::vector<const fm_op_s*> seq;
  for (int j = 0; j < k; ++j) seq.push_back(op->terms[adj ? j : k - 1 - j]);
  if (k == 1) return exec(seq[0], adj, e, b, x, y, acc, ws, s);
  int64_t maxrows = 0;
  for (int j = 0; j + 1 < k; ++j) {
    const int64_t r = out_rows(seq[j], adj);
    if (r > maxrows) maxrows = r;
  }
  const size_t mk = ws.mark();
  const size_t bytes = size_t(b.ncols * b.outer * maxrows * b.inner) * elem_bytes(e);
  char* bufs[2] = {static_cast<char*>(ws.take(bytes)), static_cast<char*>(ws.take(bytes))};
  const void* cur = x;
  int64_t cur_ld = b.ldx, cur_vs = b.xvs;
  for (int j = 0; j < k; ++j) {
    const bool last = j == k - 1;
    const int64_t rows = out_rows(seq[j], adj);
    Batch sb{b.ncols, b.outer, b.inner, cur_ld, cur_vs, 0, 0};
    void* dst;
    if (last) {
      dst = y;
      sb.ldy = b.ldy;
      sb.yvs = b.yvs;
    } else {
      dst = bufs[j & 1];
      sb.ldy = b.outer * rows * b.inner;
      sb.yvs = rows * b.inner;
    }
    FM_TRY(exec(seq[j], adj, e, sb, cur, dst, last ? acc : false, ws, s));
    cur = dst;
    cur_ld = sb.ldy;
    cur_vs = sb.yvs;
  }
  ws.release(mk);
  return FM_OK;
}

fm_status exec_kron(const fm_op_s* op, bool adj, Elem e, const Batch& b, const void* x, void* y,
                    bool acc, Workspace& ws, hipStream_t s) {
  const int d = int(op->terms.size());
  FM_CHECK_ARG(packed(b, in_rows(op, adj), out_rows(op, adj)), FM_E_UNSUPPORTED,
               "Kron: unpacked outer batch");
  std::vector<int64_t> cur(d);
  for (int l = 0; l < d; ++l) cur[l] = in_rows(op->terms[l], adj);
  // largest intermediate
  int64_t maxsz = 0;
  {
    std::vector<int64_t> c2 = cur;
    for (int k = d - 1; k > 0; --k) {
      c2[k] = out_rows(op->terms[k], adj);
      int64_t sz = 1;
      for (int l = 0; l < d; ++l) sz *= c2[l];
      if (sz > maxsz) maxsz = sz;
    }
  }
  const size_t mk = ws.mark();
  const size_t bytes = size_t(b.ncols * b.outer * maxsz * b.inner) * elem_bytes(e);
  char* bufs[2] = {nullptr, nullptr};
  if (d > 1) {
    bufs[0] = static_cast<char*>(ws.take(bytes));
    bufs[1] = static_cast<char*>(ws.take(bytes));
  }
  const void* src = x;
  int64_t src_ld = b.ldx, src_vs = b.xvs;
  int stage = 0;
  int kstart = d - 1;
  if (d >= 2 && b.inner == 1 && op->terms[d - 1]->kind == Kind::Dense && op->terms[d - 2]->kind == Kind::Fourier &&
      op->terms[d - 2]->terms.empty()) {
    // the last two factors (Fourier, small dense) in one slab pass
    const fm_op_s* F = op->terms[d - 2];
    const fm_op_s* G = op->terms[d - 1];
    const int lognf = ilog2(F->L);
    if (kron_fg_supported(e, lognf, G->m, G->n)) {
      int64_t slabs = b.outer;
      for (int l = 0; l < d - 2; ++l) slabs *= cur[l];
      const int64_t gout = out_rows(G, adj);
      const bool last = d == 2;
      void* dst = last ? y : bufs[0];
      const int64_t dst_ld = last ? b.ldy : slabs * F->L * gout;
      LAUNCH(launch_kron_fg(lognf, G->m, G->n, param(G, e), G->lda, adj, G->real_entries ? 1 : 0, b.ncols, slabs, x,
                            b.ldx, dst, dst_ld, last ? int(acc) : 0, s));
      cur[d - 1] = gout;
      cur[d - 2] = F->L;
      src = dst;
      src_ld = dst_ld;
      kstart = d - 3;
      stage = 1;
    }
  }
  for (int k = kstart; k >= 0; --k, ++stage) {
    const fm_op_s* f = op->terms[k];
    int64_t outer = 1, inner = 1;
    for (int l = 0; l < k; ++l) outer *= cur[l];
    for (int l = k + 1; l < d; ++l) inner *= cur[l];
    const int64_t rin = in_rows(f, adj), rout = out_rows(f, adj);
    const bool last = k == 0;
    void* dst;
    Batch sb;
    sb.ncols = b.ncols;
    sb.outer = b.outer * outer;
    sb.inner = inner * b.inner;
    sb.ldx = src_ld;
    sb.xvs = rin * sb.inner;
    if (last) {
      dst = y;
      sb.ldy = b.ldy;
    } else {
      dst = bufs[stage & 1];
      int64_t total = rout * sb.inner * outer;
      sb.ldy = b.outer * total;
    }
    sb.yvs = rout * sb.inner;
    FM_TRY(exec(f, adj, e, sb, src, dst, last ? acc : false, ws, s));
    cur[k] = rout;
    src = dst;
    src_ld = sb.ldy;
    (void)src_vs;
  }
  ws.release(mk);
  return FM_OK;
}

// Block matrix, general path: output slice o (+)= sum over input slices p of
// block (o, p) (forward: A_op; adjoint: A_po^H).
fm_status exec_blocks_general(const fm_op_s* op, bool adj, Elem e, const Batch& b, const void* x, void* y,
                              bool acc, Workspace& ws, hipStream_t s) {
  const int nout = adj ? op->nbc : op->nbr, nin = adj ? op->nbr : op->nbc;
  const std::vector<int64_t>& ooff = adj ? op->coff : op->roff;
  const std::vector<int64_t>& ioff = adj ? op->roff : op->coff;
  const size_t es = elem_bytes(e);
  for (int o = 0; o < nout; ++o) {
    char* ys = static_cast<char*>(y) + size_t(ooff[o] * b.inner) * es;
    for (int p = 0; p < nin; ++p) {
      const fm_op_s* blk = adj ? op->terms[size_t(p) * op->nbc + o] : op->terms[size_t(o) * op->nbc + p];
      const char* xs = static_cast<const char*>(x) + size_t(ioff[p] * b.inner) * es;
      FM_TRY(exec(blk, adj, e, b, xs, ys, p == 0 ? acc : true, ws, s));
    }
  }
  return FM_OK;
}

// Block matrix of multilevel Toeplitz blocks of one geometry: zero-pad every
// input slice into the embedding grid and transform it once, form
// Y_o = sum_p S_op .* X_p per bin (S_op = the block's spectrum, conj'ed and
// transposed for the adjoint), transform every output back once and crop.
fm_status exec_blocks_mix(const fm_op_s* op, bool adj, Elem e, const Batch& b, const void* x, void* y,
                          bool acc, Workspace& ws, hipStream_t s) {
  Batch fb;
  FM_CHECK_ARG(b.inner == 1 && fold_outer(b, op->n, op->m, &fb) && fb.outer == 1, FM_E_UNSUPPORTED,
               "block matrix along a strided axis");
  const int nout = adj ? op->nbc : op->nbr, nin = adj ? op->nbr : op->nbc;
  const std::vector<int64_t>& ooff = adj ? op->coff : op->roff;
  const std::vector<int64_t>& ioff = adj ? op->roff : op->coff;
  const int d = int(op->lv.size());
  int64_t total = 1;
  for (int l = 0; l < d; ++l) total *= op->lL[l];
  const int64_t nc = fb.ncols;
  const int nmax = nout > nin ? nout : nin;
  const size_t es = elem_bytes(e);
  const size_t mk = ws.mark();
  char* w1 = static_cast<char*>(ws.take(size_t(nmax) * size_t(nc * total) * es));
  char* w2 = static_cast<char*>(ws.take(size_t(nmax) * size_t(nc * total) * es));
  const fm_op_s* kf = op->terms[0]->terms[0];  // Kron of Fourier(L_l) of the first block
  // all blocks have the same size: slice p starts at row p * nblk; w holds
  // vector (p, c) at (p nc + c) total
  const int64_t nblk = ioff[1] - ioff[0];
  (void)ooff;
  LAUNCH(launch_box_copy(e, d, op->lv.data(), op->lv.data(), op->lL.data(), nc, x, fb.ldx, w1, total, 0, s,
                         nin, nblk, nc * total));
  Batch kin{nin * nc, 1, 1, total, total, total, total};
  FM_TRY(exec(kf, false, e, kin, w1, w2, false, ws, s));
  LAUNCH(launch_block_mix(e, nout, nin, op->nbc, int64_t(op->nbr) * op->nbc, total, op->mix_logtw, nc,
                          param(op, e), adj, w2, w1, s));
  Batch kout{nout * nc, 1, 1, total, total, total, total};
  FM_TRY(exec(kf, true, e, kout, w1, w2, false, ws, s));
  LAUNCH(launch_box_copy(e, d, op->lv.data(), op->lL.data(), op->lv.data(), nc, w2, total, y, fb.ldy, acc, s,
                         nout, nc * total, nblk));
  ws.release(mk);
  return FM_OK;
}

// Block diagonal: each block on its slice of rows; a run of consecutive
// identical blocks is one call batched over the run.
fm_status exec_blkdiag(const fm_op_s* op, bool adj, Elem e, const Batch& b, const void* x, void* y,
                       bool acc, Workspace& ws, hipStream_t s) {
  const size_t es = elem_bytes(e);
  int64_t oi = 0, oo = 0;
  const size_t nt = op->terms.size();
  for (size_t k = 0; k < nt;) {
    const fm_op_s* t = op->terms[k];
    size_t run = 1;
    while (k + run < nt && op->terms[k + run] == t) ++run;
    const int64_t ri = in_rows(t, adj), ro = out_rows(t, adj);
    const char* xs = static_cast<const char*>(x) + size_t(oi * b.inner) * es;
    char* ys = static_cast<char*>(y) + size_t(oo * b.inner) * es;
    // batched only where the run's vectors are evenly strided in x and y
    const bool even = b.ncols == 1 || (b.ldx == int64_t(run) * ri * b.inner && b.ldy == int64_t(run) * ro * b.inner);
    if (run > 1 && b.outer == 1 && even) {
      Batch rb{b.ncols, int64_t(run), b.inner, b.ldx, ri * b.inner, b.ldy, ro * b.inner};
      FM_TRY(exec(t, adj, e, rb, xs, ys, acc, ws, s));
    } else {
      run = 1;
      FM_TRY(exec(t, adj, e, b, xs, ys, acc, ws, s));
    }
    oi += int64_t(run) * ri;
    oo += int64_t(run) * ro;
    k += run;
  }
  return FM_OK;
}

}  // namespace

fm_status exec(const fm_op_s* op, bool adj, Elem e, const Batch& b, const void* x, void* y,
               bool acc, Workspace& ws, hipStream_t s) {
  if (b.ncols == 0 || b.outer == 0) return FM_OK;
  if (op->path.load(std::memory_order_acquire) == 1 && (e == Elem::C64 || e == Elem::C128)) {
    // calibrated: the dense product is faster for this operator
    LAUNCH(launch_dense(e, op->m, op->n, e == Elem::C64 ? op->dense32.p : op->dense64.p, op->m, adj, 0, b, x, y,
                        acc, s));
    return FM_OK;
  }
  switch (op->kind) {
    case Kind::Adjoint:
      return exec(op->terms[0], !adj, e, b, x, y, acc, ws, s);
    case Kind::ToeplitzInv: {  // Levinson solves with T (adjoint: T^H)
      const fm_op_s* T = op->terms[0];
      Batch fb;
      FM_CHECK_ARG(b.inner == 1 && fold_outer(b, op->n, op->n, &fb) && fb.outer == 1, FM_E_UNSUPPORTED,
                   "Toeplitz inverse along a strided axis");
      const int64_t n = op->n, nc = fb.ncols;
      const size_t es = elem_bytes(e);
      const size_t mk = ws.mark();
      void* work = ws.take(size_t(3 * n * nc) * es);
      void* dst = y;
      int64_t ldd = fb.ldy;
      if (acc) {
        dst = ws.take(size_t(n * nc) * es);
        ldd = n;
      }
      LAUNCH(launch_levinson(e, n, T->L, T->gen.p, adj ? 1 : 0, nc, x, fb.ldx, dst, ldd, work, s));
      if (acc) LAUNCH(launch_copy(e, n, Batch{nc, 1, 1, n, n, fb.ldy, fb.ldy}, dst, y, 1, s));
      ws.release(mk);
      return FM_OK;
    }
    case Kind::Conj: {  // conj(A) x = conj(A conj(x)); the same for the adjoint direction
      if (e == Elem::I32 || e == Elem::I64) return exec(op->terms[0], adj, e, b, x, y, acc, ws, s);
      const int64_t rin = in_rows(op, adj), rout = out_rows(op, adj);
      const size_t es = elem_bytes(e);
      const size_t mk = ws.mark();
      void* xc = ws.take(size_t(b.ncols * b.outer * rin * b.inner) * es);
      const Batch cb{b.ncols, b.outer, b.inner, b.ldx, b.xvs, b.outer * rin * b.inner, rin * b.inner};
      LAUNCH(launch_conj(e, rin, cb, x, xc, 0, s));
      Batch ib{b.ncols, b.outer, b.inner, b.outer * rin * b.inner, rin * b.inner, b.ldy, b.yvs};
      void* dst = y;
      if (acc) {
        dst = ws.take(size_t(b.ncols * b.outer * rout * b.inner) * es);
        ib.ldy = b.outer * rout * b.inner;
        ib.yvs = rout * b.inner;
      }
      FM_TRY(exec(op->terms[0], adj, e, ib, xc, dst, false, ws, s));
      const Batch ob{b.ncols, b.outer, b.inner, ib.ldy, ib.yvs, b.ldy, b.yvs};
      LAUNCH(launch_conj(e, rout, ob, dst, y, acc ? 1 : 0, s));
      ws.release(mk);
      return FM_OK;
    }
    case Kind::Fourier:
      return exec_fourier(op, adj, e, b, x, y, acc, ws, s);
    case Kind::Circulant:
    case Kind::Toeplitz:
      return exec_conv(op, adj, e, b, x, y, acc, ws, s);
    case Kind::Hadamard:
      return exec_hadamard(op, e, b, x, y, acc, ws, s);
    case Kind::Diag:
      LAUNCH(launch_diag(e, op->n, b, param(op, e), adj, x, y, acc, s));
      return FM_OK;
    case Kind::Dense:
      LAUNCH(launch_dense(e, op->m, op->n, param(op, e), op->lda, adj, op->real_entries, b, x, y, acc, s));
      return FM_OK;
    case Kind::Select:
      LAUNCH(launch_select(e, op->n, op->m, static_cast<const int32_t*>(op->idx.p),
                           static_cast<const int32_t*>(op->inv.p), adj, b, x, y, acc, s));
      return FM_OK;
    case Kind::MLToeplitz:
      return exec_mltoeplitz(op, adj, e, b, x, y, acc, ws, s);
    case Kind::Product:
      return exec_product(op, adj, e, b, x, y, acc, ws, s);
    case Kind::Sum: {
      for (size_t j = 0; j < op->terms.size(); ++j)
        FM_TRY(exec(op->terms[j], adj, e, b, x, y, j == 0 ? acc : true, ws, s));
      return FM_OK;
    }
    case Kind::Kron:
      return exec_kron(op, adj, e, b, x, y, acc, ws, s);
    case Kind::BlkDiag:
      return exec_blkdiag(op, adj, e, b, x, y, acc, ws, s);
    case Kind::Blocks:
      return op->mix ? exec_blocks_mix(op, adj, e, b, x, y, acc, ws, s)
                     : exec_blocks_general(op, adj, e, b, x, y, acc, ws, s);
  }
  set_error("exec: unknown operator kind");
  return FM_E_INVALID;
}

}  // namespace fm
