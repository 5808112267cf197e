// Launch interfaces of the device kernels (implemented in the *.hip files).
#pragma once

#include "common.h"

namespace fm {

// A strided batch of vectors. Vector (c, o, i) -- column c < ncols, outer
// index o < outer, inner index i < inner -- has its element r at
//   base + c*ld + o*vs + r*inner + i
// for x (ldx, xvs) and y (ldy, yvs). Contiguous vectors have outer = inner = 1.
struct Batch {
  int64_t ncols = 0, outer = 1, inner = 1;
  int64_t ldx = 0, xvs = 0, ldy = 0, yvs = 0;
};

enum class Elem { C64, C128, I32, I64 };
inline size_t elem_bytes(Elem e) {
  return e == Elem::C64 ? 8 : e == Elem::C128 ? 16 : e == Elem::I32 ? 4 : 8;
}

// ---------------------------------------------------------------- FFT
// Largest transform length held in one work-group's LDS (4096 values, 256
// threads: three to four work-groups share a CU and hide each other's
// latency; a 16384-value work-group fills a CU alone and measured slower).
inline int fft_lds_max_log(Elem) { return 12; }

// Largest strided factor 2^k of a four-step convolution that is folded into
// the row pass (the row work-group forms its row from x directly); longer
// ones get a separate strided pass. FM_MAX_FUSE overrides the default (0
// disables folding).
int conv_max_fuse();

enum FftMode { FFT_FWD = 0, FFT_INV = 1, FFT_CONV = 2 };

struct FftLaunch {
  Elem elem = Elem::C64;
  int logn = 0;            // transform length 2^logn (<= fft_lds_max_log)
  int mode = FFT_FWD;
  Batch b;
  const void* x = nullptr;
  void* y = nullptr;
  int64_t in_limit = 0;    // element (r, i) is read only when r*inner + i < in_limit
  int64_t out_limit = 0;   // and stored only when r*inner + i < out_limit
  const void* spec = nullptr;  // FFT_CONV: spectrum, entry r (+ o*spec_ostride)
  int64_t spec_ostride = 0;
  int spec_conj = 0;
  int tw_log = 0;          // > 0: multiply result r by W^(r*q), W = exp(-+2 pi j / L) with
  int tw_inv = 0;          //      L = 2^tw_log (or the table twl), q = i (strided) or o
                           //      (contiguous); tw_inv picks the + sign
  int accumulate = 0;      // y += result
  int fuse_n2 = 0;         // > 0: row o = k2 of a four-step convolution formed from the column x
                           //      (L = 2^logn * fuse_n2, logn = 12; see xform.h)
  const void* twl = nullptr;  // table W_L^m (0 <= m < L) for a four-step length that is not a
                              // power of two; NULL: taken from the power-of-two tables (L = 2^tw_log)
  // A row selection applied at the store: result position p is stored (added)
  // at row omap[p] of y's column, and not stored where omap[p] < 0 (omap: a
  // selection's inverse index map, one entry per result position).
  const int32_t* omap = nullptr;
};
fm_status launch_fft(const FftLaunch& L, hipStream_t s);

// Strided pass of a mixed four-step length L = 4096 * n2 (n2 5-smooth, not a
// power of two) for ncols columns: forward (inverse = 0) takes the n2 points
// x[n1 + 4096 j] of every column position n1 (zero at or beyond in_limit),
// their DFT times W_L^(n1 k2) into y[n1 + 4096 k2]; inverse takes the slot's
// points, their inverse DFT, stored (added with acc) where n1 + 4096 k <
// out_limit. twl: the W_L table (twiddle_table_L).
fm_status launch_mixed(Elem e, int n2, int inverse, int64_t ncols, const void* x, int64_t ldx, int64_t in_limit,
                       void* y, int64_t ldy, int64_t out_limit, const void* twl, int64_t L, int acc, hipStream_t s);

// Column-wise transpose of a row-major rows x cols matrix per column block:
// y[c*ldy + j*rows + i] (+)= x[c*ldx + i*cols + j].
fm_status launch_transpose(Elem e, int64_t ncols, int64_t rows, int64_t cols, const void* x,
                           int64_t ldx, void* y, int64_t ldy, int accumulate, hipStream_t s);

// ---------------------------------------------------------------- Walsh-Hadamard
inline int fwht_lds_max_log(Elem e) { return e == Elem::C128 ? 13 : 14; }
fm_status launch_fwht(Elem e, int logn, const Batch& b, const void* x, void* y, int accumulate,
                      hipStream_t s);

// ---------------------------------------------------------------- fused Kronecker slab
// Kron(..., F_nF, G) last two factors in one pass (see kron.hip): for each of
// the ncols * outer slabs of nF x n values (x, column stride ldx) writes the
// nF x m slab of (F (x) G) (adjoint: (F (x) G)^H with the shapes swapped).
bool kron_fg_supported(Elem e, int lognf, int64_t m, int64_t n);
fm_status launch_kron_fg(int lognf, int64_t m, int64_t n, const void* g, int64_t lda, int adjoint, int real_g,
                         int64_t ncols, int64_t outer, const void* x, int64_t ldx, void* y, int64_t ldy, int acc,
                         hipStream_t s);

// ---------------------------------------------------------------- elementwise
// y (+)= d .* x  (d conj'ed when conj) along the vector axis of the batch.
fm_status launch_diag(Elem e, int64_t n, const Batch& b, const void* d, int conj, const void* x,
                      void* y, int accumulate, hipStream_t s);
// Row selection: forward y[r] (+)= x[idx[r]] (m outputs); adjoint y = 0 except
// y[idx[r]] (+)= x[r] (n outputs), in one pass over y through inv (inv[idx[r]]
// = r, -1 elsewhere) when inv is given.
fm_status launch_select(Elem e, int64_t n_in, int64_t m, const int32_t* idx, const int32_t* inv, int adjoint,
                        const Batch& b, const void* x, void* y, int accumulate, hipStream_t s);
// inv[0..n) = -1, then inv[idx[r]] = r for the m distinct, in-range indices.
fm_status launch_invert_indices(int64_t n, int64_t m, const int32_t* idx, int32_t* inv, hipStream_t s);
// Dense complex64 product on the matrix cores (dense_mfma.hip) for m, n <= 64
// along the contiguous axis (inner == 1) of a batch; same arguments as
// launch_dense without real_a.
bool dense_mfma_supported(Elem e, int64_t m, int64_t n, const Batch& b);
fm_status launch_dense_mfma(int64_t m, int64_t n, const void* a, int64_t lda, int adjoint, const Batch& b,
                            const void* x, void* y, int acc, hipStream_t s);
// Dense mode product y[:, o, :, i] (+)= op(A) x[:, o, :, i], A m x n col-major.
// real_a: every entry of A has a zero imaginary part (only real parts used).
fm_status launch_dense(Elem e, int64_t m, int64_t n, const void* a, int64_t lda, int adjoint, int real_a,
                       const Batch& b, const void* x, void* y, int accumulate, hipStream_t s);
// Zero-pad / crop copy between multi-dimensional grids (multilevel Toeplitz):
// copies the box [0, nbox) of the source grid (dims src_dims) into the
// destination grid (dims dst_dims), zero-filling the rest of the destination.
// Vectors: (c, o) for c < ncols, o < outer, at x + c ldx + o xos and
// y + c ldy + o yos.
fm_status launch_box_copy(Elem e, int ndim, const int64_t* box, const int64_t* src_dims,
                          const int64_t* dst_dims, int64_t ncols, const void* x, int64_t ldx,
                          void* y, int64_t ldy, int accumulate, hipStream_t s, int64_t outer = 1,
                          int64_t xos = 0, int64_t yos = 0);
// Spectral mixing of a block matrix of convolutions: for o < nout, column
// c < ncols, bin f < total:
//   y[(o ncols + c) total + f] = sum_{p < nin} S(o, p)[f] x[(p ncols + c) total + f]
// with S(o, p) the spectrum of block o * ld + p (forward) or the conjugate of
// block p * ld + o (adjoint). spec: the nb spectra packed bin-tiled by
// launch_block_pack (tiles of 2^logtw bins).
fm_status launch_block_mix(Elem e, int nout, int nin, int ld, int64_t nb, int64_t total, int logtw, int64_t ncols,
                           const void* spec, int adjoint, const void* x, void* y, hipStream_t s);
// Packs nb spectra of total bins (table: DEVICE array of nb pointers) into
// out[((f >> logtw) nb + k) 2^logtw + (f mod 2^logtw)].
fm_status launch_block_pack(Elem e, int64_t nb, int64_t total, int logtw, const void* table, void* out,
                            hipStream_t s);
// y = alpha * x (contiguous, count elements of type e); alpha real.
fm_status launch_scale_copy(Elem e, int64_t count, double alpha, const void* x, void* y,
                            hipStream_t s);
// Upcast complex64 -> complex128 (count entries, contiguous).
fm_status launch_c64_to_c128(int64_t count, const void* x, void* y, hipStream_t s);
// Round complex128 -> complex64 (count entries, contiguous).
fm_status launch_c128_to_c64(int64_t count, const void* x, void* y, hipStream_t s);
// Convolution spectrum (count = L entries, rows of min(L, 4096) in the order
// the convolution reads them) rounded to complex64 in pair order: within each
// row of 16 T values, entry t + T k is stored at 2 (t + T (k / 2)) + k % 2
// (L >= 16; shorter spectra stay in natural order).
fm_status launch_spectrum_c64(int64_t count, const void* x, void* y, hipStream_t s);
// Permute a length N1*N2 spectrum from natural order X[k2 + N2 k1] into the
// four-step order P[k1 + N1 k2] (complex128).
fm_status launch_fourstep_permute(int64_t n1, int64_t n2, const void* x, void* y, hipStream_t s);
// Toeplitz generator embedded into a cyclic length-L vector (complex128):
// g[0..m-1] = col, g[L-k] = row[k] for k = 1..n-1, zero elsewhere.
fm_status launch_toeplitz_embed(int64_t m, int64_t n, int64_t L, const void* col, const void* row,
                                int elem_c64, void* g, hipStream_t s);
// Check indices. flags: n + 1 zeroed ints; flags[n] becomes nonzero if any
// idx is outside [0, n) or repeated.
fm_status launch_check_indices(int64_t n, int64_t m, const int32_t* idx, int* flags, hipStream_t s);
// Levinson solves T x = b (adjoint: T^H x = b) for ncols right-hand sides of
// the n x n Toeplitz T whose generator is embedded in gen (complex128, t_k at
// index k mod L). x may be written in place of a workspace; work holds
// 3 n ncols values of type e. A column whose leading minors are singular gets
// NaN values.
fm_status launch_levinson(Elem e, int64_t n, int64_t L, const void* gen, int adjoint, int64_t ncols, const void* b,
                          int64_t ldb, void* x, int64_t ldx, void* work, hipStream_t s);
// y (+)= conj(x) over the vectors of a batch (n rows each); plain copy for integers.
fm_status launch_conj(Elem e, int64_t n, const Batch& b, const void* x, void* y, int accumulate, hipStream_t s);
// Elementwise map of count complex128 values: mode 0 out = scale |in|^2, mode 1
// out = scale / in; flag[0] (an int, zeroed by the caller) is set to 1 when an
// inverted entry is zero or not finite.
fm_status launch_param_map(int64_t count, int mode, double scale, const void* in, void* out, int* flag,
                           hipStream_t s);
// y (+)= x over the vectors of a batch (n rows each).
fm_status launch_copy(Elem e, int64_t n, const Batch& b, const void* x, void* y, int accumulate,
                      hipStream_t s);

}  // namespace fm
