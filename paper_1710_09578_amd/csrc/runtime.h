// Runtime pieces shared by the kernels and the C ABI: per-device twiddle
// tables, device buffers, the operator tree and the executor interface.
#pragma once

#include <atomic>
#include <memory>
#include <mutex>
#include <vector>

#include "kernels.h"

namespace fm {

// Twiddle tables of every power-of-two size up to 2^logmax on the current
// device: entry [size + k] = exp(-2 pi j k / size), 0 <= k < size. Generated
// in FP64 on the host with exact octant reduction and rounded once for
// complex64. Returns nullptr on failure (error text set).
const void* twiddle_table(Elem e, int logmax);
// exp(-2 pi j k / size) in FP64 (angle reduced to at most pi/4, then exact
// quadrant rotations); size 1, 2 or a multiple of 4.
void root_of_unity(int64_t k, int64_t size, double* re, double* im);

// Owned device allocation.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      reset();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { reset(); }
  fm_status alloc(size_t n);
  void reset();
};

enum class Kind {
  Fourier,
  Hadamard,
  Diag,
  Dense,
  Circulant,
  Toeplitz,
  MLToeplitz,
  Select,
  Product,
  Sum,
  Kron,
  BlkDiag,
  Blocks,
  Adjoint,
  Conj,
  ToeplitzInv
};

// Split of a cyclic length L for one element type: L <= LDS limit runs in one
// work-group (n2 == 1); otherwise L = n1 * n2 (four-step, n1 = 2^log1
// contiguous). n2 is a power of two (log2 = log2 n2) or, for a mixed length,
// one of 3, 5, 6, 9, 10, 12, 20, 24, 30 (log2 = -1, logL = -1).
struct Split {
  int logL = 0;
  int log1 = 0, log2 = 0;
  int n2 = 1;
  bool four_step() const { return n2 > 1; }
  bool mixed() const { return n2 > 1 && (n2 & (n2 - 1)) != 0; }
};
Split split_for(Elem e, int logL);
// Split of a mixed four-step length L = 4096 * n2 (n2 not a power of two).
Split split_mixed(int64_t L);
// Four-step strided factors that are not powers of two and have strided
// passes (3, 5, 6, 9, 10, 12, 20, 24, 30).
bool mixed_n2_ok(int n2);
// Table of W_L^m = exp(-2 pi j m / L), 0 <= m < L, for a mixed length
// L = 4096 * n2, generated in FP64 with exact quadrant reduction and rounded
// once for complex64; cached per device. NULL on failure (error text set).
const void* twiddle_table_L(Elem e, int64_t L);

}  // namespace fm

struct fm_op_s {
  std::atomic<int> refs{1};
  uint32_t magic = 0x464d4f50u;  // "FMOP" while alive
  fm::Kind kind;
  fm_dtype dt;
  int64_t m = 0, n = 0;
  int device = 0;
  // leaf parameters: complex64 copy (for FM_C64 operators) and complex128 copy
  // (always, for the FP64 power iteration)
  fm::DevBuf p32, p64;
  fm::DevBuf idx;          // selection indices
  fm::DevBuf inv;          // Select: inv[idx[r]] = r, -1 for rows not selected
  int64_t lda = 0;         // dense: leading dimension of the stored copy (= m)
  bool real_entries = false;  // dense: every entry has a zero imaginary part
  int64_t L = 0;           // cyclic length (Fourier/Circulant/Toeplitz)
  fm::Split s32, s64;      // splits of L for complex64 / complex128
  std::vector<int64_t> lv, lL;  // multilevel: entries per level, embedding per level
  std::vector<fm_op> terms;     // composites (retained) / adjoint child
  // Blocks: grid shape, row / column offsets of the block rows / columns
  // (nbr + 1 and nbc + 1 entries); mix: every block is a multilevel Toeplitz
  // of one geometry (p32 / p64 then hold the blocks' spectra packed
  // bin-tiled, tiles of 2^mix_logtw bins)
  int32_t nbr = 0, nbc = 0;
  std::vector<int64_t> roff, coff;
  bool mix = false;
  int mix_logtw = 0;
  // Circulant / Toeplitz (created from a generator, not derived): the
  // embedded generator g in complex128, L values, with the operator's entry
  // (i, j) = g[(i - j) mod L]; used by the Levinson solves of a Toeplitz
  // inverse and for the columns A e_j that OMP takes
  fm::DevBuf gen;
  // evaluation path chosen by calibration (0: the structured transforms,
  // 1: a dense product with the operator's materialised matrix, column-major,
  // lda = m, in dense32 / dense64); the operator's value is the same either way
  std::atomic<int> path{0};
  fm::DevBuf dense32, dense64;
};

namespace fm {

// Stack allocator over a caller workspace; in sizing mode it only records the
// high-water mark.
struct Workspace {
  char* base = nullptr;
  size_t cap = 0, top = 0, peak = 0;
  bool sizing = false;
  void* take(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    void* p = sizing ? nullptr : base + top;
    top += bytes;
    if (top > peak) peak = top;
    return p;
  }
  size_t mark() const { return top; }
  void release(size_t m) { top = m; }
};

Elem elem_of(fm_dtype dt);

// Applies op (or op^H when adj) to a batch: y (+)= op(x). In sizing mode no
// kernel is launched; the workspace records what the call would take.
fm_status exec(const fm_op_s* op, bool adj, Elem e, const Batch& b, const void* x, void* y,
               bool accumulate, Workspace& ws, hipStream_t s);

// Rows of op^H / op in the given direction.
inline int64_t out_rows(const fm_op_s* op, bool adj) { return adj ? op->n : op->m; }
inline int64_t in_rows(const fm_op_s* op, bool adj) { return adj ? op->m : op->n; }

bool op_alive(const fm_op_s* op);

// fm_apply with its argument checks. With may_allocate = false a workspace
// that is missing or too small is an error (FM_E_WORKSPACE) instead of a
// stream-ordered allocation.
fm_status apply_op(const fm_op_s* a, fm_dir dir, int64_t ncols, const void* x, int64_t ldx, void* y, int64_t ldy,
                   void* ws, size_t ws_bytes, bool may_allocate, void* stream);

}  // namespace fm
