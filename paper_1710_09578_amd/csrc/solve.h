// Launch interfaces of the solver kernels (solve.hip).
#pragma once

#include <cmath>
#include <vector>

#include "kernels.h"

namespace fm {

// Momentum weights of the accelerated iteration (FISTA, Beck-Teboulle):
// t_1 = 1, t_{j+1} = (1 + sqrt(1 + 4 t_j^2)) / 2, and iteration k (0-based,
// the (k+1)-th gradient step) extrapolates with (t_{k+1} - 1) / t_{k+2}, so the
// first weight is 0. FP64, by the recurrence in order: every caller (solver,
// batched solver, single step) gets the same bits.
inline std::vector<double> fista_momentum_weights(int iters) {
  std::vector<double> out(size_t(iters > 0 ? iters : 0));
  double t = 1.0;
  for (int k = 0; k < iters; ++k) {
    const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
    out[size_t(k)] = (t - 1.0) / tn;
    t = tn;
  }
  return out;
}
inline double fista_momentum(int k, bool momentum) {
  if (!momentum || k < 0) return 0.0;
  return fista_momentum_weights(k + 1)[size_t(k)];
}

struct UpdateArgs {
  void* x;        // iterate x_k (overwritten by x_{k+1})
  void* y;        // extrapolated point y_k (overwritten by y_{k+1})
  const void* g;  // gradient A^H (A y_k - b)
  int64_t ldx, ldy, ldg;
  int64_t rows;
  double invL;
  const double* lam;  // per column
  double beta;        // momentum weight (t_k - 1)/t_{k+1}
  int momentum;
  const int* active;  // per column, NULL: all active
  int* status;        // per column, set to 1 on a non-finite value
  double* partial;    // per column and tile: sum |dx|^2, sum |x|^2 (NULL: not needed)
  int64_t ntiles;
  int per_thread;
};

int64_t update_tiles(int64_t rows, int* per_thread);
fm_status launch_update(Elem e, const UpdateArgs& a, int64_t ncols, hipStream_t s);
fm_status launch_stop(const double* partial, int64_t ntiles, int64_t ncols, double tol, int k, int* active,
                      int* iters, const int* status, hipStream_t s);
fm_status launch_sub(Elem e, int64_t rows, int64_t ncols, const void* b, int64_t ldb, void* r, int64_t ldr,
                     const int* active, hipStream_t s);
fm_status launch_colmax(Elem e, int64_t rows, int64_t ncols, const void* g, int64_t ldg, double rel, double* out,
                        hipStream_t s);
fm_status launch_norm2(int64_t n, const void* v, double* partial, int nparts, double* out, hipStream_t s);
fm_status launch_normalize(int64_t n, void* v, const double* nrm2, hipStream_t s);
// Partial sums of |v_i|^2 (complex128) into partial[0..nparts): the first
// kernel of launch_norm2.
fm_status launch_norm2_partial(int64_t n, const void* v, double* partial, int nparts, hipStream_t s);
// w *= 1/||w|| with ||w||^2 summed from part_w as launch_norm2 sums it; also
// stores that sum in *out_w and the sum of part_a in *out_a (complex128, n >= 1).
fm_status launch_normalize_final(int64_t n, void* w, int nparts, const double* part_w, const double* part_a,
                                 double* out_w, double* out_a, hipStream_t s);
fm_status launch_start_vector(int64_t n, uint64_t seed, void* v, hipStream_t s);
fm_status launch_fill_int(int64_t n, int* p, int v, hipStream_t s);
fm_status launch_fill_double(int64_t n, double* p, double v, hipStream_t s);
fm_status launch_zero2d(Elem e, int64_t rows, int64_t ncols, void* p, int64_t ld, hipStream_t s);
fm_status launch_copy2d(Elem e, int64_t rows, int64_t ncols, const void* src, int64_t lds, void* dst, int64_t ldd,
                        hipStream_t s);

// ---- fused solver (fista_fused.hip) for A = C or A = S C, C a circulant or
// Toeplitz leaf and S a row selection
struct FusedForm {
  const fm_op_s* conv = nullptr;  // NULL: A has another form
  const int* sel_map = nullptr;   // S's inverse index map (C's output row -> row of A, or -1), or NULL
  bool narrow = false;            // A = S C solved with 1024-point rows (L = 1024 n2, n2 >= 64)
};
// Columns up to which A = S C takes 1024-point rows.
constexpr int64_t kNarrowMaxCols = 2;
FusedForm fused_form(const fm_op_s* a, int64_t ncols);
// Partial-sum slots per column of the update pass (its work-groups per column).
int fused_nslot(const FusedForm& f, Elem e);

struct FusedRun {
  Elem e;
  const fm_op_s* conv;
  const int* sel_map;
  bool narrow;            // 1024-point rows (FusedForm::narrow)
  void* nspec;            // narrow: L values, the spectrum in that split's order (written here)
  int64_t ncols, m, n;    // A is m x n
  const void* b;
  int64_t ldb;
  void* x;
  int64_t ldx;
  void* r;     // m x ncols (ld m)
  void* y;     // n x ncols (ld n), holds y_0 on entry
  void* slot;  // L x ncols for four-step lengths
  double invL;
  const double* lam;
  int* active;
  int* status;
  int* iters;
  double* partial;  // 2 * nslot * ncols
  int64_t* pbase;   // ncols
  const void* beta; // max_iters momentum weights in the element's real type
  int* iter;        // device iteration counter (0 on entry)
  int momentum;
  int max_iters;
  double stop_tol;
};
// Runs max_iters iterations (frozen columns skip their work); synchronises
// the stream at the end when the iterations were replayed from a graph.
fm_status fista_fused_run(const FusedRun& run, hipStream_t s);

// Stream (one per device, default priority) that solver graphs are captured
// on, or NULL; and whether solver graphs are on (FM_FISTA_GRAPH != 0).
hipStream_t solver_capture_stream();
bool solver_graphs_enabled();

// Products on A = S C through the solver's passes with 1024-point rows (for
// A with fused_form(A, ncols).narrow), in the element type given to
// narrow_prepare.
struct NarrowForm {
  const fm_op_s* conv;
  const int* sel_map;
  int64_t m, n;  // A is m x n
  void* slot;    // L values per column
  void* nspec;   // L values: the spectrum in that split's order (written by narrow_prepare)
  void* zeros;   // max(m, n) values (zeroed by narrow_prepare)
};
fm_status narrow_prepare(const NarrowForm& p, Elem e, hipStream_t s);
// Power iteration, complex128: av = A v (m values), w = A^H av (n values).
fm_status power_product(const NarrowForm& p, const void* v, void* av, void* w, hipStream_t s);

}  // namespace fm
