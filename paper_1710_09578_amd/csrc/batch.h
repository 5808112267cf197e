// Internals of the batched path shared by the batched apply and the batched
// solver.
#pragma once

#include <vector>

#include "runtime.h"

namespace fm {

constexpr int kLogW = 12;   // values per work-group of the stage kernel
constexpr int kLog1 = 12;   // contiguous factor of the four-step split (complex64)

// Work items (one work-group each):
//   SINGLE  whole zero-padded convolutions of length 2^lg for `sub` columns
//   ROWF    row k2 = sub of a four-step column (L = 4096 * n2, n2 <= 2^conv_max_fuse(); the
//           item's parameter is n2), the strided n2-point transform folded into its load (reads x)
//   FS1     strided 2^lg-point transforms of one column into its slot (lg not folded)
//   FS2     row k2 = sub of a column whose FS1 pass has run (in place in the slot)
//   FS3     strided inverse 2^lg-point transforms of one column and the cropped
//           store into y (inner tile `sub`)
//   MX1/MX3 the FS1 / FS3 passes of a mixed length (L = 4096 * n2, n2 not a power of
//           two; the item's parameter is n2): tile `sub` of mixed_tiles(n2) per column
enum ItemKind : int { IT_SINGLE = 0, IT_FS1 = 1, IT_FS2 = 2, IT_FS3 = 3, IT_ROWF = 4, IT_MX1 = 5, IT_MX3 = 6 };

// Column-pass work-groups (partial-sum slots of a solve) of a four-step
// column with strided factor n2: n2 for powers of two (tiles of 4096 / n2
// positions), mixed_tiles(n2) for mixed lengths.
inline int32_t fs3_tiles(int32_t n2) {
  return (n2 & (n2 - 1)) == 0 ? n2 : (n2 > 12 ? 32 : 16);
}

struct Item {
  int32_t kind_log;  // kind | (lg << 8)
  int32_t op;
  int32_t col;  // SINGLE: first column; others: four-step column index
  int32_t sub;  // SINGLE: columns in this item; FS1/FS3: inner tile; FS2/ROWF: row k2
};

struct OpDev {
  const c64* spec;  // spectrum in the order of the operator's split, 1/L folded in
  int32_t m, n;
  int32_t logL;     // log2 L (rounded down when L is not a power of two)
  int32_t ncols;
  int64_t col_base;  // index of the operator's first column among all columns of the batch
  const c64* twl;   // four-step: table of W_L^m, 0 <= m < L (NULL for a single pass)
  int32_t n2;       // four-step: L / 4096 (1 for a single pass)
};

struct FsCol {
  int32_t op, col;
  int64_t woff;  // element offset of the column's slot in the intermediate pool
};

struct Ptrs {
  const c64* x;
  c64* y;
  int64_t ldx, ldy;
};

// Tunable parameters of a batch's work list.
struct Schedule {
  int max_fuse = 3;                         // strided factors up to 2^max_fuse folded into the row pass
  size_t region_bytes = size_t(96) << 20;   // slot region of one chunk (three rotate)
};


// Caller blocks of one operator in a batched solve.
struct User {
  const c64* b;
  c64* x;
  int64_t ldb, ldx;
};

// Epilogue of the last pass of a direction inside a batched solve:
//   kind 1 (forward):  r = A y - b        (b subtracted in the store)
//   kind 2 (adjoint):  from g = A^H r: z = y - g/L, x+ = soft(z, lam/L),
//                      y+ = x+ + beta (x+ - x), x and y updated in place, with
//                      per-slot partial sums of |x+ - x|^2 and |x+|^2 for the
//                      stopping rule and a status flag for non-finite values.
struct EpiArgs {
  int kind = 0;
  const User* user = nullptr;   // per operator
  const double* lam = nullptr;  // per batch column
  const double* L = nullptr;    // per operator
  const int64_t* pbase = nullptr;  // per batch column: first partial slot
  double* partial = nullptr;    // 2 doubles per slot
  int* status = nullptr;        // per batch column
  const float* beta = nullptr;  // momentum weight of every iteration (device)
  const int* iter = nullptr;    // current iteration (device; advanced by the stop check)
  int momentum = 1;
  bool same(const EpiArgs& o) const {
    return kind == o.kind && user == o.user && lam == o.lam && L == o.L && pbase == o.pbase &&
           partial == o.partial && status == o.status && beta == o.beta && iter == o.iter &&
           momentum == o.momentum;
  }
};

struct GraphEntry {
  bool adj;
  const void* table;
  const int* active;
  EpiArgs epi;
  hipGraphExec_t exec;
  uint64_t last_use;
};

struct BArgs {
  const Item* items;  // this stage's items
  const OpDev* ops;
  const FsCol* cols;
  const Ptrs* ptrs;
  c64* wpool;
  const c64* tw;
  int32_t adj;
  const int* active;  // per batch column; NULL: every column is active
  EpiArgs epi;
};


}  // namespace fm

struct fm_batch_s {
  uint32_t magic = 0x464d4254u;
  int device = 0;
  std::vector<fm_op> ops;
  std::vector<int64_t> ncols;
  std::vector<int64_t> col_base;  // first batch column of each operator
  int64_t total_cols = 0;
  fm::DevBuf d_items, d_ops, d_cols, d_ptrs, d_wpool;
  std::vector<int64_t> stage_off;  // stage s: items [stage_off[s], stage_off[s+1])
  fm::Schedule sched;
  // captured stage sequences, keyed by direction, pointer table and mask
  bool use_graphs = true;
  hipStream_t cap_stream = nullptr;
  std::vector<fm::GraphEntry> graphs;
  uint64_t graph_clock = 0;
  double tuned_ms = 0.0;
  // pointer tables: kTables device copies, each with a pinned staging buffer,
  // the event after its last upload and the pointers it holds
  static constexpr int kTables = 6;
  fm::Ptrs* staging = nullptr;
  hipEvent_t uploaded[kTables] = {};
  std::vector<fm::Ptrs> held[kTables];
  uint64_t used[kTables] = {};
  uint64_t clock = 0;
  std::vector<fm::Ptrs> cur;
  // solver state, allocated on the first fm_batch_fista call
  fm::DevBuf s_y, s_r, s_g, s_lam, s_L, s_active, s_status, s_iters, s_partial, s_cols, s_utiles, s_pbase, s_user,
      s_beta, s_iter;
  std::vector<int64_t> s_yoff, s_roff;  // per operator: first element in the packed n- / m-sized buffers
  int64_t s_nutiles = 0;
  std::vector<double> s_bound;  // per operator: max |DFT_L(g)|^2 (empty until computed)
};

namespace fm {
bool batch_alive(const fm_batch_s* b);
// Uploads (or finds) the device pointer table for b->cur; returns its address.
fm_status batch_pointer_table(fm_batch_s* b, hipStream_t s, const Ptrs** table);
// Launches every stage of one direction; active: per batch column or NULL.
// The stage sequence is replayed from a captured graph when possible.
fm_status batch_launch(fm_batch_s* b, bool adj, const Ptrs* table, const int* active, hipStream_t s,
                       const EpiArgs* epi = nullptr);
// Rebuilds the work list for a schedule (synchronises the device).
fm_status build_schedule(fm_batch_s* b, const Schedule& sc);
// Destroys the captured graphs.
void drop_graphs(fm_batch_s* b);
}  // namespace fm
