// Batched application of many circulant / Toeplitz operators.
//
// Work is cut into items of one work-group (4096 values) each (see batch.h):
// whole convolutions of length <= 4096 (SINGLE), and for longer embeddings
// L = 4096 * N2 the rows of the four-step split. For N2 <= 2^conv_max_fuse()
// the strided N2-point transforms are folded into the row pass (ROWF: every
// row work-group re-reads the column, which stays in L2 because the rows of
// one operator are kept on one XCD), so a column costs one read of x, one
// write and one read of the L-value intermediate and one write of y; longer
// ones get a separate strided pass first (FS1, then FS2). The last pass (FS3)
// applies the strided inverse transforms and the crop.
//
// The four-step columns are grouped into chunks whose intermediates fit a
// region sized for the memory-side cache, and the passes are software
// pipelined over the chunks: chunk c runs its first pass in stage c, its
// second in stage c+1 and (N2 >= 16) its third in stage c+2, with three
// regions in rotation; the single-pass items are spread over the stages.
// Each stage is one launch that maps work-group g to item g of the
// stage; launch boundaries order the passes, so no work-group ever waits for
// another. The rows of one column are placed at work-group indices that are
// congruent modulo 8, i.e. on one XCD, where they share the column in L2.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <unordered_set>

#include "batch.h"
#include "xform.h"

namespace fm {
namespace {

using namespace xf;

constexpr int kXcds = 8;

// Whole zero-padded convolutions of length 2^lg, it.sub columns.
template <int LOGW>
__device__ __forceinline__ void run_single(const BArgs& a, const Item& it, int lg, c64* smem) {
  const OpDev op = a.ops[it.op];
  const Ptrs pt = a.ptrs[it.op];
  Job<float> jb;
  jb.x = pt.x + int64_t(it.col) * pt.ldx;
  jb.y = pt.y + int64_t(it.col) * pt.ldy;
  jb.xbstride = pt.ldx;
  jb.ybstride = pt.ldy;
  jb.inner = 1;
  jb.nvalid = it.sub;
  jb.in_limit = a.adj ? op.m : op.n;
  jb.out_limit = a.adj ? op.n : op.m;
  jb.i0 = 0;
  jb.S = op.spec;
  jb.sbstride = 0;
  jb.q0 = 0;
  const Mode md{FFT_CONV, a.adj, 0, 0, 0};
  run_job<float, false, LOGW>(jb, md, lg, smem, a.tw);
}

// FS1 (first) or FS3: strided transforms of length 2^lg at stride 4096 over
// 4096/2^lg neighbouring inner indices.
__device__ __forceinline__ void run_strided(const BArgs& a, const Item& it, const FsCol& fc, int lg, bool first,
                                            c64* smem) {
  const OpDev op = a.ops[fc.op];
  const Ptrs pt = a.ptrs[fc.op];
  const int tpw = 1 << (kLogW - lg);
  const int i0 = it.sub * tpw;
  c64* w = a.wpool + fc.woff;
  Job<float> jb;
  jb.xbstride = jb.ybstride = 1;
  jb.inner = 1 << kLog1;
  jb.nvalid = tpw;
  jb.i0 = i0;
  jb.S = nullptr;
  jb.sbstride = 0;
  jb.q0 = i0;
  const int L = 1 << op.logL;
  if (first) {
    jb.x = pt.x + int64_t(fc.col) * pt.ldx + i0;
    jb.y = w + i0;
    jb.in_limit = a.adj ? op.m : op.n;
    jb.out_limit = L;
    const Mode md{FFT_FWD, 0, op.logL, 0, 0};
    run_job<float, true, kLogW>(jb, md, lg, smem, a.tw);
  } else {
    jb.x = w + i0;
    jb.y = pt.y + int64_t(fc.col) * pt.ldy + i0;
    jb.in_limit = L;
    jb.out_limit = a.adj ? op.n : op.m;
    const Mode md{FFT_INV, 0, 0, 0, 0};
    run_job<float, true, kLogW>(jb, md, lg, smem, a.tw);
  }
}

// FS2 / ROWF: one contiguous 4096-point row k2: transform, spectral product,
// inverse transform, twiddles W_L^-(n1 k2), into the column's slot. ROWF forms
// the row from x itself (the strided 2^fuse-point transform and W_L^(n1 k2)).
__device__ __forceinline__ void run_row(const BArgs& a, const Item& it, const FsCol& fc, int fuse, c64* smem) {
  const OpDev op = a.ops[fc.op];
  c64* row = a.wpool + fc.woff + (int64_t(it.sub) << kLog1);
  Job<float> jb;
  if (fuse) {
    const Ptrs pt = a.ptrs[fc.op];
    jb.x = pt.x + int64_t(fc.col) * pt.ldx;
    jb.in_limit = a.adj ? op.m : op.n;
    jb.fuse_log2 = fuse;
  } else {
    jb.x = row;
    jb.in_limit = 1 << kLog1;
  }
  jb.y = row;
  jb.xbstride = jb.ybstride = 0;
  jb.inner = 1;
  jb.nvalid = 1;
  jb.out_limit = 1 << kLog1;
  jb.i0 = 0;
  jb.S = op.spec + (int64_t(it.sub) << kLog1);
  jb.sbstride = 0;
  jb.q0 = it.sub;
  const Mode md{FFT_CONV, a.adj, op.logL, 1, 0};
  run_job<float, false, kLogW>(jb, md, kLog1, smem, a.tw);
}

template <int LOGW>
__global__ __launch_bounds__(Geo<LOGW>::kThreads) void stage_kernel(BArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  c64* smem = reinterpret_cast<c64*>(smem_raw);
  const Item it = a.items[blockIdx.x];
  const int kind = it.kind_log & 0xff;
  const int lg = it.kind_log >> 8;
  if (kind == IT_SINGLE) {
    if (a.active) {  // skip the item when every one of its columns is frozen
      const int64_t g0 = a.ops[it.op].col_base + it.col;
      bool any = false;
      for (int c = 0; c < it.sub; ++c) any |= a.active[g0 + c] != 0;
      if (!any) return;
    }
    run_single<LOGW>(a, it, lg, smem);
    return;
  }
  if constexpr (LOGW == kLogW) {
    const FsCol fc = a.cols[it.col];
    if (a.active && !a.active[a.ops[fc.op].col_base + fc.col]) return;
    if (kind == IT_ROWF)
      run_row(a, it, fc, lg, smem);
    else if (kind == IT_FS2)
      run_row(a, it, fc, 0, smem);
    else
      run_strided(a, it, fc, lg, kind == IT_FS1, smem);
  }
}

}  // namespace
}  // namespace fm

using namespace fm;

namespace {
std::mutex g_batch_mu;
std::unordered_set<const fm_batch_s*>& live_batches() {
  static std::unordered_set<const fm_batch_s*> s;
  return s;
}
}  // namespace

bool fm::batch_alive(const fm_batch_s* b) {
  std::lock_guard<std::mutex> lock(g_batch_mu);
  return live_batches().count(b) != 0;
}

namespace {
void destroy_batch(fm_batch_s* b) {
  {
    std::lock_guard<std::mutex> lock(g_batch_mu);
    live_batches().erase(b);
  }
  for (int k = 0; k < fm_batch_s::kTables; ++k)
    if (b->uploaded[k]) (void)hipEventSynchronize(b->uploaded[k]), (void)hipEventDestroy(b->uploaded[k]);
  if (b->staging) (void)hipHostFree(b->staging);
  for (fm_op o : b->ops) fm_op_release(o);
  b->magic = 0;
  delete b;
}
}  // namespace

fm_status fm::batch_pointer_table(fm_batch_s* b, hipStream_t s, const Ptrs** table) {
  const int nops = int(b->ops.size());
  int slot = -1;
  for (int k = 0; k < fm_batch_s::kTables && slot < 0; ++k) {
    if (b->held[k].size() != b->cur.size()) continue;
    bool same = true;
    for (int i = 0; same && i < nops; ++i)
      same = b->held[k][i].x == b->cur[i].x && b->held[k][i].y == b->cur[i].y &&
             b->held[k][i].ldx == b->cur[i].ldx && b->held[k][i].ldy == b->cur[i].ldy;
    if (same) slot = k;
  }
  Ptrs* dptrs = static_cast<Ptrs*>(b->d_ptrs.p);
  if (slot < 0) {
    // refresh the least recently used copy; the upload is ordered on the
    // stream after every earlier launch that read it
    slot = 0;
    for (int k = 1; k < fm_batch_s::kTables; ++k)
      if (b->used[k] < b->used[slot]) slot = k;
    FM_HIP(hipEventSynchronize(b->uploaded[slot]));  // its staging buffer may still be read
    Ptrs* stg = b->staging + size_t(slot) * nops;
    std::memcpy(stg, b->cur.data(), size_t(nops) * sizeof(Ptrs));
    FM_HIP(hipMemcpyAsync(dptrs + size_t(slot) * nops, stg, size_t(nops) * sizeof(Ptrs), hipMemcpyHostToDevice, s));
    FM_HIP(hipEventRecord(b->uploaded[slot], s));
    b->held[slot] = b->cur;
  }
  b->used[slot] = ++b->clock;
  *table = dptrs + size_t(slot) * nops;
  return FM_OK;
}

fm_status fm::batch_launch(fm_batch_s* b, bool adj, const Ptrs* table, const int* active, hipStream_t s) {
  const void* tw = twiddle_table(Elem::C64, 20);
  FM_CHECK_ARG(tw != nullptr, FM_E_DEVICE, "twiddle table unavailable");
  BArgs a{};
  a.ops = static_cast<const OpDev*>(b->d_ops.p);
  a.cols = static_cast<const FsCol*>(b->d_cols.p);
  a.ptrs = table;
  a.wpool = static_cast<c64*>(b->d_wpool.p);
  a.tw = static_cast<const c64*>(tw);
  a.adj = adj;
  a.active = active;
  const Item* items = static_cast<const Item*>(b->d_items.p);
  for (size_t st = 0; st + 1 < b->stage_off.size(); ++st) {
    const int64_t n = b->stage_off[st + 1] - b->stage_off[st];
    if (n == 0) continue;
    a.items = items + b->stage_off[st];
    hipLaunchKernelGGL(stage_kernel<kLogW>, dim3(unsigned(n)), dim3(Geo<kLogW>::kThreads),
                       (job_lds_bytes<float, kLogW>()), s, a);
    FM_LAUNCHED();
  }
  return FM_OK;
}

extern "C" {

fm_status fm_batch_create(fm_batch* out, int32_t nops, const fm_op* ops, const int64_t* ncols) {
  set_error("");
  FM_CHECK_ARG(out != nullptr, FM_E_INVALID, "output handle pointer is NULL");
  FM_CHECK_ARG(nops >= 1 && ops != nullptr && ncols != nullptr, FM_E_INVALID, "batch: need operators");
  int dev = 0;
  FM_HIP(hipGetDevice(&dev));
  for (int i = 0; i < nops; ++i) {
    FM_CHECK_ARG(ops[i] != nullptr, FM_E_INVALID, "batch: operator %d is NULL", i);
    FM_CHECK_ARG(op_alive(ops[i]), FM_E_RELEASED, "batch: operator %d was released", i);
    const fm_op_s* o = ops[i];
    FM_CHECK_ARG(o->kind == Kind::Circulant || o->kind == Kind::Toeplitz, FM_E_UNSUPPORTED,
                 "batch: operator %d is not a circulant or Toeplitz operator", i);
    FM_CHECK_ARG(o->dt == FM_C64, FM_E_DTYPE, "batch: operator %d is not complex64", i);
    FM_CHECK_ARG(o->device == dev, FM_E_DEVICE, "batch: operator %d lives on another device", i);
    FM_CHECK_ARG(ncols[i] >= 0 && ncols[i] < (int64_t(1) << 24), FM_E_INVALID, "batch: bad column count");
    FM_CHECK_ARG(!o->s32.four_step() || o->s32.log1 == kLog1, FM_E_UNSUPPORTED, "batch: unexpected transform split");
  }
  fm_batch_s* b = new (std::nothrow) fm_batch_s();
  FM_CHECK_ARG(b != nullptr, FM_E_NOMEM, "out of host memory");
  b->device = dev;
  std::vector<OpDev> hops(nops);
  std::vector<Item> mid;  // single-pass items
  std::vector<FsCol> cols;
  std::vector<int> col_log2;
  for (int i = 0; i < nops; ++i) {
    fm_op_s* o = ops[i];
    o->refs.fetch_add(1);
    b->ops.push_back(o);
    b->ncols.push_back(ncols[i]);
    const int logL = ilog2(o->L);
    hops[i] = OpDev{static_cast<const c64*>(o->p32.p), int32_t(o->m), int32_t(o->n), logL, int32_t(ncols[i]),
                    b->total_cols};
    b->col_base.push_back(b->total_cols);
    b->total_cols += ncols[i];
    if (logL <= kLogW) {
      const int B = 1 << (kLogW - logL);  // transforms per work-group
      for (int64_t c0 = 0; c0 < ncols[i]; c0 += B) {
        const int cnt = int(std::min<int64_t>(B, ncols[i] - c0));
        mid.push_back(Item{IT_SINGLE | (logL << 8), i, int32_t(c0), cnt});
      }
    } else {
      for (int64_t c = 0; c < ncols[i]; ++c) {
        cols.push_back(FsCol{i, int32_t(c), 0});
        col_log2.push_back(logL - kLog1);
      }
    }
  }
  // chunks of columns whose intermediates fit one region; three regions rotate
  const size_t region_elems = kRegionBytes / sizeof(c64);
  std::vector<std::vector<int>> chunks;
  {
    size_t used = region_elems;  // forces a first chunk
    for (int j = 0; j < int(cols.size()); ++j) {
      const size_t L = size_t(1) << (col_log2[j] + kLog1);
      if (used + L > region_elems) {
        chunks.emplace_back();
        used = 0;
      }
      cols[j].woff = int64_t(used);  // offset inside the chunk's region
      used += L;
      chunks.back().push_back(j);
    }
  }
  const int nchunks = int(chunks.size());
  for (int c = 0; c < nchunks; ++c)
    for (int j : chunks[c]) cols[j].woff += int64_t(c % 3) * int64_t(region_elems);
  bool unfused = false;
  const int max_fuse = conv_max_fuse();
  for (int lg2 : col_log2) unfused |= lg2 > max_fuse;
  const int nstages = nchunks > 0 ? nchunks + (unfused ? 2 : 1) : (mid.empty() ? 0 : 1);
  // per stage: reuse groups (the rows of one column, which re-read its x and
  // should share an XCD's L2)
  std::vector<std::vector<std::vector<Item>>> groups(size_t(std::max(nstages, 0)));
  for (int c = 0; c < nchunks; ++c) {
    // group the columns of one operator within the chunk
    std::vector<std::pair<int, std::vector<int>>> byop;
    for (int j : chunks[c]) {
      if (byop.empty() || byop.back().first != cols[j].op) byop.push_back({cols[j].op, {}});
      byop.back().second.push_back(j);
    }
    for (const auto& og : byop) {
      const int lg2 = col_log2[og.second[0]];
      const int n2 = 1 << lg2;
      const bool fuse = lg2 <= max_fuse;
      const int npass = fuse ? 2 : 3;
      for (int pass = 0; pass < npass; ++pass) {
        std::vector<Item> g;
        for (int j : og.second) {
          for (int t = 0; t < n2; ++t) {
            if (fuse && pass == 0)
              g.push_back(Item{IT_ROWF | (lg2 << 8), cols[j].op, j, t});
            else if (!fuse && pass == 0)
              g.push_back(Item{IT_FS1 | (lg2 << 8), cols[j].op, j, t});
            else if (!fuse && pass == 1)
              g.push_back(Item{IT_FS2 | (kLog1 << 8), cols[j].op, j, t});
            else
              g.push_back(Item{IT_FS3 | (lg2 << 8), cols[j].op, j, t});
          }
        }
        for (size_t q0 = 0; q0 < g.size(); q0 += size_t(n2))  // one reuse group per column
          groups[size_t(c + pass)].push_back(std::vector<Item>(g.begin() + q0, g.begin() + q0 + n2));
      }
    }
  }
  // middle-length single-pass items spread evenly over the stages
  for (size_t k = 0; k < mid.size(); ++k) {
    const size_t st = nstages > 0 ? k * size_t(nstages) / mid.size() : 0;
    groups[st].push_back({mid[k]});
  }
  // lay out each stage: each group goes to the currently shortest XCD queue,
  // then the queues are interleaved (work-group g runs on XCD g mod 8). A
  // column per group keeps the queues balanced; grouping whole operators
  // measured slower.
  std::vector<Item> items;
  b->stage_off.push_back(0);
  for (int st = 0; st < nstages; ++st) {
    std::vector<std::vector<Item>> q(kXcds);
    auto& gs = groups[size_t(st)];
    for (auto& g : gs) {
      int best = 0;
      for (int x = 1; x < kXcds; ++x)
        if (q[x].size() < q[best].size()) best = x;
      q[best].insert(q[best].end(), g.begin(), g.end());
    }
    size_t longest = 0;
    for (const auto& v : q) longest = std::max(longest, v.size());
    for (size_t r = 0; r < longest; ++r)
      for (int x = 0; x < kXcds; ++x)
        if (r < q[x].size()) items.push_back(q[x][r]);
    b->stage_off.push_back(int64_t(items.size()));
  }
  fm_status st = FM_OK;
  auto fail = [&](fm_status s) {
    destroy_batch(b);
    return s;
  };
  if ((st = b->d_items.alloc(std::max<size_t>(1, items.size()) * sizeof(Item))) != FM_OK) return fail(st);
  if ((st = b->d_ops.alloc(hops.size() * sizeof(OpDev))) != FM_OK) return fail(st);
  if ((st = b->d_cols.alloc(std::max<size_t>(1, cols.size()) * sizeof(FsCol))) != FM_OK) return fail(st);
  if ((st = b->d_ptrs.alloc(size_t(fm_batch_s::kTables) * nops * sizeof(Ptrs))) != FM_OK) return fail(st);
  if (nchunks > 0 && (st = b->d_wpool.alloc(size_t(std::min(3, nchunks)) * kRegionBytes)) != FM_OK)
    return fail(st);
  if (hipHostMalloc(reinterpret_cast<void**>(&b->staging), size_t(fm_batch_s::kTables) * nops * sizeof(Ptrs)) !=
      hipSuccess) {
    set_error("batch: pinned staging allocation failed");
    return fail(FM_E_NOMEM);
  }
  for (int k = 0; k < fm_batch_s::kTables; ++k) {
    if (hipEventCreateWithFlags(&b->uploaded[k], hipEventDisableTiming) != hipSuccess) {
      set_error("batch: event creation failed");
      return fail(FM_E_DEVICE);
    }
  }
  if ((!items.empty() &&
       hipMemcpy(b->d_items.p, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemcpy(b->d_ops.p, hops.data(), hops.size() * sizeof(OpDev), hipMemcpyHostToDevice) != hipSuccess ||
      (!cols.empty() &&
       hipMemcpy(b->d_cols.p, cols.data(), cols.size() * sizeof(FsCol), hipMemcpyHostToDevice) != hipSuccess)) {
    set_error("batch: upload of the work list failed");
    return fail(FM_E_DEVICE);
  }
  {
    std::lock_guard<std::mutex> lock(g_batch_mu);
    live_batches().insert(b);
  }
  *out = b;
  return FM_OK;
}

fm_status fm_batch_apply(fm_batch b, fm_dir dir, const void* const* x, const int64_t* ldx, void* const* y,
                         const int64_t* ldy, void* stream) {
  set_error("");
  FM_CHECK_ARG(b != nullptr, FM_E_INVALID, "batch handle is NULL");
  FM_CHECK_ARG(batch_alive(b), FM_E_RELEASED, "batch handle was released");
  FM_CHECK_ARG(dir == FM_FWD || dir == FM_ADJ, FM_E_INVALID, "unknown direction");
  FM_CHECK_ARG(x != nullptr && y != nullptr && ldx != nullptr && ldy != nullptr, FM_E_INVALID,
               "batch: NULL pointer array");
  const bool adj = dir == FM_ADJ;
  const int nops = int(b->ops.size());
  b->cur.resize(nops);
  for (int i = 0; i < nops; ++i) {
    const fm_op_s* o = b->ops[i];
    const int64_t rin = adj ? o->m : o->n, rout = adj ? o->n : o->m;
    const int64_t nc = b->ncols[i];
    if (nc > 0) {
      FM_CHECK_ARG(x[i] != nullptr && y[i] != nullptr, FM_E_INVALID, "batch: NULL block for operator %d", i);
      FM_CHECK_ARG(ldx[i] >= rin && ldy[i] >= rout, FM_E_SHAPE, "batch: leading dimension of operator %d", i);
      const char* xb = static_cast<const char*>(x[i]);
      const char* yb = static_cast<const char*>(y[i]);
      const size_t xl = size_t((nc - 1) * ldx[i] + rin) * 8, yl = size_t((nc - 1) * ldy[i] + rout) * 8;
      FM_CHECK_ARG(xb + xl <= yb || yb + yl <= xb, FM_E_ALIAS, "batch: x and y of operator %d overlap", i);
    }
    b->cur[i] = Ptrs{static_cast<const c64*>(x[i]), static_cast<c64*>(y[i]), ldx[i], ldy[i]};
  }
  int dev = 0;
  FM_HIP(hipGetDevice(&dev));
  FM_CHECK_ARG(dev == b->device, FM_E_DEVICE, "batch lives on device %d, current is %d", b->device, dev);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const Ptrs* table = nullptr;
  FM_TRY(batch_pointer_table(b, s, &table));
  return batch_launch(b, adj, table, nullptr, s);
}

fm_status fm_batch_release(fm_batch b) {
  set_error("");
  FM_CHECK_ARG(b != nullptr, FM_E_INVALID, "batch handle is NULL");
  FM_CHECK_ARG(batch_alive(b), FM_E_RELEASED, "batch handle was released");
  destroy_batch(b);
  return FM_OK;
}

}  // extern "C"
