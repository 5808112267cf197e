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
#include "epi.h"
#include "mixed.h"
#include "xform.h"

namespace fm {
namespace {

using namespace xf;

constexpr int kXcds = 8;

// ---------------------------------------------------------------- solver epilogues
// (epi.h; complex64 forms)
using ResidualEp = ResidualEpT<float>;
using FistaEp = FistaEpT<float>;

template <int EPI>
__device__ __forceinline__ FistaEp make_fista_ep(const BArgs& a, int op, int64_t col, bool strided, int lg) {
  const User u = a.epi.user[op];
  FistaEp ep;
  ep.X = u.x + col * u.ldx;
  ep.xstride = strided ? 0 : u.ldx;
  ep.gcol0 = a.ops[op].col_base + col;
  ep.colstride = strided ? 0 : 1;
  ep.active = a.active;
  ep.lam = a.epi.lam;
  ep.invLd = 1.0 / a.epi.L[op];
  ep.invL = float(ep.invLd);
  ep.beta = a.epi.beta[*a.epi.iter];
  ep.momentum = a.epi.momentum;
  ep.status = a.epi.status;
  ep.flush_per_slot = !strided && lg < 4;
  ep.pbase = a.epi.pbase;
  ep.partial = a.epi.partial;
  return ep;
}

// Whole zero-padded convolutions of length 2^lg, it.sub columns.
template <int LOGW, int EPI>
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
  if constexpr (EPI == 1) {
    const User u = a.epi.user[it.op];
    ResidualEp ep{u.b + int64_t(it.col) * u.ldb, u.ldb};
    run_job<float, false, LOGW, true>(jb, md, lg, smem, a.tw, &ep);
  } else if constexpr (EPI == 2) {
    FistaEp ep = make_fista_ep<EPI>(a, it.op, it.col, false, lg);
    run_job<float, false, LOGW, true>(jb, md, lg, smem, a.tw, &ep);
    fista_partials<Geo<LOGW>::kThreads>(ep, false, lg, it.sub, 0, smem);
  } else {
    run_job<float, false, LOGW, true>(jb, md, lg, smem, a.tw);
  }
}

// FS1 (first) or FS3: strided transforms of length 2^lg at stride 4096 over
// 4096/2^lg neighbouring inner indices.
template <int EPI>
__device__ __forceinline__ void run_strided_at(const BArgs& a, const Item& it, const FsCol& fc, int lg, bool first,
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
  jb.twl = op.twl;
  if (first) {
    jb.x = pt.x + int64_t(fc.col) * pt.ldx + i0;
    jb.y = w + i0;
    jb.in_limit = a.adj ? op.m : op.n;
    jb.out_limit = L;
    const Mode md{FFT_FWD, 0, op.logL, 0, 0};
    run_job<float, true, kLogW, true>(jb, md, lg, smem, a.tw);
  } else {
    jb.x = w + i0;
    jb.y = pt.y + int64_t(fc.col) * pt.ldy + i0;
    jb.in_limit = L;
    jb.out_limit = a.adj ? op.n : op.m;
    const Mode md{FFT_INV, 0, 0, 0, 0};
    if constexpr (EPI == 1) {
      const User u = a.epi.user[fc.op];
      ResidualEp ep{u.b + int64_t(fc.col) * u.ldb, 0};
      run_job<float, true, kLogW, true>(jb, md, lg, smem, a.tw, &ep);
    } else if constexpr (EPI == 2) {
      FistaEp ep = make_fista_ep<EPI>(a, fc.op, fc.col, true, lg);
      run_job<float, true, kLogW, true>(jb, md, lg, smem, a.tw, &ep);
      fista_partials<Geo<kLogW>::kThreads>(ep, true, lg, tpw, it.sub, smem);
    } else {
      run_job<float, true, kLogW, true>(jb, md, lg, smem, a.tw);
    }
  }
}

// The strided transform length as a compile-time constant (one inlined copy
// per length): unrolled steps and immediate LDS offsets, 1.700 -> 1.693 ms per
// direction on the 512-operator Toeplitz workload.
template <int EPI>
__device__ __forceinline__ void run_strided(const BArgs& a, const Item& it, const FsCol& fc, int lg, bool first,
                                            c64* smem) {
  switch (lg) {
    case 1: run_strided_at<EPI>(a, it, fc, 1, first, smem); return;
    case 2: run_strided_at<EPI>(a, it, fc, 2, first, smem); return;
    case 3: run_strided_at<EPI>(a, it, fc, 3, first, smem); return;
    case 4: run_strided_at<EPI>(a, it, fc, 4, first, smem); return;
    case 5: run_strided_at<EPI>(a, it, fc, 5, first, smem); return;
    default: break;
  }
  run_strided_at<EPI>(a, it, fc, lg, first, smem);
}

// FS2 / ROWF: one contiguous 4096-point row k2: transform, spectral product,
// inverse transform, twiddles W_L^-(n1 k2), into the column's slot. ROWF forms
// the row from x itself (the strided 2^fuse-point transform and W_L^(n1 k2)).
__device__ __forceinline__ void run_row(const BArgs& a, const Item& it, const FsCol& fc, int fuse, c64* smem) {
  const OpDev op = a.ops[fc.op];
  c64* row = a.wpool + fc.woff + (int64_t(it.sub) << kLog1);
  Job<float> jb;
  jb.twl = op.twl;
  if (fuse) {
    const Ptrs pt = a.ptrs[fc.op];
    jb.x = pt.x + int64_t(fc.col) * pt.ldx;
    jb.in_limit = a.adj ? op.m : op.n;
    jb.fuse_n2 = fuse;
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
  run_job<float, false, kLogW, true>(jb, md, kLog1, smem, a.tw);
}

// MX1 / MX3: tile `sub` of the strided pass of a mixed-length column (first:
// the forward n2-point DFTs of the zero-padded x with W_L^(n1 k2) into the
// slot; last: the inverse DFTs of the slot, cropped into y or handed to the
// solver's epilogue).
template <int EPI>
__device__ __forceinline__ void run_mixed(const BArgs& a, const Item& it, const FsCol& fc, int n2, bool first,
                                          c64* smem) {
  const OpDev op = a.ops[fc.op];
  const Ptrs pt = a.ptrs[fc.op];
  c64* w = a.wpool + fc.woff;
  const int64_t L = int64_t(op.n2) << kLog1;
  if (first) {
    mixed_tile<float, NoEp>(n2, it.sub, pt.x + int64_t(fc.col) * pt.ldx, a.adj ? op.m : op.n, w, L, false, op.twl, L,
                            0, static_cast<NoEp*>(nullptr), smem);
    return;
  }
  c64* yc = pt.y + int64_t(fc.col) * pt.ldy;
  const int64_t out_limit = a.adj ? op.n : op.m;
  if constexpr (EPI == 1) {
    const User u = a.epi.user[fc.op];
    ResidualEp ep{u.b + int64_t(fc.col) * u.ldb, 0};
    mixed_tile<float, ResidualEp>(n2, it.sub, w, L, yc, out_limit, true, op.twl, L, 0, &ep, smem);
  } else if constexpr (EPI == 2) {
    FistaEp ep = make_fista_ep<EPI>(a, fc.op, fc.col, true, 12);
    mixed_tile<float, FistaEp>(n2, it.sub, w, L, yc, out_limit, true, op.twl, L, 0, &ep, smem);
    fista_partials<Geo<kLogW>::kThreads>(ep, true, 12, 0, it.sub, smem);
  } else {
    mixed_tile<float, NoEp>(n2, it.sub, w, L, yc, out_limit, true, op.twl, L, 0, static_cast<NoEp*>(nullptr), smem);
  }
}

// Waves per SIMD the stage kernel is compiled for (its register budget):
// four fits the plain and residual forms in 128 VGPRs without spills; the
// FISTA form spills a few registers and still measured faster than at three.
#ifndef FM_STAGE_WAVES
#define FM_STAGE_WAVES 4
#endif

template <int LOGW, int EPI>
__global__ __launch_bounds__(Geo<LOGW>::kThreads, FM_STAGE_WAVES) void stage_kernel(BArgs a) {
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
    run_single<LOGW, EPI>(a, it, lg, smem);
    return;
  }
  const FsCol fc = a.cols[it.col];
  if (a.active && !a.active[a.ops[fc.op].col_base + fc.col]) return;
  if (kind == IT_MX1 || kind == IT_MX3)
    run_mixed<EPI>(a, it, fc, lg, kind == IT_MX1, smem);
  else if (kind == IT_ROWF)
    run_row(a, it, fc, lg, smem);
  else if (kind == IT_FS2)
    run_row(a, it, fc, 0, smem);
  else
    run_strided<EPI>(a, it, fc, lg, kind == IT_FS1, smem);
}

}  // namespace
}  // namespace fm

using namespace fm;

namespace {
// W_L table of a four-step operator (complex64), NULL when unavailable.
const c64* op_twiddles(const fm_op_s* o) {
  if (o->s32.mixed()) return static_cast<const c64*>(twiddle_table_L(Elem::C64, o->L));
  const void* t = twiddle_table(Elem::C64, ilog2(o->L));
  return t ? static_cast<const c64*>(t) + o->L : nullptr;
}

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
  if (!b->graphs.empty()) (void)hipDeviceSynchronize();
  drop_graphs(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
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

void fm::drop_graphs(fm_batch_s* b) {
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.exec);
  b->graphs.clear();
}

namespace {

template <int EPI>
fm_status launch_stages_t(fm_batch_s* b, const BArgs& a0, hipStream_t s) {
  BArgs a = a0;
  const Item* items = static_cast<const Item*>(b->d_items.p);
  for (size_t st = 0; st + 1 < b->stage_off.size(); ++st) {
    const int64_t n = b->stage_off[st + 1] - b->stage_off[st];
    if (n == 0) continue;
    a.items = items + b->stage_off[st];
    hipLaunchKernelGGL((stage_kernel<kLogW, EPI>), dim3(unsigned(n)), dim3(Geo<kLogW>::kThreads),
                       (job_lds_bytes<float, kLogW>()), s, a);
    FM_LAUNCHED();
  }
  return FM_OK;
}

fm_status launch_stages(fm_batch_s* b, const BArgs& a, hipStream_t s) {
  if (a.epi.kind == 1) return launch_stages_t<1>(b, a, s);
  if (a.epi.kind == 2) return launch_stages_t<2>(b, a, s);
  return launch_stages_t<0>(b, a, s);
}

// Captures the stage sequence of one (direction, table, mask) on the batch's
// own stream; nullptr when capture is not possible.
hipGraphExec_t capture(fm_batch_s* b, const BArgs& a) {
  if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
  const fm_status st = launch_stages(b, a, b->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
  if (st != FM_OK || e != hipSuccess || g == nullptr) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return nullptr;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return exec;
}

}  // namespace

fm_status fm::batch_launch(fm_batch_s* b, bool adj, const Ptrs* table, const int* active, hipStream_t s,
                           const EpiArgs* epi) {
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
  if (epi) a.epi = *epi;
  if (b->stage_off.size() < 2) return FM_OK;
  if (b->use_graphs) {
    GraphEntry* hit = nullptr;
    for (auto& g : b->graphs)
      if (g.adj == adj && g.table == table && g.active == active && g.epi.same(a.epi)) hit = &g;
    if (!hit) {
      hipGraphExec_t exec = capture(b, a);
      if (exec) {
        constexpr size_t kMaxGraphs = 16;
        if (b->graphs.size() >= kMaxGraphs) {  // evict the least recently used
          size_t lru = 0;
          for (size_t k = 1; k < b->graphs.size(); ++k)
            if (b->graphs[k].last_use < b->graphs[lru].last_use) lru = k;
          FM_HIP(hipStreamSynchronize(s));  // it may still be running
          (void)hipGraphExecDestroy(b->graphs[lru].exec);
          b->graphs.erase(b->graphs.begin() + long(lru));
        }
        b->graphs.push_back(GraphEntry{adj, table, active, a.epi, exec, 0});
        hit = &b->graphs.back();
      } else {
        b->use_graphs = false;  // this device / runtime cannot capture: launch directly from now on
      }
    }
    if (hit) {
      hit->last_use = ++b->graph_clock;
      FM_HIP(hipGraphLaunch(hit->exec, s));
      return FM_OK;
    }
  }
  return launch_stages(b, a, s);
}

// Work list of one schedule: items per stage, four-step column descriptors
// and the slot pool. Replaces the current schedule (and drops the captured
// graphs, which bake in its buffers).
fm_status fm::build_schedule(fm_batch_s* b, const Schedule& sc) {
  const int nops = int(b->ops.size());
  std::vector<Item> mid;  // single-pass items
  std::vector<FsCol> cols;
  std::vector<int> col_n2;  // strided factor L / 4096 of each four-step column
  for (int i = 0; i < nops; ++i) {
    const int64_t Lop = b->ops[i]->L;
    const int logL = ilog2(Lop);
    const int64_t nc = b->ncols[i];
    if (Lop <= (int64_t(1) << kLogW)) {
      const int B = 1 << (kLogW - logL);  // transforms per work-group
      for (int64_t c0 = 0; c0 < nc; c0 += B) {
        const int cnt = int(std::min<int64_t>(B, nc - c0));
        mid.push_back(Item{IT_SINGLE | (logL << 8), i, int32_t(c0), cnt});
      }
    } else {
      for (int64_t c = 0; c < nc; ++c) {
        cols.push_back(FsCol{i, int32_t(c), 0});
        col_n2.push_back(int(Lop >> kLog1));
      }
    }
  }
  // chunks of columns whose intermediates fit one region; three regions rotate
  const size_t region_elems = sc.region_bytes / sizeof(c64);
  std::vector<std::vector<int>> chunks;
  {
    size_t used = region_elems;  // forces a first chunk
    for (int j = 0; j < int(cols.size()); ++j) {
      const size_t L = size_t(col_n2[j]) << kLog1;
      FM_CHECK_ARG(L <= region_elems, FM_E_UNSUPPORTED, "batch: slot region smaller than one column");
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
  for (int n2 : col_n2) unfused |= n2 > (1 << sc.max_fuse);
  const int nstages = nchunks > 0 ? nchunks + (unfused ? 2 : 1) : (mid.empty() ? 0 : 1);
  // per stage: reuse groups (the rows of one column, which re-read its x and
  // should share an XCD's L2)
  std::vector<std::vector<std::vector<Item>>> groups(size_t(std::max(nstages, 0)));
  for (int c = 0; c < nchunks; ++c) {
    for (int j : chunks[c]) {
      const int n2 = col_n2[j];
      const bool mixed = (n2 & (n2 - 1)) != 0;
      const int lg2 = mixed ? 0 : ilog2(n2);
      const bool fuse = n2 <= (1 << sc.max_fuse);
      const int npass = fuse ? 2 : 3;
      for (int pass = 0; pass < npass; ++pass) {
        const bool strided = pass == npass - 1 || (!fuse && pass == 0);
        const int count = strided && mixed ? mixed_tiles(n2) : n2;
        std::vector<Item> g;
        for (int t = 0; t < count; ++t) {
          if (fuse && pass == 0)
            g.push_back(Item{IT_ROWF | (n2 << 8), cols[j].op, j, t});
          else if (!fuse && pass == 0)
            g.push_back(mixed ? Item{IT_MX1 | (n2 << 8), cols[j].op, j, t}
                              : Item{IT_FS1 | (lg2 << 8), cols[j].op, j, t});
          else if (!fuse && pass == 1)
            g.push_back(Item{IT_FS2 | (kLog1 << 8), cols[j].op, j, t});
          else
            g.push_back(mixed ? Item{IT_MX3 | (n2 << 8), cols[j].op, j, t}
                              : Item{IT_FS3 | (lg2 << 8), cols[j].op, j, t});
        }
        groups[size_t(c + pass)].push_back(std::move(g));
      }
    }
  }
  // single-pass items spread evenly over the stages
  for (size_t k = 0; k < mid.size(); ++k) {
    const size_t st = nstages > 0 ? k * size_t(nstages) / mid.size() : 0;
    groups[st].push_back({mid[k]});
  }
  // lay out each stage: each group goes to the currently shortest XCD queue,
  // then the queues are interleaved (work-group g runs on XCD g mod 8). A
  // column per group keeps the queues balanced; grouping whole operators
  // measured slower, and so did balancing the queues by an estimated cost
  // with the costliest groups first (1.77 against 1.74 ms per direction).
  std::vector<Item> items;
  std::vector<int64_t> stage_off{0};
  for (int st = 0; st < nstages; ++st) {
    std::vector<std::vector<Item>> q(kXcds);
    for (auto& g : groups[size_t(st)]) {
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
    stage_off.push_back(int64_t(items.size()));
  }
  // all work queued on the device before this call may still read the old
  // buffers: wait for it before replacing them
  FM_HIP(hipDeviceSynchronize());
  drop_graphs(b);
  FM_TRY(b->d_items.alloc(std::max<size_t>(1, items.size()) * sizeof(Item)));
  FM_TRY(b->d_cols.alloc(std::max<size_t>(1, cols.size()) * sizeof(FsCol)));
  const size_t pool = nchunks > 0 ? size_t(std::min(3, nchunks)) * sc.region_bytes : 0;
  if (b->d_wpool.bytes != pool) {
    b->d_wpool.reset();
    if (pool > 0) FM_TRY(b->d_wpool.alloc(pool));
  }
  if (!items.empty())
    FM_HIP(hipMemcpy(b->d_items.p, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice));
  if (!cols.empty())
    FM_HIP(hipMemcpy(b->d_cols.p, cols.data(), cols.size() * sizeof(FsCol), hipMemcpyHostToDevice));
  b->stage_off = std::move(stage_off);
  b->sched = sc;
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
  for (int i = 0; i < nops; ++i)
    FM_CHECK_ARG(ops[i]->L <= (int64_t(1) << kLog1) || op_twiddles(ops[i]) != nullptr, FM_E_DEVICE,
                 "batch: twiddle table unavailable: %s", last_error());
  fm_batch_s* b = new (std::nothrow) fm_batch_s();
  FM_CHECK_ARG(b != nullptr, FM_E_NOMEM, "out of host memory");
  b->device = dev;
  std::vector<OpDev> hops(nops);
  for (int i = 0; i < nops; ++i) {
    fm_op_s* o = ops[i];
    o->refs.fetch_add(1);
    b->ops.push_back(o);
    b->ncols.push_back(ncols[i]);
    const c64* twl = o->L > (int64_t(1) << kLog1) ? op_twiddles(o) : nullptr;
    hops[i] = OpDev{static_cast<const c64*>(o->p32.p), int32_t(o->m), int32_t(o->n), ilog2(o->L), int32_t(ncols[i]),
                    b->total_cols, twl, int32_t(o->L > (int64_t(1) << kLog1) ? o->L >> kLog1 : 1)};
    b->col_base.push_back(b->total_cols);
    b->total_cols += ncols[i];
  }
  fm_status st = FM_OK;
  auto fail = [&](fm_status s) {
    destroy_batch(b);
    return s;
  };
  if ((st = b->d_ops.alloc(hops.size() * sizeof(OpDev))) != FM_OK) return fail(st);
  if ((st = b->d_ptrs.alloc(size_t(fm_batch_s::kTables) * nops * sizeof(Ptrs))) != FM_OK) return fail(st);
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
  if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    set_error("batch: stream creation failed");
    return fail(FM_E_DEVICE);
  }
  if (hipMemcpy(b->d_ops.p, hops.data(), hops.size() * sizeof(OpDev), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("batch: upload of the operator table failed");
    return fail(FM_E_DEVICE);
  }
  {
    const char* e = std::getenv("FM_BATCH_GRAPH");
    b->use_graphs = !(e && std::atoi(e) == 0);
  }
  Schedule sc;
  sc.max_fuse = conv_max_fuse();
  if ((st = build_schedule(b, sc)) != FM_OK) return fail(st);
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

fm_status fm_batch_tune(fm_batch b, fm_dir dir, const void* const* x, const int64_t* ldx, void* const* y,
                        const int64_t* ldy, int32_t reps, fm_batch_schedule* chosen, void* stream) {
  set_error("");
  FM_CHECK_ARG(b != nullptr, FM_E_INVALID, "batch handle is NULL");
  FM_CHECK_ARG(batch_alive(b), FM_E_RELEASED, "batch handle was released");
  FM_CHECK_ARG(reps >= 1 && reps <= 1000, FM_E_INVALID, "tune: reps must be in 1..1000");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  FM_TRY(fm_batch_apply(b, dir, x, ldx, y, ldy, stream));  // validates the arguments
  hipEvent_t e0, e1;
  FM_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    set_error("tune: event creation failed");
    return FM_E_DEVICE;
  }
  Schedule best = b->sched;
  const Schedule entry = b->sched;
  double best_ms = -1.0;
  fm_status st = FM_OK;
  // ms per application of schedule sc: warm-up (and graph capture), then n timed
  auto time_one = [&](const Schedule& sc, int n, double* per) -> fm_status {
    FM_TRY(build_schedule(b, sc));
    FM_TRY(fm_batch_apply(b, dir, x, ldx, y, ldy, stream));
    FM_HIP(hipEventRecord(e0, s));
    for (int k = 0; k < n; ++k) FM_TRY(fm_batch_apply(b, dir, x, ldx, y, ldy, stream));
    float ms = 0.f;
    FM_HIP(hipEventRecord(e1, s));
    FM_HIP(hipEventSynchronize(e1));
    FM_HIP(hipEventElapsedTime(&ms, e0, e1));
    *per = double(ms) / n;
    return FM_OK;
  };
  // every candidate once, then the four fastest again in two interleaved
  // rounds with twice the repetitions, each keeping its minimum: a single
  // timing per candidate let a transient slowdown pick a slower schedule
  const int regions[3] = {24, 48, 96};
  std::vector<std::pair<double, Schedule>> cand;
  for (int mf = 0; mf <= 5 && st == FM_OK; ++mf) {
    for (int r = 0; r < 3 && st == FM_OK; ++r) {
      Schedule sc;
      sc.max_fuse = mf;
      sc.region_bytes = size_t(regions[r]) << 20;
      double per = 0.0;
      if ((st = time_one(sc, reps, &per)) != FM_OK) break;
      cand.emplace_back(per, sc);
    }
  }
  if (st == FM_OK) {
    std::stable_sort(cand.begin(), cand.end(), [](const auto& u, const auto& v) { return u.first < v.first; });
    if (cand.size() > 4) cand.resize(4);
    bool has_entry = false;  // the schedule in use on entry is always timed again
    for (const auto& c : cand)
      has_entry |= c.second.max_fuse == entry.max_fuse && c.second.region_bytes == entry.region_bytes;
    if (!has_entry) cand.emplace_back(1e30, entry);
    for (int round = 0; round < 2 && st == FM_OK; ++round)
      for (auto& c : cand) {
        double per = 0.0;
        if ((st = time_one(c.second, 2 * reps, &per)) != FM_OK) break;
        c.first = std::min(c.first, per);
      }
    for (const auto& c : cand)
      if (best_ms < 0 || c.first < 0.99 * best_ms) {
        best_ms = c.first;
        best = c.second;
      }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != FM_OK) {
    (void)build_schedule(b, best);
    return st;
  }
  FM_TRY(build_schedule(b, best));
  b->tuned_ms = best_ms;
  FM_TRY(fm_batch_apply(b, dir, x, ldx, y, ldy, stream));  // y from the chosen schedule
  if (chosen) FM_TRY(fm_batch_get_schedule(b, chosen));
  return FM_OK;
}

fm_status fm_batch_get_schedule(fm_batch b, fm_batch_schedule* out) {
  set_error("");
  FM_CHECK_ARG(b != nullptr && out != nullptr, FM_E_INVALID, "NULL argument");
  FM_CHECK_ARG(batch_alive(b), FM_E_RELEASED, "batch handle was released");
  out->max_fuse = b->sched.max_fuse;
  out->region_mib = int32_t(b->sched.region_bytes >> 20);
  out->graphs = b->use_graphs ? 1 : 0;
  int32_t n = 0;
  for (size_t st = 0; st + 1 < b->stage_off.size(); ++st) n += b->stage_off[st + 1] > b->stage_off[st] ? 1 : 0;
  out->stages = n;
  out->ms = b->tuned_ms;
  return FM_OK;
}

fm_status fm_batch_set_schedule(fm_batch b, const fm_batch_schedule* sc) {
  set_error("");
  FM_CHECK_ARG(b != nullptr && sc != nullptr, FM_E_INVALID, "NULL argument");
  FM_CHECK_ARG(batch_alive(b), FM_E_RELEASED, "batch handle was released");
  FM_CHECK_ARG(sc->max_fuse >= 0 && sc->max_fuse <= 5, FM_E_INVALID, "max_fuse must be in 0..5");
  FM_CHECK_ARG(sc->region_mib >= 16 && sc->region_mib <= 1024, FM_E_INVALID, "region_mib must be in 16..1024");
  Schedule s;
  s.max_fuse = sc->max_fuse;
  s.region_bytes = size_t(sc->region_mib) << 20;
  FM_TRY(build_schedule(b, s));
  b->tuned_ms = 0.0;
  return FM_OK;
}

fm_status fm_batch_release(fm_batch b) {
  set_error("");
  FM_CHECK_ARG(b != nullptr, FM_E_INVALID, "batch handle is NULL");
  FM_CHECK_ARG(batch_alive(b), FM_E_RELEASED, "batch handle was released");
  destroy_batch(b);
  return FM_OK;
}

}  // extern "C"
