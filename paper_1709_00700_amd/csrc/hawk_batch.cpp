// Batched execution behind the C ABI: many queries in one captured HIP graph
// of persistent work-queue kernels (hk_batch.hip), and the autotuner that
// picks the graph's schedule (tile size, workgroups per CU, queue order).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <set>
#include <string>
#include <vector>

#include "hawk.h"
#include "hawk_batch.h"
#include "hawk_internal.h"
#include "hawk_launch.h"

namespace {

const int64_t kBuildTile = 1 << 14;   // build rows per work item
const int64_t kFinalTile = 1 << 16;   // table slots per finalize work item
// grouped aggregations with more groups than a tile's LDS table holds get
// their own launches (spilling instead of device-scope atomics) from this size on
const int64_t kDirectRows = 1 << 20;
const int64_t kLdsBudget = 64512;     // LDS bytes of a grouped tile's table (64 KB with the static words)
enum { HEAD_BUILD = 0, HEAD_MAIN = 1, HEAD_FINAL = 6, HEAD_COUNT = 8 };

uint32_t clog2(uint64_t x) {
  uint32_t l = 0;
  while ((1ull << l) < x) ++l;
  return l;
}

uint64_t sm64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

struct hawk_batch {
  hawk_ctx* ctx = nullptr;
  std::vector<hawk_query*> qs;
  std::vector<hawk_variant> variants;   // per query (empty: none given)
  hawk_batch_opts opts{};
  std::vector<void*> allocs;            // device memory owned by the batch
  std::vector<HkBatchQuery> hq;         // per query descriptors (host copy)
  std::vector<HkBuild> hb;              // every build pipeline of every query
  std::vector<int64_t> build_rows;
  std::vector<HkFillJob> fills;
  std::vector<int64_t> fill_n;
  std::vector<std::vector<int>> res_kinds;
  // schedule-dependent device arrays
  HkBatchQuery* d_qs = nullptr;
  HkBuild* d_builds = nullptr;
  HkFillJob* d_fill = nullptr;
  int64_t* d_fill_bases = nullptr;
  int64_t fill_total = 0;
  int64_t* d_build_bases = nullptr;
  int64_t build_items = 0;
  int32_t* d_qidx[5] = {};
  int64_t* d_bases[5] = {};
  int32_t nq_shape[5] = {};
  int64_t items_shape[5] = {};
  size_t lds_shape[5] = {};
  int32_t* d_fqidx = nullptr;
  int64_t* d_fbases = nullptr;
  int32_t nfq = 0;
  int64_t final_items = 0;
  unsigned long long* d_heads = nullptr;
  int* d_err = nullptr;
  std::vector<void*> sched_allocs;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::set<hawk_result*> views;         // live result views of this batch
  // queries that run their own variant's kernels inside the graph: those
  // given a variant, and (by default) large grouped aggregations with more
  // groups than a tile's LDS table holds (spilling instead of device-scope
  // atomics). Each owns one region of device memory laid out by the
  // execution itself (exec_arena); `holder` describes its flags and results.
  struct Own {
    int32_t q;
    hawk_variant v;
    char* region;
    size_t bytes;
    hawk_result holder;
  };
  std::vector<Own> own;
  std::vector<char> is_own;
};

namespace {

hawk_status berr(hawk_batch* B, hawk_status st, const std::string& m) { return set_error(B->ctx, st, m); }

void* balloc(hawk_batch* B, size_t bytes, std::vector<void*>& list) {
  void* p = nullptr;
  if (bytes < 256) bytes = 256;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  list.push_back(p);
  return p;
}

void add_fill(hawk_batch* B, uint64_t* ptr, int64_t n, const uint64_t* pattern, int32_t period) {
  HkFillJob j;
  std::memset(&j, 0, sizeof(j));
  j.ptr = ptr;
  for (int i = 0; i < period; ++i) j.pattern[i] = pattern[i];
  j.period = period;
  B->fills.push_back(j);
  B->fill_n.push_back(n);
}

void add_zero(hawk_batch* B, uint64_t* ptr, int64_t n) {
  const uint64_t z = 0;
  add_fill(B, ptr, n, &z, 1);
}

// Whether query i runs its own kernels, and in which variant: the one given
// for it (thread_mult 0 = the tile kernels), or, without one and with
// `separate`, a grouped aggregation of at least kDirectRows rows whose groups
// do not fit a tile's LDS table runs the local strategy with linear probing
// (spilling scans without probes: one workgroup of 1024 per CU; with probes,
// which are latency-bound: about 64K rows per workgroup of 512, up to 8 per CU).
bool own_variant(const hawk_batch* B, size_t i, hawk_variant& v) {
  if (!B->variants.empty() && B->variants[i].thread_mult != 0) {
    v = B->variants[i];
    return true;
  }
  const hawk_query* q = B->qs[i];
  const int64_t n = q->main.nrows;
  if (!B->opts.separate || q->kind != 2 || q->main.ngroup == 0 || n < kDirectRows) return false;
  const int W = q->main.slot_words;
  const uint64_t groups = static_cast<uint64_t>(std::max<int64_t>(1, std::min<int64_t>(q->groups_hint, n)));
  uint32_t fit = 0;
  while ((int64_t(2) << fit) * W * 8 <= kLdsBudget) ++fit;
  const uint32_t llog2 = std::min(std::max<uint32_t>(4, clog2(groups * 2)), fit);
  if ((uint64_t(1) << llog2) >= 2 * groups) return false;
  v = hawk_variant{};
  v.proj_strategy = HAWK_MULTI_PASS;
  v.mem = HAWK_COALESCED;
  v.pred = HAWK_BRANCHED;
  v.ht = HAWK_LINEAR_PROBING;
  v.hash = HAWK_MURMUR;
  v.agg_strategy = HAWK_LOCAL;
  if (q->main.nprobes == 0) {
    v.thread_mult = 1;
    v.wg_size = 1024;
  } else {
    uint32_t tm = 1;
    while (tm < 8 && n / (static_cast<int64_t>(B->ctx->num_cus) * 2 * tm) >= 65536) tm *= 2;
    v.thread_mult = tm;
    v.wg_size = 512;
  }
  return true;
}

// device memory of every query: tables, outputs, counters (independent of the schedule)
hawk_status setup_memory(hawk_batch* B) {
  hawk_ctx* ctx = B->ctx;
  uint64_t seed = ctx->seed;
  HkHash h;
  for (int i = 0; i < HK_CUCKOO_D; ++i) h.a[i] = sm64(seed);
  B->d_heads = static_cast<unsigned long long*>(balloc(B, HEAD_COUNT * 8, B->allocs));
  B->d_err = static_cast<int*>(balloc(B, 8, B->allocs));
  if (!B->d_heads || !B->d_err) return berr(B, HAWK_E_OOM, "batch counters");
  add_zero(B, reinterpret_cast<uint64_t*>(B->d_heads), HEAD_COUNT);
  add_zero(B, reinterpret_cast<uint64_t*>(B->d_err), 1);
  const int64_t min_tile = 1 << 14;
  B->is_own.assign(B->qs.size(), 0);
  for (size_t i = 0; i < B->qs.size(); ++i) {
    const hawk_query* q = B->qs[i];
    HkBatchQuery Q;
    std::memset(&Q, 0, sizeof(Q));
    Q.plan = q->main;
    Q.plan.hash = h;
    hawk_variant ov{};
    if (own_variant(B, i, ov)) {
      // its own kernels, tables and results: nothing of the tile kernels' state
      Q.kind = q->kind == 1 ? HK_BQ_PROJECT : (Q.plan.ngroup > 0 ? HK_BQ_GROUPED : HK_BQ_SCALAR);
      Q.shape = hk_shape_of(Q.plan);
      B->hq.push_back(Q);
      B->is_own[i] = 1;
      hawk_batch::Own o{};
      o.q = static_cast<int32_t>(i);
      o.v = ov;
      B->own.push_back(o);
      continue;
    }
    // build pipelines of this query
    std::vector<HkJoinTable> tabs;
    for (const QueryBuild& qb : q->builds) {
      HkJoinTable t;
      std::memset(&t, 0, sizeof(t));
      t.log2cap = std::max<uint32_t>(4, clog2(static_cast<uint64_t>(std::max<int64_t>(1, qb.nrows)) * 2));
      if (t.log2cap > 31) return berr(B, HAWK_E_CAPACITY, "join table beyond 2^31 slots");
      t.slots = static_cast<uint64_t*>(balloc(B, (static_cast<size_t>(1) << t.log2cap) * 8, B->allocs));
      t.side = static_cast<uint64_t*>(balloc(B, 16, B->allocs));
      if (!t.slots || !t.side) return berr(B, HAWK_E_OOM, "batch join table");
      const uint64_t e = HK_EMPTY;
      add_fill(B, t.slots, int64_t(1) << t.log2cap, &e, 1);
      add_zero(B, t.side, 2);
      HkBuild b;
      std::memset(&b, 0, sizeof(b));
      b.p = qb.plan;
      b.p.hash = h;
      b.key = qb.key;
      b.payload = qb.payload;
      b.t = t;
      B->hb.push_back(b);
      B->build_rows.push_back(qb.nrows);
      tabs.push_back(t);
    }
    for (int p = 0; p < Q.plan.nprobes; ++p) Q.plan.probes[p].t = tabs[q->probe_build[p]];
    Q.shape = hk_shape_of(Q.plan);
    Q.err = B->d_err;
    Q.count = static_cast<uint64_t*>(balloc(B, 8, B->allocs));
    if (!Q.count) return berr(B, HAWK_E_OOM, "batch count");
    add_zero(B, Q.count, 1);
    const int64_t n = Q.plan.nrows;
    if (q->kind == 1) {
      Q.kind = HK_BQ_PROJECT;
      for (int c = 0; c < Q.plan.nproj; ++c) {
        Q.out.col[c] = static_cast<int64_t*>(balloc(B, static_cast<size_t>(n + 1) * 8, B->allocs));
        if (!Q.out.col[c]) return berr(B, HAWK_E_OOM, "batch projection output");
      }
      Q.out.dump = n;
      const int64_t maxtiles = std::max<int64_t>(1, (n + min_tile - 1) / min_tile);
      Q.status = static_cast<uint64_t*>(balloc(B, static_cast<size_t>(maxtiles) * 8, B->allocs));
      if (!Q.status) return berr(B, HAWK_E_OOM, "batch look-back words");
      add_zero(B, Q.status, maxtiles);
    } else {
      const bool grouped = Q.plan.ngroup > 0;
      Q.kind = grouped ? HK_BQ_GROUPED : HK_BQ_SCALAR;
      const int W = Q.plan.slot_words;
      Q.ident.nw = W;
      Q.ident.w[0] = grouped ? HK_EMPTY : 0ull;
      for (int a = 0; a < Q.plan.naggs; ++a) {
        const HkAgg& A = Q.plan.aggs[a];
        if (A.fn == HK_COUNT) continue;
        Q.ident.w[A.word] = A.fn == HK_MIN ? static_cast<uint64_t>(INT64_MAX)
                            : A.fn == HK_MAX ? static_cast<uint64_t>(INT64_MIN) : 0ull;
      }
      Q.table.slot_words = W;  // rlog2 below: one region (whole-table probing)
      if (grouped) {
        // a pipeline cannot produce more groups than it scans rows
        const uint64_t groups = static_cast<uint64_t>(std::max<int64_t>(1, std::min<int64_t>(q->groups_hint, n)));
        Q.table.log2cap = std::max<uint32_t>(6, clog2(groups * 2));
        if (Q.table.log2cap > 31) return berr(B, HAWK_E_CAPACITY, "aggregation table beyond 2^31 slots");
        Q.nslots = (int64_t(1) << Q.table.log2cap) + 1;  // + side slot for the all-ones key
        Q.table.rlog2 = Q.table.log2cap;
        uint32_t want = std::max<uint32_t>(4, clog2(groups * 4)), fit = 0;  // four slots per group
        while ((int64_t(2) << fit) * W * 8 <= kLdsBudget) ++fit;
        Q.llog2 = std::min(want, fit);
      } else {
        Q.table.log2cap = 0;
        Q.nslots = 1;
      }
      Q.table.words = static_cast<uint64_t*>(balloc(B, static_cast<size_t>(Q.nslots * W) * 8, B->allocs));
      if (!Q.table.words) return berr(B, HAWK_E_OOM, "batch aggregation table");
      add_fill(B, Q.table.words, Q.nslots * W, Q.ident.w, W);
      const int64_t cap = Q.nslots;
      for (int g = 0; g < Q.plan.ngroup; ++g) {
        Q.res.gcol[g] = static_cast<int64_t*>(balloc(B, static_cast<size_t>(cap) * 8, B->allocs));
        if (!Q.res.gcol[g]) return berr(B, HAWK_E_OOM, "batch result");
      }
      for (int a = 0; a < Q.plan.naggs; ++a) {
        const int kind = q->res_kinds[a];
        Q.res.acol[a] = balloc(B, static_cast<size_t>(cap) * (kind == HAWK_RES_I128 ? 16 : 8), B->allocs);
        if (!Q.res.acol[a]) return berr(B, HAWK_E_OOM, "batch result");
      }
      Q.res.count = static_cast<int64_t*>(balloc(B, static_cast<size_t>(cap) * 8, B->allocs));
      if (!Q.res.count) return berr(B, HAWK_E_OOM, "batch result");
      Q.res.nrows = reinterpret_cast<unsigned long long*>(Q.count);
      Q.res.keep_empty = grouped ? 0 : 1;
    }
    B->hq.push_back(Q);
  }
  // regions of the queries with their own kernels: sizes from a pass that
  // enqueues nothing, then a pass that uploads their plans (and compiles
  // their run-time kernels) with the final addresses
  for (auto& o : B->own) {
    const hawk_query* q = B->qs[o.q];
    hawk_status st = exec_arena(ctx, q, &o.v, ctx->stream, nullptr, 0, false, false, &o.holder, &o.bytes);
    if (st) return st;
    o.region = static_cast<char*>(balloc(B, o.bytes, B->allocs));
    if (!o.region) return berr(B, HAWK_E_OOM, "batch region of a query with its own variant");
    st = exec_arena(ctx, q, &o.v, ctx->stream, o.region, o.bytes, false, true, &o.holder, nullptr);
    if (st) return st;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return berr(B, HAWK_E_DEVICE, "plan upload");
  }
  return HAWK_OK;
}

void free_schedule(hawk_batch* B) {
  if (B->exec && B->ctx) (void)hipStreamSynchronize(B->ctx->stream);  // a replay may still read the arrays
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
  for (void* p : B->sched_allocs) (void)hipFree(p);
  B->sched_allocs.clear();
}

template <class T>
T* upload(hawk_batch* B, const std::vector<T>& v) {
  T* d = static_cast<T*>(balloc(B, std::max<size_t>(1, v.size()) * sizeof(T), B->sched_allocs));
  if (d && !v.empty() && hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
  return d;
}

std::vector<int64_t> prefix(const std::vector<int64_t>& n) {
  std::vector<int64_t> b(n.size() + 1, 0);
  for (size_t i = 0; i < n.size(); ++i) b[i + 1] = b[i] + n[i];
  return b;
}

// work lists, device descriptors and the captured graph for one schedule
hawk_status setup_schedule(hawk_batch* B, const hawk_batch_opts& o) {
  free_schedule(B);
  hawk_ctx* ctx = B->ctx;
  const int64_t tile = int64_t(1) << o.tile_rows_log2;
  std::vector<HkBatchQuery> hq = B->hq;
  for (auto& Q : hq) {
    Q.tile_rows = tile;
    Q.ntiles = (Q.plan.nrows + tile - 1) / tile;
  }
  // main work lists per shape class, in submission or largest-first order
  std::vector<int32_t> order(hq.size());
  std::iota(order.begin(), order.end(), 0);
  if (o.order == 1)
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return hq[a].plan.nrows > hq[b].plan.nrows; });
  for (int s = 0; s < 5; ++s) {
    std::vector<int32_t> qi;
    std::vector<int64_t> nt;
    size_t lds = 64;
    for (int32_t i : order) {
      const HkBatchQuery& Q = hq[i];
      if (Q.shape != s || Q.ntiles == 0 || B->is_own[i]) continue;
      qi.push_back(i);
      nt.push_back(Q.ntiles);
      size_t need;
      if (Q.kind == HK_BQ_PROJECT) need = (tile / 64) * 8 + (tile / 64 + 2) * 4 + 16;
      else if (Q.kind == HK_BQ_GROUPED) need = (static_cast<size_t>(1) << Q.llog2) * Q.ident.nw * 8;
      else need = static_cast<size_t>(Q.ident.nw) * 8;
      lds = std::max(lds, need);
    }
    const std::vector<int64_t> bases = prefix(nt);
    B->nq_shape[s] = static_cast<int32_t>(qi.size());
    B->items_shape[s] = bases.back();
    if (static_cast<int64_t>(lds) > std::min<int64_t>(ctx->lds_bytes, 65536))
      return berr(B, HAWK_E_INFEASIBLE, "batch tile does not fit in LDS");
    B->lds_shape[s] = lds;
    B->d_qidx[s] = upload(B, qi);
    B->d_bases[s] = upload(B, bases);
    if (!B->d_qidx[s] || !B->d_bases[s]) return berr(B, HAWK_E_OOM, "batch work lists");
  }
  // finalize list: every aggregation query's slots
  std::vector<int32_t> fq;
  std::vector<int64_t> fn;
  for (size_t i = 0; i < hq.size(); ++i)
    if (hq[i].kind != HK_BQ_PROJECT && !B->is_own[i]) {
      fq.push_back(static_cast<int32_t>(i));
      fn.push_back((hq[i].nslots + kFinalTile - 1) / kFinalTile);
    }
  const std::vector<int64_t> fb = prefix(fn);
  B->nfq = static_cast<int32_t>(fq.size());
  B->final_items = fb.back();
  B->d_fqidx = upload(B, fq);
  B->d_fbases = upload(B, fb);
  // builds
  std::vector<int64_t> bn;
  for (int64_t r : B->build_rows) bn.push_back((r + kBuildTile - 1) / kBuildTile);
  const std::vector<int64_t> bb = prefix(bn);
  B->build_items = bb.back();
  B->d_build_bases = upload(B, bb);
  B->d_builds = upload(B, B->hb);
  // fills
  const std::vector<int64_t> fillb = prefix(B->fill_n);
  B->fill_total = fillb.back();
  B->d_fill = upload(B, B->fills);
  B->d_fill_bases = upload(B, fillb);
  B->d_qs = upload(B, hq);
  if (!B->d_fqidx || !B->d_fbases || !B->d_build_bases || !B->d_builds || !B->d_fill || !B->d_fill_bases || !B->d_qs)
    return berr(B, HAWK_E_OOM, "batch descriptors");
  // capture: fill -> builds -> main kernels -> finalize
  const int64_t grid = static_cast<int64_t>(ctx->num_cus) * std::max(1, o.wgs_per_cu);
  hipError_t e = hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return berr(B, HAWK_E_DEVICE, std::string("capture: ") + hipGetErrorString(e));
  hipError_t le = hk_batch_fill(B->cap, B->d_fill, B->d_fill_bases, static_cast<int32_t>(B->fills.size()), B->fill_total);
  if (le == hipSuccess)
    le = hk_batch_build(B->cap, std::min<int64_t>(grid, std::max<int64_t>(1, B->build_items)), B->d_builds,
                        B->d_build_bases, static_cast<int32_t>(B->hb.size()), B->build_items, kBuildTile,
                        B->d_heads + HEAD_BUILD, B->d_err);
  // the queries with their own variant: their kernels over their regions
  for (auto& o : B->own) {
    if (le != hipSuccess) break;
    const hawk_status st = exec_arena(ctx, B->qs[o.q], &o.v, B->cap, o.region, o.bytes, true, false, &o.holder, nullptr);
    if (st) {
      (void)hipStreamEndCapture(B->cap, &B->graph);
      if (B->graph) (void)hipGraphDestroy(B->graph);
      B->graph = nullptr;
      return st;
    }
  }
  for (int s = 0; s < 5 && le == hipSuccess; ++s)
    le = hk_batch_main(B->cap, s, std::min<int64_t>(grid, std::max<int64_t>(1, B->items_shape[s])), 256,
                       B->lds_shape[s], B->d_qs, B->d_qidx[s], B->d_bases[s], B->nq_shape[s], B->items_shape[s],
                       B->d_heads + HEAD_MAIN + s);
  if (le == hipSuccess)
    le = hk_batch_final(B->cap, std::min<int64_t>(grid, std::max<int64_t>(1, B->final_items)), B->d_qs, B->d_fqidx,
                        B->d_fbases, B->nfq, B->final_items, kFinalTile, B->d_heads + HEAD_FINAL);
  e = hipStreamEndCapture(B->cap, &B->graph);
  if (le != hipSuccess) return berr(B, HAWK_E_DEVICE, std::string("batch launch: ") + hipGetErrorString(le));
  if (e != hipSuccess) return berr(B, HAWK_E_DEVICE, std::string("end capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return berr(B, HAWK_E_DEVICE, std::string("instantiate: ") + hipGetErrorString(e));
  B->opts = o;
  return HAWK_OK;
}

bool valid_opts(const hawk_batch_opts& o) {
  return o.tile_rows_log2 >= 14 && o.tile_rows_log2 <= 18 && o.wgs_per_cu >= 1 && o.wgs_per_cu <= 32 &&
         (o.order == 0 || o.order == 1) && (o.separate == 0 || o.separate == 1);
}

}  // namespace

void batch_forget_view(hawk_batch* B, hawk_result* r) { B->views.erase(r); }

void batch_release_device(hawk_batch* B) {
  if (!B->ctx) return;
  (void)hipStreamSynchronize(B->ctx->stream);
  for (hawk_result* r : B->views) {  // views read freed memory no more: orphan them
    if (r->ctx) r->ctx->results.erase(r);
    r->ctx = nullptr;
    r->batch = nullptr;
  }
  B->views.clear();
  free_schedule(B);
  for (void* p : B->allocs) (void)hipFree(p);
  B->allocs.clear();
  if (B->cap) (void)hipStreamDestroy(B->cap);
  B->cap = nullptr;
  B->ctx = nullptr;
}

extern "C" hawk_status hawk_batch_create(hawk_ctx* ctx, hawk_query* const* qs, int32_t n,
                                         const hawk_variant* variants, const hawk_batch_opts* opts,
                                         hawk_batch** out) {
  if (!ctx) return HAWK_E_ARG;
  if (!qs || n < 1 || !out) return set_error(ctx, HAWK_E_ARG, "null argument");
  *out = nullptr;
  if (ctx->device < 0) return set_error(ctx, HAWK_E_DEVICE, "planning context cannot execute");
  hawk_batch_opts o = opts ? *opts : hawk_batch_opts{16, 2, 1, 1};
  if (!valid_opts(o)) return set_error(ctx, HAWK_E_ARG, "batch options out of range");
  hawk_batch* B = new hawk_batch();
  B->ctx = ctx;
  for (int32_t i = 0; i < n; ++i) {
    if (!qs[i] || qs[i]->ctx != ctx) {
      delete B;
      return set_error(ctx, HAWK_E_ARG, "query of another context");
    }
    B->qs.push_back(qs[i]);
    if (variants) {
      const hawk_variant& v = variants[i];
      if (v.thread_mult != 0 && (v.mem > 1 || v.pred > 1 || v.ht > 2 || v.hash > 1 || v.agg_strategy > 1 ||
                                 v.proj_strategy > 1 || v.wg_size < 1 || v.wg_size > 1024)) {
        delete B;
        return set_error(ctx, HAWK_E_ARG, "variant value out of range");
      }
      B->variants.push_back(v);
    }
  }
  if (hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking) != hipSuccess) {
    delete B;
    return set_error(ctx, HAWK_E_DEVICE, "capture stream");
  }
  ctx->batches.insert(B);
  B->opts = o;  // setup_memory reads `separate`
  hawk_status st = setup_memory(B);
  if (!st) st = setup_schedule(B, o);
  if (st) {
    hawk_batch_free(B);
    return st;
  }
  *out = B;
  return HAWK_OK;
}

extern "C" void hawk_batch_free(hawk_batch* B) {
  if (!B) return;
  if (B->ctx) {
    B->ctx->batches.erase(B);
    batch_release_device(B);
  }
  delete B;
}

extern "C" hawk_status hawk_batch_run(hawk_batch* B) {
  if (!B || !B->ctx || !B->exec) return HAWK_E_ARG;
  for (hawk_result* r : B->views) r->checked = false;  // views report the latest run
  hipError_t e = hipGraphLaunch(B->exec, B->ctx->stream);
  if (e != hipSuccess) return berr(B, HAWK_E_DEVICE, std::string("graph launch: ") + hipGetErrorString(e));
  return HAWK_OK;
}

extern "C" hawk_status hawk_batch_time(hawk_batch* B, int32_t reps, double* median_ms) {
  if (!B || !B->ctx || reps < 1 || !median_ms) return HAWK_E_ARG;
  hawk_ctx* ctx = B->ctx;
  hawk_status st = hawk_batch_run(B);  // warm-up
  if (st) return st;
  std::vector<double> t;
  for (int32_t i = 0; i < reps; ++i) {
    (void)hipEventRecord(ctx->ev0, ctx->stream);
    st = hawk_batch_run(B);
    if (st) return st;
    (void)hipEventRecord(ctx->ev1, ctx->stream);
    hipError_t e = hipEventSynchronize(ctx->ev1);
    if (e != hipSuccess) return berr(B, HAWK_E_DEVICE, hipGetErrorString(e));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    t.push_back(ms);
  }
  int err = 0;
  if (hipMemcpy(&err, B->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return berr(B, HAWK_E_DEVICE, "flags");
  for (const auto& o : B->own) {
    int e1 = 0;
    if (hipMemcpy(&e1, o.holder.d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
      return berr(B, HAWK_E_DEVICE, "flags");
    err |= e1;
  }
  if (err & HK_ERR_DUPKEY) return berr(B, HAWK_E_DUPKEY, "a build pipeline of the batch inserted a key twice");
  if (err & (HK_ERR_CAPACITY | HK_ERR_CUCKOO)) return berr(B, HAWK_E_CAPACITY, "batch hash table overflow");
  if (err) return berr(B, HAWK_E_TIMEOUT, "a projection look-back wait of the batch gave up");
  std::sort(t.begin(), t.end());
  *median_ms = t[t.size() / 2];
  return HAWK_OK;
}

extern "C" hawk_status hawk_batch_autotune(hawk_batch* B, int32_t reps, hawk_batch_opts* best, double* best_ms) {
  if (!B || !B->ctx || reps < 1) return HAWK_E_ARG;
  const int tiles[] = {14, 15, 16, 17, 18};
  const int wgs[] = {1, 2, 4, 8};
  hawk_batch_opts bo = B->opts;
  double bt = 1e300;
  for (int order = 0; order < 2; ++order)
    for (int tl : tiles)
      for (int w : wgs) {
        hawk_batch_opts o{tl, w, order, B->opts.separate};
        hawk_status st = setup_schedule(B, o);
        if (st) return st;
        double ms = 0;
        st = hawk_batch_time(B, reps, &ms);
        if (st) return st;
        if (ms < bt) {
          bt = ms;
          bo = o;
        }
      }
  hawk_status st = setup_schedule(B, bo);
  if (st) return st;
  if (best) *best = bo;
  if (best_ms) *best_ms = bt;
  return HAWK_OK;
}

extern "C" hawk_status hawk_batch_result(hawk_batch* B, int32_t i, hawk_result** out) {
  if (!B || !B->ctx || !out || i < 0 || i >= static_cast<int32_t>(B->qs.size())) return HAWK_E_ARG;
  const HkBatchQuery& Q = B->hq[i];
  hawk_result* r = new hawk_result();
  r->ctx = B->ctx;
  r->batch = B;
  r->kind = B->qs[i]->kind;
  r->d_count = Q.count;
  r->d_err = B->d_err;
  const hawk_batch::Own* own = nullptr;
  for (const auto& o : B->own)
    if (o.q == i) own = &o;
  if (own) {
    r->d_count = own->holder.d_count;
    r->d_err = own->holder.d_err;
    r->cols = own->holder.cols;
  } else if (Q.kind == HK_BQ_PROJECT) {
    for (int c = 0; c < Q.plan.nproj; ++c) r->cols.push_back({HAWK_RES_I64, Q.out.col[c]});
  } else {
    for (int g = 0; g < Q.plan.ngroup; ++g) r->cols.push_back({HAWK_RES_I64, Q.res.gcol[g]});
    for (int a = 0; a < Q.plan.naggs; ++a) r->cols.push_back({B->qs[i]->res_kinds[a], Q.res.acol[a]});
    r->cols.push_back({HAWK_RES_I64, Q.res.count});
  }
  B->ctx->results.insert(r);
  B->views.insert(r);
  *out = r;  // a view: freeing it releases nothing of the batch
  return HAWK_OK;
}

extern "C" hawk_status hawk_batch_opts_get(const hawk_batch* B, hawk_batch_opts* out) {
  if (!B || !out) return HAWK_E_ARG;
  *out = B->opts;
  return HAWK_OK;
}
