// C ABI of the pipeline-variant library: contexts, table registry, pipeline
// program validation and lowering (Section 3.1), variant space (Section 9.2),
// the per-strategy dispatcher that sequences the kernels of a variant
// (Section 3.4: one interpreter per execution strategy routes the
// operations into one or more kernels), results and timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hawk.h"
#include "hawk_internal.h"
#include "hawk_launch.h"
#include "hawk_plan.h"

namespace {

const uint32_t kMults[7] = {1, 8, 64, 256, 1024, 16384, 65536};  // Section 9.2
const uint32_t kWgs[7] = {16, 32, 64, 128, 256, 512, 1024};       // Section 9.2
const int64_t kSpillLds = 64512;    // LDS bytes of a local table plus its spill histogram (two workgroups per CU)
const int64_t kCuLds = 163840;      // LDS bytes of a CU, and of a spill region at most
const int64_t kLdsBudget = 64512;  // LDS bytes of a local table (64 KB with the static words: two workgroups per CU)
const int kMaxAttempts = 12;

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint32_t ceil_log2(uint64_t x) {
  uint32_t l = 0;
  while ((1ull << l) < x) ++l;
  return l;
}

int dtype_bytes(int32_t t) { return t == HAWK_I8 ? 1 : t == HAWK_I32 ? 4 : 8; }

}  // namespace

// ------------------------------------------------------------------ device memory pool
void* DevicePool::get(size_t bytes) {
  if (bytes < 256) bytes = 256;
  bytes = (bytes + 255) & ~static_cast<size_t>(255);
  int best = -1;
  for (size_t i = 0; i < blocks.size(); ++i) {
    const Block& b = blocks[i];
    if (b.used || b.bytes < bytes || b.bytes > 2 * bytes + (1u << 20)) continue;
    if (best < 0 || b.bytes < blocks[best].bytes) best = static_cast<int>(i);
  }
  if (best >= 0) {
    blocks[best].used = true;
    return blocks[best].p;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    // release idle blocks and try once more
    for (auto it = blocks.begin(); it != blocks.end();) {
      if (!it->used) {
        (void)hipFree(it->p);
        it = blocks.erase(it);
      } else {
        ++it;
      }
    }
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  blocks.push_back({p, bytes, true});
  return p;
}

void DevicePool::put(void* p) {
  if (!p) return;
  for (auto& b : blocks)
    if (b.p == p) b.used = false;
}

void DevicePool::release_all() {
  for (auto& b : blocks) (void)hipFree(b.p);
  blocks.clear();
}

// ------------------------------------------------------------------ errors
hawk_status set_error(hawk_ctx* ctx, hawk_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return st;
}

static hawk_status hip_error(hawk_ctx* ctx, hipError_t e, const char* where) {
  std::string msg = std::string(where) + ": " + hipGetErrorString(e);
  if (!ctx->jit_cache.last_error.empty()) {
    msg += " (" + ctx->jit_cache.last_error + ")";
    ctx->jit_cache.last_error.clear();
  }
  return set_error(ctx, HAWK_E_DEVICE, msg);
}

// ------------------------------------------------------------------ kernel profiling
static hipEvent_t prof_event(hawk_ctx* ctx) {
  if (!ctx->prof_free.empty()) {
    hipEvent_t e = ctx->prof_free.back();
    ctx->prof_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ProfScope::ProfScope(hawk_ctx* c, const char* name) : ctx(c), idx(static_cast<size_t>(-1)) {
  if (!ctx || !ctx->prof_on) return;  // null: a launch that is not profiled
  ProfRec r{name, prof_event(ctx), prof_event(ctx)};
  if (!r.a || !r.b) return;
  (void)hipEventRecord(r.a, ctx->stream);
  ctx->prof.push_back(r);
  idx = ctx->prof.size() - 1;
}

ProfScope::~ProfScope() {
  if (idx != static_cast<size_t>(-1)) (void)hipEventRecord(ctx->prof[idx].b, ctx->stream);
}

static void prof_clear(hawk_ctx* ctx) {
  for (auto& r : ctx->prof) {
    ctx->prof_free.push_back(r.a);
    ctx->prof_free.push_back(r.b);
  }
  ctx->prof.clear();
}

extern "C" hawk_status hawk_profile_enable(hawk_ctx* ctx, int32_t on) {
  if (!ctx) return HAWK_E_ARG;
  if (ctx->device < 0) return set_error(ctx, HAWK_E_DEVICE, "planning context cannot execute");
  (void)hipStreamSynchronize(ctx->stream);
  prof_clear(ctx);
  ctx->prof_on = on != 0;
  return HAWK_OK;
}

extern "C" hawk_status hawk_profile_read(hawk_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches) {
  if (!ctx || !kernel || !total_ms || !launches) return HAWK_E_ARG;
  if (ctx->device < 0) return set_error(ctx, HAWK_E_DEVICE, "planning context cannot execute");
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return set_error(ctx, HAWK_E_DEVICE, hipGetErrorString(e));
  double t = 0;
  int64_t n = 0;
  for (auto& r : ctx->prof) {
    if (r.name != kernel) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return set_error(ctx, HAWK_E_DEVICE, "event timing");
    t += ms;
    ++n;
  }
  *total_ms = t;
  *launches = n;
  return HAWK_OK;
}

// ------------------------------------------------------------------ scratch of the non-allocating execution
// hawk_execute_noalloc places every device buffer of an execution except the
// caller's result columns in this array, one per device, held until the
// process ends. In host code its name denotes a host-side stand-in, not device
// memory: kernels and copies get the address that hipGetSymbolAddress returns
// with the device current, looked up once per device by hawk_ctx_create.
static __device__ __align__(256) unsigned char scratch[HAWK_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;  // device -> its scratch array

// with `device` current
static hipError_t scratch_lookup(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr.count(device)) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

static void* scratch_of(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  return it == g_scratch_ptr.end() ? nullptr : it->second;
}

// ------------------------------------------------------------------ context
extern "C" hawk_status hawk_ctx_create(int32_t device, void* hip_stream, hawk_ctx** out) {
  if (!out) return HAWK_E_ARG;
  *out = nullptr;
  if (device == -1) {
    // planning context: plans, variant spaces and features without a device
    hawk_ctx* c = new hawk_ctx();
    c->device = -1;
    c->num_cus = 256;
    c->lds_bytes = 160 * 1024;
    c->seed = 0x48415748ull;
    *out = c;
    return HAWK_OK;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HAWK_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return HAWK_E_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return HAWK_E_DEVICE;
  hawk_ctx* c = new hawk_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->num_cus = prop.multiProcessorCount;
  c->lds_bytes = static_cast<int64_t>(prop.sharedMemPerBlock);
  c->seed = 0x48415748ull;  // fixed: results never depend on it, timings stay reproducible
  // staging for plan uploads of up to 8 build pipelines, and the flags read
  // back by the non-allocating execution; the device's scratch address
  c->stage_bytes = sizeof(HkPlan) + 8 * sizeof(HkBuild);
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
      hipMalloc(&c->dummy, 256) != hipSuccess || hipMemset(c->dummy, 0, 256) != hipSuccess ||
      hipHostMalloc(&c->h_stage, c->stage_bytes, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c->h_flags), 16, hipHostMallocDefault) != hipSuccess ||
      scratch_lookup(device) != hipSuccess) {
    if (c->dummy) (void)hipFree(c->dummy);
    if (c->h_stage) (void)hipHostFree(c->h_stage);
    if (c->h_flags) (void)hipHostFree(c->h_flags);
    delete c;
    return HAWK_E_DEVICE;
  }
  *out = c;
  return HAWK_OK;
}

extern "C" void hawk_ctx_destroy(hawk_ctx* ctx) {
  if (!ctx) return;
  if (ctx->device >= 0) {
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
  }
  for (hawk_query* q : ctx->queries) {
    query_release_device(q);
    q->ctx = nullptr;
  }
  for (hawk_result* r : ctx->results) {
    r->owned.clear();  // the pool below returns their blocks
    r->ctx = nullptr;
  }
  for (hawk_model* m : ctx->models) model_release_device(m);
  for (hawk_batch* b : ctx->batches) batch_release_device(b);
  if (ctx->device < 0) {
    delete ctx;
    return;
  }
  ctx->pool.release_all();
  ctx->jit_cache.release();
  prof_clear(ctx);
  for (hipEvent_t e : ctx->prof_free) (void)hipEventDestroy(e);
  (void)hipEventDestroy(ctx->ev0);
  (void)hipEventDestroy(ctx->ev1);
  (void)hipFree(ctx->dummy);
  (void)hipHostFree(ctx->h_stage);
  (void)hipHostFree(ctx->h_flags);
  delete ctx;
}

extern "C" const char* hawk_last_error(const hawk_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" hawk_status hawk_ctx_set_variant_dims(hawk_ctx* ctx, uint32_t dims) {
  if (!ctx) return HAWK_E_ARG;
  if (dims & ~static_cast<uint32_t>(HAWK_DIM_ROBIN_HOOD | HAWK_DIM_UNROLL | HAWK_DIM_SIMD_FILTER))
    return set_error(ctx, HAWK_E_ARG, "unknown variant dimension");
  ctx->variant_dims = dims;
  return HAWK_OK;
}

extern "C" hawk_status hawk_ctx_set_jit(hawk_ctx* ctx, int32_t on) {
  if (!ctx) return HAWK_E_ARG;
  if (ctx->device < 0 && on) return set_error(ctx, HAWK_E_DEVICE, "planning context cannot execute");
  ctx->jit = on != 0;
  return HAWK_OK;
}

extern "C" hawk_status hawk_jit_stats(const hawk_ctx* ctx, int64_t* kernels, double* compile_ms) {
  if (!ctx) return HAWK_E_ARG;
  if (kernels) *kernels = ctx->jit_cache.compiled;
  if (compile_ms) *compile_ms = ctx->jit_cache.compile_ms;
  return HAWK_OK;
}

extern "C" hawk_status hawk_device_info(const hawk_ctx* ctx, int32_t* num_cus, int64_t* lds_bytes) {
  if (!ctx) return HAWK_E_ARG;
  if (num_cus) *num_cus = ctx->num_cus;
  if (lds_bytes) *lds_bytes = ctx->lds_bytes;
  return HAWK_OK;
}

// ------------------------------------------------------------------ tables
extern "C" hawk_status hawk_table_register(hawk_ctx* ctx, const char* name, int64_t nrows, const hawk_column* cols,
                                           int32_t ncols, int32_t* table_id) {
  if (!ctx) return HAWK_E_ARG;
  if (!name || !table_id || ncols <= 0 || (ncols > 0 && !cols)) return set_error(ctx, HAWK_E_ARG, "null argument");
  if (nrows < 0 || nrows >= (int64_t(1) << 32)) return set_error(ctx, HAWK_E_ARG, "nrows must be in [0, 2^32)");
  for (const auto& t : ctx->tables)
    if (t.live && t.name == name) return set_error(ctx, HAWK_E_ARG, std::string("duplicate table ") + name);
  TableReg t;
  t.name = name;
  t.nrows = nrows;
  t.live = true;
  for (int32_t i = 0; i < ncols; ++i) {
    if (!cols[i].name) return set_error(ctx, HAWK_E_ARG, "column without name");
    if (cols[i].dtype != HAWK_I8 && cols[i].dtype != HAWK_I32 && cols[i].dtype != HAWK_I64)
      return set_error(ctx, HAWK_E_ARG, std::string("bad dtype of column ") + cols[i].name);
    if (!cols[i].dev_ptr && nrows > 0) return set_error(ctx, HAWK_E_ARG, std::string("null column ") + cols[i].name);
    const uintptr_t esize = cols[i].dtype == HAWK_I64 ? 8 : (cols[i].dtype == HAWK_I32 ? 4 : 1);
    if (reinterpret_cast<uintptr_t>(cols[i].dev_ptr) % esize != 0)
      return set_error(ctx, HAWK_E_ARG, std::string("column not aligned to its element size: ") + cols[i].name);
    for (const auto& c : t.cols)
      if (c.name == cols[i].name) return set_error(ctx, HAWK_E_ARG, std::string("duplicate column ") + cols[i].name);
    t.cols.push_back({cols[i].name, cols[i].dtype, cols[i].scale, cols[i].dev_ptr});
  }
  ctx->tables.push_back(t);
  *table_id = static_cast<int32_t>(ctx->tables.size() - 1);
  return HAWK_OK;
}

extern "C" hawk_status hawk_table_unregister(hawk_ctx* ctx, int32_t table_id) {
  if (!ctx) return HAWK_E_ARG;
  if (table_id < 0 || table_id >= static_cast<int32_t>(ctx->tables.size()) || !ctx->tables[table_id].live)
    return set_error(ctx, HAWK_E_NOTFOUND, "unknown table id");
  ctx->tables[table_id].live = false;
  ctx->tables[table_id].cols.clear();
  return HAWK_OK;
}

// ------------------------------------------------------------------ query compilation
namespace {

struct Lowering {
  hawk_ctx* ctx;
  const TableReg* table = nullptr;
  const TableReg* inner = nullptr;  // the CROSS_JOIN table (its columns load with side 2)
  HkPlan P;
  int nreg = 0;
  // attribute name -> register; columns are loaded on first use
  std::map<std::string, int> reg_of;
  std::map<std::string, int> dtype_of;  // element type of an attribute (columns, payloads)

  Lowering(hawk_ctx* c) : ctx(c) { std::memset(&P, 0, sizeof(P)); }

  int find_col(const std::string& nm) const {
    for (size_t i = 0; i < table->cols.size(); ++i)
      if (table->cols[i].name == nm) return static_cast<int>(i);
    return -1;
  }
  int find_inner(const std::string& nm) const {
    if (!inner) return -1;
    for (size_t i = 0; i < inner->cols.size(); ++i)
      if (inner->cols[i].name == nm) return static_cast<int>(i);
    return -1;
  }
  // register holding `nm`, loading the column in `phase` (0 = A, 1 = B, 2 = C) if needed
  hawk_status attr(const char* nm, int phase, int* reg) {
    if (!nm) return set_error(ctx, HAWK_E_ARG, "missing attribute name");
    auto it = reg_of.find(nm);
    if (it != reg_of.end()) {
      *reg = it->second;
      // a filter column read again after the filters
      for (int c = 0; c < P.ncolA && phase > 0; ++c)
        if (P.colA[c].reg == it->second) P.liveA |= 1u << c;
      return HAWK_OK;
    }
    int c = find_col(nm);
    const int ci = find_inner(nm);
    if (c >= 0 && ci >= 0)
      return set_error(ctx, HAWK_E_PLAN, std::string("attribute in both tables of the CROSS_JOIN: ") + nm);
    if (c < 0 && ci < 0) return set_error(ctx, HAWK_E_NOTFOUND, std::string("unknown attribute ") + nm);
    if (nreg >= HK_NREG) return set_error(ctx, HAWK_E_PLAN, "more than 16 live attributes");
    const ColReg& cr = c >= 0 ? table->cols[c] : inner->cols[ci];
    HkCol col = {cr.ptr, static_cast<int16_t>(cr.dtype), static_cast<int16_t>(!inner ? 0 : (c >= 0 ? 1 : 2)), nreg};
    if (phase == 0) {
      if (P.ncolA >= HK_MAX_COLS_A) return set_error(ctx, HAWK_E_PLAN, "too many filter columns");
      P.colA[P.ncolA++] = col;  // read by its filter; live once read again (above)
    } else if (phase == 1) {
      if (P.ncolB >= HK_MAX_COLS_B) return set_error(ctx, HAWK_E_PLAN, "too many join-key columns");
      P.colB[P.ncolB++] = col;
    } else {
      if (P.ncolC >= HK_MAX_COLS_C) return set_error(ctx, HAWK_E_PLAN, "too many value columns");
      P.colC[P.ncolC++] = col;
    }
    reg_of[nm] = nreg;
    dtype_of[nm] = cr.dtype;
    *reg = nreg++;
    return HAWK_OK;
  }
  hawk_status new_attr(const char* nm, int dtype, int* reg) {
    if (!nm) return set_error(ctx, HAWK_E_ARG, "missing attribute name");
    if (reg_of.count(nm) || find_col(nm) >= 0 || find_inner(nm) >= 0)
      return set_error(ctx, HAWK_E_PLAN, std::string("attribute defined twice: ") + nm);
    if (nreg >= HK_NREG) return set_error(ctx, HAWK_E_PLAN, "more than 16 live attributes");
    reg_of[nm] = nreg;
    dtype_of[nm] = dtype;
    *reg = nreg++;
    return HAWK_OK;
  }
};

hawk_status lower_loop(hawk_ctx* ctx, const hawk_pipeline& p, Lowering& L) {
  if (p.nops < 2 || !p.ops || p.ops[0].kind != HAWK_LOOP)
    return set_error(ctx, HAWK_E_PLAN, "a pipeline starts with LOOP and has a sink");
  int32_t t = p.ops[0].table;
  if (t < 0 || t >= static_cast<int32_t>(ctx->tables.size()) || !ctx->tables[t].live)
    return set_error(ctx, HAWK_E_NOTFOUND, "LOOP over an unknown table");
  L.table = &ctx->tables[t];
  L.P.nrows = L.table->nrows;
  return HAWK_OK;
}

hawk_status lower_filter(hawk_ctx* ctx, const hawk_op& op, Lowering& L) {
  if (L.P.nfilters >= HK_MAX_FILTERS) return set_error(ctx, HAWK_E_PLAN, "too many filters");
  // a column of the looped table, or (after a CROSS_JOIN) of the second table
  if (L.find_col(op.a ? op.a : "") < 0 && L.find_inner(op.a ? op.a : "") < 0)
    return set_error(ctx, HAWK_E_NOTFOUND, std::string("FILTER on unknown column ") + (op.a ? op.a : "(null)"));
  int reg;
  hawk_status st = L.attr(op.a, 0, &reg);
  if (st) return st;
  HkFilter& f = L.P.filters[L.P.nfilters++];
  f.lo = op.lo;
  f.hi = op.hi;
  f.reg = reg;
  return HAWK_OK;
}

}  // namespace

// The pipeline programs in the notation of Table 2, one pipeline per line.
static std::string program_text(const hawk_ctx* ctx, const hawk_pipeline* pipes, int32_t npipes) {
  auto nm = [](const char* s) { return std::string(s ? s : "?"); };
  auto bound = [](int64_t v) {
    return v == INT64_MIN ? std::string("min") : v == INT64_MAX ? std::string("max") : std::to_string(v);
  };
  auto table = [&](int32_t t) {
    return t >= 0 && t < static_cast<int32_t>(ctx->tables.size()) ? ctx->tables[t].name : std::to_string(t);
  };
  static const char* fns[] = {"?", "COUNT", "SUM", "MIN", "MAX", "AVG"};
  static const char* ops[] = {"?", "+", "-", "*"};
  std::string out;
  for (int32_t pi = 0; pi < npipes; ++pi) {
    std::string line;
    for (int32_t k = 0; k < pipes[pi].nops; ++k) {
      const hawk_op& o = pipes[pi].ops[k];
      std::string t;
      switch (o.kind) {
        case HAWK_LOOP: t = "LOOP(" + table(o.table) + ")"; break;
        case HAWK_FILTER: t = "FILTER(" + nm(o.a) + " in [" + bound(o.lo) + ", " + bound(o.hi) + "])"; break;
        case HAWK_HASH_PUT: t = "HASH_PUT(" + nm(o.a) + " -> " + nm(o.b) + "; ht " + std::to_string(o.ht) + ")"; break;
        case HAWK_HASH_PROBE: t = "HASH_PROBE(" + nm(o.a) + " -> " + nm(o.b) + "; ht " + std::to_string(o.ht) + ")"; break;
        case HAWK_CROSS_JOIN: t = "CROSS_JOIN(" + table(o.table) + ")"; break;
        case HAWK_ARITHMETIC:
          t = "ARITHMETIC(" + nm(o.a) + " = " + (o.b ? nm(o.b) : std::to_string(o.lo)) + " " +
              ops[o.arith_op >= 1 && o.arith_op <= 3 ? o.arith_op : 0] + " " + (o.c ? nm(o.c) : std::to_string(o.hi)) + ")";
          break;
        case HAWK_PROJECT:
        case HAWK_AGGREGATE:
        case HAWK_HASH_AGGREGATE: {
          t = o.kind == HAWK_PROJECT ? "PROJECT(" : o.kind == HAWK_AGGREGATE ? "AGGREGATE(" : "HASH_AGGREGATE(";
          for (int32_t j = 0; j < o.nattrs && o.attrs; ++j) t += (j ? ", " : "") + nm(o.attrs[j]);
          if (o.kind != HAWK_PROJECT) {
            if (o.nattrs > 0) t += "; ";
            for (int32_t j = 0; j < o.naggs && o.aggs; ++j) {
              const hawk_agg& a = o.aggs[j];
              t += std::string(j ? ", " : "") + fns[a.fn >= 1 && a.fn <= 5 ? a.fn : 0];
              if (a.fn != HAWK_COUNT) t += "(" + nm(a.attr) + ")";
            }
          }
          t += ")";
          break;
        }
        default: t = "?";
      }
      line += (k ? " " : "") + t;
    }
    out += line + "\n";
  }
  return out;
}

extern "C" hawk_status hawk_query_create(hawk_ctx* ctx, const hawk_pipeline* pipes, int32_t npipes, hawk_query** out) {
  if (!ctx) return HAWK_E_ARG;
  if (!pipes || npipes < 1 || !out) return set_error(ctx, HAWK_E_ARG, "null argument");
  *out = nullptr;
  hawk_query* q = new hawk_query();
  q->ctx = ctx;
  std::map<int32_t, int> build_of_ht;  // ht id -> build index
  // build pipelines: LOOP, FILTER*, HASH_PUT
  for (int32_t pi = 0; pi + 1 < npipes; ++pi) {
    const hawk_pipeline& p = pipes[pi];
    Lowering L(ctx);
    hawk_status st = lower_loop(ctx, p, L);
    if (st) { delete q; return st; }
    QueryBuild B;
    bool put = false;
    for (int32_t k = 1; k < p.nops; ++k) {
      const hawk_op& op = p.ops[k];
      if (op.kind == HAWK_FILTER && !put) {
        st = lower_filter(ctx, op, L);
      } else if (op.kind == HAWK_HASH_PUT && !put) {
        int kc = L.find_col(op.a ? op.a : ""), pc = L.find_col(op.b ? op.b : "");
        if (kc < 0 || pc < 0) st = set_error(ctx, HAWK_E_NOTFOUND, "HASH_PUT on unknown key or payload column");
        else if (L.table->cols[kc].dtype == HAWK_I64 || L.table->cols[pc].dtype == HAWK_I64)
          st = set_error(ctx, HAWK_E_TYPE, "HASH_PUT key and payload must be at most 32-bit");
        else if (build_of_ht.count(op.ht)) st = set_error(ctx, HAWK_E_PLAN, "hash table built twice");
        else {
          B.key = {L.table->cols[kc].ptr, static_cast<int16_t>(L.table->cols[kc].dtype), 0, 0};
          B.payload = {L.table->cols[pc].ptr, static_cast<int16_t>(L.table->cols[pc].dtype), 0, 0};
          B.payload_dtype = L.table->cols[pc].dtype;
          B.ht_id = op.ht;
          put = true;
        }
      } else if (op.kind == HAWK_PROJECT && put) {
        // a build pipeline may materialise attributes (Table 2); payloads are what probes see
      } else {
        st = set_error(ctx, HAWK_E_PLAN, "build pipelines are LOOP, FILTER*, HASH_PUT");
      }
      if (st) { delete q; return st; }
    }
    if (!put) { delete q; return set_error(ctx, HAWK_E_PLAN, "non-final pipeline without HASH_PUT"); }
    B.plan = L.P;
    B.nrows = L.P.nrows;
    build_of_ht[B.ht_id] = static_cast<int>(q->builds.size());
    q->builds.push_back(B);
  }
  // main pipeline
  const hawk_pipeline& p = pipes[npipes - 1];
  Lowering L(ctx);
  hawk_status st = lower_loop(ctx, p, L);
  if (st) { delete q; return st; }
  int stage = 0;  // 0 filters, 1 probes, 2 arithmetic, 3 sink seen
  for (int32_t k = 1; k < p.nops && !st; ++k) {
    const hawk_op& op = p.ops[k];
    if (stage == 3) { st = set_error(ctx, HAWK_E_PLAN, "operations after the sink"); break; }
    switch (op.kind) {
      case HAWK_FILTER:
        if (stage > 0) st = set_error(ctx, HAWK_E_PLAN, "FILTER after HASH_PROBE/ARITHMETIC is not supported");
        else st = lower_filter(ctx, op, L);
        break;
      case HAWK_CROSS_JOIN: {
        // the pipeline now loops over the product of its table and this one
        if (stage > 0 || L.inner) { st = set_error(ctx, HAWK_E_PLAN, "one CROSS_JOIN, before probes and arithmetic"); break; }
        if (op.table < 0 || op.table >= static_cast<int32_t>(ctx->tables.size()) || !ctx->tables[op.table].live) {
          st = set_error(ctx, HAWK_E_NOTFOUND, "CROSS_JOIN of an unknown table");
          break;
        }
        const TableReg* u = &ctx->tables[op.table];
        for (const auto& c : u->cols)
          if (L.find_col(c.name) >= 0) { st = set_error(ctx, HAWK_E_PLAN, "column name in both tables of the CROSS_JOIN: " + c.name); break; }
        if (st) break;
        const uint64_t prod = static_cast<uint64_t>(L.P.nrows) * static_cast<uint64_t>(u->nrows);
        if (prod >= (uint64_t(1) << 32)) { st = set_error(ctx, HAWK_E_PLAN, "CROSS_JOIN of 2^32 or more pairs"); break; }
        L.inner = u;
        // columns loaded so far (filters on the looped table) address its rows
        for (int c = 0; c < L.P.ncolA; ++c) L.P.colA[c].side = 1;
        L.P.xinner = static_cast<uint32_t>(u->nrows);
        L.P.xmagic = u->nrows > 1 ? ~0ull / static_cast<uint64_t>(u->nrows) + 1 : 0;
        L.P.nrows = static_cast<int64_t>(prod);
        break;
      }
      case HAWK_HASH_PROBE: {
        if (stage > 1) { st = set_error(ctx, HAWK_E_PLAN, "HASH_PROBE after ARITHMETIC"); break; }
        stage = 1;
        auto it = build_of_ht.find(op.ht);
        if (it == build_of_ht.end()) { st = set_error(ctx, HAWK_E_PLAN, "HASH_PROBE of a table no pipeline builds"); break; }
        if (L.P.nprobes >= HK_MAX_PROBES) { st = set_error(ctx, HAWK_E_PLAN, "too many probes"); break; }
        // the key is a column of the looped table or (after a CROSS_JOIN) of the second one
        const int c = L.find_col(op.a ? op.a : ""), ci = L.find_inner(op.a ? op.a : "");
        if (c < 0 && ci < 0) { st = set_error(ctx, HAWK_E_NOTFOUND, "HASH_PROBE on unknown column"); break; }
        if ((c >= 0 ? L.table->cols[c] : L.inner->cols[ci]).dtype == HAWK_I64) {
          st = set_error(ctx, HAWK_E_TYPE, "join keys are at most 32-bit");
          break;
        }
        int fk, pay;
        if ((st = L.attr(op.a, 1, &fk))) break;
        if ((st = L.new_attr(op.b, q->builds[it->second].payload_dtype, &pay))) break;
        HkProbe& pr = L.P.probes[L.P.nprobes++];
        std::memset(&pr, 0, sizeof(pr));
        pr.fk_reg = fk;
        pr.pay_reg = pay;
        q->probe_build.push_back(it->second);
        break;
      }
      case HAWK_ARITHMETIC: {
        stage = 2;
        if (L.P.narith >= HK_MAX_ARITH) { st = set_error(ctx, HAWK_E_PLAN, "too many arithmetic steps"); break; }
        if (op.arith_op < HAWK_ADD || op.arith_op > HAWK_MUL) { st = set_error(ctx, HAWK_E_ARG, "bad arithmetic operator"); break; }
        HkArith A;
        std::memset(&A, 0, sizeof(A));
        A.op = static_cast<int8_t>(op.arith_op);
        int r;
        if (op.b) { if ((st = L.attr(op.b, 2, &r))) break; A.x = static_cast<int8_t>(r); }
        else { A.xc = 1; A.cx = op.lo; }
        if (op.c) { if ((st = L.attr(op.c, 2, &r))) break; A.y = static_cast<int8_t>(r); }
        else { A.yc = 1; A.cy = op.hi; }
        if ((st = L.new_attr(op.a, HAWK_I64, &r))) break;
        A.dst = static_cast<int8_t>(r);
        L.P.arith[L.P.narith++] = A;
        break;
      }
      case HAWK_PROJECT: {
        stage = 3;
        q->kind = 1;
        if (op.nattrs < 1 || op.nattrs > HK_MAX_PROJ || !op.attrs) { st = set_error(ctx, HAWK_E_PLAN, "PROJECT takes 1..4 attributes"); break; }
        for (int32_t j = 0; j < op.nattrs && !st; ++j) {
          int r;
          if (!(st = L.attr(op.attrs[j], 2, &r))) L.P.preg[L.P.nproj++] = r;
        }
        break;
      }
      case HAWK_AGGREGATE:
      case HAWK_HASH_AGGREGATE: {
        stage = 3;
        q->kind = 2;
        const bool grouped = op.kind == HAWK_HASH_AGGREGATE;
        if (grouped && (op.nattrs < 1 || op.nattrs > 2 || !op.attrs)) { st = set_error(ctx, HAWK_E_PLAN, "HASH_AGGREGATE groups by 1 or 2 attributes"); break; }
        if (op.naggs < 1 || op.naggs > HK_MAX_AGGS || !op.aggs) { st = set_error(ctx, HAWK_E_PLAN, "1..8 aggregates"); break; }
        if (grouped) {
          for (int32_t j = 0; j < op.nattrs && !st; ++j) {
            int r;
            if ((st = L.attr(op.attrs[j], 2, &r))) break;
            int dt = L.dtype_of[op.attrs[j]];
            if (dt == HAWK_I64) { st = set_error(ctx, HAWK_E_TYPE, "group attributes are at most 32-bit"); break; }
            L.P.greg[L.P.ngroup++] = r;
          }
          if (st) break;
        }
        int word = 2;  // [key, count, aggregates...]
        for (int32_t j = 0; j < op.naggs && !st; ++j) {
          const hawk_agg& ag = op.aggs[j];
          if (ag.fn < HAWK_COUNT || ag.fn > HAWK_AVG) { st = set_error(ctx, HAWK_E_ARG, "bad aggregate function"); break; }
          HkAgg A;
          std::memset(&A, 0, sizeof(A));
          A.fn = static_cast<int8_t>(ag.fn);
          A.wide = static_cast<int8_t>(ag.fn == HAWK_SUM && ag.wide ? 1 : 0);
          if (ag.fn != HAWK_COUNT) {
            int r;
            if ((st = L.attr(ag.attr, 2, &r))) break;
            A.reg = static_cast<int8_t>(r);
            // AVG divides the exact sum. A 64-bit accumulator is exact for
            // 8- and 32-bit attributes (fewer than 2^32 rows of |x| <= 2^31
            // sum to less than 2^63 in magnitude); 64-bit attributes, and
            // arithmetic results, take the 128-bit one.
            if (ag.fn == HAWK_AVG && (ag.wide || L.dtype_of[ag.attr] == HAWK_I64)) A.wide = 1;
            A.word = word;
            word += A.wide ? 2 : 1;
          }
          L.P.aggs[L.P.naggs++] = A;
          q->res_kinds.push_back(ag.fn == HAWK_AVG ? HAWK_RES_F64 : (ag.fn == HAWK_SUM && A.wide ? HAWK_RES_I128 : HAWK_RES_I64));
        }
        L.P.slot_words = word;
        q->groups_hint = grouped ? std::max<int64_t>(1, op.groups_hint) : 1;
        break;
      }
      default:
        st = set_error(ctx, HAWK_E_PLAN, "unsupported operation in the main pipeline");
    }
  }
  if (!st && stage != 3) st = set_error(ctx, HAWK_E_PLAN, "main pipeline has no PROJECT/AGGREGATE/HASH_AGGREGATE");
  if (st) { delete q; return st; }
  // unused column slots read the context's zero block, so kernels may load
  // every slot of their shape class without a per-slot condition
  for (int c = L.P.ncolA; c < HK_MAX_COLS_A; ++c) L.P.colA[c] = HkCol{ctx->dummy, HK_T_I64, 0, 0};
  for (int c = L.P.ncolB; c < HK_MAX_COLS_B; ++c) L.P.colB[c] = HkCol{ctx->dummy, HK_T_I64, 0, 0};
  for (int c = L.P.ncolC; c < HK_MAX_COLS_C; ++c) L.P.colC[c] = HkCol{ctx->dummy, HK_T_I64, 0, 0};
  q->main = L.P;
  q->has_table = L.P.nprobes > 0 || L.P.ngroup > 0;
  q->program = program_text(ctx, pipes, npipes);
  ctx->queries.insert(q);
  *out = q;
  return HAWK_OK;
}

void query_release_device(hawk_query* q) {
  if (!q->ctx || q->ctx->device < 0) return;
  if (q->d_plans || !q->jt.empty()) (void)hipStreamSynchronize(q->ctx->stream);
  for (auto& t : q->jt) {
    if (t.slots) (void)hipFree(t.slots);
    if (t.side) (void)hipFree(t.side);
  }
  q->jt.clear();
  if (q->d_plans) (void)hipFree(q->d_plans);
  if (q->h_stage) (void)hipHostFree(q->h_stage);
  if (q->up_ev) (void)hipEventDestroy(q->up_ev);
  q->d_plans = q->h_stage = nullptr;
  q->up_ev = nullptr;
}

extern "C" void hawk_query_free(hawk_query* q) {
  if (!q) return;
  if (q->ctx) {
    query_release_device(q);
    q->ctx->queries.erase(q);
  }
  delete q;
}

extern "C" hawk_status hawk_query_program(const hawk_query* q, char* buf, int64_t cap, int64_t* len) {
  if (!q || !len) return HAWK_E_ARG;
  *len = static_cast<int64_t>(q->program.size());
  if (!buf) return HAWK_OK;
  if (cap < *len + 1) return set_error(q->ctx, HAWK_E_ARG, "buffer too small");
  std::memcpy(buf, q->program.c_str(), q->program.size() + 1);
  return HAWK_OK;
}

extern "C" hawk_status hawk_query_kind(const hawk_query* q, int32_t* kind) {
  if (!q || !kind) return HAWK_E_ARG;
  *kind = q->kind;
  return HAWK_OK;
}

// ------------------------------------------------------------------ variant space
static void push_variant(std::vector<hawk_variant>& v, int ps, int mem, int pred, int ht, int hash, int as, uint32_t tm,
                         uint32_t wg) {
  hawk_variant x;
  std::memset(&x, 0, sizeof(x));
  x.proj_strategy = static_cast<uint8_t>(ps);
  x.mem = static_cast<uint8_t>(mem);
  x.pred = static_cast<uint8_t>(pred);
  x.ht = static_cast<uint8_t>(ht);
  x.hash = static_cast<uint8_t>(hash);
  x.agg_strategy = static_cast<uint8_t>(as);
  x.thread_mult = tm;
  x.wg_size = wg;
  v.push_back(x);
}

// The variant space of Section 9.2 (32 projection / 896 aggregation
// variants), with the context's extra dimensions multiplied in where they
// apply: robin-hood join tables for pipelines with probes, loop unrolling
// (1, 2, 4 rows per iteration) for multi-pass coalesced projections and the
// SIMD filter for those without probes.
std::vector<hawk_variant> variant_space(const hawk_query* q) {
  std::vector<hawk_variant> v;
  const uint32_t dims = q->ctx ? q->ctx->variant_dims : 0;
  const int nht = !q->has_table ? 1 : (dims & HAWK_DIM_ROBIN_HOOD) && q->main.nprobes > 0 ? 3 : 2;
  const int nhs = q->has_table ? 2 : 1;
  // the SIMD filter: filters without probes or a cross join, over 16-byte aligned columns
  bool simd_ok = q->main.nprobes == 0 && q->main.nfilters > 0 && q->main.xinner == 0;
  for (int c = 0; c < q->main.ncolA && simd_ok; ++c)
    simd_ok = reinterpret_cast<uintptr_t>(q->main.colA[c].ptr) % 16 == 0;
  if (q->kind == 1) {
    for (int ps = 0; ps < 2; ++ps)
      for (int mem = 0; mem < 2; ++mem)
        for (int pred = 0; pred < 2; ++pred)
          for (int ht = 0; ht < nht; ++ht)
            for (int hs = 0; hs < nhs; ++hs) {
              if (ps == HAWK_SINGLE_PASS) {
                push_variant(v, ps, mem, pred, ht, hs, 0, 1, 64);
                continue;
              }
              for (uint32_t tm : kMults) {
                push_variant(v, ps, mem, pred, ht, hs, 0, tm, 256);
                if (mem != HAWK_COALESCED) continue;
                if (dims & HAWK_DIM_UNROLL)
                  for (uint8_t u : {uint8_t(2), uint8_t(1)}) {
                    push_variant(v, ps, mem, pred, ht, hs, 0, tm, 256);
                    v.back().unroll = u;
                  }
                if ((dims & HAWK_DIM_SIMD_FILTER) && simd_ok) {
                  push_variant(v, ps, mem, pred, ht, hs, 0, tm, 256);
                  v.back().filter_mode = HAWK_FILTER_SIMD;
                }
              }
            }
  } else {
    for (int as = 0; as < 2; ++as)
      for (int mem = 0; mem < 2; ++mem)
        for (int pred = 0; pred < 2; ++pred)
          for (int ht = 0; ht < nht; ++ht)
            for (int hs = 0; hs < nhs; ++hs) {
              if (as == HAWK_LOCAL) {
                for (uint32_t tm : kMults)
                  for (uint32_t wg : kWgs) push_variant(v, 1, mem, pred, ht, hs, as, tm, wg);
              } else {
                for (uint32_t wg : kWgs) push_variant(v, 1, mem, pred, ht, hs, as, 1, wg);
              }
            }
  }
  return v;
}

extern "C" hawk_status hawk_variant_space(const hawk_query* q, hawk_variant* out, int64_t cap, int64_t* n) {
  if (!q || !n) return HAWK_E_ARG;
  std::vector<hawk_variant> v = variant_space(q);
  *n = static_cast<int64_t>(v.size());
  if (out) {
    if (cap < *n) return HAWK_E_ARG;
    std::copy(v.begin(), v.end(), out);
  }
  return HAWK_OK;
}

extern "C" hawk_status hawk_variant_format(const hawk_variant* v, char* buf, int32_t cap) {
  if (!v || !buf || cap <= 0) return HAWK_E_ARG;
  int k = std::snprintf(buf, static_cast<size_t>(cap), "strat=%s,mem=%s,pred=%s,ht=%s,hash=%s,agg=%s,tm=%u,wg=%u%s%s%s",
                        v->proj_strategy ? "mp" : "sp", v->mem ? "coal" : "seq", v->pred ? "pred" : "br",
                        v->ht == HAWK_ROBIN_HOOD ? "robin" : v->ht ? "cuckoo" : "lin", v->hash ? "mulshift" : "murmur",
                        v->agg_strategy ? "global" : "local", v->thread_mult, v->wg_size,
                        v->unroll == 1 ? ",unroll=1" : v->unroll == 2 ? ",unroll=2" : "",
                        v->filter_mode ? ",filter=simd" : "", "");
  return k < cap ? HAWK_OK : HAWK_E_ARG;
}

// ------------------------------------------------------------------ results
static void result_release(hawk_result* r) {
  if (!r) return;
  for (void* p : r->owned) r->ctx->pool.put(p);
  r->owned.clear();
}

extern "C" void hawk_result_free(hawk_result* r) {
  if (!r) return;
  if (r->batch) batch_forget_view(r->batch, r);
  if (r->ctx) {
    result_release(r);
    r->ctx->results.erase(r);
  }
  delete r;
}

static hawk_status result_check(hawk_result* r) {
  if (r->checked) return r->status;
  hawk_ctx* ctx = r->ctx;
  if (!ctx) return HAWK_E_ARG;  // its context was destroyed
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_error(ctx, e, "stream synchronize");
  int err = 0;
  uint64_t n = 0;
  if ((e = hipMemcpy(&err, r->d_err, sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess) return hip_error(ctx, e, "read flags");
  if ((e = hipMemcpy(&n, r->d_count, sizeof(uint64_t), hipMemcpyDeviceToHost)) != hipSuccess) return hip_error(ctx, e, "read count");
  r->checked = true;
  r->err_bits = err;
  r->nrows = static_cast<int64_t>(n);
  if (err & HK_ERR_DUPKEY) r->status = set_error(ctx, HAWK_E_DUPKEY, "a build pipeline inserted a key twice");
  else if (err & (HK_ERR_CAPACITY | HK_ERR_CUCKOO)) r->status = set_error(ctx, HAWK_E_CAPACITY, "hash table overflow");
  else if (err & HK_ERR_TIMEOUT)
    r->status = set_error(ctx, HAWK_E_TIMEOUT, "a bounded wait for another workgroup's result gave up");
  else r->status = HAWK_OK;
  return r->status;
}

extern "C" hawk_status hawk_result_info(hawk_result* r, int64_t* nrows, int32_t* ncols) {
  if (!r || !r->ctx) return HAWK_E_ARG;  // orphaned: its memory is gone
  hawk_status st = result_check(r);
  if (st) return st;
  if (nrows) *nrows = r->nrows;
  if (ncols) *ncols = static_cast<int32_t>(r->cols.size());
  return HAWK_OK;
}

extern "C" hawk_status hawk_result_column(hawk_result* r, int32_t col, int32_t* elem_kind, const void** dev_ptr) {
  if (!r) return HAWK_E_ARG;
  if (!r->ctx) return HAWK_E_ARG;
  if (col < 0 || col >= static_cast<int32_t>(r->cols.size())) return set_error(r->ctx, HAWK_E_ARG, "bad column index");
  if (elem_kind) *elem_kind = r->cols[col].kind;
  if (dev_ptr) *dev_ptr = r->cols[col].ptr;
  return HAWK_OK;
}

extern "C" hawk_status hawk_result_copy_column(hawk_result* r, int32_t col, void* host_dst, int64_t cap_bytes) {
  if (!r || !r->ctx) return HAWK_E_ARG;
  hawk_status st = result_check(r);
  if (st) return st;
  if (col < 0 || col >= static_cast<int32_t>(r->cols.size())) return set_error(r->ctx, HAWK_E_ARG, "bad column index");
  const int64_t bytes = r->nrows * (r->cols[col].kind == HAWK_RES_I128 ? 16 : 8);
  if (bytes > cap_bytes || (!host_dst && bytes > 0)) return set_error(r->ctx, HAWK_E_ARG, "destination too small");
  if (bytes == 0) return HAWK_OK;
  hipError_t e = hipMemcpy(host_dst, r->cols[col].ptr, static_cast<size_t>(bytes), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_error(r->ctx, e, "copy column");
  return HAWK_OK;
}

// ------------------------------------------------------------------ execution
hawk_status agg_config(hawk_ctx* ctx, const HkPlan& P, const HkAggTable& T, int64_t groups_hint,
                       const hawk_variant* v, int64_t groups, AggConfig& c) {
  const int W = P.slot_words;
  c = AggConfig{};
  c.groups = groups;
  c.llog2 = 0;
  c.reps = 1;
  c.rlog2 = T.log2cap;
  // A grid of at most one workgroup per CU lets each take the CU's LDS (less
  // 1 KB for static words); a wider grid keeps two workgroups per CU. The
  // table then leaves 8 KB for a spill histogram.
  const bool whole_cu = groups <= ctx->num_cus;
  int64_t wg_lds = whole_cu ? std::min<int64_t>(ctx->lds_bytes, kCuLds) - 1024 : kSpillLds;
  int64_t table_budget = whole_cu ? wg_lds - 8192 : kLdsBudget;
  // The run-time kernel copies small join tables into LDS, in plan order
  // while they take at most half of a workgroup's LDS (all of it without a
  // local table): their lookups then wait on LDS alone, not behind the
  // column loads in flight. The local table takes what remains.
  if (ctx->jit && v->ht == HAWK_LINEAR_PROBING && P.xinner == 0) {
    int64_t budget = v->agg_strategy == HAWK_LOCAL ? wg_lds / 2 : wg_lds;
    if (v->agg_strategy != HAWK_LOCAL) {
      // without a local table the copies alone bound the resident
      // workgroups: they leave room for at least 16 waves per CU
      const int64_t waves = std::max<int64_t>(1, (v->wg_size + 63) / 64);
      const int64_t wgs = (16 + waves - 1) / waves;
      budget = std::min<int64_t>(budget, kCuLds / wgs - 1024);
    }
    for (int i = 0; i < P.nprobes; ++i) {
      const int64_t tb = int64_t(8) << P.probes[i].t.log2cap;
      if (P.probes[i].t.log2cap >= 4 && c.stage_bytes + tb <= budget) {
        c.stage[c.nstage++] = i;
        c.stage_bytes += tb;
      }
    }
    wg_lds -= c.stage_bytes;
    table_budget = std::min(table_budget, wg_lds - (whole_cu ? 8192 : 0));
  }
  if (v->agg_strategy == HAWK_LOCAL) {
    // four slots per expected group: few keys then share a group of four
    // slots (a lookup reads one group)
    const uint32_t want = std::max<uint32_t>(4, ceil_log2(static_cast<uint64_t>(groups_hint) * 4));
    uint32_t fit = 0;
    while ((int64_t(2) << fit) * W * 8 <= table_budget) ++fit;
    c.llog2 = std::min(want, fit);
    if ((int64_t(1) << c.llog2) * W * 8 > ctx->lds_bytes)
      return set_error(ctx, HAWK_E_INFEASIBLE, "local table does not fit in LDS");
    // copies of the aggregate words while they fit the budget (up to one per
    // lane); a table of few groups gives up slots (down to two per group, at
    // least 16) for more copies: its rows' atomics then meet on fewer
    // addresses
    auto copies = [&](uint32_t l2) {
      const int64_t lc = int64_t(1) << l2;
      int32_t r = 1;
      while (r < 64 && (lc + (W - 1) * (2 * r) * lc) * 8 <= table_budget) r *= 2;
      return r;
    };
    c.reps = copies(c.llog2);
    const uint32_t floor2 = std::max<uint32_t>(4, ceil_log2(static_cast<uint64_t>(groups_hint) * 2));
    while (c.reps < 64 && c.llog2 > floor2 && copies(c.llog2 - 1) > c.reps) {
      --c.llog2;
      c.reps = copies(c.llog2);
    }
  }
  // Overflow partitioning: with the local strategy and linear probing, when
  // the LDS table cannot hold every group, rows that miss it are spilled and
  // aggregated per table region by the region's owner workgroup instead of
  // each updating the table with device-scope atomics. A region (aggregated
  // in LDS by its owner) takes at most 64 KB; the partition histogram of a
  // workgroup sits beside its LDS table.
  // Regions as large as one workgroup's LDS allows (up to 160 KB: fewer,
  // larger regions spread the spilled rows over fewer buckets), but at least
  // 256 of them (so that the regions' owners fill the device) while they
  // keep 64 slots.
  const int64_t region_lds = std::min<int64_t>(ctx->lds_bytes, kCuLds);
  uint32_t rlog2 = 0;
  while ((int64_t(2) << rlog2) * W * 8 <= region_lds) ++rlog2;
  if (T.log2cap >= 14 && T.log2cap - 8 < rlog2) rlog2 = T.log2cap - 8;
  else if (T.log2cap < 14 && rlog2 > 6) rlog2 = 6;
  const int64_t nparts = T.log2cap > rlog2 ? int64_t(1) << (T.log2cap - rlog2) : 1;
  const int64_t LC = int64_t(1) << c.llog2;
  const int64_t table_bytes = (LC + (W - 1) * c.reps * LC) * 8;
  c.spill = v->agg_strategy == HAWK_LOCAL && v->ht == HAWK_LINEAR_PROBING && T.log2cap > c.llog2 && rlog2 >= 6 &&
            nparts >= 2 && table_bytes + nparts * 4 <= wg_lds && nparts * groups <= (int64_t(1) << 26) &&
            P.nrows > 0 && ctx->lds_bytes >= kSpillLds;
  if (c.spill) {
    c.rlog2 = rlog2;
    c.nparts = nparts;
    HkSpill& sp = c.sp;
    sp.nparts = static_cast<int32_t>(nparts);
    for (int a = 0; a < P.naggs; ++a) {
      if (P.aggs[a].fn == HK_COUNT) continue;
      bool seen = false;
      for (int j = 0; j < sp.ncols; ++j) seen = seen || sp.reg[j] == P.aggs[a].reg;
      if (!seen) sp.reg[sp.ncols++] = P.aggs[a].reg;
    }
    sp.ew = 1 + sp.ncols;
    // one 32-bit group attribute and one input value: 12-byte entries
    sp.e12 = sp.ew == 2 && P.ngroup == 1 ? 1 : 0;
    sp.nrows = P.nrows;
    sp.bs = static_cast<int32_t>(v->wg_size);
    sp.coal = v->mem == HAWK_COALESCED ? 1 : 0;
    sp.fcap = static_cast<int32_t>(int64_t(1) << c.llog2);
    // Merge entries pay where a grid of at most one workgroup per CU holds
    // large LDS tables: few workgroups, many distinct slots each. A wider
    // grid merges its (smaller, more alike) tables with device-scope atomics.
    sp.merge = groups <= ctx->num_cus ? 1 : 0;
    // a 64K-bit admission filter on grids of at most one workgroup per CU
    // (elsewhere its LDS would cost resident workgroups)
    sp.door_log2 = whole_cu && table_bytes + nparts * 4 + 8192 <= wg_lds ? 16 : 0;
  }
  return HAWK_OK;
}

hipError_t agg_kernel_launch(hawk_ctx* ctx, hipStream_t st, const hawk_variant* v, const HkPlan& P,
                             const HkAggTable& T, const AggConfig& c, const uint64_t* ident, int32_t W, int* err,
                             const HkSpill* sp, bool allow_jit) {
  const int32_t wg = static_cast<int32_t>(v->wg_size);
  if (allow_jit && ctx->jit && v->ht == HAWK_LINEAR_PROBING && P.xinner == 0) {
    HkIdent id = {};
    for (int i = 0; i < W; ++i) id.w[i] = ident[i];
    id.nw = W;
    std::string msg;
    const hipError_t e = jit_agg_launch(ctx->jit_cache, msg, st, P, T, v->mem, v->pred, v->hash, v->agg_strategy,
                                        c.groups, wg, c.llog2, id, err, sp, c.reps, c.stage, c.nstage);
    if (e != hipSuccess && !msg.empty()) ctx->jit_cache.last_error = msg;
    if (e != hipErrorNotSupported) return e;
  }
  return hk_agg(st, P, T, v->mem, v->pred, v->ht, v->hash, v->agg_strategy, c.groups, wg, c.llog2, ident, W, err,
                sp, c.reps);
}

// the AGGREGATE kernel without grouping of variant v: compiled at run time
// for the plan when the context does so (linear probing), else the
// precompiled one
hipError_t scalar_kernel_launch(hawk_ctx* ctx, hipStream_t st, const hawk_variant* v, const HkPlan& P,
                                const HkAggTable& T, int64_t groups, int32_t wg, const uint64_t* ident, int32_t W,
                                int* err, bool allow_jit) {
  if (allow_jit && ctx->jit && v->ht == HAWK_LINEAR_PROBING && P.xinner == 0) {
    HkIdent id = {};
    for (int i = 0; i < W; ++i) id.w[i] = ident[i];
    id.nw = W;
    std::string msg;
    const hipError_t e = jit_scalar_launch(ctx->jit_cache, msg, st, P, T, v->mem, v->pred, v->hash, v->agg_strategy,
                                           groups, wg, id);
    if (e != hipSuccess && !msg.empty()) ctx->jit_cache.last_error = msg;
    if (e != hipErrorNotSupported) return e;
  }
  return hk_scalar_agg(st, P, T, v->mem, v->pred, v->ht, v->hash, v->agg_strategy, groups, wg, ident, W, err);
}

namespace {

// Where the device buffers of one execution come from.
//  POOL: the context's pool; result columns are owned by the result.
//  ARENA: consecutive 256-byte aligned pieces of one region [base, base+cap),
//   handed out in call order. A pass with base == nullptr enqueues nothing and
//   only measures the bytes (and result rows) that a pass over a real region
//   then uses at the same offsets. Result columns are the caller's (`outs`,
//   `out_rows` elements each) or, without `outs`, pieces of the region too.
enum ExecMem { EXEC_POOL = 0, EXEC_ARENA = 1 };

struct Exec {
  hawk_ctx* ctx;
  const hawk_query* q;
  const hawk_variant* v;
  hawk_result* res;
  std::vector<void*> scratch;
  int attempt;
  hipStream_t st;
  int mem = EXEC_POOL;
  char* base = nullptr;
  size_t cap = 0, used = 0;
  bool launch = true;          // enqueue kernels and fills (false: addresses and sizes only)
  bool upload = true;          // copy the plans to the device in this pass
  bool allow_jit = true;       // kernels compiled at run time may be used (and compiled)
  void* const* outs = nullptr; // caller's result columns (ARENA)
  int32_t nouts = 0;
  int64_t out_rows = 0;
  int32_t next_out = 0;
  int64_t need_rows = 0;       // largest result column requested so far
  const void* d_plans = nullptr;  // device copy of [main plan][builds] read by build and finalize kernels
  bool robin = false;            // the variant's join tables use robin-hood linear probing

  bool sizing() const { return mem == EXEC_ARENA && !base; }
  void* get(size_t bytes, bool owned) {
    if (mem == EXEC_ARENA) {
      bytes = bytes < 256 ? 256 : (bytes + 255) & ~static_cast<size_t>(255);
      const size_t at = used;
      used += bytes;
      if (!base) return reinterpret_cast<void*>(static_cast<uintptr_t>(256));  // sizing: never dereferenced
      return used <= cap ? base + at : nullptr;
    }
    void* p = ctx->pool.get(bytes);
    if (p) (owned ? res->owned : scratch).push_back(p);
    return p;
  }
  // profiled launches: pool executions on the context stream only
  hawk_ctx* prof() const { return mem == EXEC_POOL && launch ? ctx : nullptr; }
  ~Exec() {
    for (void* p : scratch) ctx->pool.put(p);
  }
};

#define HIPCHK(call, where)                          \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hip_error(X.ctx, e_, where); \
  } while (0)
#define ALLOC(ptr, type, bytes, owned)                                        \
  do {                                                                        \
    ptr = static_cast<type>(X.get((bytes), (owned)));                         \
    if (!ptr) return set_error(X.ctx, HAWK_E_OOM, "device allocation failed"); \
  } while (0)
// a kernel launch or device fill of the execution (skipped by address-only passes)
#define LAUNCH(call, where)                                      \
  do {                                                           \
    if (X.launch) {                                              \
      hipError_t e_ = (call);                                    \
      if (e_ != hipSuccess) return hip_error(X.ctx, e_, where);  \
    }                                                            \
  } while (0)

// One result column of `rows` elements of `kind`: a pool block the result
// owns, a piece of the arena, or the caller's next column (which must hold
// `rows` elements).
hawk_status result_col(Exec& X, int32_t kind, int64_t rows, void** ptr) {
  const size_t esize = kind == HAWK_RES_I128 ? 16 : 8;
  X.need_rows = std::max(X.need_rows, rows);
  if (X.mem == EXEC_ARENA && X.outs) {
    if (X.next_out >= X.nouts) return set_error(X.ctx, HAWK_E_ARG, "fewer result columns than the query produces");
    if (rows > X.out_rows)
      return set_error(X.ctx, HAWK_E_ARG, "result columns hold " + std::to_string(X.out_rows) + " rows, the query needs " +
                                              std::to_string(rows));
    *ptr = X.outs[X.next_out++];
    if (!*ptr) return set_error(X.ctx, HAWK_E_ARG, "null result column");
    return HAWK_OK;
  }
  *ptr = X.get(static_cast<size_t>(rows) * esize, true);
  if (!*ptr) return set_error(X.ctx, HAWK_E_OOM, "device allocation failed");
  return HAWK_OK;
}

HkHash make_hash(hawk_ctx* ctx, const hawk_variant* v, int attempt) {
  uint64_t s = ctx->seed + 0x1000193ull * static_cast<uint64_t>(attempt);
  HkHash h;
  for (int i = 0; i < HK_CUCKOO_D; ++i) {
    uint64_t a = splitmix(s);
    h.a[i] = v->hash == HAWK_MULTIPLY_SHIFT ? (a | 1ull) : a;
  }
  return h;
}

// Uploads the main plan and the build plans to the query's device buffer when
// they differ from the last upload (new hash seeds or tables); the copy is
// ordered on the context stream from a pinned staging buffer.
hawk_status upload_plans(Exec& X, const HkPlan& main, const std::vector<HkBuild>& builds) {
  hawk_query* q = const_cast<hawk_query*>(X.q);
  const size_t bytes = sizeof(HkPlan) + builds.size() * sizeof(HkBuild);
  if (X.mem == EXEC_ARENA) {
    // the plans take a piece of the arena and are copied from the context's
    // pinned staging buffer (the caller synchronises before it is reused)
    void* d;
    ALLOC(d, void*, bytes, false);
    X.d_plans = d;
    if (X.sizing() || !X.upload) return HAWK_OK;
    if (bytes > X.ctx->stage_bytes) return set_error(X.ctx, HAWK_E_PLAN, "too many build pipelines for the staging buffer");
    std::memcpy(X.ctx->h_stage, &main, sizeof(HkPlan));
    if (!builds.empty())
      std::memcpy(static_cast<char*>(X.ctx->h_stage) + sizeof(HkPlan), builds.data(), builds.size() * sizeof(HkBuild));
    HIPCHK(hipMemcpyAsync(d, X.ctx->h_stage, bytes, hipMemcpyHostToDevice, X.st), "plan upload");
    return HAWK_OK;
  }
  X.d_plans = q->d_plans;
  std::vector<char> now(bytes);
  std::memcpy(now.data(), &main, sizeof(HkPlan));
  if (!builds.empty()) std::memcpy(now.data() + sizeof(HkPlan), builds.data(), builds.size() * sizeof(HkBuild));
  if (!q->d_plans) {
    if (hipMalloc(&q->d_plans, bytes) != hipSuccess) return set_error(X.ctx, HAWK_E_OOM, "plan buffer");
    if (hipHostMalloc(&q->h_stage, bytes, hipHostMallocDefault) != hipSuccess)
      return set_error(X.ctx, HAWK_E_OOM, "plan staging buffer");
    if (hipEventCreateWithFlags(&q->up_ev, hipEventDisableTiming) != hipSuccess)
      return set_error(X.ctx, HAWK_E_DEVICE, "plan upload event");
    X.d_plans = q->d_plans;
  }
  if (now == q->uploaded) return HAWK_OK;
  if (q->up_pending) HIPCHK(hipEventSynchronize(q->up_ev), "plan upload wait");
  std::memcpy(q->h_stage, now.data(), bytes);
  HIPCHK(hipMemcpyAsync(q->d_plans, q->h_stage, bytes, hipMemcpyHostToDevice, X.st), "plan upload");
  HIPCHK(hipEventRecord(q->up_ev, X.st), "plan upload event");
  q->up_pending = true;
  q->uploaded.swap(now);
  return HAWK_OK;
}

const HkPlan* dev_main(const Exec& X) { return static_cast<const HkPlan*>(X.d_plans); }
const HkBuild* dev_build(const Exec& X, size_t i) {
  return reinterpret_cast<const HkBuild*>(static_cast<const char*>(X.d_plans) + sizeof(HkPlan)) + i;
}

// slots of a join table (log2): at least twice the build's rows, doubled per retry
uint32_t join_log2cap(int64_t build_rows, int grow) {
  return std::max<uint32_t>(4, ceil_log2(static_cast<uint64_t>(std::max<int64_t>(1, build_rows)) * 2)) + grow;
}

hawk_status run_builds(Exec& X, HkPlan& main, const HkHash& h, int grow) {
  hawk_query* q = const_cast<hawk_query*>(X.q);
  if (q->jt.size() != q->builds.size()) q->jt.resize(q->builds.size());
  std::vector<HkBuild> bs;
  for (size_t i = 0; i < q->builds.size(); ++i) {
    const QueryBuild& B = q->builds[i];
    JoinTableMem& m = q->jt[i];
    const uint32_t l2 = join_log2cap(B.nrows, grow);
    if (l2 > 31) return set_error(X.ctx, HAWK_E_CAPACITY, "join table beyond 2^31 slots");
    uint64_t *slots = m.slots, *side = m.side;
    if (X.mem == EXEC_ARENA) {
      ALLOC(slots, uint64_t*, (static_cast<size_t>(1) << l2) * 8, false);
      ALLOC(side, uint64_t*, 16, false);
    } else if (!m.slots || m.log2cap != l2) {
      if (m.slots) {
        HIPCHK(hipStreamSynchronize(X.st), "synchronize");
        (void)hipFree(m.slots);
        (void)hipFree(m.side);
        m.slots = m.side = nullptr;
      }
      if (hipMalloc(&m.slots, (static_cast<size_t>(1) << l2) * 8) != hipSuccess || hipMalloc(&m.side, 16) != hipSuccess)
        return set_error(X.ctx, HAWK_E_OOM, "join table allocation failed");
      m.log2cap = l2;
      slots = m.slots;
      side = m.side;
    }
    HkBuild b;
    std::memset(&b, 0, sizeof(b));
    b.p = B.plan;
    b.p.hash = h;
    b.key = B.key;
    b.payload = B.payload;
    b.t.slots = slots;
    b.t.side = side;
    b.t.robin = X.robin ? 1 : 0;
    b.t.log2cap = l2;
    bs.push_back(b);
  }
  for (int i = 0; i < main.nprobes; ++i) main.probes[i].t = bs[q->probe_build[i]].t;
  hawk_status st = upload_plans(X, main, bs);
  if (st) return st;
  // every table and its side words cleared in one launch, then every build
  // in one launch (the builds are independent)
  HkFills f{};
  int32_t k = 0;
  for (size_t i = 0; i < bs.size(); ++i) {
    f.p[k] = bs[i].t.slots;
    f.n[k] = int64_t(1) << bs[i].t.log2cap;
    f.v[k++] = HK_EMPTY;
    f.p[k] = bs[i].t.side;
    f.n[k] = 2;
    f.v[k++] = 0;
    if (k + 2 > HK_MAX_FILLS || i + 1 == bs.size()) {
      LAUNCH(hk_fill_multi(X.st, f, k), "fill join tables");
      k = 0;
    }
  }
  if (!bs.empty()) {
    ProfScope ps(X.prof(), "k_build");
    LAUNCH(hk_build(X.st, bs.data(), dev_build(X, 0), static_cast<int32_t>(bs.size()), X.v->ht, X.v->hash,
                    X.res->d_err), "build");
  }
  return HAWK_OK;
}

hawk_status run_projection(Exec& X, const HkPlan& P) {
  hawk_ctx* ctx = X.ctx;
  const hawk_variant* v = X.v;
  const int64_t n = P.nrows;
  hawk_result* res = X.res;
  int64_t* out[HK_MAX_PROJ] = {};
  for (int c = 0; c < P.nproj; ++c) {
    void* p;
    hawk_status rst = result_col(X, HAWK_RES_I64, n + 1, &p);  // + the dump slot of predicated writes
    if (rst) return rst;
    out[c] = static_cast<int64_t*>(p);
    res->cols.push_back({HAWK_RES_I64, out[c]});
  }
  if (v->proj_strategy == HAWK_MULTI_PASS) {
    const int64_t T = static_cast<int64_t>(v->thread_mult) * ctx->num_cus;  // threads (Section 9.2)
    const int64_t threads = std::max<int64_t>(256, (T + 255) / 256 * 256);
    const int64_t nblk = (n + 63) / 64;
    uint64_t* masks;
    ALLOC(masks, uint64_t*, static_cast<size_t>(nblk) * 8, false);
    int64_t m, nact = 0;
    if (v->mem == HAWK_COALESCED) {
      m = nblk;
    } else {
      int64_t chunk = (n + threads - 1) / threads;
      chunk = (chunk + 63) / 64 * 64;
      nact = chunk > 0 ? (n + chunk - 1) / chunk : 0;
      m = nact;
    }
    uint32_t *counts, *offsets, *tmp;
    ALLOC(counts, uint32_t*, static_cast<size_t>(m) * 4, false);
    ALLOC(offsets, uint32_t*, static_cast<size_t>(m) * 4, false);
    ALLOC(tmp, uint32_t*, static_cast<size_t>(hk_scan_tmp_words(m)) * 4, false);
    if (v->filter_mode == HAWK_FILTER_SIMD) {
      // vector loads of 4 rows: a coalesced scan of filter columns without probes, 16-byte aligned
      bool ok = v->mem == HAWK_COALESCED && P.nprobes == 0 && P.nfilters > 0 && P.xinner == 0;
      for (int c = 0; c < P.ncolA && ok; ++c) ok = reinterpret_cast<uintptr_t>(P.colA[c].ptr) % 16 == 0;
      if (!ok) return set_error(ctx, HAWK_E_INFEASIBLE, "the SIMD filter needs a coalesced scan of 16-byte aligned "
                                                        "filter columns without probes");
    }
    // kernels compiled at run time for the plan's structure when the context does so
    const bool jit = X.allow_jit && ctx->jit && P.xinner == 0;
    std::string jmsg;
    auto jit_err = [&](hipError_t e) {
      if (e != hipSuccess && !jmsg.empty()) ctx->jit_cache.last_error = jmsg;
      return e;
    };
    {
      ProfScope ps(X.prof(), "k_mp_filter");
      hipError_t je = hipErrorNotSupported;
      if (jit && X.launch)  // (a sizing pass enqueues nothing)
        je = jit_err(jit_mp_filter_launch(ctx->jit_cache, jmsg, X.st, P, v->filter_mode, v->mem, v->pred, v->ht,
                                          v->hash, v->unroll, threads, masks, counts));
      if (je != hipErrorNotSupported) LAUNCH(je, "filter kernel");
      else
        LAUNCH(hk_mp_filter(X.st, P, v->mem, v->pred, v->ht, v->hash, threads, masks, counts, v->unroll,
                            v->filter_mode),
               "filter kernel");
    }
    {
      ProfScope ps(X.prof(), "k_scan");
      LAUNCH(hk_scan(X.st, counts, offsets, m, tmp, res->d_count, res->d_err), "prefix sum");
    }
    {
      ProfScope ps(X.prof(), "k_mp_project");
      hipError_t je = hipErrorNotSupported;
      if (jit && X.launch) {  // (a sizing pass enqueues nothing)
        HkOut O = {};
        for (int c = 0; c < P.nproj; ++c) O.col[c] = out[c];
        O.dump = n;
        je = jit_err(jit_mp_project_launch(ctx->jit_cache, jmsg, X.st, P, v->mem, v->pred, v->ht, v->hash, threads,
                                           masks, offsets, res->d_count, nact, O));
      }
      if (je != hipErrorNotSupported) LAUNCH(je, "projection kernel");
      else
        LAUNCH(hk_mp_project(X.st, P, v->mem, v->pred, v->ht, v->hash, threads, masks, offsets, res->d_count, nact,
                             out, n), "projection kernel");
    }
  } else {
    const int64_t inst = ctx->num_cus;  // one pipeline instance per compute unit
    int64_t chunk = (n + inst - 1) / inst;
    chunk = (chunk + 63) / 64 * 64;
    int64_t region, nregions;
    if (v->mem == HAWK_COALESCED) {
      region = chunk + 1;
      nregions = inst;
    } else {
      region = chunk / 64 + 1;
      nregions = inst * 64;
    }
    int64_t* tmp[HK_MAX_PROJ] = {};
    for (int c = 0; c < P.nproj; ++c) ALLOC(tmp[c], int64_t*, static_cast<size_t>(region * nregions) * 8, false);
    uint32_t *counts, *offsets, *stmp;
    ALLOC(counts, uint32_t*, static_cast<size_t>(nregions) * 4, false);
    ALLOC(offsets, uint32_t*, static_cast<size_t>(nregions) * 4, false);
    ALLOC(stmp, uint32_t*, static_cast<size_t>(hk_scan_tmp_words(nregions)) * 4, false);
    {
      ProfScope ps(X.prof(), "k_sp");
      LAUNCH(hk_sp(X.st, P, v->mem, v->pred, v->ht, v->hash, inst, tmp, region, counts), "single-pass kernel");
    }
    {
      ProfScope ps(X.prof(), "k_scan");
      LAUNCH(hk_scan(X.st, counts, offsets, nregions, stmp, res->d_count, res->d_err), "prefix sum");
    }
    {
      ProfScope ps(X.prof(), "k_sp_concat");
      LAUNCH(hk_sp_concat(X.st, tmp, P.nproj, region, nregions, counts, offsets, out), "concatenation");
    }
  }
  return HAWK_OK;
}

void identity_words(const HkPlan& P, bool grouped, uint64_t* w) {
  w[0] = grouped ? HK_EMPTY : 0ull;
  w[1] = 0;
  for (int a = 0; a < P.naggs; ++a) {
    const HkAgg& A = P.aggs[a];
    if (A.fn == HK_COUNT) continue;
    w[A.word] = A.fn == HK_MIN ? static_cast<uint64_t>(INT64_MAX) : A.fn == HK_MAX ? static_cast<uint64_t>(INT64_MIN) : 0ull;
    if (A.wide) w[A.word + 1] = 0;
  }
}

hawk_status run_aggregation(Exec& X, const HkPlan& P, int grow) {
  hawk_ctx* ctx = X.ctx;
  const hawk_variant* v = X.v;
  hawk_result* res = X.res;
  const bool grouped = P.ngroup > 0;
  const int W = P.slot_words;
  uint64_t ident[2 + 2 * HK_MAX_AGGS] = {};
  identity_words(P, grouped, ident);
  HkAggTable T;
  T.slot_words = W;
  int64_t nslots;
  if (grouped) {
    T.log2cap = std::max<uint32_t>(6, ceil_log2(static_cast<uint64_t>(X.q->groups_hint) * 2)) + grow;
    if (T.log2cap > 31) return set_error(ctx, HAWK_E_CAPACITY, "aggregation table beyond 2^31 slots");
    nslots = (int64_t(1) << T.log2cap) + 1;  // + side slot for the all-ones key
    T.rlog2 = T.log2cap;
  } else {
    T.log2cap = 0;
    T.rlog2 = 0;
    nslots = 1;
  }
  ALLOC(T.words, uint64_t*, static_cast<size_t>(nslots * W) * 8, false);
  const int32_t wg = static_cast<int32_t>(v->wg_size);
  if (wg < 1 || wg > 1024) return set_error(ctx, HAWK_E_ARG, "wg_size must be in [1, 1024]");
  int64_t groups;
  if (v->agg_strategy == HAWK_LOCAL) groups = static_cast<int64_t>(v->thread_mult) * ctx->num_cus;  // N tables
  else groups = static_cast<int64_t>(ctx->num_cus) * std::max(1, 2048 / wg);                      // fill the device
  if (groups < 1 || groups > 0x7FFFFFFF) return set_error(ctx, HAWK_E_ARG, "thread_mult out of range");
  AggConfig cfg{};
  if (grouped) {
    hawk_status cst = agg_config(ctx, P, T, X.q->groups_hint, v, groups, cfg);
    if (cst) return cst;
    T.rlog2 = cfg.rlog2;
  }
  // Spilling, the regions' owners write the groups as result rows and the
  // table's regions are never read: only its side slot (the all-ones key)
  // needs the identity and the final extraction.
  const bool direct = grouped && cfg.spill && cfg.sp.merge;
  HkAggTable Tside = T;
  Tside.words = T.words + (nslots - 1) * W;
  {
    ProfScope ps(X.prof(), "k_init_aggtable");
    LAUNCH(direct ? hk_init_aggtable(X.st, Tside.words, 1, ident, W) : hk_init_aggtable(X.st, T.words, nslots, ident, W),
           "init table");
  }
  // result columns: groups, aggregates, count
  const int64_t cap = nslots;
  int64_t* gcols[2] = {};
  hawk_status rst;
  for (int g = 0; g < P.ngroup; ++g) {
    void* p;
    if ((rst = result_col(X, HAWK_RES_I64, cap, &p))) return rst;
    gcols[g] = static_cast<int64_t*>(p);
    res->cols.push_back({HAWK_RES_I64, gcols[g]});
  }
  void* acols[HK_MAX_AGGS] = {};
  for (int a = 0; a < P.naggs; ++a) {
    const int kind = X.q->res_kinds[a];
    if ((rst = result_col(X, kind, cap, &acols[a]))) return rst;
    res->cols.push_back({kind, acols[a]});
  }
  int64_t* cnt;
  {
    void* p;
    if ((rst = result_col(X, HAWK_RES_I64, cap, &p))) return rst;
    cnt = static_cast<int64_t*>(p);
  }
  res->cols.push_back({HAWK_RES_I64, cnt});
  if (grouped) {
    if (cfg.spill) {
      HkSpill sp = cfg.sp;
      const int64_t m = cfg.nparts * groups;
      uint32_t *offs, *stmp;
      uint64_t *total, *part, *scratch;
      // 12-byte entries: keys, then values from a 16-byte boundary (SpillArr)
      const size_t spill_bytes = static_cast<size_t>(
          sp.e12 ? (P.nrows * 4 + 15) / 16 * 16 + P.nrows * 8 : P.nrows * 8 * sp.ew);
      ALLOC(sp.buf, uint64_t*, spill_bytes, false);
      ALLOC(sp.hist, uint32_t*, static_cast<size_t>(m) * 4, false);
      ALLOC(sp.cnt, uint32_t*, static_cast<size_t>(groups) * 4, false);
      ALLOC(offs, uint32_t*, static_cast<size_t>(m) * 4, false);
      ALLOC(stmp, uint32_t*, static_cast<size_t>(hk_scan_tmp_words(m)) * 4, false);
      ALLOC(total, uint64_t*, 8, false);
      ALLOC(part, uint64_t*, spill_bytes, false);
      scratch = nullptr;
      if (sp.merge) {
        ALLOC(sp.flush, uint64_t*, static_cast<size_t>(groups * sp.fcap * W) * 8, false);
        ALLOC(sp.foffs, uint32_t*, static_cast<size_t>(groups * (cfg.nparts + 1)) * 4, false);
        ALLOC(scratch, uint64_t*, static_cast<size_t>(cfg.nparts) * 32 * 8, false);
      }
      HkResOut O = {};
      for (int g = 0; g < P.ngroup; ++g) O.gcol[g] = gcols[g];
      for (int a = 0; a < P.naggs; ++a) O.acol[a] = acols[a];
      O.count = cnt;
      O.nrows = reinterpret_cast<unsigned long long*>(res->d_count);
      {
        ProfScope ps(X.prof(), "k_agg");
        LAUNCH(agg_kernel_launch(ctx, X.st, v, P, T, cfg, ident, W, res->d_err, &sp, X.allow_jit), "aggregation kernel");
      }
      {
        ProfScope ps(X.prof(), "k_scan");
        LAUNCH(hk_scan(X.st, sp.hist, offs, m, stmp, total, res->d_err), "spill offsets");
      }
      {
        ProfScope ps(X.prof(), "k_spill_scatter");
        LAUNCH(hk_spill(X.st, 0, P, T, v->hash, sp, ident, W, offs, total, groups, part, res->d_err), "spill regrouping");
      }
      {
        ProfScope ps(X.prof(), "k_spill_agg");
        LAUNCH(hk_spill(X.st, 1, P, T, v->hash, sp, ident, W, offs, total, groups, part, res->d_err,
                        direct ? &O : nullptr, scratch),
               "spill aggregation");
      }
    } else {
      ProfScope ps(X.prof(), "k_agg");
      LAUNCH(agg_kernel_launch(ctx, X.st, v, P, T, cfg, ident, W, res->d_err, nullptr, X.allow_jit), "aggregation kernel");
    }
  } else {
    ProfScope ps(X.prof(), "k_scalar_agg");
    LAUNCH(scalar_kernel_launch(ctx, X.st, v, P, T, groups, wg, ident, W, res->d_err, X.allow_jit),
           "aggregation kernel");
  }
  {
    ProfScope ps(X.prof(), "k_finalize");
    LAUNCH(direct ? hk_finalize(X.st, P, dev_main(X), Tside, 1, gcols, acols, cnt, res->d_count, 0)
                  : hk_finalize(X.st, P, dev_main(X), T, nslots, gcols, acols, cnt, res->d_count, grouped ? 0 : 1),
           "finalize");
  }
  return HAWK_OK;
}

// One execution of (X.q, X.v) as set up in X: the flags cleared, the build
// pipelines, then the main pipeline's kernels.
hawk_status run_query(Exec& X, int grow) {
  if (X.v->mem > 1 || X.v->pred > 1 || X.v->ht > 2 || X.v->hash > 1 || X.v->agg_strategy > 1 ||
      X.v->proj_strategy > 1 || X.v->thread_mult < 1 || X.v->unroll > 4 || X.v->filter_mode > 1)
    return set_error(X.ctx, HAWK_E_ARG, "variant value out of range");
  // robin-hood join tables: the kernels of linear probing, the tables marked
  hawk_variant vk = *X.v;
  if (vk.ht == HAWK_ROBIN_HOOD) {
    if (X.q->main.nprobes == 0) return set_error(X.ctx, HAWK_E_INFEASIBLE, "robin hood applies to join tables");
    vk.ht = HAWK_LINEAR_PROBING;
    X.robin = true;
  }
  X.v = &vk;
  const hawk_variant* v = X.v;
  void* flags;
  ALLOC(flags, void*, 16, true);
  X.res->d_count = static_cast<uint64_t*>(flags);
  X.res->d_err = reinterpret_cast<int*>(X.res->d_count + 1);
  LAUNCH(hk_fill_u64(X.st, X.res->d_count, 2, 0), "clear flags");
  HkPlan P = X.q->main;
  P.hash = make_hash(X.ctx, v, X.attempt);
  hawk_status st = run_builds(X, P, P.hash, grow);
  if (!st) st = X.q->kind == 1 ? run_projection(X, P) : run_aggregation(X, P, grow);
  return st;
}

hawk_status execute_once(hawk_ctx* ctx, const hawk_query* q, const hawk_variant* v, int attempt, int grow,
                         hawk_result** out) {
  if (ctx->device < 0) return set_error(ctx, HAWK_E_DEVICE, "planning context cannot execute");
  if (q->ctx != ctx) return set_error(ctx, HAWK_E_ARG, "query of another context");
  hawk_result* res = new hawk_result();
  res->ctx = ctx;
  res->kind = q->kind;
  ctx->results.insert(res);
  Exec X{ctx, q, v, res, {}, attempt, ctx->stream};
  hawk_status st = run_query(X, grow);
  if (st) {
    hawk_result_free(res);
    return st;
  }
  *out = res;
  return HAWK_OK;
}

}  // namespace

static hawk_status prepare_run_time_kernel(hawk_ctx* ctx, const hawk_query* q, const hawk_variant* v);

hawk_status exec_arena(hawk_ctx* ctx, const hawk_query* q, const hawk_variant* v, hipStream_t st, char* base,
                       size_t cap, bool launch, bool upload, hawk_result* holder, size_t* used) {
  if (ctx->device < 0) return set_error(ctx, HAWK_E_DEVICE, "planning context cannot execute");
  if (q->ctx != ctx) return set_error(ctx, HAWK_E_ARG, "query of another context");
  if (upload && base) {
    // a run-time kernel is compiled before any launch of it is recorded
    hawk_status pst = prepare_run_time_kernel(ctx, q, v);
    if (pst) return pst;
  }
  holder->ctx = ctx;
  holder->kind = q->kind;
  holder->cols.clear();
  Exec X{ctx, q, v, holder, {}, 0, st};
  X.mem = EXEC_ARENA;
  X.base = base;
  X.cap = cap;
  X.launch = launch;
  X.upload = upload;
  hawk_status rst = run_query(X, 0);
  if (used) *used = X.used;
  return rst;
}

extern "C" hawk_status hawk_execute_async(hawk_ctx* ctx, const hawk_query* q, const hawk_variant* v, hawk_result** out) {
  if (!ctx) return HAWK_E_ARG;
  if (!q || !v || !out) return set_error(ctx, HAWK_E_ARG, "null argument");
  *out = nullptr;
  return execute_once(ctx, q, v, 0, 0, out);
}

extern "C" hawk_status hawk_execute(hawk_ctx* ctx, const hawk_query* q, const hawk_variant* v, hawk_result** out) {
  if (!ctx) return HAWK_E_ARG;
  if (!q || !v || !out) return set_error(ctx, HAWK_E_ARG, "null argument");
  *out = nullptr;
  int grow = 0;
  for (int attempt = 0; attempt < kMaxAttempts; ++attempt) {
    hawk_result* r = nullptr;
    hawk_status st = execute_once(ctx, q, v, attempt, grow, &r);
    if (st) return st;
    st = result_check(r);
    if (st == HAWK_OK) {
      *out = r;
      return HAWK_OK;
    }
    const int bits = r->err_bits;
    hawk_result_free(r);
    if (st != HAWK_E_CAPACITY) return st;
    // a full linear-probing table doubles; a failed cuckoo chain first gets new
    // hash seeds (the next attempt), then more room
    if (bits & HK_ERR_CAPACITY) grow += 1;
    else if (attempt >= 1) grow += 1;
  }
  return set_error(ctx, HAWK_E_CAPACITY, "hash table overflow after retries");
}

extern "C" hawk_status hawk_execute_noalloc(hawk_ctx* ctx, const hawk_query* q, const hawk_variant* v,
                                            void* const* cols, int32_t ncols, int64_t cap_rows, int64_t* nrows) {
  if (!ctx) return HAWK_E_ARG;
  if (!q || !v || !nrows || (cols && (ncols < 1 || cap_rows < 0))) return set_error(ctx, HAWK_E_ARG, "bad argument");
  if (q->ctx != ctx) return set_error(ctx, HAWK_E_ARG, "query of another context");
  if (cols && ctx->device < 0) return set_error(ctx, HAWK_E_DEVICE, "planning context cannot execute");
  // The result holds the flags and the column list only; it owns nothing.
  hawk_result res;
  res.ctx = ctx;
  res.kind = q->kind;
  // pass 1: scratch bytes and result rows the execution needs (nothing enqueued)
  Exec S{ctx, q, v, &res, {}, 0, ctx->stream};
  S.mem = EXEC_ARENA;
  S.launch = false;
  S.allow_jit = false;
  S.outs = cols;
  S.nouts = ncols;
  S.out_rows = cap_rows;
  hawk_status st = run_query(S, 0);
  if (st) return st;
  if (!cols) {
    *nrows = S.need_rows;
    return HAWK_OK;
  }
  if (S.next_out != ncols)
    return set_error(ctx, HAWK_E_ARG, "the query produces " + std::to_string(S.next_out) + " result columns");
  if (S.used > HAWK_NOALLOC_SCRATCH_BYTES)
    return set_error(ctx, HAWK_E_CAPACITY, "the execution needs " + std::to_string(S.used) +
                                               " bytes of scratch, more than the " +
                                               std::to_string(HAWK_NOALLOC_SCRATCH_BYTES) + " the library holds");
  // pass 2: the same buffers at the same offsets of this device's scratch
  void* base = scratch_of(ctx->device);
  if (!base) return set_error(ctx, HAWK_E_DEVICE, "no scratch address for this device");
  res.cols.clear();
  Exec X{ctx, q, v, &res, {}, 0, ctx->stream};
  X.mem = EXEC_ARENA;
  X.base = static_cast<char*>(base);
  X.cap = HAWK_NOALLOC_SCRATCH_BYTES;
  X.allow_jit = false;
  X.outs = cols;
  X.nouts = ncols;
  X.out_rows = cap_rows;
  st = run_query(X, 0);
  if (st) {
    (void)hipStreamSynchronize(ctx->stream);
    return st;
  }
  hipError_t e = hipMemcpyAsync(ctx->h_flags, res.d_count, 16, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_error(ctx, e, "read flags");
  const int err = static_cast<int>(ctx->h_flags[1] & 0xffffffffu);
  if (err & HK_ERR_DUPKEY) return set_error(ctx, HAWK_E_DUPKEY, "a build pipeline inserted a key twice");
  if (err & (HK_ERR_CAPACITY | HK_ERR_CUCKOO))
    return set_error(ctx, HAWK_E_CAPACITY, "hash table overflow (no retry without allocation; raise the group hint)");
  if (err & HK_ERR_TIMEOUT) return set_error(ctx, HAWK_E_TIMEOUT, "a bounded wait for another workgroup's result gave up");
  *nrows = static_cast<int64_t>(ctx->h_flags[0]);
  return HAWK_OK;
}

// ------------------------------------------------------------------ timing
// Compiles the run-time kernel that executing (q, v) will launch, so that a
// timed run measures the kernels and not the compiler.
static hawk_status prepare_run_time_kernel(hawk_ctx* ctx, const hawk_query* q, const hawk_variant* vin) {
  // robin-hood join tables run the kernels of linear probing
  hawk_variant vv = *vin;
  if (vv.ht == HAWK_ROBIN_HOOD) vv.ht = HAWK_LINEAR_PROBING;
  const hawk_variant* v = &vv;
  if (ctx->jit && q->kind == 1 && v->proj_strategy == HAWK_MULTI_PASS && q->main.xinner == 0 && v->ht <= 1) {
    // the multi-pass projection's filter and projection kernels
    const int ht = v->ht;
    std::string msg;
    const int which = v->filter_mode ? JIT_MP_FILTER_SIMD : JIT_MP_FILTER;
    // a refused kernel (hipErrorNotSupported) leaves the execution to the precompiled one
    for (const hipError_t e : {jit_proj_prepare(ctx->jit_cache, msg, q->main, which, v->mem, v->pred, ht, v->hash,
                                                v->unroll),
                               jit_proj_prepare(ctx->jit_cache, msg, q->main, JIT_MP_PROJECT, v->mem, v->pred, ht,
                                                v->hash, 0)})
      if (e != hipSuccess && e != hipErrorNotSupported)
        return set_error(ctx, HAWK_E_DEVICE, "run-time compilation: " + msg);
    return HAWK_OK;
  }
  if (!ctx->jit || q->kind == 1 || v->ht == HAWK_CUCKOO || q->main.xinner > 0)
    return HAWK_OK;  // (plans with a CROSS_JOIN run the kernels compiled ahead of time)
  if (v->wg_size < 1 || v->wg_size > 1024 || v->thread_mult < 1) return HAWK_OK;  // execution reports it
  if (q->main.ngroup == 0) {
    // AGGREGATE without grouping attributes
    std::string msg;
    const hipError_t e = jit_scalar_prepare(ctx->jit_cache, msg, q->main, v->mem, v->pred, v->hash, v->agg_strategy,
                                            static_cast<int32_t>(v->wg_size));
    if (e != hipSuccess && e != hipErrorNotSupported)
      return set_error(ctx, HAWK_E_DEVICE, "run-time compilation: " + msg);
    return HAWK_OK;
  }
  HkAggTable T{};
  T.slot_words = q->main.slot_words;
  T.log2cap = std::max<uint32_t>(6, ceil_log2(static_cast<uint64_t>(q->groups_hint) * 2));
  T.rlog2 = T.log2cap;
  const int64_t groups = v->agg_strategy == HAWK_LOCAL
                             ? static_cast<int64_t>(v->thread_mult) * ctx->num_cus
                             : static_cast<int64_t>(ctx->num_cus) * std::max<int64_t>(1, 2048 / v->wg_size);
  // the join tables' sizes as the builds will make them
  HkPlan P = q->main;
  for (int i = 0; i < P.nprobes; ++i)
    P.probes[i].t.log2cap = join_log2cap(q->builds[q->probe_build[i]].nrows, 0);
  AggConfig c;
  if (agg_config(ctx, P, T, q->groups_hint, v, groups, c)) {
    ctx->err.clear();  // the execution reports it
    return HAWK_OK;
  }
  std::string msg;
  const hipError_t e = jit_agg_prepare(ctx->jit_cache, msg, P, v->mem, v->pred, v->hash, v->agg_strategy,
                                       static_cast<int32_t>(v->wg_size), c.llog2, q->main.slot_words, c.reps,
                                       c.spill ? &c.sp : nullptr, c.stage, c.nstage);
  if (e != hipSuccess && e != hipErrorNotSupported) return set_error(ctx, HAWK_E_DEVICE, "run-time compilation: " + msg);
  return HAWK_OK;
}

extern "C" hawk_status hawk_jit_compile_check(hawk_ctx* ctx, const hawk_query* q, const hawk_variant* v) {
  if (!ctx) return HAWK_E_ARG;
  if (!q || !v) return set_error(ctx, HAWK_E_ARG, "bad argument");
  const bool was = ctx->jit;
  ctx->jit = true;
  ctx->jit_cache.compile_only = true;
  const hawk_status st = prepare_run_time_kernel(ctx, q, v);
  ctx->jit_cache.compile_only = false;
  ctx->jit = was;
  return st;
}

extern "C" hawk_status hawk_time_variant(hawk_ctx* ctx, const hawk_query* q, const hawk_variant* v, int32_t reps,
                                         double limit_ms, double* median_ms) {
  if (!ctx) return HAWK_E_ARG;
  if (!q || !v || !median_ms || reps < 1) return set_error(ctx, HAWK_E_ARG, "bad argument");
  if (ctx->device < 0) return set_error(ctx, HAWK_E_DEVICE, "planning context cannot execute");
  hawk_status pst = prepare_run_time_kernel(ctx, q, v);
  if (pst) return pst;
  hawk_result* r = nullptr;
  // untimed first run: checks the variant end to end (retries included)
  hipError_t e = hipEventRecord(ctx->ev0, ctx->stream);
  if (e != hipSuccess) return hip_error(ctx, e, "event");
  hawk_status st = hawk_execute(ctx, q, v, &r);
  if (st) return st;
  hawk_result_free(r);
  (void)hipEventRecord(ctx->ev1, ctx->stream);
  (void)hipEventSynchronize(ctx->ev1);
  float first = 0.f;
  (void)hipEventElapsedTime(&first, ctx->ev0, ctx->ev1);
  if (limit_ms > 0 && first > limit_ms) {
    *median_ms = first;
    return set_error(ctx, HAWK_E_TIMEOUT, "variant slower than the time limit");
  }
  std::vector<double> t;
  for (int32_t i = 0; i < reps; ++i) {
    (void)hipEventRecord(ctx->ev0, ctx->stream);
    st = hawk_execute_async(ctx, q, v, &r);
    if (st) return st;
    (void)hipEventRecord(ctx->ev1, ctx->stream);
    e = hipEventSynchronize(ctx->ev1);
    if (e != hipSuccess) {
      hawk_result_free(r);
      return hip_error(ctx, e, "event synchronize");
    }
    st = result_check(r);
    hawk_result_free(r);
    if (st) return st;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    t.push_back(ms);
    if (limit_ms > 0 && ms > limit_ms) {
      *median_ms = ms;
      return set_error(ctx, HAWK_E_TIMEOUT, "variant slower than the time limit");
    }
  }
  std::sort(t.begin(), t.end());
  *median_ms = t[t.size() / 2];
  return HAWK_OK;
}
