// Host-side state behind the opaque handles of hawk.h.
#pragma once
#include <hip/hip_runtime.h>

#include <set>
#include <string>
#include <vector>

#include "hawk.h"
#include "hawk_jit.h"
#include "hawk_plan.h"

// Device memory pool of the context: blocks are hipMalloc'ed once and reused
// (stream order makes reuse safe; nothing is returned to the driver before
// hawk_ctx_destroy), so steady-state execution allocates nothing.
struct DevicePool {
  struct Block { void* p; size_t bytes; bool used; };
  std::vector<Block> blocks;
  void* get(size_t bytes);
  void put(void* p);
  void release_all();
};

struct ColReg { std::string name; int32_t dtype; int32_t scale; const void* ptr; };
struct TableReg { std::string name; int64_t nrows; std::vector<ColReg> cols; bool live; };

// one profiled kernel launch: HIP events around it on the context stream
struct ProfRec { std::string name; hipEvent_t a, b; };

struct hawk_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cus = 0;
  int64_t lds_bytes = 0;
  uint64_t seed = 0;
  std::string err;
  std::vector<TableReg> tables;
  DevicePool pool;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  void* dummy = nullptr;  // 256 zero bytes in device memory: the column of a plan's unused column slots
  void* h_stage = nullptr;      // pinned staging of plan uploads into an arena
  size_t stage_bytes = 0;
  uint64_t* h_flags = nullptr;  // pinned: row count and error flags read back by the non-allocating execution
  bool jit = false;       // grouped aggregation runs kernels specialised at run time for the plan
  uint32_t variant_dims = 0;  // extra variant dimensions in variant spaces (HAWK_DIM_*)
  JitCache jit_cache;
  // live handles; destroying the context releases their device state and
  // orphans them (their *_free then only releases host memory)
  std::set<struct hawk_query*> queries;
  std::set<struct hawk_result*> results;
  std::set<struct hawk_model*> models;
  std::set<struct hawk_batch*> batches;
  bool prof_on = false;
  std::vector<ProfRec> prof;           // launches recorded since profiling was enabled
  std::vector<hipEvent_t> prof_free;   // recycled events
};

// brackets one launch with events when profiling is on
struct ProfScope {
  hawk_ctx* ctx;
  size_t idx;
  ProfScope(hawk_ctx* c, const char* name);
  ~ProfScope();
};

// a lowered build pipeline (LOOP, FILTER*, HASH_PUT)
struct QueryBuild {
  HkPlan plan;  // filter part
  HkCol key, payload;
  int32_t payload_dtype = 0;
  int32_t ht_id = 0;
  int64_t nrows = 0;
};

// a join table owned by a query (kept across executions)
struct JoinTableMem { uint64_t* slots = nullptr; uint64_t* side = nullptr; uint32_t log2cap = 0; };

struct hawk_query {
  hawk_ctx* ctx = nullptr;
  // device copies of the lowered plans read by the kernels: [main HkPlan][HkBuild x builds]
  void* d_plans = nullptr;
  void* h_stage = nullptr;           // pinned staging buffer of the upload
  hipEvent_t up_ev = nullptr;        // completes when the last upload has been read
  bool up_pending = false;
  std::vector<char> uploaded;        // bytes of the last upload
  std::vector<JoinTableMem> jt;      // one per build pipeline
  int kind = 0;                      // 1 projection, 2 aggregation
  std::vector<QueryBuild> builds;
  std::vector<int> probe_build;      // build index of each probe of the main pipeline
  HkPlan main;                       // lowered main pipeline (tables and hash seeds filled per execution)
  std::vector<int> res_kinds;        // result kind of each aggregate
  int64_t groups_hint = 1;
  double stat_selectivity = 1.0;     // catalog statistic: fraction of rows reaching the sink
  bool has_table = false;            // probes or grouping: hash-table dimensions apply
  std::string program;               // the pipeline programs as text (hawk_query_program)
};

struct ResCol { int32_t kind; void* ptr; };

struct hawk_result {
  hawk_ctx* ctx = nullptr;
  int kind = 0;
  uint64_t* d_count = nullptr;       // rows of the result (device)
  int* d_err = nullptr;              // kernel error flags (device)
  std::vector<ResCol> cols;
  std::vector<void*> owned;          // pool blocks released by hawk_result_free
  bool checked = false;
  int err_bits = 0;
  hawk_status status = HAWK_OK;
  int64_t nrows = -1;
  struct hawk_batch* batch = nullptr;  // set for a view of a batch's result (owns nothing)
};

hawk_status set_error(hawk_ctx* ctx, hawk_status st, const std::string& msg);

// launch configuration of a grouped aggregation: workgroups, LDS table size
// and copies, and whether (and how) rows that miss the LDS table spill
struct AggConfig {
  int64_t groups;
  uint32_t llog2;
  int32_t reps;
  bool spill;
  uint32_t rlog2;   // table region (log2 slots); the whole table without spilling
  int64_t nparts;
  HkSpill sp;       // sizes and registers; buffers are the caller's
  // join tables that the run-time kernel copies into each workgroup's LDS
  // (probe indices in plan order) and their bytes
  int32_t nstage;
  int32_t stage[HK_MAX_PROBES];
  int64_t stage_bytes;
};
hawk_status agg_config(hawk_ctx* ctx, const HkPlan& P, const HkAggTable& T, int64_t groups_hint,
                       const hawk_variant* v, int64_t groups, AggConfig& c);
// the aggregation kernel of variant v: compiled at run time for the plan when
// the context does so (linear probing), else the precompiled one
// the same for AGGREGATE without grouping attributes
hipError_t scalar_kernel_launch(hawk_ctx* ctx, hipStream_t st, const hawk_variant* v, const HkPlan& P,
                                const HkAggTable& T, int64_t groups, int32_t wg, const uint64_t* ident, int32_t W,
                                int* err, bool allow_jit = true);
hipError_t agg_kernel_launch(hawk_ctx* ctx, hipStream_t st, const hawk_variant* v, const HkPlan& P,
                             const HkAggTable& T, const AggConfig& c, const uint64_t* ident, int32_t W, int* err,
                             const HkSpill* sp, bool allow_jit = true);
// One execution of (q, v) over an arena [base, base + cap): every device
// buffer, result columns included, is the next 256-byte aligned piece, in an
// order that depends only on (q, v). base == nullptr: nothing is enqueued and
// *used receives the bytes needed. launch: the kernels and fills are enqueued
// on `st` (stream capture allowed: nothing else is called on the device);
// upload (with a base): the plans are copied on `st` from the context's
// staging buffer (the caller synchronises before the next upload) and a
// run-time kernel is compiled first. `holder` receives the flags and result
// columns (pieces of the arena; it owns nothing). No retry on overflow.
hawk_status exec_arena(hawk_ctx* ctx, const hawk_query* q, const hawk_variant* v, hipStream_t st, char* base,
                       size_t cap, bool launch, bool upload, hawk_result* holder, size_t* used);
void query_release_device(hawk_query* q);
void model_release_device(struct hawk_model* m);
void batch_release_device(struct hawk_batch* b);
void batch_forget_view(struct hawk_batch* b, hawk_result* r);
std::vector<hawk_variant> variant_space(const hawk_query* q);
hawk_status query_features(const hawk_query* q, const hawk_variant* v, int num_cus, float* f);
