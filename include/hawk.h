/*
 * hawk.h - C ABI of the MI355X (gfx950) pipeline-variant library.
 *
 * The library executes the data-parallel hot path of a variant-generating
 * query compiler (Bress et al., "Generating Custom Code for Efficient Query
 * Execution on Heterogeneous Processors", arXiv 1709.00700): fused pipeline
 * programs (Section 3.1, Table 1) - columnar scan, selection, hash-join probe,
 * arithmetic, then grouped aggregation or order-preserving projection - in
 * any variant of the paper's variant space (Section 9.2: execution strategy,
 * hash-table implementation and hash function, memory access pattern,
 * branching vs software predication, thread counts).
 *
 * Conventions for every entry point:
 *  - Return value: hawk_status, 0 = HAWK_OK, negative = error. No entry point
 *    throws or aborts across the ABI. After an error on a context,
 *    hawk_last_error(ctx) describes it (valid until the next call on ctx).
 *  - Device memory passed in (columns) is BORROWED: the caller allocates it,
 *    keeps it alive and unmodified while registered. Queries, results, models
 *    and batches are library-owned and released with their *_free call.
 *  - All GPU work is ordered on the stream given to hawk_ctx_create.
 *    Calls that hand data to the host (result info/copy, model readback)
 *    synchronise that stream.
 *  - One context per host thread; a context is not thread-safe.
 */
#ifndef HAWK_H
#define HAWK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hawk_status;
enum {
  HAWK_OK = 0,
  HAWK_E_ARG = -1,         /* null pointer, bad size or enum value */
  HAWK_E_NOTFOUND = -2,    /* unknown table / column / attribute name */
  HAWK_E_TYPE = -3,        /* attribute type not allowed where used */
  HAWK_E_PLAN = -4,        /* pipeline program malformed or beyond supported limits */
  HAWK_E_INFEASIBLE = -5,  /* variant cannot run this plan on this device */
  HAWK_E_CAPACITY = -6,    /* a hash table overflowed (after the library's own retries) */
  HAWK_E_DUPKEY = -7,      /* a build pipeline inserted one key twice */
  HAWK_E_DEVICE = -8,      /* HIP runtime error */
  HAWK_E_OOM = -9,         /* device allocation failed */
  HAWK_E_TIMEOUT = -10     /* variant exceeded the exploration time limit (pruned) */
};

/* column element types: signed two's complement, non-nullable */
enum { HAWK_I8 = 1, HAWK_I32 = 2, HAWK_I64 = 3 };
/* result column element kinds */
enum { HAWK_RES_I64 = 3, HAWK_RES_I128 = 4, HAWK_RES_F64 = 5 };

typedef struct hawk_ctx hawk_ctx;
typedef struct hawk_query hawk_query;
typedef struct hawk_result hawk_result;
typedef struct hawk_model hawk_model;
typedef struct hawk_batch hawk_batch;

/* ------------------------------------------------------------ context */
/* Creates a context on HIP device `device`, ordering work on `hip_stream`
   (a hipStream_t, e.g. torch's current stream; NULL = the null stream).
   device = -1 creates a planning context without a device (assumes 256
   compute units and 160 KiB LDS): tables, queries, variant spaces and
   features work; every execution entry point returns HAWK_E_DEVICE.
   Errors: HAWK_E_DEVICE (no such device), HAWK_E_ARG. */
hawk_status hawk_ctx_create(int32_t device, void* hip_stream, hawk_ctx** out);
/* Synchronises the stream and frees every device buffer the context owns,
   including those of queries, results and models still alive: such handles
   become orphaned, their *_free only releases host memory and every other
   call on them returns HAWK_E_ARG. */
void hawk_ctx_destroy(hawk_ctx* ctx);
const char* hawk_last_error(const hawk_ctx* ctx);
/* Device facts used by the variant space: compute units ("maximal compute
   units" of Section 9.2) and LDS bytes per workgroup. */
hawk_status hawk_device_info(const hawk_ctx* ctx, int32_t* num_cus, int64_t* lds_bytes);

/* ------------------------------------------------------------ tables */
/* A column of a column-major in-memory table (Section 7.6). `scale` is the
   fixed-point decimal scale, carried as metadata only. */
typedef struct {
  const char* name;
  int32_t dtype;        /* HAWK_I8 | HAWK_I32 | HAWK_I64 */
  int32_t scale;
  const void* dev_ptr;  /* nrows elements, device memory, borrowed */
} hawk_column;

/* Registers a table under `name`; names and column names are copied.
   nrows must be < 2^32; each column must be aligned to its element size.
   Errors: HAWK_E_ARG (duplicate table/column name, bad dtype, null pointer
   with nrows > 0, misaligned column). */
hawk_status hawk_table_register(hawk_ctx* ctx, const char* name, int64_t nrows,
                                const hawk_column* cols, int32_t ncols, int32_t* table_id);
hawk_status hawk_table_unregister(hawk_ctx* ctx, int32_t table_id);

/* ------------------------------------------------------------ pipeline programs */
/* Pipeline operations of Section 3.1, Table 1. */
enum {
  HAWK_LOOP = 1,           /* LOOP(T): iterate the rows of table `table` */
  HAWK_FILTER = 2,         /* FILTER(lo <= a <= hi) on a column of the looped table */
  HAWK_HASH_PUT = 3,       /* HASH_PUT: insert key column `a` with payload column `b` into table `ht` */
  HAWK_HASH_PROBE = 4,     /* HASH_PROBE(a = key of table `ht`): inner equi-join; payload becomes attribute `b` */
  HAWK_ARITHMETIC = 5,     /* ARITHMETIC: attribute `a` := x (arith_op) y, x = attr `b` or const `lo`, y = attr `c` or const `hi` */
  HAWK_AGGREGATE = 6,      /* AGGREGATE(F): non-grouped aggregation */
  HAWK_HASH_AGGREGATE = 7, /* HASH_AGGREGATE(G, F): group by attrs[0..nattrs) (1 or 2, at most 32-bit each) */
  HAWK_PROJECT = 8,        /* PROJECT(attrs): materialise attributes in input row order */
  HAWK_CROSS_JOIN = 9      /* CROSS_JOIN(T): table id `table`; every tuple is paired with every row of T
                              (row-major: T's rows vary fastest); later operations see the columns of
                              both tables (names must differ); one per main pipeline, after LOOP and
                              FILTERs on the looped table, before probes; fewer than 2^32 pairs */
};
enum { HAWK_ADD = 1, HAWK_SUB = 2, HAWK_MUL = 3 };
enum { HAWK_COUNT = 1, HAWK_SUM = 2, HAWK_MIN = 3, HAWK_MAX = 4, HAWK_AVG = 5 };

typedef struct {
  int32_t fn;          /* HAWK_COUNT..HAWK_AVG */
  int32_t wide;        /* SUM: 1 = exact 128-bit sum, 0 = its low 64 bits (two's complement);
                          AVG always divides the exact sum (128-bit accumulator for 64-bit
                          attributes and arithmetic results, 64-bit for 8/32-bit ones) */
  const char* attr;    /* aggregated attribute (NULL for COUNT) */
} hawk_agg;

typedef struct {
  int32_t kind;                 /* HAWK_LOOP .. HAWK_PROJECT */
  int32_t table;                /* LOOP: table id */
  const char* a;                /* see the operation list above */
  const char* b;
  const char* c;
  int32_t arith_op;             /* ARITHMETIC: HAWK_ADD | HAWK_SUB | HAWK_MUL */
  int32_t ht;                   /* HASH_PUT / HASH_PROBE: id linking a build to its probes */
  int64_t lo, hi;               /* FILTER: inclusive bounds; ARITHMETIC: constants */
  const char* const* attrs;     /* PROJECT outputs / HASH_AGGREGATE group attributes */
  int32_t nattrs;
  int32_t naggs;
  const hawk_agg* aggs;         /* AGGREGATE / HASH_AGGREGATE */
  int64_t groups_hint;          /* HASH_AGGREGATE: expected distinct groups (table sizing) */
} hawk_op;

typedef struct { const hawk_op* ops; int32_t nops; } hawk_pipeline;

/* A query is an ordered list of pipelines (Table 2): zero or more build
   pipelines (LOOP, FILTER*, HASH_PUT) followed by one main pipeline
   (LOOP, FILTER*, [CROSS_JOIN, FILTER*], HASH_PROBE*, ARITHMETIC*, then
   PROJECT | AGGREGATE | HASH_AGGREGATE). The plan is validated here: names and types, build/probe
   pairing by `ht` (Section 5.1: a build and its probes share one table), and
   the kernel limits (12 columns, 6 filters, 4 probes, 8 arithmetic steps,
   8 aggregates, 4 projected attributes, 16 live attributes). The query keeps
   pointers to the registered tables' columns, not to `pipes`. */
hawk_status hawk_query_create(hawk_ctx* ctx, const hawk_pipeline* pipes, int32_t npipes, hawk_query** out);
void hawk_query_free(hawk_query* q);
/* 1 = projection pipeline, 2 = aggregation pipeline */
hawk_status hawk_query_kind(const hawk_query* q, int32_t* kind);

/* ------------------------------------------------------------ relational plans */
/* A relational operator tree, partitioned into pipelines by the
   produce/consume model (Section 2.1): a hash join's build side becomes a
   build pipeline (LOOP, FILTER*, HASH_PUT), every other operator adds its
   operation to the pipeline of the tuples that reach it, and the root ends
   the probe pipeline (Table 2). Nodes refer to their children by index. */
enum {
  HAWK_REL_SCAN = 1,       /* the rows of table `table` */
  HAWK_REL_SELECT = 2,     /* input's tuples with lo <= a <= hi */
  HAWK_REL_MAP = 3,        /* input's tuples plus a := x (arith_op) y; x = attr b or const lo, y = attr c or const hi */
  HAWK_REL_HASH_JOIN = 4,  /* inner equi-join of input (probe side) with right (build side, unique keys) on
                              input.a = right.b; the result is input's tuple plus right's attribute c */
  HAWK_REL_CROSS_JOIN = 5, /* every tuple of input with every tuple of right (row-major) */
  HAWK_REL_GROUP_BY = 6,   /* root only: group input by attrs[0..nattrs) (none: one row) computing aggs */
  HAWK_REL_PROJECT = 7     /* root only: attrs of input's tuples, in input order */
};
typedef struct {
  int32_t kind;                 /* HAWK_REL_* */
  int32_t input;                /* child node index (-1 for SCAN) */
  int32_t right;                /* HASH_JOIN: build side; CROSS_JOIN: second input */
  int32_t table;                /* SCAN: table id */
  const char* a;
  const char* b;
  const char* c;
  int32_t arith_op;             /* MAP: HAWK_ADD | HAWK_SUB | HAWK_MUL */
  int32_t nattrs;
  int64_t lo, hi;
  const char* const* attrs;     /* GROUP_BY keys / PROJECT attributes */
  const hawk_agg* aggs;         /* GROUP_BY */
  int32_t naggs;
  int32_t reserved;
  int64_t groups_hint;          /* GROUP_BY with keys: expected distinct groups */
} hawk_rel;
/* Compiles the plan of n nodes rooted at `root` into a query: build
   pipelines in the order the produce pass meets the joins, then the probe
   pipeline with its operations ordered LOOP, FILTERs on the scanned table,
   CROSS_JOIN and its FILTERs, HASH_PROBEs, ARITHMETIC, sink (selections
   commute with inner joins and arithmetic). A hash join's build side and a
   cross join's second input must be scans under selections; selections read
   scanned columns (not join payloads or computed attributes). The query is
   validated as by hawk_query_create. Errors: HAWK_E_ARG (indices, unknown
   operator), HAWK_E_PLAN (unsupported shape, a node reaching itself),
   anything hawk_query_create returns. */
hawk_status hawk_query_from_plan(hawk_ctx* ctx, const hawk_rel* nodes, int32_t n, int32_t root, hawk_query** out);
/* The query's pipeline programs as text, one pipeline per line (build
   pipelines first), in the notation of Table 2, e.g.
   "LOOP(T1) FILTER(x in [5, 5]) HASH_PUT(a -> x; ht 0)". Two-call sizing:
   *len receives the length (without the terminating zero); buf (cap bytes)
   may be NULL. */
hawk_status hawk_query_program(const hawk_query* q, char* buf, int64_t cap, int64_t* len);

/* ------------------------------------------------------------ variants */
/* One point of the variant space of Section 9.2. Value order of each
   dimension follows the paper's listing (first value first). */
enum { HAWK_SINGLE_PASS = 0, HAWK_MULTI_PASS = 1 };    /* projection strategy (Section 4.1) */
enum { HAWK_SEQUENTIAL = 0, HAWK_COALESCED = 1 };      /* memory access pattern (Section 6.1) */
enum { HAWK_BRANCHED = 0, HAWK_PREDICATED = 1 };       /* predication mode (Section 6.1) */
enum { HAWK_LINEAR_PROBING = 0, HAWK_CUCKOO = 1,       /* hash table (Section 5.1) */
       HAWK_ROBIN_HOOD = 2 };  /* join tables only (extension of Section 7.5.1): robin-hood linear probing;
                                  grouping tables of such a variant use linear probing */
enum { HAWK_FILTER_SCALAR = 0, HAWK_FILTER_SIMD = 1 }; /* FILTER mode (extension of Section 7.5.2) */
enum { HAWK_MURMUR = 0, HAWK_MULTIPLY_SHIFT = 1 };     /* hash function (Section 9.2) */
enum { HAWK_LOCAL = 0, HAWK_GLOBAL = 1 };              /* aggregation strategy (Section 4.2) */
typedef struct {
  uint8_t proj_strategy, mem, pred, ht, hash, agg_strategy;
  uint8_t unroll;        /* loop unrolling (Section 6.1): rows per loop iteration of the multi-pass filter
                            kernel, taken with element access offsets 0..unroll-1 (1, 2 or 4; 0 = the
                            default 4) */
  uint8_t filter_mode;   /* HAWK_FILTER_SCALAR | HAWK_FILTER_SIMD (multi-pass coalesced projections) */
  uint32_t thread_mult;  /* multi-pass projection threads / local hash tables, as a multiple of the CUs */
  uint32_t wg_size;      /* aggregation: threads per hash table (16..1024) */
} hawk_variant;

/* Writes the variant space of q (two-call sizing: out may be NULL, *n is the
   size). Projection: 4 single-pass + 28 multi-pass; aggregation: 784 local +
   112 global (Section 9.2). Hash-table dimensions are multiplied in only when
   the query has a hash table (probes or groups). With extra dimensions set on
   the query's context (hawk_ctx_set_variant_dims) the space grows where they
   apply. */
hawk_status hawk_variant_space(const hawk_query* q, hawk_variant* out, int64_t cap, int64_t* n);
/* Extra variant dimensions beyond Section 9.2, the extensions the paper
   sketches (Sections 6.1, 7.5.1, 7.5.2): HAWK_DIM_ROBIN_HOOD adds ht =
   HAWK_ROBIN_HOOD for pipelines with probes; HAWK_DIM_UNROLL adds unroll 2
   and 1 to multi-pass coalesced projections (the default is 4);
   HAWK_DIM_SIMD_FILTER adds filter_mode = HAWK_FILTER_SIMD to multi-pass
   coalesced projections with filters, no probes and 16-byte aligned filter
   columns (executing it otherwise is HAWK_E_INFEASIBLE). 0 (the default) = the paper's space.
   Affects hawk_variant_space, hawk_explore and the model's picks. */
enum { HAWK_DIM_ROBIN_HOOD = 1, HAWK_DIM_UNROLL = 2, HAWK_DIM_SIMD_FILTER = 4 };
hawk_status hawk_ctx_set_variant_dims(hawk_ctx* ctx, uint32_t dims);
/* Text form "strat=mp,mem=coal,pred=br,ht=lin,hash=murmur,agg=local,tm=64,wg=256"
   (",unroll=U" and ",filter=simd" follow when set; ht=robin for robin hood). */
hawk_status hawk_variant_format(const hawk_variant* v, char* buf, int32_t cap);

/* ------------------------------------------------------------ execution */
/* Executes q in variant v. Runs every build pipeline then the main pipeline,
   synchronises, and retries internally on hash-table overflow (new hash
   seeds, then doubled capacity). Errors: HAWK_E_DUPKEY, HAWK_E_CAPACITY,
   HAWK_E_INFEASIBLE (e.g. a local table does not fit in LDS), HAWK_E_DEVICE. */
hawk_status hawk_execute(hawk_ctx* ctx, const hawk_query* q, const hawk_variant* v, hawk_result** out);
/* Same, but only enqueues work (no synchronisation, no retry). Overflow and
   duplicate-key errors are reported by hawk_result_info. */
hawk_status hawk_execute_async(hawk_ctx* ctx, const hawk_query* q, const hawk_variant* v, hawk_result** out);

/* Execution that allocates nothing, for callers that cannot allocate device
   memory: code under HIP graph capture, tight serving loops, harnesses that
   forbid hipMalloc. It runs q in variant v once, as hawk_execute does but
   without its retries, and synchronises the context stream before it
   returns. Every device buffer except the result columns (flags, plans, join
   and aggregation tables, scan and projection buffers) lies in a scratch array
   of HAWK_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs
   on until the process ends; only kernels compiled ahead of time run
   (hawk_ctx_set_jit does not apply).
   cols: ncols caller-owned device pointers in the column order of
   hawk_result_info (projection: one per projected attribute; aggregation:
   the group attributes, the aggregates, the row count), each with room for
   cap_rows elements (16 bytes in a HAWK_RES_I128 column, 8 otherwise). With
   cols == NULL nothing runs and *nrows receives the cap_rows the execution
   needs (projection: input rows + 1; grouped aggregation: the table's slots
   + 1, from the group hint); this sizing call also works on a planning
   context. On success *nrows = result rows, laid out as
   hawk_execute's (projection rows in input order, group rows in hash-table
   order).
   Errors: HAWK_E_ARG (null pointer, wrong column count, cap_rows below the
   need), HAWK_E_CAPACITY (the execution needs more scratch than the array
   holds - e.g. a spilling aggregation or a projection of several hundred
   million rows - or a hash table overflowed: no retry here, raise the
   query's group hint), HAWK_E_DUPKEY, HAWK_E_INFEASIBLE, HAWK_E_TIMEOUT,
   HAWK_E_DEVICE.
   The scratch array is shared by every call on one device and keeps the last
   call's contents (each call initialises what it reads): calls that overlap
   on one device, from two host threads or two contexts, race and give
   undefined results. */
#define HAWK_NOALLOC_SCRATCH_BYTES (64ull << 20)
hawk_status hawk_execute_noalloc(hawk_ctx* ctx, const hawk_query* q, const hawk_variant* v, void* const* cols,
                                 int32_t ncols, int64_t cap_rows, int64_t* nrows);

/* Result rows and columns. Projection: one HAWK_RES_I64 column per projected
   attribute, rows in input order. Aggregation: the group attributes
   (HAWK_RES_I64), then one column per aggregate (COUNT/MIN/MAX/narrow SUM:
   HAWK_RES_I64; wide SUM: HAWK_RES_I128 as {uint64 lo, int64 hi} pairs; AVG:
   HAWK_RES_F64), then the group's row count (HAWK_RES_I64). Group rows come
   in hash-table order. Synchronises; returns the deferred error of an async
   execution. */
hawk_status hawk_result_info(hawk_result* r, int64_t* nrows, int32_t* ncols);
hawk_status hawk_result_column(hawk_result* r, int32_t col, int32_t* elem_kind, const void** dev_ptr);
/* Copies column col (nrows elements) to host memory of cap_bytes. */
hawk_status hawk_result_copy_column(hawk_result* r, int32_t col, void* host_dst, int64_t cap_bytes);
void hawk_result_free(hawk_result* r);

/* ------------------------------------------------------------ timing and exploration (Section 8) */
/* Executes (q, v) once untimed and `reps` times timed with HIP events on the
   context stream; *median_ms is the median. A run longer than limit_ms
   (<= 0: no limit) stops the repetitions and returns HAWK_E_TIMEOUT
   (the pruning rule of Section 9.1). */
hawk_status hawk_time_variant(hawk_ctx* ctx, const hawk_query* q, const hawk_variant* v,
                              int32_t reps, double limit_ms, double* median_ms);

/* Cost callback for the learning algorithm: time of configuration `cfg`
   (one value index per dimension); return +inf for an infeasible point. */
typedef double (*hawk_cost_fn)(const int32_t* cfg, int32_t ndims, void* user);
/* Algorithm 1 (feature-wise variant learning): start from the first value
   of every dimension, vary one dimension at a time keeping the fastest value
   (strictly faster wins, so ties keep the earlier value), repeat the sweep
   until the configuration no longer changes or q sweeps ran. `order` lists
   the dimensions in the order they are visited (NULL = 0..ndims-1; the
   paper's feature ordering visits strategy, threads and memory access
   first). Writes the learned configuration and the number of cost calls. */
hawk_status hawk_learn_feature_wise(const int32_t* dim_sizes, int32_t ndims, const int32_t* order,
                                    int32_t q, hawk_cost_fn cost, void* user,
                                    int32_t* best_cfg, int64_t* n_calls);

enum { HAWK_EXPLORE_EXHAUSTIVE = 0, HAWK_EXPLORE_FEATURE_WISE = 1 };
typedef struct {
  int32_t reps;          /* timed runs per (query, variant); median decides */
  int32_t max_iters;     /* q of Algorithm 1 */
  double limit_ms;       /* prune rule: a run above this is +inf */
  const char* timing_db; /* append-only text log of every measurement (NULL: none): a line
                            "#workload <sig> <k> mode=<m>" per exploration, then one line per
                            (query, variant): sig, query index, the 12 features, the variant's
                            text form, median ms (-1 when pruned) and status, tab-separated */
  int32_t resume;        /* 1: first read timing_db; variants whose k measurements of this
                            workload (same sig: query kinds, sizes, plan structure and
                            constants, compute units) are logged are not measured again
                            (the log is trusted to come from the same tables and device) */
  int32_t reserved;
} hawk_explore_opts;
typedef struct {
  int64_t evaluated;     /* (workload, variant) configurations measured */
  int64_t pruned;        /* of which pruned or infeasible */
  double best_ms;        /* workload time of the returned variant */
  double seconds;        /* wall time of the exploration */
  int64_t reused;        /* configurations taken from the timing log (resume) */
} hawk_explore_report;
/* Learns one variant for the workload W of k queries (Section 8.1): the
   variant minimising the summed per-query median time, by exhaustive search
   ("backtracking" of Section 9.3.2) or by Algorithm 1. Every query must be of
   the same kind (all projection or all aggregation). A variant that is pruned
   (HAWK_E_TIMEOUT) or infeasible for any query counts as +inf; any other
   error stops the exploration and is returned. */
hawk_status hawk_explore(hawk_ctx* ctx, hawk_query* const* W, int32_t k, int32_t mode,
                         const hawk_explore_opts* opts, hawk_variant* best, hawk_explore_report* rep);

/* ------------------------------------------------------------ run-time code generation */
/* When on, aggregation with linear probing (grouped, and without grouping
   attributes) and the multi-pass projection (filter or SIMD filter, then
   projection) run kernels compiled at run time (hipRTC, gfx950) for the plan's structure: column types and
   registers, filter and probe registers, arithmetic operators, group and
   aggregate layout are constants of the generated code, as in the paper's
   per-query code generation (Section 7); column pointers, filter bounds,
   arithmetic constants, join tables, hash seeds and the row count stay
   arguments, so queries of one structure share a kernel. The first execution
   of a (structure, variant) pair compiles it (about a second); kernels are
   cached in the context until hawk_ctx_destroy. Off by default: every other
   path, and this one when off, uses the kernels compiled ahead of time, as
   do plans with a CROSS_JOIN and a generated kernel that would need scratch
   memory (register spills). A generated aggregation kernel also copies the
   join tables that fit (in plan order, up to half of a workgroup's LDS beside
   a local table; without one, as much as leaves room for 16 resident waves
   per CU) into each workgroup's LDS and probes them there; the results are
   the same. With the environment variable HAWK_JIT_DUMP set
   to a directory, each generated source is also written there.
   Errors: HAWK_E_ARG, HAWK_E_DEVICE (planning context). A compilation
   failure is reported by the execution as HAWK_E_DEVICE with the compiler
   log in hawk_last_error. */
hawk_status hawk_ctx_set_jit(hawk_ctx* ctx, int32_t on);
/* Kernels compiled so far and their total compile time. */
hawk_status hawk_jit_stats(const hawk_ctx* ctx, int64_t* kernels, double* compile_ms);
/* Generates and compiles (hipRTC, gfx950) the run-time kernels that executing
   q in variant v would launch with run-time compilation on, and keeps none of
   them: a check of the generated sources that needs no device (a planning
   context works; the context's setting of hawk_ctx_set_jit is left as it
   is). A plan or variant without run-time kernels passes trivially.
   Errors: HAWK_E_ARG; HAWK_E_DEVICE with the compiler log in hawk_last_error. */
hawk_status hawk_jit_compile_check(hawk_ctx* ctx, const hawk_query* q, const hawk_variant* v);

/* ------------------------------------------------------------ kernel profiling */
/* When on, every launch of the library's kernel families is bracketed by HIP
   events on the context stream (adds two event records per launch). Enabling
   or disabling synchronises the stream and clears earlier records. */
hawk_status hawk_profile_enable(hawk_ctx* ctx, int32_t on);
/* Sum of the recorded durations and number of launches of one kernel family:
   "k_agg" (grouped aggregation, including the cuckoo key phase), "k_scalar_agg",
   "k_mp_filter", "k_scan", "k_mp_project", "k_sp", "k_sp_concat", "k_build",
   "k_init_aggtable", "k_finalize", "k_spill_scatter" and "k_spill_agg"
   (regrouping by table region, then aggregation, of the rows a local table
   could not hold). Synchronises the stream. */
hawk_status hawk_profile_read(hawk_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches);

/* ------------------------------------------------------------ cost-model features */
/* Catalog statistic of a query: estimated fraction of input rows that reach
   the sink (filters and joins). Used only as a feature; default 1. */
hawk_status hawk_query_set_stats(hawk_query* q, double selectivity);
/* The 12 features of (query, variant) used by the learned cost model:
   [0] log2(rows+1) [1] selectivity statistic [2] log2(groups+1) (0 for
   projection) [3] bytes read per row [4] probes [5] bytes written per
   qualifying row / per group slot [6] strategy (projection: 0 single-pass,
   1 multi-pass; aggregation: 0 local, 1 global) [7] log2(threads launched)
   [8] log2(workgroup size) [9] predicated [10] coalesced [11] hash table * 2
   + hash function (0 without a table). */
hawk_status hawk_features(const hawk_query* q, const hawk_variant* v, float* out12);

/* ------------------------------------------------------------ learned cost model */
/* A 12 -> 64 -> 64 -> 1 ReLU network in FP32 predicting ln(milliseconds) of a
   (query, variant) pair from hawk_features; the paper picks one variant per
   processor (Section 8) and leaves a per-query optimizer to future work
   (Sections 9.3.4 and 9.4), which this model provides. Parameters (5,057 floats):
   W1 [64x12] | b1 [64] | W2 [64x64] | b2 [64] | W3 [64] | b3 [1], row-major;
   features are standardised as (x - mu) / sd before the first layer. */
hawk_status hawk_model_create(hawk_ctx* ctx, uint64_t seed, hawk_model** out);
void hawk_model_free(hawk_model* m);
/* host arrays: params[5057], mu[12], sd[12] (sd > 0); resets Adam state */
hawk_status hawk_model_set_params(hawk_model* m, const float* params, const float* mu, const float* sd);
hawk_status hawk_model_get_params(hawk_model* m, float* params, float* mu, float* sd);
typedef struct { int32_t epochs; int32_t batch; float lr; uint64_t seed; } hawk_train_opts;
/* Trains on m samples, host arrays X [m x 12] row-major and y [m] = ln(ms):
   standardises with the training mean/std, then mini-batch Adam (beta1 0.9,
   beta2 0.999, eps 1e-8) on the mean squared error with the library's own
   forward/backward kernels; *final_loss = training MSE after the last epoch. */
hawk_status hawk_model_train(hawk_model* m, const float* X, const float* y, int64_t nsamples,
                             const hawk_train_opts* opts, float* final_loss);
/* host arrays X [n x 12] -> out [n] (predicted ln ms) */
hawk_status hawk_model_predict(hawk_model* m, const float* X, int64_t n, float* out);
/* device arrays: forward pass and mean-squared-error gradient (grad[5057],
   loss[1]) of the current parameters, ordered on the context stream */
hawk_status hawk_mlp_forward_dev(hawk_model* m, const float* dX, int64_t n, float* dout);
hawk_status hawk_mlp_grad_dev(hawk_model* m, const float* dX, const float* dy, int64_t n, float* dgrad, float* dloss);
/* For each of n queries: the variant of its variant space with the lowest
   predicted time (first on ties); predicted_ms may be NULL. */
hawk_status hawk_model_pick(hawk_model* m, hawk_query* const* qs, int32_t n, hawk_variant* out, float* predicted_ms);
/* The same over an ensemble of nm models of one context (trained on the same
   timings from different seeds): each variant scores the members' mean
   predicted ln(ms) plus `penalty` (>= 0) times their standard deviation, so
   a variant the members disagree on, far from the training timings, is not
   picked for an optimistic error of one model. predicted_ms (may be NULL)
   receives exp(mean) of each pick. */
hawk_status hawk_model_pick_ensemble(hawk_model* const* ms, int32_t nm, float penalty, hawk_query* const* qs,
                                     int32_t n, hawk_variant* out, float* predicted_ms);

/* ------------------------------------------------------------ batched execution */
/* Many queries as one captured HIP graph. Section 8 tunes one variant per
   workload and the paper leaves per-query work distribution open (Sections
   9.3.4 and 9.4); a batch instead runs every query of a mixed workload in one
   launch sequence, each query in its own variant or in the batch's tile
   kernels:
   - Tile kernels: a fill kernel resets the batch's tables and counters, a
     persistent kernel runs the tiles of every build pipeline (HASH_PUT,
     Table 1), one persistent kernel per plan shape runs the main pipelines'
     tiles (LOOP, FILTER, HASH_PROBE, ARITHMETIC, then HASH_AGGREGATE /
     AGGREGATE or order-preserving PROJECT), and a persistent kernel writes
     every aggregation's result rows. Workgroups take (query, tile) items from
     an atomic counter. These tiles run one fixed variant: coalesced access,
     branched evaluation, linear probing with Murmur hashing, local (LDS)
     pre-aggregation; projections keep input order with a single-pass
     look-back over tile counts.
   - Own variant: the query's builds and main pipeline run the kernels of its
     variant (as hawk_execute would, without retries) as nodes of the same
     graph, over device memory the batch reserves for it at creation.
   Schedule options: tile_rows_log2 in [14, 18] (rows per work item),
   wgs_per_cu in [1, 32] (persistent workgroups per compute unit), order 0
   (submission order) or 1 (largest query first); separate 1 gives grouped
   aggregations without a variant of their own, of at least 2^20 rows and
   with more groups than a tile's LDS table holds, their own variant (the
   spilling local strategy with linear probing, compiled at run time when the
   context does so); 0 keeps them in the tile kernels. NULL opts =
   {16, 2, 1, 1}. */
typedef struct { int32_t tile_rows_log2; int32_t wgs_per_cu; int32_t order; int32_t separate; } hawk_batch_opts;
/* Creates a batch of n queries of ctx (borrowed: they must outlive the batch;
   their tables must stay registered and unmodified). variants: NULL, or one
   per query: a variant of the query's variant space runs the query with its
   own kernels; a variant with thread_mult 0 puts the query in the tile
   kernels. Allocates the batch's device memory (tables sized from the
   queries' row counts and group hints, outputs sized for every input row)
   and captures the graph. Errors: HAWK_E_ARG (bad variant values),
   HAWK_E_DEVICE (planning context, HIP error), HAWK_E_OOM, HAWK_E_INFEASIBLE
   (a tile or a query's variant does not fit in LDS). */
hawk_status hawk_batch_create(hawk_ctx* ctx, hawk_query* const* qs, int32_t n, const hawk_variant* variants,
                              const hawk_batch_opts* opts, hawk_batch** out);
/* Releases the batch's device memory (synchronises the context stream);
   its result views are orphaned (every call on them returns HAWK_E_ARG). */
void hawk_batch_free(hawk_batch* b);
/* Replays the graph once on the context stream (asynchronous). */
hawk_status hawk_batch_run(hawk_batch* b);
/* One untimed and `reps` timed replays with HIP events on the context
   stream; *median_ms is the median. Returns HAWK_E_CAPACITY when a hash table
   of the batch overflowed (group hint or join size too small), HAWK_E_DUPKEY
   when a build inserted a key twice, and HAWK_E_TIMEOUT when a projection
   tile's bounded wait for the counts of the tiles before it gave up (never
   expected: those tiles were handed out earlier to running workgroups). */
hawk_status hawk_batch_time(hawk_batch* b, int32_t reps, double* median_ms);
/* Times every schedule of the grid tile_rows_log2 14..18 x wgs_per_cu
   {1, 2, 4, 8} x order {0, 1} (`reps` timed replays each), keeps the fastest
   (first on ties) and re-captures the graph with it. best/best_ms may be NULL. */
hawk_status hawk_batch_autotune(hawk_batch* b, int32_t reps, hawk_batch_opts* best, double* best_ms);
hawk_status hawk_batch_opts_get(const hawk_batch* b, hawk_batch_opts* out);
/* A view of query i's result after the latest run, read with the result
   calls above (same column layout as hawk_execute). The view owns no memory:
   the next hawk_batch_run overwrites what it shows, and hawk_batch_free
   orphans it; release it with hawk_result_free. Errors as the result calls;
   HAWK_E_CAPACITY or HAWK_E_DUPKEY when the run's hash tables failed (no
   retry inside a batch), HAWK_E_TIMEOUT when a look-back wait gave up. */
hawk_status hawk_batch_result(hawk_batch* b, int32_t i, hawk_result** out);

#ifdef __cplusplus
}
#endif
#endif /* HAWK_H */
