/*
 * CPU oracle for pipeline programs: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, column-at-a-time interpreter of one query (build pipelines +
 * one probe/main pipeline) following the operation semantics of the paper's
 * pipeline-program table (Section 3.1, Table 1) and its example query plan
 * (Table 2). Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it. It shares no code, header or helper with the GPU
 * library; it has no hash tables and no hash functions.
 */
#ifndef HAWK_ORACLE_H
#define HAWK_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* element types: signed, non-nullable */
enum { ORC_I8 = 1, ORC_I32 = 2, ORC_I64 = 3 };
enum { ORC_ADD = 1, ORC_SUB = 2, ORC_MUL = 3 };
enum { ORC_COUNT = 1, ORC_SUM = 2, ORC_MIN = 3, ORC_MAX = 4, ORC_AVG = 5 };
enum { ORC_PROJECT = 1, ORC_AGGREGATE = 2 };
enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_DUPKEY = -7 };

typedef struct { const void* data; int32_t dtype; int32_t pad; } orc_col;
typedef struct { int32_t col; int32_t pad; int64_t lo; int64_t hi; } orc_filter; /* lo <= x <= hi */

typedef struct {
  int64_t nrows; const orc_col* cols; int32_t ncols;
  int32_t nfilters; const orc_filter* filters;
  int32_t key_col; int32_t payload_col;
} orc_build;

/* Attribute ids of the main pipeline: [0, ncols) table columns, then
   [ncols, ncols + ninner) the columns of the CROSS_JOIN table (if any), then
   one per probe (its payload), then one per arithmetic step (its output). */
typedef struct { int32_t fk_col; int32_t build; } orc_probe;
typedef struct { int32_t op; int32_t x_const, y_const; int32_t x, y; int32_t pad; int64_t xc, yc; } orc_arith;
typedef struct { int32_t fn; int32_t attr; int32_t wide; int32_t pad; } orc_agg;

typedef struct {
  int64_t nrows; const orc_col* cols; int32_t ncols;
  int32_t nfilters; const orc_filter* filters;       /* FILTERs before the CROSS_JOIN (table columns) */
  /* CROSS_JOIN (Table 1): every surviving row is paired with every row of a
     second table, in row-major order; ninner = 0: no CROSS_JOIN */
  int64_t inner_nrows; const orc_col* inner_cols; int32_t ninner;
  int32_t nfilters2; const orc_filter* filters2;     /* FILTERs after it (either table's columns) */
  int32_t nprobes; const orc_probe* probes;
  int32_t narith; const orc_arith* arith;
  int32_t kind;
  int32_t nproj; const int32_t* proj;
  int32_t ngroup; const int32_t* group;
  int32_t naggs; const orc_agg* aggs;
} orc_main;

typedef struct orc_result orc_result;

/* Runs the query. On success *out receives a result the caller frees. */
int32_t orc_run(const orc_build* builds, int32_t nbuilds, const orc_main* m, orc_result** out);
/* The same result, with the main pipeline's rows split into nthreads
   contiguous ranges interpreted on as many threads (the ranges' rows
   concatenated in order, their groups merged): the oracle on all host cores. */
int32_t orc_run_parallel(const orc_build* builds, int32_t nbuilds, const orc_main* m, int32_t nthreads,
                         orc_result** out);
void orc_free(orc_result* r);
int64_t orc_rows(const orc_result* r);
/* projection: column c (int64, row order) */
void orc_project_column(const orc_result* r, int32_t c, int64_t* dst);
/* aggregation (rows sorted by group key): group attribute g as int64 */
void orc_group_key(const orc_result* r, int32_t g, int64_t* dst);
void orc_group_count(const orc_result* r, int64_t* dst);
/* aggregate a: lo/hi halves of the exact value (hi = sign-carrying upper 64 bits);
   for narrow SUM/MIN/MAX/COUNT hi is the sign extension of lo */
void orc_agg_value(const orc_result* r, int32_t a, uint64_t* lo, int64_t* hi);
/* AVG aggregate a as double */
void orc_agg_avg(const orc_result* r, int32_t a, double* dst);

#ifdef __cplusplus
}
#endif
#endif
