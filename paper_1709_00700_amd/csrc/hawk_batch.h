// Batched execution (hk_batch.hip): per-query descriptors read by the
// persistent kernels, fill jobs, and the launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hawk_plan.h"

enum { HK_BQ_PROJECT = 1, HK_BQ_GROUPED = 2, HK_BQ_SCALAR = 3 };

// fill ptr[0..n) with pattern[i % period] (n comes from the job's range)
struct HkFillJob { uint64_t* ptr; uint64_t pattern[2 + 2 * HK_MAX_AGGS]; int32_t period; };

struct HkBatchQuery {
  HkPlan plan;              // lowered main pipeline (tables and hash functions filled in)
  int32_t kind;             // HK_BQ_*
  int32_t shape;            // shape class of the plan
  int64_t tile_rows;        // rows per work item (multiple of 128)
  int64_t ntiles;
  HkAggTable table;         // aggregation: global table (+ side slot); scalar: one slot
  int64_t nslots;
  uint32_t llog2;           // LDS table slots of a grouped tile (log2)
  HkIdent ident;            // identity words of a slot
  HkOut out;                // projection outputs
  uint64_t* status;         // projection: one look-back word per tile
  uint64_t* count;          // projected rows / group rows
  int* err;
  HkResOut res;             // aggregation result columns
};

hipError_t hk_batch_fill(hipStream_t st, const HkFillJob* jobs, const int64_t* bases, int32_t njobs, int64_t total);
hipError_t hk_batch_build(hipStream_t st, int64_t grid, const HkBuild* builds, const int64_t* bases, int32_t nb,
                          int64_t nitems, int64_t tile_rows, unsigned long long* head, int* err);
hipError_t hk_batch_main(hipStream_t st, int shape, int64_t grid, int32_t wg, size_t lds, const HkBatchQuery* qs,
                         const int32_t* qidx, const int64_t* bases, int32_t nq, int64_t nitems,
                         unsigned long long* head);
hipError_t hk_batch_final(hipStream_t st, int64_t grid, const HkBatchQuery* qs, const int32_t* qidx,
                          const int64_t* bases, int32_t nq, int64_t nitems, int64_t tile_slots,
                          unsigned long long* head);
