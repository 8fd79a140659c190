// Host-side launchers of the gfx950 kernels (hk_*.hip).
// Each maps the runtime variant values onto template instantiations and
// enqueues on `st`; none synchronises.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hawk_plan.h"

// Pipeline kernels take the lowered plan by value (a kernel argument); each
// launcher picks the shape class that holds the plan. Build and finalize
// kernels read the copy the query keeps in device memory (dB / dP).

hipError_t hk_fill_u64(hipStream_t st, uint64_t* p, int64_t n, uint64_t v);
// fills 0..k-1 of f (k <= HK_MAX_FILLS) in one launch
#define HK_MAX_FILLS 16
struct HkFills {
  uint64_t* p[HK_MAX_FILLS];
  int64_t n[HK_MAX_FILLS];
  uint64_t v[HK_MAX_FILLS];
};
hipError_t hk_fill_multi(hipStream_t st, const HkFills& f, int32_t k);
hipError_t hk_init_aggtable(hipStream_t st, uint64_t* words, int64_t nslots, const uint64_t* ident, int32_t nw);

// build pipelines: FILTER part of B.p (colA columns), then HASH_PUT of key ->
// payload into B.t, for the nb builds B[0..nb) in one launch (one grid row
// each); B is the host copy (sizes), dB the same array in device memory (read
// by the kernels)
hipError_t hk_build(hipStream_t st, const HkBuild* B, const HkBuild* dB, int32_t nb, int ht, int hash, int* err);

// multi-pass projection: filter kernel, scan, projection kernel
// unroll (coalesced): rows per loop iteration, 1, 2 or 4 (0 = 4); simd: FILTER
// in SIMD mode (4 rows per lane from vector loads; coalesced, no probes)
hipError_t hk_mp_filter(hipStream_t st, const HkPlan& P, int mem, int pred, int ht, int hash, int64_t threads,
                        uint64_t* masks, uint32_t* counts, int unroll = 0, int simd = 0);
hipError_t hk_mp_project(hipStream_t st, const HkPlan& P, int mem, int pred, int ht, int hash, int64_t threads,
                         const uint64_t* masks, const uint32_t* offsets, const uint64_t* total, int64_t nact,
                         int64_t* const* out, int64_t dump);

// single-pass projection into per-instance regions, then in-order concatenation
hipError_t hk_sp(hipStream_t st, const HkPlan& P, int mem, int pred, int ht, int hash, int64_t instances,
                 int64_t* const* tmp, int64_t region, uint32_t* counts);
hipError_t hk_sp_concat(hipStream_t st, int64_t* const* tmp, int32_t nproj, int64_t region, int64_t nregions,
                        const uint32_t* counts, const uint32_t* offsets, int64_t* const* out);

// exclusive scan of m u32 counts; tmp needs hk_scan_tmp_words(m) u32 words,
// 8-byte aligned; *total = sum; err (may be null) gets HK_ERR_TIMEOUT if a
// tile's bounded wait for the tiles before it gives up
int64_t hk_scan_tmp_words(int64_t m);
hipError_t hk_scan(hipStream_t st, const uint32_t* in, uint32_t* out, int64_t m, uint32_t* tmp, uint64_t* total,
                   int* err = nullptr);

// grouped aggregation (cuckoo: key phase first; reps: copies of the aggregate
// words of the LDS table, a power of two), non-grouped aggregation, result extraction
// sp != null: spill mode of the local strategy with linear probing (LDS misses
// are appended to sp's regions instead of updating the table, and the LDS
// tables end as merge entries in sp.flush); hk_spill step 0 then regroups the
// entries by table region (offs = exclusive scan of sp.hist, *total = entries)
// into `part`, step 1 aggregates each region in LDS from the identity (a
// region of 2^T.rlog2 slots must fit in one workgroup's LDS)
hipError_t hk_agg(hipStream_t st, const HkPlan& P, const HkAggTable& T, int mem, int pred, int ht, int hash,
                  int strat, int64_t groups, int32_t wg, uint32_t llog2, const uint64_t* ident, int32_t nw, int* err,
                  const HkSpill* sp = nullptr, int32_t reps = 1);
// dynamic LDS bytes of one aggregation workgroup (local table, its copies,
// the spill histogram)
inline size_t hk_agg_lds_bytes(int strat, uint32_t llog2, int32_t nw, int32_t reps, const HkSpill* sp) {
  size_t lds = 0;
  if (strat == HK_LOCAL) {
    const size_t LC = static_cast<size_t>(1) << llog2;
    lds = (LC + static_cast<size_t>(nw - 1) * reps * LC) * sizeof(uint64_t);
  }
  if (sp) lds += static_cast<size_t>(sp->nparts) * sizeof(uint32_t);
  if (sp && sp->door_log2 > 0) lds += (static_cast<size_t>(1) << sp->door_log2) / 8;
  return lds;
}
// step 1 with `out`: the groups become result rows (rows reserved by atomics
// on out->nrows; scratch: 32 words per region) instead of returning to the table
hipError_t hk_spill(hipStream_t st, int step, const HkPlan& P, const HkAggTable& T, int hash, const HkSpill& sp,
                    const uint64_t* ident, int32_t nw, const uint32_t* offs, const uint64_t* total, int64_t nwg,
                    uint64_t* part, int* err, const HkResOut* out = nullptr, uint64_t* scratch = nullptr);
hipError_t hk_scalar_agg(hipStream_t st, const HkPlan& P, const HkAggTable& T, int mem, int pred, int ht, int hash,
                         int strat, int64_t groups, int32_t wg, const uint64_t* ident, int32_t nw, int* err);
hipError_t hk_finalize(hipStream_t st, const HkPlan& P, const HkPlan* dP, const HkAggTable& T, int64_t nslots, int64_t* const* gcols,
                       void* const* acols, int64_t* count, uint64_t* nrows, int keep_empty);
