// Entry points of the pipeline kernels: pick the smallest shape class that
// holds the plan (hk_shape_of) and call that class's launcher, compiled in
// its own translation unit (hk_agg.hip, hk_proj.hip, hk_scalar.hip built once
// per class).
#include <hip/hip_runtime.h>

#include <cstring>

#include "hawk_device.h"
#include "hawk_launch.h"

template <class S>
hipError_t hk_agg_shape(hipStream_t st, const HkPlan& P, const HkAggTable& T, int mem, int pred, int ht, int hash,
                        int strat, int64_t groups, int32_t wg, uint32_t llog2, const HkIdent& id, int* err,
                        const HkSpill* sp, int32_t reps);
template <class S>
hipError_t hk_spill_shape(hipStream_t st, int step, const HkPlan& P, const HkAggTable& T, int hash, const HkSpill& sp,
                          const HkIdent& id, const uint32_t* offs, const uint64_t* total, int64_t nwg, uint64_t* part,
                          int* err, const HkResOut& O, uint64_t* scratch);
template <class S>
hipError_t hk_scalar_shape(hipStream_t st, const HkPlan& P, const HkAggTable& T, int mem, int pred, int ht, int hash,
                           int strat, int64_t groups, int32_t wg, const HkIdent& id);
template <class S>
hipError_t hk_mp_filter_shape(hipStream_t st, const HkPlan& P, int mem, int pred, int ht, int hash, int64_t threads,
                              uint64_t* masks, uint32_t* counts, int unroll, int simd);
template <class S>
hipError_t hk_mp_project_shape(hipStream_t st, const HkPlan& P, int mem, int pred, int ht, int hash, int64_t threads,
                               const uint64_t* masks, const uint32_t* offsets, const uint64_t* total, int64_t nact,
                               const HkOut& O);
template <class S>
hipError_t hk_sp_shape(hipStream_t st, const HkPlan& P, int mem, int pred, int ht, int hash, int64_t instances,
                       const HkOut& O, int64_t region, uint32_t* counts);

#define BY_SHAPE(P, CALL)                                  \
  switch (hk_shape_of(P)) {                                \
    case HK_SHAPE_A: { using S = HkShapeA; return CALL; }  \
    case HK_SHAPE_F: { using S = HkShapeF; return CALL; }  \
    case HK_SHAPE_J: { using S = HkShapeJ; return CALL; }  \
    case HK_SHAPE_W: { using S = HkShapeW; return CALL; }  \
    default: { using S = HkShapeG; return CALL; }          \
  }

static HkIdent make_ident(const uint64_t* ident, int32_t nw) {
  HkIdent id = {};
  for (int i = 0; i < nw; ++i) id.w[i] = ident[i];
  id.nw = nw;
  return id;
}

hipError_t hk_agg(hipStream_t st, const HkPlan& P, const HkAggTable& T, int mem, int pred, int ht, int hash, int strat,
                  int64_t groups, int32_t wg, uint32_t llog2, const uint64_t* ident, int32_t nw, int* err,
                  const HkSpill* sp, int32_t reps) {
  const HkIdent id = make_ident(ident, nw);
  BY_SHAPE(P, hk_agg_shape<S>(st, P, T, mem, pred, ht, hash, strat, groups, wg, llog2, id, err, sp, reps));
}

hipError_t hk_spill(hipStream_t st, int step, const HkPlan& P, const HkAggTable& T, int hash, const HkSpill& sp,
                    const uint64_t* ident, int32_t nw, const uint32_t* offs, const uint64_t* total, int64_t nwg,
                    uint64_t* part, int* err, const HkResOut* out, uint64_t* scratch) {
  const HkIdent id = make_ident(ident, nw);
  HkResOut O;
  std::memset(&O, 0, sizeof(O));
  if (out) {
    if (!scratch || !out->nrows) return hipErrorInvalidValue;
    O = *out;
  }
  BY_SHAPE(P, hk_spill_shape<S>(st, step, P, T, hash, sp, id, offs, total, nwg, part, err, O, scratch));
}

hipError_t hk_scalar_agg(hipStream_t st, const HkPlan& P, const HkAggTable& T, int mem, int pred, int ht, int hash,
                         int strat, int64_t groups, int32_t wg, const uint64_t* ident, int32_t nw, int* err) {
  (void)err;
  const HkIdent id = make_ident(ident, nw);
  BY_SHAPE(P, hk_scalar_shape<S>(st, P, T, mem, pred, ht, hash, strat, groups, wg, id));
}

hipError_t hk_mp_filter(hipStream_t st, const HkPlan& P, int mem, int pred, int ht, int hash, int64_t threads,
                        uint64_t* masks, uint32_t* counts, int unroll, int simd) {
  BY_SHAPE(P, hk_mp_filter_shape<S>(st, P, mem, pred, ht, hash, threads, masks, counts, unroll, simd));
}

hipError_t hk_mp_project(hipStream_t st, const HkPlan& P, int mem, int pred, int ht, int hash, int64_t threads,
                         const uint64_t* masks, const uint32_t* offsets, const uint64_t* total, int64_t nact,
                         int64_t* const* out, int64_t dump) {
  HkOut O = {};
  for (int c = 0; c < P.nproj; ++c) O.col[c] = out[c];
  O.dump = dump;
  BY_SHAPE(P, hk_mp_project_shape<S>(st, P, mem, pred, ht, hash, threads, masks, offsets, total, nact, O));
}

hipError_t hk_sp(hipStream_t st, const HkPlan& P, int mem, int pred, int ht, int hash, int64_t instances,
                 int64_t* const* tmp, int64_t region, uint32_t* counts) {
  HkOut O = {};
  for (int c = 0; c < P.nproj; ++c) O.col[c] = tmp[c];
  BY_SHAPE(P, hk_sp_shape<S>(st, P, mem, pred, ht, hash, instances, O, region, counts));
}
