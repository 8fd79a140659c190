// AGGREGATE without grouping attributes (Table 1), compiled once per shape
// class; the body is in hk_scalar_body.h.
#include <hip/hip_runtime.h>

#include "hawk_device.h"
#include "hawk_launch.h"
#include "hk_scalar_body.h"

#ifndef HK_SHAPE_CLASS
#error "compile once per shape class with -DHK_SHAPE_CLASS=HkShapeX"
#endif

template <int MEM, int PRED, int HT, int HASH, int STRAT, class S>
__global__ void __launch_bounds__(1024) k_scalar_agg(HkPlan P, HkAggTable T, HkIdent id, int64_t nwg) {
  scalar_body<MEM, PRED, HT, HASH, STRAT, S>(P, T, id, nwg);
}

template <class S>
hipError_t hk_scalar_shape(hipStream_t st, const HkPlan& P, const HkAggTable& T, int mem, int pred, int ht, int hash,
                           int strat, int64_t groups, int32_t wg, const HkIdent& id) {
  const dim3 g = hk_wg_grid(groups), b(static_cast<uint32_t>(wg));
  DISPATCH2(mem, M, DISPATCH2(pred, PR, DISPATCH2(ht, HT, DISPATCH2(hash, HS, DISPATCH2(strat, SG,
            hipLaunchKernelGGL((k_scalar_agg<M, PR, HT, HS, SG, S>), g, b, 0, st, P, T, id, groups))))));
  return hipGetLastError();
}

template hipError_t hk_scalar_shape<HK_SHAPE_CLASS>(hipStream_t, const HkPlan&, const HkAggTable&, int, int, int, int, int,
                                                    int64_t, int32_t, const HkIdent&);
