// Grouped aggregation (HASH_AGGREGATE, Section 4.2): local (per-workgroup LDS
// tables merged into a global table) and global (one table) strategies,
// linear probing or cuckoo hashing (whose keys are inserted first by
// k_agg_keys). Compiled once per shape class: the build passes
// -DHK_SHAPE_CLASS=HkShapeX and this file instantiates hk_agg_shape for it.
#include <hip/hip_runtime.h>

#include "hawk_device.h"
#include "hawk_launch.h"

#ifndef HK_SHAPE_CLASS
#error "compile once per shape class with -DHK_SHAPE_CLASS=HkShapeX"
#endif

template <int MEM, int PRED, int HT, int HASH, int STRAT, class S>
__global__ void __launch_bounds__(1024) k_agg(HkPlan P, HkAggTable T, uint32_t llog2, HkIdent id, int64_t nwg,
                                              int* err) {
  // workgroups may come as a 2-D grid (HSA counts grid sizes in work-items as 32-bit values)
  const int64_t wgid = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  if (wgid >= nwg) return;  // padding workgroup: leaves before any barrier
  extern __shared__ uint64_t lds[];
  const int64_t LC = STRAT == HK_LOCAL ? (static_cast<int64_t>(1) << llog2) : 0;
  if (STRAT == HK_LOCAL) {
    for (int w = 0; w < id.nw; ++w)
      for (int64_t i = threadIdx.x; i < LC; i += blockDim.x) lds[w * LC + i] = id.w[w];
    __syncthreads();
  }
  v16i64 r = {};
  const int64_t n = P.nrows;
  const int64_t Tn = nwg * blockDim.x;
  const int64_t gt = wgid * blockDim.x + threadIdx.x;
  int64_t b, e, step;
  if (MEM == HK_COAL) { b = gt; e = n; step = Tn; }
  else { seq_range(n, gt, Tn, 1, b, e); step = 1; }
  for (int64_t row = b; row < e; row += step) {
    const bool pass = eval_row<PRED, HT, HASH, true, S>(P, row, r);
    if (PRED == HK_BR && !pass) continue;
    const uint64_t key = group_key(P, r);
    if (STRAT == HK_LOCAL && key != HK_EMPTY) {
      const int32_t s = lslot<HT, HASH>(lds, llog2, P.hash, key);
      if (s >= 0) {
        agg_apply<PRED, true, S>(lds + s, LC, P, r, pass);
        continue;
      }
    }
    uint64_t* g = gslot<HT, HASH>(T, P.hash, key, err);
    if (g) agg_apply<PRED, false, S>(g, 1, P, r, pass);
  }
  if (STRAT == HK_LOCAL) {
    __syncthreads();
    for (int64_t s = threadIdx.x; s < LC; s += blockDim.x) {
      const uint64_t key = lds[s];
      if (key == HK_EMPTY || lds[LC + s] == 0) continue;
      uint64_t* g = gslot<HT, HASH>(T, P.hash, key, err);
      if (g) agg_merge<S>(g, lds + s, LC, P);
    }
  }
}


// cuckoo aggregation, phase 1: insert every group key that reaches the sink
template <int MEM, int PRED, int HASH, class S>
__global__ void __launch_bounds__(256) k_agg_keys(HkPlan P, HkAggTable T, int* err) {
  v16i64 r = {};
  const int64_t n = P.nrows;
  const int64_t Tn = (int64_t)gridDim.x * blockDim.x;
  const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t b, e, step;
  if (MEM == HK_COAL) { b = gt; e = n; step = Tn; }
  else { seq_range(n, gt, Tn, 1, b, e); step = 1; }
  for (int64_t row = b; row < e; row += step) {
    const bool pass = eval_row<PRED, HK_CUCKOO, HASH, true, S>(P, row, r);
    if (PRED == HK_BR && !pass) continue;
    gkey_cuckoo_insert<HASH>(T, P.hash, group_key(P, r), err);
  }
}

template <class S>
hipError_t hk_agg_shape(hipStream_t st, const HkPlan& P, const HkAggTable& T, int mem, int pred, int ht, int hash,
                        int strat, int64_t groups, int32_t wg, uint32_t llog2, const HkIdent& id, int* err) {
  if (ht == HK_CUCKOO) {
    const dim3 gk(hk_grid_for(P.nrows, 256, 8192)), bk(256);
    DISPATCH2(mem, M, DISPATCH2(pred, PR, DISPATCH2(hash, HS,
              hipLaunchKernelGGL((k_agg_keys<M, PR, HS, S>), gk, bk, 0, st, P, T, err))));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const dim3 g = hk_wg_grid(groups), b(static_cast<uint32_t>(wg));
  const size_t lds = strat == HK_LOCAL ? (static_cast<size_t>(1) << llog2) * id.nw * sizeof(uint64_t) : 0;
  DISPATCH2(mem, M, DISPATCH2(pred, PR, DISPATCH2(ht, HT, DISPATCH2(hash, HS, DISPATCH2(strat, SG,
            hipLaunchKernelGGL((k_agg<M, PR, HT, HS, SG, S>), g, b, lds, st, P, T, llog2, id, groups, err))))));
  return hipGetLastError();
}

template hipError_t hk_agg_shape<HK_SHAPE_CLASS>(hipStream_t, const HkPlan&, const HkAggTable&, int, int, int, int, int,
                                                 int64_t, int32_t, uint32_t, const HkIdent&, int*);
