// Grouped aggregation (HASH_AGGREGATE, Section 4.2), global hash-table strategy.
#include <hip/hip_runtime.h>

#include "hawk_device.h"
#include "hawk_launch.h"

#define HK_CHECK_LAUNCH() return hipGetLastError()

hipError_t hk_agg_local(hipStream_t st, const HkPlan& P, const HkPlan* dP, const HkAggTable& T, int mem, int pred, int ht, int hash,
                        int64_t groups, int32_t wg, uint32_t llog2, const HkIdent& id, int* err);
hipError_t hk_agg_global(hipStream_t st, const HkPlan& P, const HkPlan* dP, const HkAggTable& T, int mem, int pred, int ht, int hash,
                         int64_t groups, int32_t wg, uint32_t llog2, const HkIdent& id, int* err);

template <int MEM, int PRED, int HT, int HASH, int STRAT>
__global__ void __launch_bounds__(1024) k_agg(const HkPlan* Pp, HkAggTable T, uint32_t llog2, HkIdent id, int64_t nwg,
                                              int* err) {
  const HkPlan& P = *Pp;  // plan in device memory, read where used
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
    const bool pass = eval_row<PRED, HT, HASH, true>(P, row, r);
    if (PRED == HK_BR && !pass) continue;
    const uint64_t key = group_key(P, r);
    if (STRAT == HK_LOCAL && key != HK_EMPTY) {
      const int32_t s = lslot<HT, HASH>(lds, llog2, P.hash, key);
      if (s >= 0) {
        agg_apply<PRED, true>(lds + s, LC, P, r, pass);
        continue;
      }
    }
    uint64_t* g = gslot<HT, HASH>(T, P.hash, key, err);
    if (g) agg_apply<PRED, false>(g, 1, P, r, pass);
  }
  if (STRAT == HK_LOCAL) {
    __syncthreads();
    for (int64_t s = threadIdx.x; s < LC; s += blockDim.x) {
      const uint64_t key = lds[s];
      if (key == HK_EMPTY || lds[LC + s] == 0) continue;
      uint64_t* g = gslot<HT, HASH>(T, P.hash, key, err);
      if (g) agg_merge(g, lds + s, LC, P);
    }
  }
}


hipError_t hk_agg_global(hipStream_t st, const HkPlan& P, const HkPlan* dP, const HkAggTable& T, int mem, int pred, int ht, int hash,
                      int64_t groups, int32_t wg, uint32_t llog2, const HkIdent& id, int* err) {
  const dim3 g = hk_wg_grid(groups), b(static_cast<uint32_t>(wg));
  const size_t lds = 0;
  DISPATCH2(mem, M, DISPATCH2(pred, PR, DISPATCH2(ht, HT, DISPATCH2(hash, HS,
            hipLaunchKernelGGL((k_agg<M, PR, HT, HS, 1>), g, b, lds, st, dP, T, llog2, id, groups, err)))));
  HK_CHECK_LAUNCH();
}

// cuckoo aggregation, phase 1: insert every group key that reaches the sink
template <int MEM, int PRED, int HASH>
__global__ void __launch_bounds__(256) k_agg_keys(const HkPlan* Pp, HkAggTable T, int* err) {
  const HkPlan& P = *Pp;  // plan in device memory, read where used
  v16i64 r = {};
  const int64_t n = P.nrows;
  const int64_t Tn = (int64_t)gridDim.x * blockDim.x;
  const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t b, e, step;
  if (MEM == HK_COAL) { b = gt; e = n; step = Tn; }
  else { seq_range(n, gt, Tn, 1, b, e); step = 1; }
  for (int64_t row = b; row < e; row += step) {
    const bool pass = eval_row<PRED, HK_CUCKOO, HASH, true>(P, row, r);
    if (PRED == HK_BR && !pass) continue;
    gkey_cuckoo_insert<HASH>(T, P.hash, group_key(P, r), err);
  }
}

hipError_t hk_agg_keys(hipStream_t st, const HkPlan& P, const HkPlan* dP, const HkAggTable& T, int mem, int pred, int hash, int* err) {
  const dim3 gk(hk_grid_for(P.nrows, 256, 8192)), bk(256);
  DISPATCH2(mem, M, DISPATCH2(pred, PR, DISPATCH2(hash, HS,
            hipLaunchKernelGGL((k_agg_keys<M, PR, HS>), gk, bk, 0, st, dP, T, err))));
  HK_CHECK_LAUNCH();
}

hipError_t hk_agg(hipStream_t st, const HkPlan& P, const HkPlan* dP, const HkAggTable& T, int mem, int pred, int ht, int hash,
                  int strat, int64_t groups, int32_t wg, uint32_t llog2, const uint64_t* ident, int32_t nw, int* err) {
  HkIdent id = {};
  for (int i = 0; i < nw; ++i) id.w[i] = ident[i];
  id.nw = nw;
  if (ht == HK_CUCKOO) {
    hipError_t e = hk_agg_keys(st, P, dP, T, mem, pred, hash, err);
    if (e != hipSuccess) return e;
  }
  if (strat == HK_LOCAL) return hk_agg_local(st, P, dP, T, mem, pred, ht, hash, groups, wg, llog2, id, err);
  return hk_agg_global(st, P, dP, T, mem, pred, ht, hash, groups, wg, llog2, id, err);
}
