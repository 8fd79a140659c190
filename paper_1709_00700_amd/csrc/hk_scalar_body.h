// Body of the AGGREGATE kernel without grouping attributes (Table 1). As in
// the paper's AGGREGATE fragment (Section 7.4), every thread keeps its own
// running aggregates in registers while it walks its rows; at the end each
// thread merges them once, into its workgroup's LDS slot (local strategy,
// then one merge per workgroup into the global slot) or straight into the
// single global slot (global strategy). The ahead-of-time kernels
// (hk_scalar.hip) call it with the plan as a kernel argument; a kernel
// compiled at run time for one plan calls it with the plan's structure as
// constants.
#pragma once
#include "hawk_device.h"

template <bool LDS>
__device__ __forceinline__ void merge_partial(uint64_t* tgt, const HkPlan& P, uint64_t cnt, const uint64_t* lo,
                                              const int64_t* hi) {
  at_add<LDS>(tgt + 1, cnt);
#pragma unroll
  for (int a = 0; a < HK_MAX_AGGS; ++a) {
    if (a >= P.naggs) break;
    const HkAgg& A = P.aggs[a];
    uint64_t* w = tgt + A.word;
    if (A.fn == HK_SUM || A.fn == HK_AVG) {
      if (A.wide) at_add128_pair<LDS>(w, w + 1, lo[a], hi[a]);
      else at_add<LDS>(w, lo[a]);
    } else if (A.fn == HK_MIN) {
      at_min<LDS>(w, static_cast<int64_t>(lo[a]));
    } else if (A.fn == HK_MAX) {
      at_max<LDS>(w, static_cast<int64_t>(lo[a]));
    }
  }
}

template <int MEM, int PRED, int HT, int HASH, int STRAT, class S>
__device__ __forceinline__ void scalar_body(const HkPlan& P, const HkAggTable& T, const HkIdent& id, int64_t nwg) {
  const int64_t wgid = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  if (wgid >= nwg) return;  // padding workgroup of a 2-D grid
  if (wg_without_rows<MEM>(P.nrows, wgid, nwg, blockDim.x)) return;  // nothing to fold
  __shared__ uint64_t lw[2 + 2 * HK_MAX_AGGS];
  if (STRAT == HK_LOCAL) {
    if (threadIdx.x == 0)
      for (int j = 0; j < id.nw; ++j) lw[j] = id.w[j];
    __syncthreads();
  }
  uint64_t cnt = 0;
  uint64_t lo[HK_MAX_AGGS];
  int64_t hi[HK_MAX_AGGS];
#pragma unroll
  for (int a = 0; a < HK_MAX_AGGS; ++a) {
    const int fn = a < P.naggs ? P.aggs[a].fn : 0;
    lo[a] = fn == HK_MIN ? static_cast<uint64_t>(INT64_MAX) : (fn == HK_MAX ? static_cast<uint64_t>(INT64_MIN) : 0ull);
    hi[a] = 0;
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
    cnt += PRED == HK_PRED ? static_cast<uint64_t>(pass) : 1ull;
#pragma unroll
    for (int a = 0; a < S::aggs; ++a) {
      if (a >= P.naggs) break;
      const HkAgg& A = P.aggs[a];
      const int64_t x = r[A.reg];
      if (A.fn == HK_SUM || A.fn == HK_AVG) {
        // predication: a dropped row adds x * result_increment = 0
        const uint64_t v = static_cast<uint64_t>(PRED == HK_PRED ? (pass ? x : 0) : x);
        const uint64_t old = lo[a];
        lo[a] = old + v;
        hi[a] += static_cast<int64_t>(lo[a] < old) - static_cast<int64_t>(v >> 63);
      } else if (A.fn == HK_MIN) {
        const int64_t v = PRED == HK_PRED ? (pass ? x : INT64_MAX) : x;
        lo[a] = static_cast<uint64_t>(v < static_cast<int64_t>(lo[a]) ? v : static_cast<int64_t>(lo[a]));
      } else if (A.fn == HK_MAX) {
        const int64_t v = PRED == HK_PRED ? (pass ? x : INT64_MIN) : x;
        lo[a] = static_cast<uint64_t>(v > static_cast<int64_t>(lo[a]) ? v : static_cast<int64_t>(lo[a]));
      }
    }
  }
  if (STRAT == HK_LOCAL) {
    merge_partial<true>(lw, P, cnt, lo, hi);
    __syncthreads();
    if (threadIdx.x == 0) agg_merge<S>(T.words, lw, 1, P);
  } else {
    merge_partial<false>(T.words, P, cnt, lo, hi);
  }
}

