// Grouped aggregation (HASH_AGGREGATE, Section 4.2): local (per-workgroup LDS
// tables merged into a global table) and global (one table) strategies,
// linear probing or cuckoo hashing (whose keys are inserted first by
// k_agg_keys). Compiled once per shape class: the build passes
// -DHK_SHAPE_CLASS=HkShapeX and this file instantiates hk_agg_shape for it.
#include <hip/hip_runtime.h>

#include <cstring>

#include "hawk_device.h"
#include "hawk_launch.h"

#ifndef HK_SHAPE_CLASS
#error "compile once per shape class with -DHK_SHAPE_CLASS=HkShapeX"
#endif

// The local table in LDS: keys[LC], then for each word j >= 1 (count,
// aggregates) `reps` copies of the LC slots, RS words apart (padded by one
// word when reps > 1 so the copies of a slot sit in different banks). Lane l
// updates copy l % reps: lanes of one instruction that hit the same group
// then mostly hit different addresses. The copies are folded before the
// table is merged into the global table.
template <int MEM, int PRED, int HT, int HASH, int STRAT, class S, bool SPILL>
__global__ void __launch_bounds__(1024) k_agg(HkPlan P, HkAggTable T, uint32_t llog2, HkIdent id, int64_t nwg,
                                              int* err, HkSpill sp, int32_t reps) {
  // workgroups may come as a 2-D grid (HSA counts grid sizes in work-items as 32-bit values)
  const int64_t wgid = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  if (wgid >= nwg) return;  // padding workgroup: leaves before any barrier
  // a workgroup without rows has nothing to aggregate (spill mode: its
  // histogram column and count are still written, as zeros)
  if (wg_without_rows<MEM>(P.nrows, wgid, nwg, blockDim.x)) {
    if (SPILL) {
      for (int p = threadIdx.x; p < sp.nparts; p += blockDim.x) sp.hist[static_cast<int64_t>(p) * nwg + wgid] = 0;
      if (threadIdx.x == 0) sp.cnt[wgid] = 0;
    }
    return;
  }
  extern __shared__ uint64_t lds[];
  __shared__ uint32_t spill_cursor;
  const int64_t LC = STRAT == HK_LOCAL ? (static_cast<int64_t>(1) << llog2) : 0;
  const int64_t RS = reps > 1 ? LC + 1 : LC;
  const int64_t WS = reps * RS;  // from word j to word j + 1 of one copy
  uint64_t* lw1 = lds + LC;      // word 1 of copy 0 of slot 0
  const int64_t q = __lane_id() & (reps - 1);
  // spill mode: the partition histogram follows the LDS table
  uint32_t* hist = reinterpret_cast<uint32_t*>(lds + LC + (id.nw - 1) * WS);
  uint32_t* cursor = &spill_cursor;
  if (STRAT == HK_LOCAL) {
    for (int64_t i = threadIdx.x; i < LC; i += blockDim.x) lds[i] = id.w[0];
    for (int w = 1; w < id.nw; ++w)
      for (int64_t i = threadIdx.x; i < WS; i += blockDim.x) lw1[(w - 1) * WS + i] = id.w[w];
    if (SPILL) {
      for (int i = threadIdx.x; i < sp.nparts; i += blockDim.x) hist[i] = 0;
      if (threadIdx.x == 0) *cursor = 0;
    }
    __syncthreads();
  }
  v16i64 r = {};
  const int64_t n = P.nrows;
  const int64_t Tn = nwg * blockDim.x;
  const int64_t gt = wgid * blockDim.x + threadIdx.x;
  int64_t b, e, step;
  if (MEM == HK_COAL) { b = gt; e = n; step = Tn; }
  else { seq_range(n, gt, Tn, 1, b, e); step = 1; }
  int64_t rcap = 0;
  uint64_t* region = nullptr;
  if (SPILL) {
    const int64_t r0 = spill_region_start(sp, nwg, wgid);
    rcap = spill_region_start(sp, nwg, wgid + 1) - r0;
    region = sp.buf + r0 * sp.ew;
  }
  auto row_step = [&](int64_t row, const HkFirst<S>& f) {
    const bool pass = eval_row_f<PRED, HT, HASH, true, S, true>(P, row, f, r);
    bool spill = false;
    uint64_t key = 0;
    if (PRED != HK_BR || pass) {
      key = group_key(P, r);
      bool done = false;
      if (STRAT == HK_LOCAL && key != HK_EMPTY) {
        const int32_t s = lslot<HT, HASH>(lds, llog2, P.hash, key);
        if (s >= 0) {
          agg_apply_w1<PRED, true, S>(lw1 + q * RS + s, WS, P, r, pass);
          done = true;
        }
      }
      if (!done) {
        if (SPILL && key != HK_EMPTY) {
          spill = pass;  // a predicated row that did not pass contributes nothing
        } else {
          uint64_t* g = gslot<HT, HASH>(T, P.hash, key, err);
          if (g) agg_apply<PRED, false, S>(g, 1, P, r, pass);
          // this path's returning atomics end here: the rows fetched ahead
          // then stay in flight on the common path
          __builtin_amdgcn_s_waitcnt(0);
        }
      }
    }
    if (SPILL) {
      // one LDS cursor update per wave: the spilled lanes write consecutive entries
      const uint64_t m = __ballot(spill);
      if (m) {
        const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
        uint32_t base = 0;
        if (__lane_id() == leader) base = atomicAdd(cursor, static_cast<uint32_t>(__popcll(m)));
        base = __shfl(base, leader, WAVE);
        if (spill) {
          const int64_t pos = static_cast<int64_t>(base) + __popcll(m & lanemask_lt());
          if (pos < rcap) {
            uint64_t* ent = region + pos * sp.ew;
            ent[0] = key;
            for (int j = 0; j < sp.ncols; ++j) ent[1 + j] = static_cast<uint64_t>(r[sp.reg[j]]);
            atomicAdd(&hist[hslot<HASH>(key, P.hash.a[0], T.log2cap) >> T.rlog2], 1u);
          } else {
            set_err(err, HK_ERR_CAPACITY);  // never expected: a region holds every row its workgroup scans
          }
        }
      }
    }
  };
  // software pipeline over the thread's rows: the first load phase of the
  // next AH rows is in flight while a row is evaluated. The loop is unrolled
  // by the ring size so every buffer index is a constant (no register copies,
  // which would wait for the loads in flight).
  constexpr int AH = HkFirst<S>::A + HkFirst<S>::B + HkFirst<S>::C <= 3 ? 3 : 1;
  constexpr int NB = AH + 1;
  HkFirst<S> f[NB] = {};
  // rows past the thread's range fetch its last row again (the fetch count
  // stays fixed); a thread without rows fetches nothing
  const int64_t last = e - 1;
  if (b < e) {
#pragma unroll
    for (int k = 0; k < AH; ++k) fetch_first<S>(P, b + k * step < e ? b + k * step : last, f[k]);
  }
  for (int64_t row = b; row < e; row += NB * step) {
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int64_t rk = row + k * step;
      if (rk >= e) break;
      const int64_t ahead = rk + AH * step;
      fetch_first<S>(P, ahead < e ? ahead : last, f[(k + AH) % NB]);
      row_step(rk, f[k]);
    }
  }
  if (STRAT == HK_LOCAL) {
    __syncthreads();
    for (int64_t s = threadIdx.x; s < LC; s += blockDim.x) {
      const uint64_t key = lds[s];
      if (key == HK_EMPTY) continue;
      uint64_t* c0 = lw1 + s;
      for (int32_t c = 1; c < reps; ++c) agg_fold_w1<S>(c0, c0 + c * RS, WS, P);
      if (c0[0] == 0) continue;  // only predicated rows that did not pass reached this group
      uint64_t* g = gslot<HT, HASH>(T, P.hash, key, err);
      if (g) agg_merge_w1<S>(g, c0, WS, P);
    }
    if (SPILL) {
      for (int p = threadIdx.x; p < sp.nparts; p += blockDim.x) sp.hist[static_cast<int64_t>(p) * nwg + wgid] = hist[p];
      if (threadIdx.x == 0) sp.cnt[wgid] = *cursor < rcap ? *cursor : static_cast<uint32_t>(rcap);
    }
  }
}

// spill, step 2: each workgroup moves its region's entries to their
// partitions (offsets = exclusive scan of the partition-major histogram)
template <int HASH>
__global__ void __launch_bounds__(256) k_spill_scatter(HkSpill sp, const uint32_t* __restrict__ offs, int64_t nwg,
                                                       HkHash h, uint32_t log2cap, uint32_t rlog2,
                                                       uint64_t* __restrict__ out) {
  const int64_t wgid = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  if (wgid >= nwg) return;
  extern __shared__ uint32_t cur[];
  for (int p = threadIdx.x; p < sp.nparts; p += blockDim.x) cur[p] = offs[static_cast<int64_t>(p) * nwg + wgid];
  __syncthreads();
  const int64_t cnt = sp.cnt[wgid];
  const uint64_t* region = sp.buf + spill_region_start(sp, nwg, wgid) * sp.ew;
  for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) {
    const uint64_t* ent = region + i * sp.ew;
    const uint64_t key = ent[0];
    const uint32_t pos = atomicAdd(&cur[hslot<HASH>(key, h.a[0], log2cap) >> rlog2], 1u);
    uint64_t* dst = out + static_cast<int64_t>(pos) * sp.ew;
    dst[0] = key;
    for (int j = 0; j < sp.ncols; ++j) dst[1 + j] = ent[1 + j];
  }
}

// spill, step 3: workgroup p owns table region p for the whole kernel: it
// copies the region into LDS, aggregates partition p's entries there (LDS
// atomics, probing confined to the region as in the table) and writes the
// region back
template <int HASH, class S>
__global__ void __launch_bounds__(256) k_spill_agg(HkPlan P, HkAggTable T, HkSpill sp, const uint32_t* __restrict__ offs,
                                                   const uint64_t* total, int64_t nwg, const uint64_t* __restrict__ in,
                                                   int* err) {
  const int64_t p = blockIdx.x;
  const int64_t b = offs[p * nwg];
  const int64_t e = p + 1 < sp.nparts ? static_cast<int64_t>(offs[(p + 1) * nwg]) : static_cast<int64_t>(*total);
  if (b >= e) return;  // nothing spilled here (uniform over the workgroup)
  extern __shared__ uint64_t lt[];  // word w of region slot i at lt[w * R + i]
  const int64_t R = static_cast<int64_t>(1) << T.rlog2;
  const int W = T.slot_words;
  uint64_t* g = T.words + p * R * W;
  for (int64_t i = threadIdx.x; i < R * W; i += blockDim.x) lt[(i % W) * R + i / W] = g[i];
  __syncthreads();
  const uint32_t rmask = static_cast<uint32_t>(R - 1);
  v16i64 r = {};
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
    const uint64_t* ent = in + i * sp.ew;
    const uint64_t key = ent[0];
    for (int j = 0; j < sp.ncols; ++j) r[sp.reg[j]] = static_cast<long long>(ent[1 + j]);
    uint32_t s = hslot<HASH>(key, P.hash.a[0], T.log2cap) & rmask;
    int32_t found = -1;
    for (uint32_t k = 0; k <= rmask; ++k) {
      uint64_t cur = lt[s];
      if (cur == HK_EMPTY) cur = at_cas<true>(&lt[s], HK_EMPTY, key);
      if (cur == HK_EMPTY || cur == key) {
        found = static_cast<int32_t>(s);
        break;
      }
      s = (s + 1) & rmask;
    }
    if (found < 0) {
      set_err(err, HK_ERR_CAPACITY);  // the region is full: the caller retries with a larger table
      continue;
    }
    agg_apply<HK_BR, true, S>(lt + found, R, P, r, true);
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < R * W; i += blockDim.x) g[i] = lt[(i % W) * R + i / W];
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
                        int strat, int64_t groups, int32_t wg, uint32_t llog2, const HkIdent& id, int* err,
                        const HkSpill* sp, int32_t reps) {
  if (reps < 1 || reps > 64 || (reps & (reps - 1)) != 0) return hipErrorInvalidValue;
  if (ht == HK_CUCKOO) {
    const dim3 gk(hk_grid_for(P.nrows, 256, 8192)), bk(256);
    DISPATCH2(mem, M, DISPATCH2(pred, PR, DISPATCH2(hash, HS,
              hipLaunchKernelGGL((k_agg_keys<M, PR, HS, S>), gk, bk, 0, st, P, T, err))));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const dim3 g = hk_wg_grid(groups), b(static_cast<uint32_t>(wg));
  size_t lds = 0;
  if (strat == HK_LOCAL) {
    const size_t LC = static_cast<size_t>(1) << llog2;
    lds = (LC + (id.nw - 1) * reps * (reps > 1 ? LC + 1 : LC)) * sizeof(uint64_t);
  }
  if (sp) {
    // spill mode exists for the local strategy with linear probing
    if (strat != HK_LOCAL || ht != HK_LIN) return hipErrorInvalidValue;
    lds += static_cast<size_t>(sp->nparts) * sizeof(uint32_t);
    const HkSpill S1 = *sp;
    DISPATCH2(mem, M, DISPATCH2(pred, PR, DISPATCH2(hash, HS,
              hipLaunchKernelGGL((k_agg<M, PR, HK_LIN, HS, HK_LOCAL, S, true>), g, b, lds, st, P, T, llog2, id,
                                 groups, err, S1, reps))));
    return hipGetLastError();
  }
  HkSpill none;
  std::memset(&none, 0, sizeof(none));
  DISPATCH2(mem, M, DISPATCH2(pred, PR, DISPATCH2(ht, HT, DISPATCH2(hash, HS, DISPATCH2(strat, SG,
            hipLaunchKernelGGL((k_agg<M, PR, HT, HS, SG, S, false>), g, b, lds, st, P, T, llog2, id, groups, err,
                               none, reps))))));
  return hipGetLastError();
}

template <class S>
hipError_t hk_spill_shape(hipStream_t st, int step, const HkPlan& P, const HkAggTable& T, int hash, const HkSpill& sp,
                          const uint32_t* offs, const uint64_t* total, int64_t nwg, uint64_t* part, int* err) {
  if (step == 0) {
    const size_t lds = static_cast<size_t>(sp.nparts) * sizeof(uint32_t);
    DISPATCH2(hash, HS, hipLaunchKernelGGL((k_spill_scatter<HS>), hk_wg_grid(nwg), dim3(256), lds, st, sp, offs, nwg,
                                           P.hash, T.log2cap, T.rlog2, part));
  } else {
    const size_t lds = (static_cast<size_t>(1) << T.rlog2) * T.slot_words * sizeof(uint64_t);
    DISPATCH2(hash, HS, hipLaunchKernelGGL((k_spill_agg<HS, S>), dim3(static_cast<uint32_t>(sp.nparts)), dim3(256),
                                           lds, st, P, T, sp, offs, total, nwg, part, err));
  }
  return hipGetLastError();
}

template hipError_t hk_agg_shape<HK_SHAPE_CLASS>(hipStream_t, const HkPlan&, const HkAggTable&, int, int, int, int, int,
                                                 int64_t, int32_t, uint32_t, const HkIdent&, int*, const HkSpill*,
                                                 int32_t);
template hipError_t hk_spill_shape<HK_SHAPE_CLASS>(hipStream_t, int, const HkPlan&, const HkAggTable&, int, const HkSpill&,
                                                   const uint32_t*, const uint64_t*, int64_t, uint64_t*, int*);
