// Body of the grouped-aggregation kernel (HASH_AGGREGATE, Section 4.2) for
// one variant: local strategy (per-workgroup LDS tables merged into the
// global table, with spilling of LDS misses) or global strategy (every row
// updates the global table). The ahead-of-time kernels (hk_agg.hip) call it
// with the plan as a kernel argument; a kernel compiled at run time for one
// plan calls it with the plan's structure as constants.
#pragma once
#include "hawk_device.h"

// The local table in LDS: keys[LC], then for each word j >= 1 (count,
// aggregates) the slots' `reps` copies side by side (copy c of slot s at
// s * reps + c). Lane l updates copy l % reps: lanes of one instruction that
// hit the same group then hit different addresses, and with 32 or more
// copies every lane's word sits in a bank of its own whichever slots the
// lanes hit. The copies are folded (a tree over the workgroup) before the
// table is merged into the global table.
template <int MEM, int PRED, int HT, int HASH, int STRAT, class S, bool SPILL>
__device__ __forceinline__ void agg_body(const HkPlan& P, const HkAggTable& T, uint32_t llog2, const HkIdent& id,
                                         int64_t nwg, int* err, const HkSpill& sp, int32_t reps, uint64_t* lds) {
  // workgroups may come as a 2-D grid (HSA counts grid sizes in work-items as 32-bit values)
  const int64_t wgid = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  if (wgid >= nwg) return;  // padding workgroup: leaves before any barrier
  // a workgroup without rows has nothing to aggregate (spill mode: its
  // histogram column and count are still written, as zeros)
  if (wg_without_rows<MEM>(P.nrows, wgid, nwg, blockDim.x)) {
    if (SPILL) {
      for (int p = threadIdx.x; p < sp.nparts; p += blockDim.x) sp.hist[static_cast<int64_t>(p) * nwg + wgid] = 0;
      if (sp.merge)
        for (int p = threadIdx.x; p <= sp.nparts; p += blockDim.x) sp.foffs[wgid * (sp.nparts + 1) + p] = 0;
      if (threadIdx.x == 0) sp.cnt[wgid] = 0;
    }
    return;
  }
  __shared__ uint32_t spill_cursor;
  __shared__ uint32_t wave_tot[1024 / WAVE];
  const int64_t LC = STRAT == HK_LOCAL ? (static_cast<int64_t>(1) << llog2) : 0;
  const int64_t WS = reps * LC;  // from word j to word j + 1 of one copy
  uint64_t* lw1 = lds + LC;      // word 1 of copy 0 of slot 0
  const int64_t q = __lane_id() & (reps - 1);
  // spill mode: the partition histogram follows the LDS table, then the
  // admission filter's words
  uint32_t* hist = reinterpret_cast<uint32_t*>(lds + LC + (id.nw - 1) * WS);
  uint32_t* door = hist + (SPILL ? sp.nparts : 0);
  const uint32_t dl2 = SPILL && sp.door_log2 > 0 ? static_cast<uint32_t>(sp.door_log2) : 0u;
  uint32_t* cursor = &spill_cursor;
  if (STRAT == HK_LOCAL) {
    for (int64_t i = threadIdx.x; i < LC; i += blockDim.x) lds[i] = id.w[0];
    for (int w = 1; w < id.nw; ++w)
      for (int64_t i = threadIdx.x; i < WS; i += blockDim.x) lw1[(w - 1) * WS + i] = id.w[w];
    if (SPILL) {
      for (int i = threadIdx.x; i < sp.nparts; i += blockDim.x) hist[i] = 0;
      for (int i = threadIdx.x; i < (dl2 ? (1 << dl2) / 32 : 0); i += blockDim.x) door[i] = 0;
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
  int64_t rcap = 0, r0 = 0;
  uint64_t* region = nullptr;
  if (SPILL) {
    r0 = spill_region_start(sp, nwg, wgid);
    rcap = spill_region_start(sp, nwg, wgid + 1) - r0;
    region = sp.buf + r0 * sp.ew;  // (entries of ew words)
  }
  // the aggregation of one evaluated row (registers rr, result_increment pass)
  auto agg_row = [&](const v16i64& rr, bool pass) {
    bool spill = false;
    uint64_t key = 0;
    if (PRED != HK_BR || pass) {
      key = group_key(P, rr);
      bool done = false;
      if (STRAT == HK_LOCAL && key != HK_EMPTY) {
        const int32_t s = lslot<HT, HASH, SPILL>(lds, llog2, P.hash, key, door, dl2);
        if (s >= 0) {
          agg_apply_w1<PRED, true, S>(lw1 + s * reps + q, WS, P, rr, pass);
          done = true;
        }
      }
      if (!done) {
        if (SPILL && key != HK_EMPTY) {
          spill = pass;  // a predicated row that did not pass contributes nothing
        } else {
          uint64_t* g = gslot<HT, HASH>(T, P.hash, key, err);
          if (g) agg_apply<PRED, false, S>(g, 1, P, rr, pass);
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
            if (sp.e12) {
              // consecutive spilling lanes write consecutive keys and values
              HkE12 e3;
              e3.k = static_cast<uint32_t>(key);
              e3.v = static_cast<uint64_t>(rr[sp.reg[0]]);
              SpillArr<HkE12>(sp.buf, sp.nrows, r0).put(pos, e3);
            } else if (sp.ew == 2) {
              // consecutive spilling lanes write consecutive 16-byte entries: one store each
              ulonglong2 e2;
              e2.x = key;
              e2.y = static_cast<uint64_t>(rr[sp.reg[0]]);
              reinterpret_cast<ulonglong2*>(region)[pos] = e2;
            } else {
              uint64_t* ent = region + pos * sp.ew;
              ent[0] = key;
              for (int j = 0; j < sp.ncols; ++j) ent[1 + j] = static_cast<uint64_t>(rr[sp.reg[j]]);
            }
            atomicAdd(&hist[hslot<HASH>(key, P.hash.a[0], T.log2cap) >> T.rlog2], 1u);
          } else {
            set_err(err, HK_ERR_CAPACITY);  // never expected: a region holds every row its workgroup scans
          }
        }
      }
    }
  };
  auto row_step = [&](int64_t row, const HkFirst<S>& f) {
    const bool pass = eval_row_f<PRED, HT, HASH, true, S, true>(P, row, f, r);
    agg_row(r, pass);
  };
  // software pipeline over the thread's rows: the first load phase of the
  // next AH rows is in flight while a row is evaluated (more rows ahead for
  // fewer columns). The loop is unrolled by the ring size so every buffer
  // index is a constant (no register copies, which would wait for the loads
  // in flight).
  constexpr int NF = HkFirst<S>::A + HkFirst<S>::B + HkFirst<S>::C;
  constexpr int AH = NF <= 2 ? 4 : (NF <= 3 ? 3 : 1);
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
    // the copies of each slot folded into copy 0, halving the copies each round
    for (int32_t d = reps >> 1; d >= 1; d >>= 1) {
      __syncthreads();
      const int32_t ld = __ffs(d) - 1;
      for (int64_t i = threadIdx.x; i < (LC << ld); i += blockDim.x) {
        const int64_t s = i >> ld;
        if (lds[s] == HK_EMPTY) continue;
        uint64_t* a = lw1 + s * reps + (i & (d - 1));
        agg_fold_w1<S>(a, a + d, WS, P);
      }
    }
  }
  if (STRAT == HK_LOCAL && (!SPILL || !sp.merge)) {
    __syncthreads();
    for (int64_t s = threadIdx.x; s < LC; s += blockDim.x) {
      const uint64_t key = lds[s];
      if (key == HK_EMPTY) continue;
      const uint64_t* c0 = lw1 + s * reps;
      if (c0[0] == 0) continue;  // only predicated rows that did not pass reached this group
      uint64_t* g = gslot<HT, HASH>(T, P.hash, key, err);
      if (g) agg_merge_w1<S>(g, c0, WS, P);
    }
  }
  if (STRAT == HK_LOCAL && SPILL) {
    // the spill histogram goes out, then (merge entries) the same LDS words
    // count this table's slots by region and, scanned, place them
    __syncthreads();
    for (int p = threadIdx.x; p < sp.nparts; p += blockDim.x) sp.hist[static_cast<int64_t>(p) * nwg + wgid] = hist[p];
    if (threadIdx.x == 0) sp.cnt[wgid] = *cursor < rcap ? *cursor : static_cast<uint32_t>(rcap);
    if (!sp.merge) return;
    __syncthreads();
    for (int p = threadIdx.x; p < sp.nparts; p += blockDim.x) hist[p] = 0;
    __syncthreads();
    for (int64_t s = threadIdx.x; s < LC; s += blockDim.x) {
      const uint64_t key = lds[s];
      if (key == HK_EMPTY) continue;
      if (lw1[s * reps] == 0) continue;  // only predicated rows that did not pass reached this group
      atomicAdd(&hist[hslot<HASH>(key, P.hash.a[0], T.log2cap) >> T.rlog2], 1u);
    }
    __syncthreads();
    wg_exclusive_scan(hist, sp.nparts, sp.foffs + wgid * (sp.nparts + 1), wave_tot);
    const int W = T.slot_words;
    uint64_t* fl = sp.flush + wgid * sp.fcap * W;
    for (int64_t s = threadIdx.x; s < LC; s += blockDim.x) {
      const uint64_t key = lds[s];
      if (key == HK_EMPTY) continue;
      const uint64_t* c0 = lw1 + s * reps;  // copy 0, the folded slot
      if (c0[0] == 0) continue;
      const uint32_t pos = atomicAdd(&hist[hslot<HASH>(key, P.hash.a[0], T.log2cap) >> T.rlog2], 1u);
      uint64_t* ent = fl + static_cast<int64_t>(pos) * W;
      ent[0] = key;
      for (int j = 1; j < W; ++j) ent[j] = c0[(j - 1) * WS];
    }
  }
}

