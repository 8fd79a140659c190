// Grouped aggregation (HASH_AGGREGATE, Section 4.2): local (per-workgroup LDS
// tables merged into a global table) and global (one table) strategies,
// linear probing or cuckoo hashing (whose keys are inserted first by
// k_agg_keys). Compiled once per shape class: the build passes
// -DHK_SHAPE_CLASS=HkShapeX and this file instantiates hk_agg_shape for it.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

#include "hawk_device.h"
#include "hawk_launch.h"
#include "hk_agg_body.h"

#ifndef HK_SHAPE_CLASS
#error "compile once per shape class with -DHK_SHAPE_CLASS=HkShapeX"
#endif

template <int MEM, int PRED, int HT, int HASH, int STRAT, class S, bool SPILL>
__global__ void __launch_bounds__(1024) k_agg(HkPlan P, HkAggTable T, uint32_t llog2, HkIdent id, int64_t nwg,
                                              int* err, HkSpill sp, int32_t reps) {
  // the local table (hk_agg_lds_bytes), read in 32-byte groups
  extern __shared__ __attribute__((aligned(32))) uint64_t lds[];
  agg_body<MEM, PRED, HT, HASH, STRAT, S, SPILL>(P, T, llog2, id, nwg, err, sp, reps, lds);
}

// spill, step 2: each workgroup moves its region's entries to their
// partitions (offsets = exclusive scan of the partition-major histogram).
// Each thread handles SU entries per round: their loads are all issued before
// the first cursor update; two-word entries move as one 16-byte store.
#define SPILL_SU 8
template <int HASH>
__global__ void __launch_bounds__(1024) k_spill_scatter(HkSpill sp, const uint32_t* __restrict__ offs, int64_t nwg,
                                                        HkHash h, uint32_t log2cap, uint32_t rlog2,
                                                        uint64_t* __restrict__ out) {
  const int64_t wgid = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  if (wgid >= nwg) return;
  extern __shared__ uint32_t cur[];
  for (int p = threadIdx.x; p < sp.nparts; p += blockDim.x) cur[p] = offs[static_cast<int64_t>(p) * nwg + wgid];
  __syncthreads();
  const int64_t cnt = sp.cnt[wgid];
  const int64_t start = spill_region_start(sp, nwg, wgid);
  const uint64_t* region = sp.buf + start * sp.ew;  // (entries of ew words)
  const int64_t stride = static_cast<int64_t>(blockDim.x) * SPILL_SU;
  auto move = [&](auto tag) {
    using E = decltype(tag);
    const SpillArr<E> src(sp.buf, sp.nrows, start), dst(out, sp.nrows, 0);
    for (int64_t i0 = threadIdx.x; i0 < cnt; i0 += stride) {
      E v[SPILL_SU];
#pragma unroll
      for (int u = 0; u < SPILL_SU; ++u) {
        const int64_t i = i0 + u * static_cast<int64_t>(blockDim.x);
        if (i < cnt) v[u] = src.get(i);
      }
#pragma unroll
      for (int u = 0; u < SPILL_SU; ++u) {
        const int64_t i = i0 + u * static_cast<int64_t>(blockDim.x);
        if (i < cnt) dst.put(atomicAdd(&cur[hslot<HASH>(spill_key(v[u]), h.a[0], log2cap) >> rlog2], 1u), v[u]);
      }
    }
  };
  if (sp.e12) {
    move(HkE12{});
    return;
  }
  if (sp.ew == 2) {
    move(ulonglong2{});
    return;
  }
  for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) {
    const uint64_t* ent = region + i * sp.ew;
    const uint64_t key = ent[0];
    const uint32_t pos = atomicAdd(&cur[hslot<HASH>(key, h.a[0], log2cap) >> rlog2], 1u);
    uint64_t* d = out + static_cast<int64_t>(pos) * sp.ew;
    d[0] = key;
    for (int j = 0; j < sp.ncols; ++j) d[1 + j] = ent[1 + j];
  }
}

// spill, step 2 for two-word entries: the region is moved in tiles of
// SU * 1024 entries that are first sorted by partition in LDS (counting sort:
// ranks from LDS atomics, offsets from a workgroup scan), so that consecutive
// lanes store consecutive entries of one partition instead of 64 scattered
// 16-byte stores per instruction. LDS: the tile, then per partition the
// running output cursor, the tile counts and the tile offsets (nparts + 1),
// then one word per wave.
template <int HASH, int SU, class E>
__global__ void __launch_bounds__(1024) k_spill_scatter_lds(HkSpill sp, const uint32_t* __restrict__ offs,
                                                            int64_t nwg, HkHash h, uint32_t log2cap, uint32_t rlog2,
                                                            uint64_t* __restrict__ out) {
  const int64_t wgid = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  if (wgid >= nwg) return;
  constexpr int TE = SU * 1024;
  extern __shared__ uint64_t sm[];
  const SpillArr<E> tile(sm, TE, 0);  // (12-byte entries: TE keys, then TE values)
  const int np = sp.nparts;
  uint32_t* gcur = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(sm) + spill_tile_bytes<E>(TE));
  uint32_t* tcnt = gcur + np;
  uint32_t* toff = tcnt + np;
  uint32_t* wave_tot = toff + np + 1;
  const int t = threadIdx.x, bs = blockDim.x;
  for (int p = t; p < np; p += bs) gcur[p] = offs[static_cast<int64_t>(p) * nwg + wgid];
  const int64_t cnt = sp.cnt[wgid];
  const SpillArr<E> src(sp.buf, sp.nrows, spill_region_start(sp, nwg, wgid)), dst(out, sp.nrows, 0);
  for (int64_t base = 0; base < cnt; base += TE) {
    const int n = cnt - base < TE ? static_cast<int>(cnt - base) : TE;
    for (int p = t; p < np; p += bs) tcnt[p] = 0;
    __syncthreads();
    E v[SU];
    uint32_t pr[SU], rk[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int i = t + u * bs;
      if (i < n) v[u] = src.get(base + i);
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int i = t + u * bs;
      if (i < n) {
        pr[u] = hslot<HASH>(spill_key(v[u]), h.a[0], log2cap) >> rlog2;
        rk[u] = atomicAdd(&tcnt[pr[u]], 1u);
      }
    }
    __syncthreads();
    wg_exclusive_scan(tcnt, np, toff, wave_tot);  // toff[p]: first tile slot of partition p; toff[np] = n
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int i = t + u * bs;
      if (i < n) tile.put(toff[pr[u]] + rk[u], v[u]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int j = t + u * bs;
      if (j < n) {
        const E e = tile.get(j);
        const uint32_t p = hslot<HASH>(spill_key(e), h.a[0], log2cap) >> rlog2;
        dst.put(static_cast<int64_t>(gcur[p]) + (j - toff[p]), e);
      }
    }
    __syncthreads();
    for (int p = t; p < np; p += bs) gcur[p] += toff[p + 1] - toff[p];
    // the next tile's counts are cleared after this barrier
    __syncthreads();
  }
}

// spill, step 3: workgroup p owns table region p for the whole kernel. With
// merge entries no other kernel writes the region's slots, so it starts from
// the identity in LDS and merges the workgroups' merge entries of region p;
// else it starts from the region's contents in the table. Then it aggregates
// partition p's spilled entries (LDS atomics, probing confined to the region
// as in the table). With O.nrows set its groups become result rows directly,
// else the region is written back to the table.
template <int HASH, class S>
__global__ void __launch_bounds__(1024) k_spill_agg(HkPlan P, HkAggTable T, HkSpill sp, HkIdent id,
                                                   const uint32_t* __restrict__ offs, const uint64_t* total,
                                                   int64_t nwg, const uint64_t* __restrict__ in, int* err,
                                                   HkResOut O, uint64_t* scratch) {
  const int64_t p = blockIdx.x;
  const int64_t b = offs[p * nwg];
  const int64_t e = p + 1 < sp.nparts ? static_cast<int64_t>(offs[(p + 1) * nwg]) : static_cast<int64_t>(*total);
  const int64_t fstride = sp.nparts + 1;
  // The region may take all the LDS a workgroup can have, so this kernel
  // holds no static LDS: the flag below is the region's first word, read
  // before the region is initialised.
  extern __shared__ uint64_t lt[];  // word w of region slot i at lt[w * R + i]
  bool merges = false;
  if (sp.merge) {
    uint32_t* flag = reinterpret_cast<uint32_t*>(lt);
    if (threadIdx.x == 0) *flag = 0;
    __syncthreads();
    for (int64_t w = threadIdx.x; w < nwg; w += blockDim.x)
      if (sp.foffs[w * fstride + p + 1] > sp.foffs[w * fstride + p]) atomicOr(flag, 1u);
    __syncthreads();
    merges = *flag != 0;
    __syncthreads();
  }
  // nothing spilled and no merge entries here: the region keeps its contents
  // (the identity with merge entries, else what the table holds)
  if (!merges && b >= e) return;
  const int64_t R = static_cast<int64_t>(1) << T.rlog2;
  const int W = T.slot_words;
  uint64_t* g = T.words + p * R * W;
  const uint32_t RW = static_cast<uint32_t>(R * W);  // at most the LDS words of a workgroup
  if (sp.merge) {
    for (uint32_t i = threadIdx.x; i < RW; i += blockDim.x) lt[i] = id.w[i >> T.rlog2];
  } else {
    const uint32_t W32 = static_cast<uint32_t>(W);
    for (uint32_t i = threadIdx.x; i < RW; i += blockDim.x) lt[(i % W32) * R + i / W32] = g[i];
  }
  __syncthreads();
  const uint32_t rmask = static_cast<uint32_t>(R - 1);
  // the region slot of a key (inserted if new); -1 when the region is full
  auto find = [&](uint64_t key) -> int32_t {
    uint32_t s = hslot<HASH>(key, P.hash.a[0], T.log2cap) & rmask;
    for (uint32_t k = 0; k <= rmask; ++k) {
      uint64_t cur = lt[s];
      if (cur == HK_EMPTY) cur = at_cas<true>(&lt[s], HK_EMPTY, key);
      if (cur == HK_EMPTY || cur == key) return static_cast<int32_t>(s);
      s = (s + 1) & rmask;
    }
    set_err(err, HK_ERR_CAPACITY);  // the region is full: the caller retries with a larger table
    return -1;
  };
  // merge entries: K threads per source workgroup (one when the sources
  // outnumber the threads), each taking every K-th of its entries
  const int64_t K = nwg < blockDim.x ? blockDim.x / nwg : 1;
  for (int64_t x = threadIdx.x; merges && x < nwg * K; x += blockDim.x) {
    const int64_t w = x % nwg;
    const int64_t mb = sp.foffs[w * fstride + p], me = sp.foffs[w * fstride + p + 1];
    const uint64_t* src = sp.flush + w * sp.fcap * W;
    for (int64_t i = mb + x / nwg; i < me; i += K) {
      const uint64_t* ent = src + i * W;
      const int32_t s = find(ent[0]);
      if (s >= 0) agg_merge_into<true, S>(lt + s, R, ent + 1, 1, P);
    }
  }
  v16i64 r = {};
  auto apply = [&](uint64_t key) {
    const int32_t found = find(key);
    if (found >= 0) agg_apply<HK_BR, true, S>(lt + found, R, P, r, true);
  };
  // one input value per entry: SU entries per thread and round; the next
  // round's entries are loaded while this round's are applied (the applies
  // wait only on LDS, so the loads in flight stay in flight)
  auto apply_all = [&](auto tag) {
    using E = decltype(tag);
    const SpillArr<E> src(const_cast<uint64_t*>(in), sp.nrows, 0);
    const int reg = sp.reg[0];
    const int64_t bd = blockDim.x;
    const int64_t stride = bd * SPILL_SU;
    E v[SPILL_SU] = {}, nx[SPILL_SU] = {};
    int64_t i0 = b + threadIdx.x;
#pragma unroll
    for (int u = 0; u < SPILL_SU; ++u)
      if (i0 + u * bd < e) v[u] = src.get(i0 + u * bd);
    for (; i0 < e; i0 += stride) {
      const int64_t n0 = i0 + stride;
#pragma unroll
      for (int u = 0; u < SPILL_SU; ++u)
        if (n0 + u * bd < e) nx[u] = src.get(n0 + u * bd);
#pragma unroll
      for (int u = 0; u < SPILL_SU; ++u) {
        if (i0 + u * bd < e) {
          r[reg] = spill_value(v[u]);
          apply(spill_key(v[u]));
        }
      }
#pragma unroll
      for (int u = 0; u < SPILL_SU; ++u) v[u] = nx[u];
    }
  };
  if (sp.e12) {
    apply_all(HkE12{});
  } else if (sp.ew == 2) {
    apply_all(ulonglong2{});
  } else {
    for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
      const uint64_t* ent = in + i * sp.ew;
      for (int j = 0; j < sp.ncols; ++j) r[sp.reg[j]] = static_cast<long long>(ent[1 + j]);
      apply(ent[0]);
    }
  }
  __syncthreads();
  if (!O.nrows) {
    // the region goes back to the table (whose reader extracts the groups)
    const uint32_t W32 = static_cast<uint32_t>(W);
    for (uint32_t i = threadIdx.x; i < RW; i += blockDim.x) g[i] = lt[(i % W32) * R + i / W32];
    return;
  }
  // The region's groups go straight to the result columns: each wave counts
  // the live slots it will write, one device atomic per workgroup reserves
  // the rows. The region takes all of the LDS, so the per-wave counts and
  // the base pass through this region's words of `scratch` (global memory,
  // ordered within the workgroup by the barriers).
  const int wave = threadIdx.x / WAVE, nwv = (blockDim.x + WAVE - 1) / WAVE;
  uint64_t* sc = scratch + p * 32;
  uint32_t live = 0;
  for (int64_t s = threadIdx.x; s < R; s += blockDim.x) live += lt[R + s] != 0 ? 1u : 0u;
  for (int off = WAVE / 2; off > 0; off >>= 1) live += __shfl_xor(live, off, WAVE);
  if (__lane_id() == 0) sc[wave] = live;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (int w = 0; w < nwv; ++w) tot += sc[w];
    sc[16] = tot ? atomicAdd(O.nrows, tot) : 0ull;
  }
  __syncthreads();
  uint64_t pos = sc[16];
  for (int w = 0; w < wave; ++w) pos += sc[w];
  for (int64_t s0 = 0; s0 < R; s0 += blockDim.x) {
    const int64_t s = s0 + threadIdx.x;
    const bool on = s < R && lt[R + s] != 0;
    const uint64_t m = __ballot(on);
    if (on) write_group_row_s(P, lt + s, R, static_cast<int64_t>(pos) + __popcll(m & lanemask_lt()), O);
    pos += __popcll(m);
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

// the LDS a workgroup may hold on `dev` (queried once per device)
static int device_max_lds(int dev) {
  static std::mutex mu;
  static std::vector<std::pair<int, int>> known;
  std::lock_guard<std::mutex> g(mu);
  for (const auto& k : known)
    if (k.first == dev) return k.second;
  int maxl = 0;
  if (hipDeviceGetAttribute(&maxl, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
  known.emplace_back(dev, maxl);
  return maxl;
}

// a launch whose static plus dynamic LDS exceeds one workgroup's maximum
// would abort the queue: such a launch is refused here instead (the
// kernel's static LDS is queried once per kernel)
static hipError_t lds_fits_fn(const void* kernel, size_t dyn) {
  static std::mutex mu;
  static std::vector<std::pair<const void*, size_t>> known;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const size_t maxl = static_cast<size_t>(device_max_lds(dev));
  {
    std::lock_guard<std::mutex> g(mu);
    for (const auto& k : known)
      if (k.first == kernel) return k.second + dyn <= maxl ? hipSuccess : hipErrorInvalidValue;
  }
  hipFuncAttributes a;
  if ((e = hipFuncGetAttributes(&a, kernel)) != hipSuccess) return e;
  {
    std::lock_guard<std::mutex> g(mu);
    known.emplace_back(kernel, a.sharedSizeBytes);
  }
  return a.sharedSizeBytes + dyn <= maxl ? hipSuccess : hipErrorInvalidValue;
}

template <class K>
static hipError_t lds_fits(K kernel, size_t dyn) {
  return lds_fits_fn(reinterpret_cast<const void*>(kernel), dyn);
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
  const size_t lds = hk_agg_lds_bytes(strat, llog2, id.nw, reps, sp);
  if (sp) {
    // spill mode exists for the local strategy with linear probing
    if (strat != HK_LOCAL || ht != HK_LIN) return hipErrorInvalidValue;
    const HkSpill S1 = *sp;
    hipError_t le = hipSuccess;
    DISPATCH2(mem, M, DISPATCH2(pred, PR, DISPATCH2(hash, HS, {
      le = lds_fits(k_agg<M, PR, HK_LIN, HS, HK_LOCAL, S, true>, lds);
      if (le == hipSuccess)
        hipLaunchKernelGGL((k_agg<M, PR, HK_LIN, HS, HK_LOCAL, S, true>), g, b, lds, st, P, T, llog2, id, groups,
                           err, S1, reps);
    })));
    return le != hipSuccess ? le : hipGetLastError();
  }
  HkSpill none;
  std::memset(&none, 0, sizeof(none));
  hipError_t le = hipSuccess;
  DISPATCH2(mem, M, DISPATCH2(pred, PR, DISPATCH2(ht, HT, DISPATCH2(hash, HS, DISPATCH2(strat, SG, {
    le = lds_fits(k_agg<M, PR, HT, HS, SG, S, false>, lds);
    if (le == hipSuccess)
      hipLaunchKernelGGL((k_agg<M, PR, HT, HS, SG, S, false>), g, b, lds, st, P, T, llog2, id, groups, err, none,
                         reps);
  })))));
  return le != hipSuccess ? le : hipGetLastError();
}

template <class S>
hipError_t hk_spill_shape(hipStream_t st, int step, const HkPlan& P, const HkAggTable& T, int hash, const HkSpill& sp,
                          const HkIdent& id, const uint32_t* offs, const uint64_t* total, int64_t nwg, uint64_t* part,
                          int* err, const HkResOut& O, uint64_t* scratch) {
  if (step == 0) {
    // two-word entries with 1024 threads: tiles sorted in LDS (8192 entries,
    // else 4096, whichever fits with the partition arrays)
    int dev = 0;
    const hipError_t ae = hipGetDevice(&dev);
    if (ae != hipSuccess) return ae;
    const int maxl = device_max_lds(dev);
    const size_t side = (3 * static_cast<size_t>(sp.nparts) + 1) * sizeof(uint32_t) + (1024 / WAVE) * sizeof(uint32_t);
    const size_t l8 = (sp.e12 ? spill_tile_bytes<HkE12>(8192) : spill_tile_bytes<ulonglong2>(8192)) + side;
    const size_t l4 = (sp.e12 ? spill_tile_bytes<HkE12>(4096) : spill_tile_bytes<ulonglong2>(4096)) + side;
    auto tiles = [&](auto su, auto* ent, size_t l) {
      constexpr int SU = decltype(su)::value;
      using E = typename std::remove_pointer<decltype(ent)>::type;
      hipError_t le = hipSuccess;
      DISPATCH2(hash, HS, {
        le = lds_fits(k_spill_scatter_lds<HS, SU, E>, l);
        if (le == hipSuccess)
          hipLaunchKernelGGL((k_spill_scatter_lds<HS, SU, E>), hk_wg_grid(nwg), dim3(1024), l, st, sp, offs, nwg,
                             P.hash, T.log2cap, T.rlog2, part);
      });
      return le;
    };
    using su8 = std::integral_constant<int, 8>;
    using su4 = std::integral_constant<int, 4>;
    if (sp.ew == 2 && l8 <= static_cast<size_t>(maxl)) {
      const hipError_t le = sp.e12 ? tiles(su8{}, static_cast<HkE12*>(nullptr), l8)
                                   : tiles(su8{}, static_cast<ulonglong2*>(nullptr), l8);
      if (le != hipSuccess) return le;
    } else if (sp.ew == 2 && l4 <= static_cast<size_t>(maxl)) {
      const hipError_t le = sp.e12 ? tiles(su4{}, static_cast<HkE12*>(nullptr), l4)
                                   : tiles(su4{}, static_cast<ulonglong2*>(nullptr), l4);
      if (le != hipSuccess) return le;
    } else {
      const size_t lds = static_cast<size_t>(sp.nparts) * sizeof(uint32_t);
      DISPATCH2(hash, HS, hipLaunchKernelGGL((k_spill_scatter<HS>), hk_wg_grid(nwg), dim3(1024), lds, st, sp, offs,
                                             nwg, P.hash, T.log2cap, T.rlog2, part));
    }
  } else {
    // a region larger than half the LDS of a CU: one workgroup per CU, of 1024 threads
    const size_t lds = (static_cast<size_t>(1) << T.rlog2) * T.slot_words * sizeof(uint64_t);
    const uint32_t threads = lds > 81920 ? 1024 : 512;
    hipError_t le = hipSuccess;
    DISPATCH2(hash, HS, {
      le = lds_fits(k_spill_agg<HS, S>, lds);
      if (le == hipSuccess)
        hipLaunchKernelGGL((k_spill_agg<HS, S>), dim3(static_cast<uint32_t>(sp.nparts)), dim3(threads), lds, st, P, T,
                           sp, id, offs, total, nwg, part, err, O, scratch);
    });
    if (le != hipSuccess) return le;
  }
  return hipGetLastError();
}

template hipError_t hk_agg_shape<HK_SHAPE_CLASS>(hipStream_t, const HkPlan&, const HkAggTable&, int, int, int, int, int,
                                                 int64_t, int32_t, uint32_t, const HkIdent&, int*, const HkSpill*,
                                                 int32_t);
template hipError_t hk_spill_shape<HK_SHAPE_CLASS>(hipStream_t, int, const HkPlan&, const HkAggTable&, int, const HkSpill&,
                                                   const HkIdent&, const uint32_t*, const uint64_t*, int64_t, uint64_t*,
                                                   int*, const HkResOut&, uint64_t*);
