// Batched execution of many pipelines in persistent, work-queue kernels that
// one captured HIP graph replays: a fill kernel resets the batch's tables and
// counters, a persistent build kernel runs every build pipeline's tiles, one
// persistent main kernel per shape class runs the main pipelines' tiles, and
// a persistent finalize kernel extracts every aggregation's groups.
//
// Workgroups take (query, tile) items from an atomic counter. Every query in
// a batch runs the batch's own tile-parallel strategy: a tile is a contiguous
// row range scanned by one workgroup with coalesced access and branched
// evaluation; aggregation tiles pre-aggregate in an LDS table (linear
// probing, Murmur hash) merged into the query's global table; projection
// tiles keep input row order with a single-pass decoupled look-back over the
// tiles' counts (a tile waits only for lower tiles of its query, which were
// handed out earlier to running workgroups, so the lowest unfinished tile
// never waits; every wait is also bounded and reports an error instead of
// hanging).
#include <hip/hip_runtime.h>

#include "hawk_batch.h"
#include "hawk_device.h"

#define LB_AGG 1ull       // look-back word holds this tile's count
#define LB_INCL 2ull      // look-back word holds the inclusive prefix
#define LB_SPIN_LIMIT (1 << 26)

__device__ __forceinline__ uint64_t lb_pack(uint64_t state, uint64_t v) { return (state << 62) | v; }

// (query index, tile) of a work item: items of query k are [bases[k], bases[k+1])
__device__ __forceinline__ void decode_item(const int64_t* bases, int32_t nq, int64_t item, int32_t& k, int64_t& t) {
  int32_t lo = 0, hi = nq - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (bases[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  k = lo;
  t = item - bases[lo];
}

// next work item for the whole workgroup
__device__ __forceinline__ int64_t next_item(unsigned long long* head, int64_t* sh) {
  __syncthreads();
  if (threadIdx.x == 0) *sh = static_cast<int64_t>(atomicAdd(head, 1ull));
  __syncthreads();
  return *sh;
}

// ------------------------------------------------------------------ fill
__global__ void __launch_bounds__(256) k_batch_fill(const HkFillJob* __restrict__ jobs, const int64_t* __restrict__ bases,
                                                    int32_t njobs, int64_t total) {
  const int64_t T = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += T) {
    int32_t j;
    int64_t w;
    decode_item(bases, njobs, i, j, w);
    const HkFillJob& J = jobs[j];
    J.ptr[w] = J.pattern[w % J.period];
  }
}

// ------------------------------------------------------------------ builds
__global__ void __launch_bounds__(256) k_batch_build(const HkBuild* __restrict__ builds, const int64_t* __restrict__ bases,
                                                     int32_t nb, int64_t nitems, int64_t tile_rows,
                                                     unsigned long long* head, int* err) {
  __shared__ int64_t sh;
  v16i64 r = {};
  for (;;) {
    const int64_t item = next_item(head, &sh);
    if (item >= nitems) break;
    int32_t b;
    int64_t t;
    decode_item(bases, nb, item, b, t);
    const HkBuild B = builds[b];
    const int64_t r0 = t * tile_rows, r1 = r0 + tile_rows < B.p.nrows ? r0 + tile_rows : B.p.nrows;
    for (int64_t row = r0 + threadIdx.x; row < r1; row += blockDim.x) {
      if (!eval_row<HK_BR, HK_LIN, HK_MURMUR, false, HkShapeG>(B.p, row, r)) continue;
      join_insert<HK_LIN, HK_MURMUR>(B.t, B.p.hash, static_cast<int32_t>(load_col(B.key, row)),
                                     static_cast<int32_t>(load_col(B.payload, row)), err);
    }
  }
}

// ------------------------------------------------------------------ main tiles
template <class S>
__device__ void tile_aggregate(const HkPlan& P, const HkBatchQuery& Q, int64_t r0, int64_t r1, uint64_t* lds) {
  const int64_t LC = static_cast<int64_t>(1) << Q.llog2;
  const int nw = Q.ident.nw;
  for (int w = 0; w < nw; ++w)
    for (int64_t i = threadIdx.x; i < LC; i += blockDim.x) lds[w * LC + i] = Q.ident.w[w];
  __syncthreads();
  v16i64 r = {};
  for (int64_t row = r0 + threadIdx.x; row < r1; row += blockDim.x) {
    if (!eval_row<HK_BR, HK_LIN, HK_MURMUR, true, S>(P, row, r)) continue;
    const uint64_t key = group_key(P, r);
    if (key != HK_EMPTY) {
      const int32_t s = lslot<HK_LIN, HK_MURMUR, false>(lds, Q.llog2, P.hash, key);
      if (s >= 0) {
        agg_apply<HK_BR, true, S>(lds + s, LC, P, r, true);
        continue;
      }
    }
    uint64_t* g = gslot<HK_LIN, HK_MURMUR>(Q.table, P.hash, key, Q.err);
    if (g) agg_apply<HK_BR, false, S>(g, 1, P, r, true);
  }
  __syncthreads();
  for (int64_t s = threadIdx.x; s < LC; s += blockDim.x) {
    const uint64_t key = lds[s];
    if (key == HK_EMPTY || lds[LC + s] == 0) continue;
    uint64_t* g = gslot<HK_LIN, HK_MURMUR>(Q.table, P.hash, key, Q.err);
    if (g) agg_merge<S>(g, lds + s, LC, P);
  }
}

// AGGREGATE without groups: each thread folds its rows into one LDS slot,
// which the workgroup then merges into the query's single global slot
template <class S>
__device__ void tile_scalar(const HkPlan& P, const HkBatchQuery& Q, int64_t r0, int64_t r1, uint64_t* lds) {
  if (threadIdx.x < Q.ident.nw) lds[threadIdx.x] = Q.ident.w[threadIdx.x];
  __syncthreads();
  v16i64 r = {};
  for (int64_t row = r0 + threadIdx.x; row < r1; row += blockDim.x) {
    if (!eval_row<HK_BR, HK_LIN, HK_MURMUR, true, S>(P, row, r)) continue;
    agg_apply<HK_BR, true, S>(lds, 1, P, r, true);
  }
  __syncthreads();
  if (threadIdx.x == 0 && lds[1] != 0) agg_merge<S>(Q.table.words, lds, 1, P);
}

// projection tile: flags into LDS, tile count, look-back for the tile's
// output offset, then the qualifying rows' values at their positions
template <class S>
__device__ void tile_project(const HkPlan& P, const HkBatchQuery& Q, int64_t t, int64_t r0, int64_t r1,
                             uint64_t* lds) {
  const int64_t nwords = (r1 - r0 + WAVE - 1) / WAVE;
  uint64_t* masks = lds;                                   // nwords
  uint32_t* pre = reinterpret_cast<uint32_t*>(lds + Q.tile_rows / WAVE);  // nwords + 1
  int64_t* sh = reinterpret_cast<int64_t*>(pre + Q.tile_rows / WAVE + 2);
  v16i64 r = {};
  for (int64_t c0 = r0; c0 < r1; c0 += blockDim.x) {
    const int64_t row = c0 + threadIdx.x;
    bool pass = false;
    if (row < r1) pass = eval_row<HK_BR, HK_LIN, HK_MURMUR, false, S>(P, row, r);
    const uint64_t m = __ballot(pass);
    if (__lane_id() == 0 && row - __lane_id() < r1) masks[(row - __lane_id() - r0) / WAVE] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // exclusive prefix of the words' counts and the tile total
    uint32_t acc = 0;
    for (int64_t i = 0; i < nwords; ++i) {
      pre[i] = acc;
      acc += static_cast<uint32_t>(__popcll(masks[i]));
    }
    const uint64_t cnt = acc;
    uint64_t excl = 0;
    if (t == 0) {
      __hip_atomic_store(&Q.status[0], lb_pack(LB_INCL, cnt), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_store(&Q.status[t], lb_pack(LB_AGG, cnt), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      int64_t p = t - 1;
      int spins = 0;
      while (p >= 0) {
        const uint64_t s = __hip_atomic_load(&Q.status[p], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t st = s >> 62, v = s & ((1ull << 62) - 1);
        if (st == LB_INCL) {
          excl += v;
          break;
        }
        if (st == LB_AGG) {
          excl += v;
          --p;
          continue;
        }
        if (++spins > LB_SPIN_LIMIT) {  // never expected: report instead of hanging
          set_err(Q.err, HK_ERR_TIMEOUT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      __hip_atomic_store(&Q.status[t], lb_pack(LB_INCL, excl + cnt), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    *sh = static_cast<int64_t>(excl);
    if (t == Q.ntiles - 1) *Q.count = excl + cnt;
  }
  __syncthreads();
  const int64_t excl = *sh;
  for (int64_t c0 = r0; c0 < r1; c0 += blockDim.x) {
    const int64_t row = c0 + threadIdx.x;
    if (row >= r1) continue;
    const int64_t wi = (row - r0) / WAVE;
    const uint64_t m = masks[wi];
    if (!((m >> __lane_id()) & 1ull)) continue;
    eval_row<HK_BR, HK_LIN, HK_MURMUR, true, S>(P, row, r);
    write_proj<S>(P, Q.out, excl + pre[wi] + __popcll(m & lanemask_lt()), r);
  }
}

template <class S>
__global__ void __launch_bounds__(256) k_batch_main(const HkBatchQuery* __restrict__ qs, const int32_t* __restrict__ qidx,
                                                    const int64_t* __restrict__ bases, int32_t nq, int64_t nitems,
                                                    unsigned long long* head) {
  extern __shared__ __attribute__((aligned(32))) uint64_t lds[];  // tables read in 32-byte groups
  __shared__ int64_t sh;
  for (;;) {
    const int64_t item = next_item(head, &sh);
    if (item >= nitems) break;
    int32_t k;
    int64_t t;
    decode_item(bases, nq, item, k, t);
    const HkBatchQuery& Q = qs[qidx[k]];
    const HkPlan P = Q.plan;  // this tile's plan fields, loaded once
    const int64_t r0 = t * Q.tile_rows, r1 = r0 + Q.tile_rows < P.nrows ? r0 + Q.tile_rows : P.nrows;
    if (Q.kind == HK_BQ_PROJECT) tile_project<S>(P, Q, t, r0, r1, lds);
    else if (Q.kind == HK_BQ_GROUPED) tile_aggregate<S>(P, Q, r0, r1, lds);
    else tile_scalar<S>(P, Q, r0, r1, lds);
  }
}

// ------------------------------------------------------------------ finalize
__global__ void __launch_bounds__(256) k_batch_final(const HkBatchQuery* __restrict__ qs, const int32_t* __restrict__ qidx,
                                                     const int64_t* __restrict__ bases, int32_t nq, int64_t nitems,
                                                     int64_t tile_slots, unsigned long long* head) {
  __shared__ int64_t sh;
  for (;;) {
    const int64_t item = next_item(head, &sh);
    if (item >= nitems) break;
    int32_t k;
    int64_t t;
    decode_item(bases, nq, item, k, t);
    const HkBatchQuery& Q = qs[qidx[k]];
    const int64_t W = Q.table.slot_words;
    const int64_t s0 = t * tile_slots, s1 = s0 + tile_slots < Q.nslots ? s0 + tile_slots : Q.nslots;
    for (int64_t base = s0 + threadIdx.x - __lane_id(); base < s1; base += blockDim.x) {
      const int64_t s = base + __lane_id();
      const uint64_t* p = Q.table.words + s * W;
      const bool live = s < s1 && (p[1] != 0 || Q.kind == HK_BQ_SCALAR);
      const uint64_t m = __ballot(live);
      if (m == 0) continue;
      unsigned long long start = 0;
      if (__lane_id() == 0) start = atomicAdd(reinterpret_cast<unsigned long long*>(Q.count), static_cast<unsigned long long>(__popcll(m)));
      start = __shfl(start, 0, WAVE);
      if (!live) continue;
      const int64_t pos = static_cast<int64_t>(start) + __popcll(m & lanemask_lt());
      write_group_row(Q.plan, p, pos, Q.res);
    }
  }
}

// ================================================================== launchers
hipError_t hk_batch_fill(hipStream_t st, const HkFillJob* jobs, const int64_t* bases, int32_t njobs, int64_t total) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_fill, dim3(hk_grid_for(total, 256, 16384)), dim3(256), 0, st, jobs, bases, njobs, total);
  return hipGetLastError();
}

hipError_t hk_batch_build(hipStream_t st, int64_t grid, const HkBuild* builds, const int64_t* bases, int32_t nb,
                          int64_t nitems, int64_t tile_rows, unsigned long long* head, int* err) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_build, dim3(static_cast<uint32_t>(grid)), dim3(256), 0, st, builds, bases, nb, nitems,
                     tile_rows, head, err);
  return hipGetLastError();
}

hipError_t hk_batch_main(hipStream_t st, int shape, int64_t grid, int32_t wg, size_t lds, const HkBatchQuery* qs,
                         const int32_t* qidx, const int64_t* bases, int32_t nq, int64_t nitems,
                         unsigned long long* head) {
  if (nitems <= 0) return hipSuccess;
  const dim3 g(static_cast<uint32_t>(grid)), b(static_cast<uint32_t>(wg));
  switch (shape) {
    case HK_SHAPE_A: hipLaunchKernelGGL(k_batch_main<HkShapeA>, g, b, lds, st, qs, qidx, bases, nq, nitems, head); break;
    case HK_SHAPE_F: hipLaunchKernelGGL(k_batch_main<HkShapeF>, g, b, lds, st, qs, qidx, bases, nq, nitems, head); break;
    case HK_SHAPE_J: hipLaunchKernelGGL(k_batch_main<HkShapeJ>, g, b, lds, st, qs, qidx, bases, nq, nitems, head); break;
    case HK_SHAPE_W: hipLaunchKernelGGL(k_batch_main<HkShapeW>, g, b, lds, st, qs, qidx, bases, nq, nitems, head); break;
    default: hipLaunchKernelGGL(k_batch_main<HkShapeG>, g, b, lds, st, qs, qidx, bases, nq, nitems, head); break;
  }
  return hipGetLastError();
}

hipError_t hk_batch_final(hipStream_t st, int64_t grid, const HkBatchQuery* qs, const int32_t* qidx,
                          const int64_t* bases, int32_t nq, int64_t nitems, int64_t tile_slots,
                          unsigned long long* head) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_final, dim3(static_cast<uint32_t>(grid)), dim3(256), 0, st, qs, qidx, bases, nq, nitems,
                     tile_slots, head);
  return hipGetLastError();
}
