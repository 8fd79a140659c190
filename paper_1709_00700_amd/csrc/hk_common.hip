// Kernels shared by every pipeline kind: table initialisation, build
// pipelines (HASH_PUT), the exclusive scan of the multi-pass strategy, the
// concatenation of single-pass regions and aggregation result extraction.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "hawk_device.h"
#include "hawk_launch.h"

#define HK_CHECK_LAUNCH() return hipGetLastError()

// ------------------------------------------------------------------ fill / init
__global__ void __launch_bounds__(256) k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// several fills in one launch, one per grid row
__global__ void __launch_bounds__(256) k_fill_multi(HkFills f) {
  uint64_t* p = f.p[blockIdx.y];
  const int64_t n = f.n[blockIdx.y];
  const uint64_t v = f.v[blockIdx.y];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void __launch_bounds__(256) k_init_aggtable(uint64_t* words, int64_t nslots, HkIdent id) {
  __shared__ uint64_t w[2 + 2 * HK_MAX_AGGS];
  if (threadIdx.x == 0)
    for (int j = 0; j < id.nw; ++j) w[j] = id.w[j];
  __syncthreads();
  const int64_t total = nslots * id.nw;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    words[i] = w[i % id.nw];
}

// The build kernels take an array of builds, one per grid row (blockIdx.y):
// the builds of a query are independent (each fills its own table), so one
// launch runs them all.
template <int HT, int HASH>
__global__ void __launch_bounds__(256) k_build(const HkBuild* Bp, int* err) {
  const HkBuild& B = Bp[blockIdx.y];  // build plan in device memory
  v16i64 r = {};
  const int64_t T = (int64_t)gridDim.x * blockDim.x;
  for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < B.p.nrows; row += T) {
    if (!eval_row<HK_BR, HT, HASH, false, HkShapeG>(B.p, row, r)) continue;
    join_insert<HT, HASH>(B.t, B.p.hash, static_cast<int32_t>(load_col(B.key, row)),
                          static_cast<int32_t>(load_col(B.payload, row)), err);
  }
}

// a cuckoo table may hold two copies of a key inserted twice; count copies
template <int HASH>
__global__ void __launch_bounds__(256) k_build_verify(const HkBuild* Bp, int* err) {
  const HkBuild& B = Bp[blockIdx.y];  // build plan in device memory
  v16i64 r = {};
  const int64_t T = (int64_t)gridDim.x * blockDim.x;
  for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < B.p.nrows; row += T) {
    if (!eval_row<HK_BR, HK_CUCKOO, HASH, false, HkShapeG>(B.p, row, r)) continue;
    const int32_t key = static_cast<int32_t>(load_col(B.key, row));
    if (key == -1) continue;
    uint32_t pos[HK_CUCKOO_D];
    int copies = 0;
#pragma unroll
    for (int i = 0; i < HK_CUCKOO_D; ++i) {
      pos[i] = hslot<HASH>(static_cast<uint32_t>(key), B.p.hash.a[i], B.t.log2cap);
      bool seen = false;
#pragma unroll
      for (int j = 0; j < i; ++j) seen = seen || pos[j] == pos[i];
      const uint64_t w = B.t.slots[pos[i]];
      if (!seen && w != HK_EMPTY && static_cast<uint32_t>(w >> 32) == static_cast<uint32_t>(key)) ++copies;
    }
    if (copies > 1) set_err(err, HK_ERR_DUPKEY);
    if (copies == 0) set_err(err, HK_ERR_CUCKOO);
  }
}

// Robin-hood builds insert concurrently: two insertions of one key may both
// land. Every qualifying build row counts the copies of its key within the
// largest displacement from its home slot: two or more is a duplicate key,
// none an insertion that failed.
template <int HASH>
__global__ void __launch_bounds__(256) k_build_verify_robin(const HkBuild* Bp, int* err) {
  const HkBuild& B = Bp[blockIdx.y];
  v16i64 r = {};
  const int64_t T = (int64_t)gridDim.x * blockDim.x;
  const uint32_t mask = (1u << B.t.log2cap) - 1u;
  for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < B.p.nrows; row += T) {
    if (!eval_row<HK_BR, HK_LIN, HASH, false, HkShapeG>(B.p, row, r)) continue;
    const int32_t key = static_cast<int32_t>(load_col(B.key, row));
    if (key == -1) continue;
    const uint32_t maxd = static_cast<uint32_t>(B.t.side[1]);
    uint32_t pos = hslot<HASH>(static_cast<uint32_t>(key), B.p.hash.a[0], B.t.log2cap);
    int copies = 0;
    for (uint32_t d = 0; d <= maxd && d <= mask; ++d) {
      const uint64_t w = B.t.slots[pos];
      if (w == HK_EMPTY) break;
      copies += static_cast<uint32_t>(w >> 32) == static_cast<uint32_t>(key);
      pos = (pos + 1) & mask;
    }
    if (copies > 1) set_err(err, HK_ERR_DUPKEY);
    if (copies == 0) set_err(err, HK_ERR_CAPACITY);
  }
}

// ------------------------------------------------------------------ exclusive scan (u32 counts -> u32 offsets)
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint32_t t = __shfl_up(v, d, WAVE);
    if (__lane_id() >= d) v += t;
  }
  return v;
}
// exclusive scan of one value per thread over a 1024-thread block; returns the block total in *tot
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* tot) {
  const int lane = __lane_id(), wid = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  const uint32_t inc = wave_incl_scan(v);
  if (lane == WAVE - 1) sh[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    const uint32_t x = lane < nw ? sh[lane] : 0u;
    const uint32_t xs = wave_incl_scan(x);
    if (lane < nw) sh[lane] = xs - x;
    if (lane == nw - 1) sh[WAVE] = xs;
  }
  __syncthreads();
  const uint32_t res = sh[wid] + inc - v;
  *tot = sh[WAVE];
  __syncthreads();
  return res;
}

// Single-pass exclusive scan (decoupled look-back). A tile is 1024 threads x
// 16 consecutive counts per thread (vector loads and stores). Tiles take
// their index from an atomic counter, so every tile that one waits for was
// handed out earlier to a running workgroup; a tile publishes its total,
// then its inclusive prefix once the tiles before it have theirs. A scan of
// one tile (up to 16384 counts) needs neither the counter nor the status
// words. The waits are bounded: past the bound the tile reports
// HK_ERR_TIMEOUT instead of hanging.
#define SCAN_ITEMS 16
#define SCAN_TILE (1024 * SCAN_ITEMS)
#define SCAN_PART 1ull   // status word: the tile's own total
#define SCAN_INCL 2ull   // status word: the inclusive prefix through the tile
#define SCAN_SPIN_LIMIT (1 << 24)

__global__ void __launch_bounds__(1024) k_scan_lb(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                  int64_t m, uint64_t* status, unsigned int* counter,
                                                  uint64_t* total, int* err) {
  __shared__ uint32_t sh[WAVE + 1];
  __shared__ uint32_t tile_sh;
  __shared__ uint64_t excl_sh;
  const int64_t ntiles = (m + SCAN_TILE - 1) / SCAN_TILE;
  if (m <= 0) {
    if (total && threadIdx.x == 0) *total = 0;
    return;
  }
  uint32_t tile = 0;
  if (ntiles > 1) {
    if (threadIdx.x == 0) tile_sh = atomicAdd(counter, 1u);
    __syncthreads();
    tile = tile_sh;
  }
  const int64_t j0 = static_cast<int64_t>(tile) * SCAN_TILE + static_cast<int64_t>(threadIdx.x) * SCAN_ITEMS;
  const bool vec = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15u) == 0;
  uint32_t v[SCAN_ITEMS];
  if (vec && j0 + SCAN_ITEMS <= m) {
    const uint4* src = reinterpret_cast<const uint4*>(in + j0);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS / 4; ++i) {
      const uint4 x = src[i];
      v[4 * i] = x.x;
      v[4 * i + 1] = x.y;
      v[4 * i + 2] = x.z;
      v[4 * i + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) v[i] = j0 + i < m ? in[j0 + i] : 0u;
  }
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) s += v[i];
  uint32_t tot;
  const uint32_t pre = block_excl_scan(s, sh, &tot);
  if (threadIdx.x == 0) {
    uint64_t excl = 0;
    if (ntiles > 1) {
      if (tile == 0) {
        __hip_atomic_store(&status[0], (SCAN_INCL << 62) | tot, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        __hip_atomic_store(&status[tile], (SCAN_PART << 62) | tot, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int64_t p = static_cast<int64_t>(tile) - 1;
        int spins = 0;
        while (p >= 0) {
          const uint64_t w = __hip_atomic_load(&status[p], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
          const uint64_t st = w >> 62, val = w & ((1ull << 62) - 1);
          if (st == SCAN_INCL) {
            excl += val;
            break;
          }
          if (st == SCAN_PART) {
            excl += val;
            --p;
            continue;
          }
          if (++spins > SCAN_SPIN_LIMIT) {  // never expected: report instead of hanging
            if (err) set_err(err, HK_ERR_TIMEOUT);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        __hip_atomic_store(&status[tile], (SCAN_INCL << 62) | (excl + tot), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    excl_sh = excl;
    if (total && tile == ntiles - 1) *total = excl + tot;
  }
  __syncthreads();
  uint32_t run = static_cast<uint32_t>(excl_sh) + pre;
  if (vec && j0 + SCAN_ITEMS <= m) {
    uint4* dst = reinterpret_cast<uint4*>(out + j0);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS / 4; ++i) {
      uint4 x;
      x.x = run;
      run += v[4 * i];
      x.y = run;
      run += v[4 * i + 1];
      x.z = run;
      run += v[4 * i + 2];
      x.w = run;
      run += v[4 * i + 3];
      dst[i] = x;
    }
  } else {
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
      if (j0 + i < m) out[j0 + i] = run;
      run += v[i];
    }
  }
}

// concatenation of the single-pass regions: one wave per region
__global__ void __launch_bounds__(256) k_sp_concat(HkOut tmp, int32_t nproj, int64_t region, int64_t nregions,
                                                   const uint32_t* __restrict__ counts,
                                                   const uint32_t* __restrict__ offsets, HkOut out) {
  const int64_t waves = (int64_t)gridDim.x * blockDim.x / WAVE;
  for (int64_t g = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / WAVE; g < nregions; g += waves) {
    const int64_t c = counts[g], o = offsets[g];
    for (int64_t i = __lane_id(); i < c; i += WAVE)
      for (int k = 0; k < HK_MAX_PROJ; ++k)
        if (k < nproj) out.col[k][o + i] = tmp.col[k][g * region + i];
  }
}

// ------------------------------------------------------------------ finalize
// Each workgroup takes a contiguous chunk of slots: it counts the chunk's
// live slots, reserves their result rows with one atomic, then writes them
// in slot order (wave offsets from a per-round prefix in LDS).
__global__ void __launch_bounds__(256) k_finalize(const HkPlan* Pp, HkAggTable T, int64_t nslots, int64_t chunk,
                                                  HkResOut O) {
  const HkPlan& P = *Pp;  // plan in device memory, read where used
  const int64_t W = T.slot_words;
  const int64_t s0 = blockIdx.x * chunk;
  const int64_t s1 = s0 + chunk < nslots ? s0 + chunk : nslots;
  __shared__ uint32_t wcount[256 / WAVE];
  __shared__ unsigned long long base;
  const int wave = threadIdx.x / WAVE, nwaves = blockDim.x / WAVE;
  uint32_t mine = 0;
  for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) mine += (T.words[s * W + 1] != 0 || O.keep_empty) ? 1u : 0u;
  for (int off = WAVE / 2; off > 0; off >>= 1) mine += __shfl_xor(mine, off, WAVE);
  if (__lane_id() == 0) wcount[wave] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (int w = 0; w < nwaves; ++w) tot += wcount[w];
    base = tot ? atomicAdd(O.nrows, tot) : 0ull;
  }
  __syncthreads();
  unsigned long long pos0 = base;
  for (int64_t r0 = s0; r0 < s1; r0 += blockDim.x) {
    const int64_t s = r0 + threadIdx.x;
    const uint64_t* p = T.words + s * W;
    const bool live = s < s1 && (p[1] != 0 || O.keep_empty);
    const uint64_t m = __ballot(live);
    __syncthreads();  // the previous round's offsets are read
    if (__lane_id() == 0) wcount[wave] = static_cast<uint32_t>(__popcll(m));
    __syncthreads();
    unsigned long long before = 0, round = 0;
    for (int w = 0; w < nwaves; ++w) {
      if (w < wave) before += wcount[w];
      round += wcount[w];
    }
    if (live) write_group_row(P, p, static_cast<int64_t>(pos0 + before) + __popcll(m & lanemask_lt()), O);
    pos0 += round;
  }
}


// ================================================================== host launchers
hipError_t hk_fill_u64(hipStream_t st, uint64_t* p, int64_t n, uint64_t v) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(hk_grid_for(n, 256, 8192)), dim3(256), 0, st, p, n, v);
  HK_CHECK_LAUNCH();
}

hipError_t hk_init_aggtable(hipStream_t st, uint64_t* words, int64_t nslots, const uint64_t* ident, int32_t nw) {
  HkIdent id = {};
  for (int i = 0; i < nw; ++i) id.w[i] = ident[i];
  id.nw = nw;
  hipLaunchKernelGGL(k_init_aggtable, dim3(hk_grid_for(nslots * nw, 256, 8192)), dim3(256), 0, st, words, nslots, id);
  HK_CHECK_LAUNCH();
}

hipError_t hk_fill_multi(hipStream_t st, const HkFills& f, int32_t k) {
  if (k <= 0) return hipSuccess;
  if (k > HK_MAX_FILLS) return hipErrorInvalidValue;
  int64_t n = 1;
  for (int32_t i = 0; i < k; ++i) n = std::max(n, f.n[i]);
  hipLaunchKernelGGL(k_fill_multi, dim3(hk_grid_for(n, 256, 8192), static_cast<uint32_t>(k)), dim3(256), 0, st, f);
  HK_CHECK_LAUNCH();
}

hipError_t hk_build(hipStream_t st, const HkBuild* B, const HkBuild* dB, int32_t nb, int ht, int hash, int* err) {
  if (nb <= 0) return hipSuccess;
  int64_t rows = 1;
  bool robin = false;
  for (int32_t i = 0; i < nb; ++i) {
    rows = std::max(rows, B[i].p.nrows);
    robin = robin || B[i].t.robin;
  }
  const dim3 g(hk_grid_for(rows, 256, 4096), static_cast<uint32_t>(nb)), b(256);
  DISPATCH2(ht, HT, DISPATCH2(hash, HS, hipLaunchKernelGGL((k_build<HT, HS>), g, b, 0, st, dB, err)));
  if (ht == HK_CUCKOO) {
    DISPATCH2(hash, HS, hipLaunchKernelGGL((k_build_verify<HS>), g, b, 0, st, dB, err));
  } else if (robin) {
    DISPATCH2(hash, HS, hipLaunchKernelGGL((k_build_verify_robin<HS>), g, b, 0, st, dB, err));
  }
  HK_CHECK_LAUNCH();
}

hipError_t hk_sp_concat(hipStream_t st, int64_t* const* tmp, int32_t nproj, int64_t region, int64_t nregions,
                        const uint32_t* counts, const uint32_t* offsets, int64_t* const* out) {
  HkOut T = {}, O = {};
  for (int c = 0; c < nproj; ++c) { T.col[c] = tmp[c]; O.col[c] = out[c]; }
  hipLaunchKernelGGL(k_sp_concat, dim3(hk_grid_for(nregions * WAVE, 256, 4096)), dim3(256), 0, st, T, nproj, region,
                     nregions, counts, offsets, O);
  HK_CHECK_LAUNCH();
}

// the status words (one per tile) and the tile counter, in u32 words
int64_t hk_scan_tmp_words(int64_t m) { return ((m + SCAN_TILE - 1) / SCAN_TILE + 1) * 2 + 2; }

hipError_t hk_scan(hipStream_t st, const uint32_t* in, uint32_t* out, int64_t m, uint32_t* tmp, uint64_t* total,
                   int* err) {
  const int64_t ntiles = m > 0 ? (m + SCAN_TILE - 1) / SCAN_TILE : 1;
  uint64_t* status = reinterpret_cast<uint64_t*>(tmp);
  unsigned int* counter = reinterpret_cast<unsigned int*>(status + ntiles);
  if (ntiles > 1) {
    // status words and counter start at zero (a kernel, not a memset node: the
    // scan may run inside a captured graph)
    const hipError_t e = hk_fill_u64(st, status, ntiles + 1, 0);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_scan_lb, dim3(static_cast<uint32_t>(ntiles)), dim3(1024), 0, st, in, out, m, status, counter,
                     total, err);
  HK_CHECK_LAUNCH();
}

hipError_t hk_finalize(hipStream_t st, const HkPlan& P, const HkPlan* dP, const HkAggTable& T, int64_t nslots, int64_t* const* gcols,
                       void* const* acols, int64_t* count, uint64_t* nrows, int keep_empty) {
  HkResOut O = {};
  for (int g = 0; g < P.ngroup; ++g) O.gcol[g] = gcols[g];
  for (int a = 0; a < P.naggs; ++a) O.acol[a] = acols[a];
  O.count = count;
  O.nrows = reinterpret_cast<unsigned long long*>(nrows);
  O.keep_empty = keep_empty;
  if (nslots <= 0) return hipSuccess;
  const int64_t nwg = std::min<int64_t>(1024, (nslots + 2047) / 2048);
  const int64_t chunk = (nslots + nwg - 1) / nwg;
  hipLaunchKernelGGL(k_finalize, dim3(static_cast<uint32_t>(nwg)), dim3(256), 0, st, dP, T, nslots, chunk, O);
  HK_CHECK_LAUNCH();
}
