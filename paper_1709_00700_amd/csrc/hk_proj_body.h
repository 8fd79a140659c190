// Bodies of the multi-pass projection kernels (Section 4.1): the filter
// kernel (scalar, unrolled, or FILTER in SIMD mode) and the projection
// kernel. The ahead-of-time kernels (hk_proj.hip, one build per shape class)
// take the plan as an argument; a kernel compiled at run time for one plan
// (hawk_jit.cpp) calls the same bodies with the plan's structure as
// constants.
#pragma once
#include "hawk_device.h"

// ------------------------------------------------------------------ projection: multi-pass (Section 4.1)
// Phase 1, filter kernel: evaluates filters and probes and records one flag
// bit per row (64-bit words, one per 64-row block) plus the number of flags
// per scan unit (a 64-row block for coalesced access, a thread's chunk for
// sequential access).
// U (coalesced access): rows per loop iteration, the loop unrolled U times
// with element access offsets 0..U-1 (Section 6.1); the first load phase of
// the next U-1 rows is in flight while one is evaluated.
template <int MEM, int PRED, int HT, int HASH, class S, int U>
__device__ __forceinline__ void mp_filter_body(const HkPlan& P, uint64_t* __restrict__ masks,
                                               uint32_t* __restrict__ counts) {
  v16i64 r = {};
  const int64_t n = P.nrows;
  const int64_t T = (int64_t)gridDim.x * blockDim.x;
  const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (MEM == HK_COAL) {
    // lanes of one wave cover one 64-row block per iteration: id = thread,
    // id += threads. Software pipeline: the first load phase of the next AH
    // blocks is in flight while a block is evaluated; the loop is unrolled by
    // the ring size so every buffer index is a constant.
    constexpr int NB = U, AH = U - 1;
    HkFirst<S> f[NB] = {};
    const int64_t b0 = gt - __lane_id();
    // rows past the end fetch the last row again (the fetch count stays fixed)
    auto at = [&](int64_t row) { return row < n ? row : n - 1; };
    if (b0 < n) {
#pragma unroll
      for (int k = 0; k < AH; ++k) fetch_first<S>(P, at(b0 + k * T + __lane_id()), f[k]);
    }
    for (int64_t base = b0; base < n; base += NB * T) {
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const int64_t bk = base + k * T;
        if (bk >= n) break;  // uniform over the wave
        fetch_first<S>(P, at(bk + AH * T + __lane_id()), f[(k + AH) % NB]);
        const int64_t row = bk + __lane_id();
        bool pass = false;
        if (row < n) pass = eval_row_f<PRED, HT, HASH, false, S, true>(P, row, f[k], r);
        const uint64_t m = __ballot(pass);
        if (__lane_id() == 0) {
          masks[bk >> 6] = m;
          counts[bk >> 6] = static_cast<uint32_t>(__popcll(m));
        }
      }
    }
  } else {
    int64_t b, e;
    seq_range(n, gt, T, WAVE, b, e);
    if (b >= e) return;  // threads past the last chunk own no scan entry
    uint32_t cnt = 0;
    for (int64_t w0 = b; w0 < e; w0 += WAVE) {
      uint64_t m = 0;
      const int64_t we = w0 + WAVE < e ? w0 + WAVE : e;
      for (int64_t row = w0; row < we; ++row) {
        const bool pass = eval_row<PRED, HT, HASH, false, S>(P, row, r);
        if (PRED == HK_PRED) m |= static_cast<uint64_t>(pass) << (row - w0);
        else if (pass) m |= 1ull << (row - w0);
      }
      masks[w0 >> 6] = m;
      cnt += static_cast<uint32_t>(__popcll(m));
    }
    counts[gt] = cnt;
  }
}

// Phase 1 with FILTER in SIMD mode (coalesced, no probes): the scan of Zhou
// and Ross checks the predicate on several tuples at once. Each lane loads 4
// consecutive rows of every filter column with one vector load and evaluates
// the conjunction on all 4; a wave covers 256 rows, whose four 64-bit flag
// words are interleaved from four ballots (lane i's row j is bit 4i + j of
// its word). Filter columns are 16-byte aligned (checked on the host).
__device__ __forceinline__ uint64_t spread4(uint64_t x) {  // bit i -> bit 4i, i < 16
  x &= 0xFFFFull;
  x = (x | (x << 24)) & 0x000000FF000000FFull;
  x = (x | (x << 12)) & 0x000F000F000F000Full;
  x = (x | (x << 6)) & 0x0303030303030303ull;
  x = (x | (x << 3)) & 0x1111111111111111ull;
  return x;
}

__device__ __forceinline__ void load4(const HkCol& c, int64_t r0, int64_t* v) {
  if (c.dtype == HK_T_I32) {
    const int4 q = *reinterpret_cast<const int4*>(static_cast<const int32_t*>(c.ptr) + r0);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  } else if (c.dtype == HK_T_I64) {
    const longlong2 a = *reinterpret_cast<const longlong2*>(static_cast<const int64_t*>(c.ptr) + r0);
    const longlong2 b = *reinterpret_cast<const longlong2*>(static_cast<const int64_t*>(c.ptr) + r0 + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  } else {
    const int32_t q = *reinterpret_cast<const int32_t*>(static_cast<const int8_t*>(c.ptr) + r0);
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = static_cast<int8_t>(static_cast<uint32_t>(q) >> (8 * j));
  }
}

template <class S>
__device__ __forceinline__ void mp_filter_simd_body(const HkPlan& P, uint64_t* __restrict__ masks,
                                                    uint32_t* __restrict__ counts) {
  const int64_t n = P.nrows;
  const int64_t T = (int64_t)gridDim.x * blockDim.x;
  const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int lane = __lane_id();
  for (int64_t base = 4 * (gt - lane); base < n; base += 4 * T) {
    const int64_t r0 = base + 4 * lane;
    int64_t v[S::colA > 0 ? S::colA : 1][4];
    if (r0 + 3 < n) {
#pragma unroll
      for (int c = 0; c < S::colA; ++c)
        if (c < P.ncolA) load4(P.colA[c], r0, v[c]);
    } else {
      // the last rows, one at a time (no load past the column's end)
#pragma unroll
      for (int c = 0; c < S::colA; ++c)
        if (c < P.ncolA)
#pragma unroll
          for (int j = 0; j < 4; ++j) v[c][j] = r0 + j < n ? load_col(P.colA[c], r0 + j) : 0;
    }
    uint32_t m4 = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bool pass = r0 + j < n;
#pragma unroll
      for (int f = 0; f < S::filters; ++f) {
        if (f >= P.nfilters) break;
        int64_t x = 0;
#pragma unroll
        for (int c = 0; c < S::colA; ++c)
          if (c < P.ncolA && P.colA[c].reg == P.filters[f].reg) x = v[c][j];
        pass = pass & (x >= P.filters[f].lo) & (x <= P.filters[f].hi);
      }
      m4 |= static_cast<uint32_t>(pass) << j;
    }
    uint64_t b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = __ballot((m4 >> j) & 1u);
    if (lane < 4 && base + 64 * lane < n) {
      uint64_t w = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) w |= spread4(b[j] >> (16 * lane)) << j;
      masks[(base >> 6) + lane] = w;
      counts[(base >> 6) + lane] = static_cast<uint32_t>(__popcll(w));
    }
  }
}

// Phase 3, projection kernel: repeats the probes to get the payloads, computes
// the arithmetic and writes each qualifying row at its scanned position.
template <int MEM, int PRED, int HT, int HASH, class S>
__device__ __forceinline__ void mp_project_body(const HkPlan& P, const uint64_t* __restrict__ masks,
                                                const uint32_t* __restrict__ offsets, const uint64_t* total,
                                                int64_t nact, const HkOut& O) {
  v16i64 r = {};
  const int64_t n = P.nrows;
  const int64_t T = (int64_t)gridDim.x * blockDim.x;
  const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (MEM == HK_COAL && PRED == HK_BR) {
    // The wave's blocks j = 0, 1, ... start at b0 + j * threads. Their
    // passing rows are handed to the lanes densely: for 64 blocks at a time,
    // lane l holds block j0 + l's flag word, offset and (scanned over the
    // lanes) the rank of its first passing row among those blocks; then the
    // i-th passing row goes to lane i % 64 of round i / 64, which finds its
    // block by a search over the ranks and its row as the matching set bit.
    // All lanes of a round evaluate rows, not a few lanes per block.
    const int64_t b0 = gt - __lane_id();
    if (b0 >= n) return;  // uniform over the wave
    const int64_t nbw = (n - b0 + T - 1) / T;  // blocks of this wave
    uint64_t mnext = 0;
    uint32_t onext = 0;
    auto load_batch = [&](int64_t j0, uint64_t& ml, uint32_t& ol) {
      const int64_t j = j0 + __lane_id();
      ml = 0;
      ol = 0;
      if (j < nbw) {
        const int64_t bi = (b0 + j * T) >> 6;
        ml = masks[bi];
        ol = offsets[bi];
      }
    };
    load_batch(0, mnext, onext);
    for (int64_t j0 = 0; j0 < nbw; j0 += WAVE) {
      const uint64_t ml = mnext;
      const uint32_t ol = onext;
      load_batch(j0 + WAVE, mnext, onext);  // the next 64 blocks' words in flight
      const uint32_t cl = static_cast<uint32_t>(__popcll(ml));
      // inclusive scan of the counts over the lanes
      uint32_t incl = cl;
#pragma unroll
      for (int d = 1; d < WAVE; d <<= 1) {
        const uint32_t t = __shfl_up(incl, d, WAVE);
        if (__lane_id() >= d) incl += t;
      }
      const uint32_t excl = incl - cl;
      const uint32_t total = __builtin_amdgcn_readlane(incl, WAVE - 1);
      for (uint32_t c0 = 0; c0 < total; c0 += WAVE) {
        const uint32_t i = c0 + __lane_id();
        // the last lane whose first rank is <= i holds row i (it has a
        // passing row: the next lane's first rank exceeds i)
        int src = 0;
#pragma unroll
        for (int step = WAVE / 2; step >= 1; step >>= 1) {
          const uint32_t e = __shfl(excl, src + step, WAVE);
          if (e <= i) src += step;
        }
        const uint64_t m = (static_cast<uint64_t>(static_cast<uint32_t>(__shfl(static_cast<int>(ml >> 32), src, WAVE))) << 32) |
                           static_cast<uint32_t>(__shfl(static_cast<int>(ml), src, WAVE));
        const uint32_t o = static_cast<uint32_t>(__shfl(static_cast<int>(ol), src, WAVE));
        uint32_t k = i - static_cast<uint32_t>(__shfl(static_cast<int>(excl), src, WAVE));
        const uint32_t rank = k;
        // position of the k-th set bit of m
        uint64_t x = m;
        int bit = 0;
#pragma unroll
        for (int w = 32; w >= 1; w >>= 1) {
          const uint32_t c = static_cast<uint32_t>(__popcll(x & ((1ull << w) - 1)));
          if (k >= c) {
            k -= c;
            x >>= w;
            bit += w;
          }
        }
        if (i < total) {
          const int64_t row = b0 + (j0 + src) * T + bit;
          HkAll<S> f;
          fetch_all<S>(P, row, f);
          eval_passing_row<HT, HASH, S>(P, row, f, r);
          write_proj<S>(P, O, static_cast<int64_t>(o) + rank, r);
        }
      }
    }
  } else if (MEM == HK_COAL) {
    // predicated: every row is evaluated and written (a dropped row to the
    // dump slot); the flag word and offset of the next AH blocks are in
    // flight while a block is projected
    constexpr int AH = 3, NB = AH + 1;
    uint64_t mk[NB] = {};
    uint32_t ok[NB] = {};
    const int64_t b0 = gt - __lane_id();
    const int64_t lastb = n > 0 ? (n - 1) >> 6 : 0;
    auto blk = [&](int64_t base) { return base < n ? base >> 6 : lastb; };
    if (b0 < n) {
#pragma unroll
      for (int k = 0; k < AH; ++k) {
        mk[k] = masks[blk(b0 + k * T)];
        ok[k] = offsets[blk(b0 + k * T)];
      }
    }
    for (int64_t base0 = b0; base0 < n; base0 += NB * T) {
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const int64_t base = base0 + k * T;
        if (base >= n) break;  // uniform over the wave
        mk[(k + AH) % NB] = masks[blk(base + AH * T)];
        ok[(k + AH) % NB] = offsets[blk(base + AH * T)];
        const uint64_t m = mk[k];
        const int64_t row = base + __lane_id();
        const bool pass = (m >> __lane_id()) & 1ull;
        const int64_t pos = ok[k] + __popcll(m & lanemask_lt());
        if (row < n) {
          eval_row<HK_PRED, HT, HASH, true, S>(P, row, r);
          write_proj<S>(P, O, pass ? pos : O.dump, r);
        }
      }
    }
  } else {
    int64_t b, e;
    seq_range(n, gt, T, WAVE, b, e);
    if (b >= e) return;
    int64_t pos = offsets[gt];
    if (PRED == HK_BR) {
      for (int64_t w0 = b; w0 < e; w0 += WAVE) {
        uint64_t m = masks[w0 >> 6];
        while (m) {
          const int bit = __ffsll(static_cast<unsigned long long>(m)) - 1;
          m &= m - 1;
          eval_row<HK_BR, HT, HASH, true, S>(P, w0 + bit, r);
          write_proj<S>(P, O, pos++, r);
        }
      }
    } else {
      // write every row, advance by result_increment; a trailing write past
      // this thread's range goes to the dump slot
      const int64_t end = gt + 1 < nact ? static_cast<int64_t>(offsets[gt + 1]) : static_cast<int64_t>(*total);
      for (int64_t row = b; row < e; ++row) {
        const bool pass = (masks[row >> 6] >> (row & 63)) & 1ull;
        eval_row<HK_PRED, HT, HASH, true, S>(P, row, r);
        write_proj<S>(P, O, pos < end ? pos : O.dump, r);
        pos += pass;
      }
    }
  }
}

