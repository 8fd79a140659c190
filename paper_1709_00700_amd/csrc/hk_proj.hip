// Projection pipelines (Section 4.1): the multi-pass (fine-grained) strategy
// with its filter and projection kernels, and the single-pass (coarse-grained)
// strategy with one pipeline instance per compute unit. Compiled once per
// shape class (-DHK_SHAPE_CLASS=HkShapeX).
#include <hip/hip_runtime.h>

#include "hawk_device.h"
#include "hawk_launch.h"

#ifndef HK_SHAPE_CLASS
#error "compile once per shape class with -DHK_SHAPE_CLASS=HkShapeX"
#endif

// ------------------------------------------------------------------ projection: multi-pass (Section 4.1)
// Phase 1, filter kernel: evaluates filters and probes and records one flag
// bit per row (64-bit words, one per 64-row block) plus the number of flags
// per scan unit (a 64-row block for coalesced access, a thread's chunk for
// sequential access).
template <int MEM, int PRED, int HT, int HASH, class S>
__global__ void __launch_bounds__(256) k_mp_filter(HkPlan P, uint64_t* __restrict__ masks, uint32_t* __restrict__ counts) {
  v16i64 r = {};
  const int64_t n = P.nrows;
  const int64_t T = (int64_t)gridDim.x * blockDim.x;
  const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (MEM == HK_COAL) {
    // lanes of one wave cover one 64-row block per iteration: id = thread, id += threads
    for (int64_t base = gt - __lane_id(); base < n; base += T) {
      const int64_t row = base + __lane_id();
      bool pass = false;
      if (row < n) pass = eval_row<PRED, HT, HASH, false, S>(P, row, r);
      const uint64_t m = __ballot(pass);
      if (__lane_id() == 0) {
        masks[base >> 6] = m;
        counts[base >> 6] = static_cast<uint32_t>(__popcll(m));
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

// Phase 3, projection kernel: repeats the probes to get the payloads, computes
// the arithmetic and writes each qualifying row at its scanned position.
template <int MEM, int PRED, int HT, int HASH, class S>
__global__ void __launch_bounds__(256) k_mp_project(HkPlan P, const uint64_t* __restrict__ masks,
                                                    const uint32_t* __restrict__ offsets, const uint64_t* total,
                                                    int64_t nact, HkOut O) {
  v16i64 r = {};
  const int64_t n = P.nrows;
  const int64_t T = (int64_t)gridDim.x * blockDim.x;
  const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (MEM == HK_COAL) {
    for (int64_t base = gt - __lane_id(); base < n; base += T) {
      const uint64_t m = masks[base >> 6];
      if (PRED == HK_BR && m == 0) continue;
      const int64_t row = base + __lane_id();
      const bool pass = (m >> __lane_id()) & 1ull;
      const int64_t pos = offsets[base >> 6] + __popcll(m & lanemask_lt());
      if (PRED == HK_BR) {
        if (pass) {
          eval_row<HK_BR, HT, HASH, true, S>(P, row, r);
          write_proj<S>(P, O, pos, r);
        }
      } else if (row < n) {
        eval_row<HK_PRED, HT, HASH, true, S>(P, row, r);
        write_proj<S>(P, O, pass ? pos : O.dump, r);
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

// ------------------------------------------------------------------ projection: single-pass (Section 4.1)
// Coarse-grained: one pipeline instance per compute unit (one wavefront each)
// runs the whole pipeline over a contiguous chunk and appends results to its
// own region; the regions are concatenated in order afterwards.
//   coalesced: the wave walks its chunk 64 rows at a time; ballot + mbcnt keep row order
//   sequential: each lane walks a sub-chunk and owns a region of sub + 1 slots
template <int MEM, int PRED, int HT, int HASH, class S>
__global__ void __launch_bounds__(64) k_sp(HkPlan P, HkOut tmp, int64_t region, uint32_t* __restrict__ counts) {
  v16i64 r = {};
  const int64_t n = P.nrows;
  const int64_t inst = blockIdx.x;
  int64_t b, e;
  seq_range(n, inst, gridDim.x, WAVE, b, e);
  if (MEM == HK_COAL) {
    const int64_t rs = inst * region;  // region holds chunk + 1 slots
    int64_t wpos = 0;
    for (int64_t base = b; base < e; base += WAVE) {
      const int64_t row = base + __lane_id();
      if (PRED == HK_BR) {
        bool pass = false;
        if (row < e) pass = eval_row<HK_BR, HT, HASH, true, S>(P, row, r);
        const uint64_t m = __ballot(pass);
        if (pass) write_proj<S>(P, tmp, rs + wpos + __popcll(m & lanemask_lt()), r);
        wpos += __popcll(m);
      } else {
        bool pass = false;
        if (row < e) pass = eval_row<HK_PRED, HT, HASH, true, S>(P, row, r);
        const uint64_t m = __ballot(pass);
        if (row < e) write_proj<S>(P, tmp, pass ? rs + wpos + __popcll(m & lanemask_lt()) : rs + region - 1, r);
        wpos += __popcll(m);
      }
    }
    if (__lane_id() == 0) counts[inst] = static_cast<uint32_t>(wpos);
  } else {
    int64_t lb, le;
    seq_range(e - b, __lane_id(), WAVE, 1, lb, le);
    lb += b;
    le += b;
    const int64_t rs = (inst * WAVE + __lane_id()) * region;  // region holds sub + 1 slots
    int64_t pos = 0;
    for (int64_t row = lb; row < le; ++row) {
      if (PRED == HK_BR) {
        if (eval_row<HK_BR, HT, HASH, true, S>(P, row, r)) write_proj<S>(P, tmp, rs + pos++, r);
      } else {
        const bool pass = eval_row<HK_PRED, HT, HASH, true, S>(P, row, r);
        write_proj<S>(P, tmp, rs + pos, r);
        pos += pass;
      }
    }
    counts[inst * WAVE + __lane_id()] = static_cast<uint32_t>(pos);
  }
}


// ================================================================== launchers for one shape class
template <class S>
hipError_t hk_mp_filter_shape(hipStream_t st, const HkPlan& P, int mem, int pred, int ht, int hash, int64_t threads,
                              uint64_t* masks, uint32_t* counts) {
  const dim3 g(static_cast<uint32_t>((threads + 255) / 256)), b(256);
  DISPATCH2(mem, M, DISPATCH2(pred, PR, DISPATCH2(ht, HT, DISPATCH2(hash, HS,
            hipLaunchKernelGGL((k_mp_filter<M, PR, HT, HS, S>), g, b, 0, st, P, masks, counts)))));
  return hipGetLastError();
}

template <class S>
hipError_t hk_mp_project_shape(hipStream_t st, const HkPlan& P, int mem, int pred, int ht, int hash, int64_t threads,
                               const uint64_t* masks, const uint32_t* offsets, const uint64_t* total, int64_t nact,
                               const HkOut& O) {
  const dim3 g(static_cast<uint32_t>((threads + 255) / 256)), b(256);
  DISPATCH2(mem, M, DISPATCH2(pred, PR, DISPATCH2(ht, HT, DISPATCH2(hash, HS,
            hipLaunchKernelGGL((k_mp_project<M, PR, HT, HS, S>), g, b, 0, st, P, masks, offsets, total, nact, O)))));
  return hipGetLastError();
}

template <class S>
hipError_t hk_sp_shape(hipStream_t st, const HkPlan& P, int mem, int pred, int ht, int hash, int64_t instances,
                       const HkOut& O, int64_t region, uint32_t* counts) {
  const dim3 g(static_cast<uint32_t>(instances)), b(WAVE);
  DISPATCH2(mem, M, DISPATCH2(pred, PR, DISPATCH2(ht, HT, DISPATCH2(hash, HS,
            hipLaunchKernelGGL((k_sp<M, PR, HT, HS, S>), g, b, 0, st, P, O, region, counts)))));
  return hipGetLastError();
}

template hipError_t hk_mp_filter_shape<HK_SHAPE_CLASS>(hipStream_t, const HkPlan&, int, int, int, int, int64_t,
                                                       uint64_t*, uint32_t*);
template hipError_t hk_mp_project_shape<HK_SHAPE_CLASS>(hipStream_t, const HkPlan&, int, int, int, int, int64_t,
                                                        const uint64_t*, const uint32_t*, const uint64_t*, int64_t,
                                                        const HkOut&);
template hipError_t hk_sp_shape<HK_SHAPE_CLASS>(hipStream_t, const HkPlan&, int, int, int, int, int64_t, const HkOut&,
                                                int64_t, uint32_t*);
