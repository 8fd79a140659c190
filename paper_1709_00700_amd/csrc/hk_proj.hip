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

#include "hk_proj_body.h"

// ------------------------------------------------------------------ multi-pass kernels (bodies in hk_proj_body.h)
template <int MEM, int PRED, int HT, int HASH, class S, int U>
__global__ void __launch_bounds__(256) k_mp_filter(HkPlan P, uint64_t* __restrict__ masks, uint32_t* __restrict__ counts) {
  mp_filter_body<MEM, PRED, HT, HASH, S, U>(P, masks, counts);
}

template <class S>
__global__ void __launch_bounds__(256) k_mp_filter_simd(HkPlan P, uint64_t* __restrict__ masks,
                                                         uint32_t* __restrict__ counts) {
  mp_filter_simd_body<S>(P, masks, counts);
}

template <int MEM, int PRED, int HT, int HASH, class S>
__global__ void __launch_bounds__(256) k_mp_project(HkPlan P, const uint64_t* __restrict__ masks,
                                                    const uint32_t* __restrict__ offsets, const uint64_t* total,
                                                    int64_t nact, HkOut O) {
  mp_project_body<MEM, PRED, HT, HASH, S>(P, masks, offsets, total, nact, O);
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
                              uint64_t* masks, uint32_t* counts, int unroll, int simd) {
  const dim3 g(static_cast<uint32_t>((threads + 255) / 256)), b(256);
  if (simd) {
    // coalesced scans of filter columns only (no probes)
    if constexpr (S::filters > 0) {
      if (mem != HK_COAL || P.nprobes > 0) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_mp_filter_simd<S>), g, b, 0, st, P, masks, counts);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (mem == HK_COAL) {
    const int u = unroll == 1 ? 1 : unroll == 2 ? 2 : 4;  // 0: the default 4
    DISPATCH2(pred, PR, DISPATCH2(ht, HT, DISPATCH2(hash, HS, switch (u) {
      case 1: hipLaunchKernelGGL((k_mp_filter<HK_COAL, PR, HT, HS, S, 1>), g, b, 0, st, P, masks, counts); break;
      case 2: hipLaunchKernelGGL((k_mp_filter<HK_COAL, PR, HT, HS, S, 2>), g, b, 0, st, P, masks, counts); break;
      default: hipLaunchKernelGGL((k_mp_filter<HK_COAL, PR, HT, HS, S, 4>), g, b, 0, st, P, masks, counts);
    })));
  } else {
    DISPATCH2(pred, PR, DISPATCH2(ht, HT, DISPATCH2(hash, HS,
              hipLaunchKernelGGL((k_mp_filter<HK_SEQ, PR, HT, HS, S, 1>), g, b, 0, st, P, masks, counts))));
  }
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
                                                       uint64_t*, uint32_t*, int, int);
template hipError_t hk_mp_project_shape<HK_SHAPE_CLASS>(hipStream_t, const HkPlan&, int, int, int, int, int64_t,
                                                        const uint64_t*, const uint32_t*, const uint64_t*, int64_t,
                                                        const HkOut&);
template hipError_t hk_sp_shape<HK_SHAPE_CLASS>(hipStream_t, const HkPlan&, int, int, int, int, int64_t, const HkOut&,
                                                int64_t, uint32_t*);
