// Run-time specialisation of the grouped-aggregation kernel for one plan
// structure (the variant generation of Section 7, done with hipRTC): the
// kernel body of hk_agg_body.h is compiled with the plan's structure
// (column types and registers, operators, aggregates, counts) as constants,
// while data that differs between queries of one structure (column
// pointers, filter bounds, arithmetic constants, join tables, hash seeds,
// row count) stays a kernel argument. The local table is a static LDS array
// of the launch's size. Kernels are cached per context by their generated
// source.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "hawk_plan.h"

// fn == nullptr: compiled but refused (the launch functions then return
// hipErrorNotSupported and the caller runs the ahead-of-time kernel)
struct JitKernel { hipModule_t module; hipFunction_t fn; };
struct JitCache {
  std::map<std::string, JitKernel> kernels;
  bool compile_only = false;  // compile, load nothing and keep nothing (hawk_jit_compile_check)
  int64_t compiled = 0;
  double compile_ms = 0;
  std::string last_error;  // compiler log of the last failed compilation
  void release();
};

// Generated source of the specialised kernel `hk_jit_agg` for (P, variant).
// The join tables of probes stage[0..nstage) (sizes from P) are copied into
// each workgroup's LDS after its lds_bytes of local table.
std::string jit_agg_source(const HkPlan& P, int mem, int pred, int ht, int hash, int strat, bool spill,
                           size_t lds_bytes, int32_t wg, const int32_t* stage, int32_t nstage);
// Compiles the specialised kernel unless the cache holds it (no GPU work).
hipError_t jit_agg_prepare(JitCache& cache, std::string& err_msg, const HkPlan& P, int mem, int pred, int hash,
                           int strat, int32_t wg, uint32_t llog2, int32_t nw, int32_t reps, const HkSpill* sp,
                           const int32_t* stage, int32_t nstage);
// Compiles (or finds) and launches the specialised kernel; same arguments and
// launch shape as the ahead-of-time k_agg. Linear probing only.
hipError_t jit_agg_launch(JitCache& cache, std::string& err_msg, hipStream_t st, const HkPlan& P,
                          const HkAggTable& T, int mem, int pred, int hash, int strat, int64_t groups, int32_t wg,
                          uint32_t llog2, const HkIdent& id, int* err, const HkSpill* sp, int32_t reps,
                          const int32_t* stage, int32_t nstage);

// Run-time specialisation of the AGGREGATE kernel without grouping
// attributes (body in hk_scalar_body.h), `hk_jit_scalar`; same arguments and
// launch shape as the ahead-of-time k_scalar_agg. Linear probing only.
std::string jit_scalar_source(const HkPlan& P, int mem, int pred, int hash, int strat, int32_t wg);
hipError_t jit_scalar_prepare(JitCache& cache, std::string& err_msg, const HkPlan& P, int mem, int pred, int hash,
                              int strat, int32_t wg);
hipError_t jit_scalar_launch(JitCache& cache, std::string& err_msg, hipStream_t st, const HkPlan& P,
                             const HkAggTable& T, int mem, int pred, int hash, int strat, int64_t groups, int32_t wg,
                             const HkIdent& id);

// Run-time specialisation of the multi-pass projection kernels (bodies in
// hk_proj_body.h) for one plan structure, same arguments and launch shape as
// the ahead-of-time kernels.
enum { JIT_MP_FILTER = 0, JIT_MP_FILTER_SIMD = 1, JIT_MP_PROJECT = 2 };
std::string jit_proj_source(const HkPlan& P, int which, int mem, int pred, int ht, int hash, int unroll);
hipError_t jit_proj_prepare(JitCache& cache, std::string& err_msg, const HkPlan& P, int which, int mem, int pred,
                            int ht, int hash, int unroll);
hipError_t jit_mp_filter_launch(JitCache& cache, std::string& err_msg, hipStream_t st, const HkPlan& P, int simd,
                                int mem, int pred, int ht, int hash, int unroll, int64_t threads, uint64_t* masks,
                                uint32_t* counts);
hipError_t jit_mp_project_launch(JitCache& cache, std::string& err_msg, hipStream_t st, const HkPlan& P, int mem,
                                 int pred, int ht, int hash, int64_t threads, const uint64_t* masks,
                                 const uint32_t* offsets, const uint64_t* total, int64_t nact, const HkOut& O);
