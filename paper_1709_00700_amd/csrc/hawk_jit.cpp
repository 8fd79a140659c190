// Run-time specialisation of the grouped-aggregation kernel (see hawk_jit.h).
#include "hawk_jit.h"

#include <hip/hiprtc.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <sstream>

#include "hawk_device.h"
#include "hawk_launch.h"

namespace {

// the device headers, embedded at build time (raw string literals)
#include "hk_jit_sources.inc"

void emit_col(std::ostringstream& o, const char* arr, int c, const HkCol& col) {
  o << "  P." << arr << "[" << c << "].ptr = Prt." << arr << "[" << c << "].ptr; P." << arr << "[" << c
    << "].dtype = " << col.dtype << "; P." << arr << "[" << c << "].side = " << col.side << "; P." << arr << "["
    << c << "].reg = " << col.reg << ";\n";
}

}  // namespace

void JitCache::release() {
  for (auto& k : kernels)
    if (k.second.module) (void)hipModuleUnload(k.second.module);
  kernels.clear();
}

namespace {

// `P`'s structure as constants of a local plan P; the data that differs
// between queries of one structure is copied from the argument Prt
void emit_structure(std::ostringstream& o, const HkPlan& P) {
  o << "  HkPlan P;\n"
       "  P.nrows = Prt.nrows;\n  P.hash = Prt.hash;\n";
  o << "  P.ncolA = " << P.ncolA << "; P.ncolB = " << P.ncolB << "; P.ncolC = " << P.ncolC
    << "; P.nfilters = " << P.nfilters << "; P.liveA = " << P.liveA << "u; P.xinner = 0;\n";
  for (int c = 0; c < P.ncolA; ++c) emit_col(o, "colA", c, P.colA[c]);
  for (int c = 0; c < P.ncolB; ++c) emit_col(o, "colB", c, P.colB[c]);
  for (int c = 0; c < P.ncolC; ++c) emit_col(o, "colC", c, P.colC[c]);
  for (int f = 0; f < P.nfilters; ++f)
    o << "  P.filters[" << f << "].lo = Prt.filters[" << f << "].lo; P.filters[" << f << "].hi = Prt.filters[" << f
      << "].hi; P.filters[" << f << "].reg = " << P.filters[f].reg << ";\n";
  o << "  P.nprobes = " << P.nprobes << "; P.narith = " << P.narith << "; P.ngroup = " << P.ngroup
    << "; P.naggs = " << P.naggs << ";\n";
  for (int p = 0; p < P.nprobes; ++p)
    o << "  P.probes[" << p << "].t = Prt.probes[" << p << "].t; P.probes[" << p << "].fk_reg = " << P.probes[p].fk_reg
      << "; P.probes[" << p << "].pay_reg = " << P.probes[p].pay_reg << ";\n";
  for (int k = 0; k < P.narith; ++k) {
    const HkArith& A = P.arith[k];
    o << "  P.arith[" << k << "].cx = Prt.arith[" << k << "].cx; P.arith[" << k << "].cy = Prt.arith[" << k
      << "].cy; P.arith[" << k << "].op = " << int(A.op) << "; P.arith[" << k << "].dst = " << int(A.dst)
      << "; P.arith[" << k << "].x = " << int(A.x) << "; P.arith[" << k << "].y = " << int(A.y) << "; P.arith[" << k
      << "].xc = " << int(A.xc) << "; P.arith[" << k << "].yc = " << int(A.yc) << ";\n";
  }
  o << "  P.greg[0] = " << P.greg[0] << "; P.greg[1] = " << P.greg[1] << ";\n";
  for (int a = 0; a < P.naggs; ++a) {
    const HkAgg& A = P.aggs[a];
    o << "  P.aggs[" << a << "].fn = " << int(A.fn) << "; P.aggs[" << a << "].wide = " << int(A.wide) << "; P.aggs["
      << a << "].reg = " << int(A.reg) << "; P.aggs[" << a << "].word = " << A.word << ";\n";
  }
  o << "  P.nproj = " << P.nproj << ";\n";
  for (int c = 0; c < P.nproj; ++c) o << "  P.preg[" << c << "] = " << P.preg[c] << ";\n";
  o << "  P.slot_words = " << P.slot_words << ";\n";
}

// the compile-time shape of exactly this plan's counts
std::string exact_shape(const HkPlan& P, int naggs, int nproj) {
  std::ostringstream o;
  o << "HkShape<" << P.ncolA << ", " << P.nfilters << ", " << P.ncolB << ", " << P.nprobes << ", " << P.ncolC << ", "
    << P.narith << ", " << naggs << ", " << nproj << ">";
  return o.str();
}

}  // namespace

std::string jit_agg_source(const HkPlan& P, int mem, int pred, int ht, int hash, int strat, bool spill,
                           size_t lds_bytes, int32_t wg, const int32_t* stage, int32_t nstage) {
  std::ostringstream o;
  // the local table is a static LDS array of the launch's size (no dynamic
  // LDS), followed by the join tables copied into LDS (32-byte aligned)
  const size_t table_words = (lds_bytes + 31) / 32 * 4;
  size_t words = table_words;
  for (int32_t i = 0; i < nstage; ++i) words += size_t(1) << P.probes[stage[i]].t.log2cap;
  if (words == 0) words = 1;
  o << "#include \"hk_agg_body.h\"\n"
       "extern \"C\" __global__ void __launch_bounds__(" << wg << ") hk_jit_agg(HkPlan Prt, HkAggTable T, uint32_t llog2,\n"
       "    HkIdent id, int64_t nwg, int* err, HkSpill sp, int32_t reps) {\n"
       "  __shared__ __attribute__((aligned(32))) uint64_t lds[" << words << "];\n";
  HkPlan Q = P;
  Q.nproj = 0;
  emit_structure(o, Q);
  if (nstage > 0) {
    size_t off = table_words;
    for (int32_t i = 0; i < nstage; ++i) {
      const uint32_t l2 = P.probes[stage[i]].t.log2cap;
      o << "  stage_join(P.probes[" << stage[i] << "].t, lds + " << off << ", " << l2 << "u);\n";
      off += size_t(1) << l2;
    }
    o << "  __syncthreads();\n";
  }
  o << "  agg_body<" << mem << ", " << pred << ", " << ht << ", " << hash << ", " << strat << ", "
    << exact_shape(P, P.naggs, 0) << ", " << (spill ? "true" : "false") << ">(P, T, llog2, id, nwg, err, sp, reps, lds);\n}\n";
  return o.str();
}

std::string jit_scalar_source(const HkPlan& P, int mem, int pred, int hash, int strat, int32_t wg) {
  std::ostringstream o;
  o << "#include \"hk_scalar_body.h\"\n"
       "extern \"C\" __global__ void __launch_bounds__(" << wg << ") hk_jit_scalar(HkPlan Prt, HkAggTable T,\n"
       "    HkIdent id, int64_t nwg) {\n";
  HkPlan Q = P;
  Q.nproj = 0;
  emit_structure(o, Q);
  o << "  scalar_body<" << mem << ", " << pred << ", " << HK_LIN << ", " << hash << ", " << strat << ", "
    << exact_shape(P, P.naggs, 0) << ">(P, T, id, nwg);\n}\n";
  return o.str();
}

std::string jit_proj_source(const HkPlan& P, int which, int mem, int pred, int ht, int hash, int unroll) {
  std::ostringstream o;
  const std::string S = exact_shape(P, 0, P.nproj);
  const int u = unroll == 1 ? 1 : unroll == 2 ? 2 : 4;
  o << "#include \"hk_proj_body.h\"\n";
  if (which == JIT_MP_PROJECT) {
    o << "extern \"C\" __global__ void __launch_bounds__(256) hk_jit_proj(HkPlan Prt, const uint64_t* masks,\n"
         "    const uint32_t* offsets, const uint64_t* total, int64_t nact, HkOut O) {\n";
    emit_structure(o, P);
    o << "  mp_project_body<" << mem << ", " << pred << ", " << ht << ", " << hash << ", " << S
      << ">(P, masks, offsets, total, nact, O);\n}\n";
  } else {
    o << "extern \"C\" __global__ void __launch_bounds__(256) hk_jit_proj(HkPlan Prt, uint64_t* masks,\n"
         "    uint32_t* counts) {\n";
    emit_structure(o, P);
    if (which == JIT_MP_FILTER_SIMD) o << "  mp_filter_simd_body<" << S << ">(P, masks, counts);\n}\n";
    else
      o << "  mp_filter_body<" << mem << ", " << pred << ", " << ht << ", " << hash << ", " << S << ", "
        << (mem == HK_COAL ? u : 1) << ">(P, masks, counts);\n}\n";
  }
  return o.str();
}

namespace {

hipError_t get_kernel(JitCache& cache, std::string& err_msg, const std::string& src, hipFunction_t& fn,
                      const char* name = "hk_jit_agg") {
  auto it = cache.kernels.find(src);
  if (it == cache.kernels.end()) {
    const auto t0 = std::chrono::steady_clock::now();
    // HAWK_JIT_DUMP=<dir>: each generated source is also written there (for
    // reading or compiling it ahead of time with the library's headers)
    if (const char* dir = std::getenv("HAWK_JIT_DUMP")) {
      const std::string path = std::string(dir) + "/hk_jit_" + std::to_string(std::hash<std::string>{}(src)) + ".hip";
      if (FILE* f = std::fopen(path.c_str(), "w")) {
        std::fputs(src.c_str(), f);
        std::fclose(f);
      }
    }
    hiprtcProgram prog;
    const char* hs[] = {kSrcPlan, kSrcDevice, kSrcAggBody, kSrcProjBody, kSrcScalarBody};
    const char* hn[] = {"hawk_plan.h", "hawk_device.h", "hk_agg_body.h", "hk_proj_body.h", "hk_scalar_body.h"};
    if (hiprtcCreateProgram(&prog, src.c_str(), "hk_jit.hip", 5, hs, hn) != HIPRTC_SUCCESS) {
      err_msg = "hipRTC: program creation failed";
      return hipErrorInvalidValue;
    }
    const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                          "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, 7, opts);
    if (r != HIPRTC_SUCCESS) {
      size_t ls = 0;
      (void)hiprtcGetProgramLogSize(prog, &ls);
      std::string log(ls, '\0');
      if (ls) (void)hiprtcGetProgramLog(prog, &log[0]);
      (void)hiprtcDestroyProgram(&prog);
      err_msg = std::string("hipRTC: ") + hiprtcGetErrorString(r) + ": " + log.substr(0, 2000);
      return hipErrorInvalidValue;
    }
    size_t cs = 0;
    (void)hiprtcGetCodeSize(prog, &cs);
    std::vector<char> code(cs);
    (void)hiprtcGetCode(prog, code.data());
    (void)hiprtcDestroyProgram(&prog);
    if (cache.compile_only) {
      fn = nullptr;
      if (cs == 0) {
        err_msg = "hipRTC: empty code object";
        return hipErrorInvalidValue;
      }
      return hipSuccess;
    }
    JitKernel k{};
    hipError_t e = hipModuleLoadData(&k.module, code.data());
    if (e != hipSuccess) {
      err_msg = "module load of the specialised kernel failed";
      return e;
    }
    e = hipModuleGetFunction(&k.fn, k.module, name);
    if (e != hipSuccess) {
      (void)hipModuleUnload(k.module);
      err_msg = "specialised kernel not found in its module";
      return e;
    }
    // the kernel's LDS must fit one workgroup's maximum (a launch beyond it would abort the queue)
    int shared = 0, dev = 0, maxl = 0;
    if (hipFuncGetAttribute(&shared, HIP_FUNC_ATTRIBUTE_SHARED_SIZE_BYTES, k.fn) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&maxl, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || shared > maxl) {
      (void)hipModuleUnload(k.module);
      err_msg = "the specialised kernel's LDS exceeds a workgroup's maximum";
      return hipErrorInvalidValue;
    }
    cache.compile_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    ++cache.compiled;
    // a kernel that spills registers to scratch memory is not launched: the
    // caller runs the kernel compiled ahead of time instead (kept as refused)
    int priv = 0;
    if (hipFuncGetAttribute(&priv, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, k.fn) != hipSuccess || priv > 0) {
      (void)hipModuleUnload(k.module);
      k = JitKernel{};
    }
    it = cache.kernels.emplace(src, k).first;
  }
  fn = it->second.fn;
  if (!fn) {
    err_msg = "the specialised kernel needs scratch memory";
    return hipErrorNotSupported;
  }
  return hipSuccess;
}

}  // namespace

hipError_t jit_agg_prepare(JitCache& cache, std::string& err_msg, const HkPlan& P, int mem, int pred, int hash,
                           int strat, int32_t wg, uint32_t llog2, int32_t nw, int32_t reps, const HkSpill* sp,
                           const int32_t* stage, int32_t nstage) {
  hipFunction_t fn;
  const size_t lds = hk_agg_lds_bytes(strat, llog2, nw, reps, sp);
  return get_kernel(cache, err_msg,
                    jit_agg_source(P, mem, pred, HK_LIN, hash, strat, sp != nullptr, lds, wg, stage, nstage), fn);
}

hipError_t jit_agg_launch(JitCache& cache, std::string& err_msg, hipStream_t st, const HkPlan& P,
                          const HkAggTable& T, int mem, int pred, int hash, int strat, int64_t groups, int32_t wg,
                          uint32_t llog2, const HkIdent& id, int* err, const HkSpill* sp, int32_t reps,
                          const int32_t* stage, int32_t nstage) {
  hipFunction_t fn;
  const size_t lds = hk_agg_lds_bytes(strat, llog2, id.nw, reps, sp);
  const hipError_t ge = get_kernel(
      cache, err_msg, jit_agg_source(P, mem, pred, HK_LIN, hash, strat, sp != nullptr, lds, wg, stage, nstage), fn);
  if (ge != hipSuccess) return ge;
  HkSpill none;
  std::memset(&none, 0, sizeof(none));
  HkPlan Pa = P;
  HkAggTable Ta = T;
  HkIdent ida = id;
  HkSpill spa = sp ? *sp : none;
  int64_t nwg = groups;
  int* erra = err;
  uint32_t ll = llog2;
  int32_t rp = reps;
  void* args[] = {&Pa, &Ta, &ll, &ida, &nwg, &erra, &spa, &rp};
  const dim3 g = hk_wg_grid(groups);
  return hipModuleLaunchKernel(fn, g.x, g.y, 1, static_cast<uint32_t>(wg), 1, 1, 0, st, args, nullptr);
}

hipError_t jit_scalar_prepare(JitCache& cache, std::string& err_msg, const HkPlan& P, int mem, int pred, int hash,
                              int strat, int32_t wg) {
  hipFunction_t fn;
  return get_kernel(cache, err_msg, jit_scalar_source(P, mem, pred, hash, strat, wg), fn, "hk_jit_scalar");
}

hipError_t jit_scalar_launch(JitCache& cache, std::string& err_msg, hipStream_t st, const HkPlan& P,
                             const HkAggTable& T, int mem, int pred, int hash, int strat, int64_t groups, int32_t wg,
                             const HkIdent& id) {
  hipFunction_t fn;
  const hipError_t ge =
      get_kernel(cache, err_msg, jit_scalar_source(P, mem, pred, hash, strat, wg), fn, "hk_jit_scalar");
  if (ge != hipSuccess) return ge;
  HkPlan Pa = P;
  HkAggTable Ta = T;
  HkIdent ida = id;
  int64_t nwg = groups;
  void* args[] = {&Pa, &Ta, &ida, &nwg};
  const dim3 g = hk_wg_grid(groups);
  return hipModuleLaunchKernel(fn, g.x, g.y, 1, static_cast<uint32_t>(wg), 1, 1, 0, st, args, nullptr);
}

hipError_t jit_proj_prepare(JitCache& cache, std::string& err_msg, const HkPlan& P, int which, int mem, int pred,
                            int ht, int hash, int unroll) {
  hipFunction_t fn;
  return get_kernel(cache, err_msg, jit_proj_source(P, which, mem, pred, ht, hash, unroll), fn, "hk_jit_proj");
}

hipError_t jit_mp_filter_launch(JitCache& cache, std::string& err_msg, hipStream_t st, const HkPlan& P, int simd,
                                int mem, int pred, int ht, int hash, int unroll, int64_t threads, uint64_t* masks,
                                uint32_t* counts) {
  hipFunction_t fn;
  const int which = simd ? JIT_MP_FILTER_SIMD : JIT_MP_FILTER;
  const hipError_t ge =
      get_kernel(cache, err_msg, jit_proj_source(P, which, mem, pred, ht, hash, unroll), fn, "hk_jit_proj");
  if (ge != hipSuccess) return ge;
  HkPlan Pa = P;
  void* args[] = {&Pa, &masks, &counts};
  return hipModuleLaunchKernel(fn, static_cast<uint32_t>((threads + 255) / 256), 1, 1, 256, 1, 1, 0, st, args, nullptr);
}

hipError_t jit_mp_project_launch(JitCache& cache, std::string& err_msg, hipStream_t st, const HkPlan& P, int mem,
                                 int pred, int ht, int hash, int64_t threads, const uint64_t* masks,
                                 const uint32_t* offsets, const uint64_t* total, int64_t nact, const HkOut& O) {
  hipFunction_t fn;
  const hipError_t ge =
      get_kernel(cache, err_msg, jit_proj_source(P, JIT_MP_PROJECT, mem, pred, ht, hash, 0), fn, "hk_jit_proj");
  if (ge != hipSuccess) return ge;
  HkPlan Pa = P;
  HkOut Oa = O;
  int64_t na = nact;
  void* args[] = {&Pa, &masks, &offsets, &total, &na, &Oa};
  return hipModuleLaunchKernel(fn, static_cast<uint32_t>((threads + 255) / 256), 1, 1, 256, 1, 1, 0, st, args, nullptr);
}
