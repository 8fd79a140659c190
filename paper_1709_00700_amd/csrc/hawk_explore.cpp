// Variant exploration (Section 8): Algorithm 1 (feature-wise learning),
// exhaustive search ("backtracking", Section 9.3.2) as its judge, the pruning
// rule of Section 9.1 (variants above a time limit count as infinitely slow),
// a memo of measured configurations and an append-only timing log. Also the
// query/variant feature vector used by the learned cost model.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <string>
#include <vector>

#include "hawk.h"
#include "hawk_internal.h"

namespace {

const double kInf = std::numeric_limits<double>::infinity();
const uint32_t kMults[7] = {1, 8, 64, 256, 1024, 16384, 65536};
const uint32_t kWgs[7] = {16, 32, 64, 128, 256, 512, 1024};

}  // namespace

// ------------------------------------------------------------------ Algorithm 1
extern "C" hawk_status hawk_learn_feature_wise(const int32_t* dim_sizes, int32_t ndims, const int32_t* order, int32_t q,
                                               hawk_cost_fn cost, void* user, int32_t* best_cfg, int64_t* n_calls) {
  if (!dim_sizes || ndims < 1 || !cost || !best_cfg || q < 1) return HAWK_E_ARG;
  for (int32_t i = 0; i < ndims; ++i)
    if (dim_sizes[i] < 1) return HAWK_E_ARG;
  std::vector<int32_t> ord(static_cast<size_t>(ndims));
  for (int32_t i = 0; i < ndims; ++i) ord[i] = order ? order[i] : i;
  std::vector<char> seen(static_cast<size_t>(ndims), 0);
  for (int32_t i : ord) {
    if (i < 0 || i >= ndims || seen[i]) return HAWK_E_ARG;
    seen[i] = 1;
  }
  std::map<std::vector<int32_t>, double> memo;
  int64_t calls = 0;
  auto eval = [&](const std::vector<int32_t>& c) {
    auto it = memo.find(c);
    if (it != memo.end()) return it->second;
    ++calls;
    double t = cost(c.data(), ndims, user);
    if (std::isnan(t)) t = kInf;
    memo[c] = t;
    return t;
  };
  // start from the first value of every dimension
  std::vector<int32_t> v(static_cast<size_t>(ndims), 0);
  for (int32_t iter = 0; iter < q; ++iter) {
    const std::vector<int32_t> last = v;
    for (int32_t i : ord) {
      // vary dimension i only; keep the value with the lowest time (a strictly
      // lower time replaces the incumbent, so ties keep the earlier value)
      double best_t = kInf;
      int32_t best_d = -1;
      for (int32_t d = 0; d < dim_sizes[i]; ++d) {
        std::vector<int32_t> w = v;
        w[i] = d;
        const double t = eval(w);
        if (t < best_t) {
          best_t = t;
          best_d = d;
        }
      }
      if (best_d >= 0) v[i] = best_d;  // every value infeasible: keep the current one
    }
    if (v == last) break;  // fixed point: no faster configuration found in this sweep
  }
  std::memcpy(best_cfg, v.data(), sizeof(int32_t) * ndims);
  if (n_calls) *n_calls = calls;
  return HAWK_OK;
}

// ------------------------------------------------------------------ features
static double log2p1(double x) { return std::log2(x + 1.0); }

hawk_status query_features(const hawk_query* q, const hawk_variant* v, int num_cus, float* f) {
  const HkPlan& P = q->main;
  int bytes = 0;
  auto w = [](int32_t t) { return t == HK_T_I8 ? 1 : t == HK_T_I32 ? 4 : 8; };
  for (int i = 0; i < P.ncolA; ++i) bytes += w(P.colA[i].dtype);
  for (int i = 0; i < P.ncolB; ++i) bytes += w(P.colB[i].dtype);
  for (int i = 0; i < P.ncolC; ++i) bytes += w(P.colC[i].dtype);
  f[0] = static_cast<float>(log2p1(static_cast<double>(P.nrows)));
  f[1] = static_cast<float>(q->stat_selectivity);
  f[2] = static_cast<float>(q->kind == 2 ? log2p1(static_cast<double>(q->groups_hint)) : 0.0);
  f[3] = static_cast<float>(bytes);
  f[4] = static_cast<float>(P.nprobes);
  f[5] = static_cast<float>(q->kind == 1 ? 8 * P.nproj : 8 * P.slot_words);
  double threads, wg, strat;
  if (q->kind == 1) {
    strat = v->proj_strategy;
    threads = v->proj_strategy ? static_cast<double>(v->thread_mult) * num_cus : static_cast<double>(num_cus) * 64;
    wg = v->proj_strategy ? 256 : 64;
  } else {
    strat = v->agg_strategy;
    const double wgs = v->wg_size ? v->wg_size : 256;
    threads = v->agg_strategy == HAWK_LOCAL ? static_cast<double>(v->thread_mult) * num_cus * wgs
                                            : static_cast<double>(num_cus) * std::max(1.0, std::floor(2048.0 / wgs)) * wgs;
    wg = wgs;
  }
  f[6] = static_cast<float>(strat);
  f[7] = static_cast<float>(std::log2(threads));
  f[8] = static_cast<float>(std::log2(wg));
  // the extra dimensions share ordinal codes with the paper's: SIMD filter
  // with predication, unrolling with the access pattern (the default 4 rows
  // per iteration codes as 0), robin hood as a third table kind
  f[9] = static_cast<float>(v->pred + 2 * v->filter_mode);
  f[10] = static_cast<float>(v->mem + 2 * (v->unroll == 2 ? 1 : v->unroll == 1 ? 2 : 0));
  f[11] = static_cast<float>(q->has_table ? v->ht * 2 + v->hash : 0);
  return HAWK_OK;
}

extern "C" hawk_status hawk_features(const hawk_query* q, const hawk_variant* v, float* out12) {
  if (!q || !v || !out12 || !q->ctx) return HAWK_E_ARG;
  return query_features(q, v, q->ctx->num_cus, out12);
}

extern "C" hawk_status hawk_query_set_stats(hawk_query* q, double selectivity) {
  if (!q || !(selectivity >= 0.0 && selectivity <= 1.0)) return HAWK_E_ARG;
  q->stat_selectivity = selectivity;
  return HAWK_OK;
}

// ------------------------------------------------------------------ workload exploration
namespace {

// dimensions explored for a workload of one pipeline kind, in feature order
// (strategy, threads, memory access first; Section 8.2)
struct Space {
  int kind;
  bool table;
  std::vector<int32_t> sizes;
  int iu = -1, isimd = -1;  // positions of the unrolling and filter-mode dimensions (extra dimensions)
  hawk_variant at(const std::vector<int32_t>& c) const {
    hawk_variant v;
    std::memset(&v, 0, sizeof(v));
    if (kind == 1) {
      v.proj_strategy = static_cast<uint8_t>(c[0]);
      v.thread_mult = v.proj_strategy ? kMults[c[1]] : 1;  // single-pass: one instance per CU
      v.mem = static_cast<uint8_t>(c[2]);
      v.pred = static_cast<uint8_t>(c[3]);
      v.wg_size = v.proj_strategy ? 256 : 64;
      if (table) {
        v.ht = static_cast<uint8_t>(c[4]);
        v.hash = static_cast<uint8_t>(c[5]);
      }
      v.agg_strategy = 0;
      static const uint8_t kUnroll[3] = {0, 2, 1};  // the default 4 rows per iteration first
      if (iu >= 0) v.unroll = kUnroll[c[iu]];
      if (isimd >= 0) v.filter_mode = static_cast<uint8_t>(c[isimd]);
    } else {
      v.proj_strategy = 1;
      v.agg_strategy = static_cast<uint8_t>(c[0]);
      v.thread_mult = v.agg_strategy == HAWK_LOCAL ? kMults[c[1]] : 1;  // global: one table
      v.wg_size = kWgs[c[2]];
      v.mem = static_cast<uint8_t>(c[3]);
      v.pred = static_cast<uint8_t>(c[4]);
      if (table) {
        v.ht = static_cast<uint8_t>(c[5]);
        v.hash = static_cast<uint8_t>(c[6]);
      }
    }
    return v;
  }
};

std::string vkey(const hawk_variant& v) {
  char buf[160];
  hawk_variant_format(&v, buf, sizeof(buf));
  return buf;
}

// Identity of a workload in the timing log: the kind, sizes and structure of
// its queries (no device addresses), so that a later exploration of the same
// workload can take its measurements from the log (Section 8.3: learned
// configurations are stored and reused).
std::string workload_signature(hawk_query* const* W, int32_t k, int num_cus) {
  uint64_t h = 0xcbf29ce484222325ull;  // FNV-1a over a canonical text
  auto mix = [&](const std::string& t) {
    for (unsigned char c : t) h = (h ^ c) * 0x100000001b3ull;
  };
  char buf[256];
  std::snprintf(buf, sizeof(buf), "cus=%d;k=%d;", num_cus, k);
  mix(buf);
  for (int32_t i = 0; i < k; ++i) {
    const hawk_query* q = W[i];
    const HkPlan& P = q->main;
    std::snprintf(buf, sizeof(buf), "q%d:kind=%d,n=%lld,g=%lld,f=%d,p=%d,a=%d,gr=%d,ag=%d,pj=%d,w=%d;", i, q->kind,
                  static_cast<long long>(P.nrows), static_cast<long long>(q->groups_hint), P.nfilters, P.nprobes,
                  P.narith, P.ngroup, P.naggs, P.nproj, P.slot_words);
    mix(buf);
    for (int f = 0; f < P.nfilters; ++f) {
      std::snprintf(buf, sizeof(buf), "F%d:%lld:%lld;", P.filters[f].reg, static_cast<long long>(P.filters[f].lo),
                    static_cast<long long>(P.filters[f].hi));
      mix(buf);
    }
    for (int c = 0; c < P.ncolA + P.ncolB + P.ncolC; ++c) {
      const HkCol& col = c < P.ncolA ? P.colA[c] : c < P.ncolA + P.ncolB ? P.colB[c - P.ncolA]
                                                                        : P.colC[c - P.ncolA - P.ncolB];
      std::snprintf(buf, sizeof(buf), "C%d:%d;", col.dtype, col.reg);
      mix(buf);
    }
    for (int a = 0; a < P.narith; ++a) {
      const HkArith& A = P.arith[a];
      std::snprintf(buf, sizeof(buf), "A%d:%d:%d:%d:%d:%d:%lld:%lld;", A.op, A.dst, A.x, A.y, A.xc, A.yc,
                    static_cast<long long>(A.cx), static_cast<long long>(A.cy));
      mix(buf);
    }
    for (int a = 0; a < P.naggs; ++a) {
      std::snprintf(buf, sizeof(buf), "G%d:%d:%d;", P.aggs[a].fn, P.aggs[a].wide, P.aggs[a].reg);
      mix(buf);
    }
    for (const QueryBuild& B : q->builds) {
      std::snprintf(buf, sizeof(buf), "B%lld:%d;", static_cast<long long>(B.nrows), B.plan.nfilters);
      mix(buf);
      for (int f = 0; f < B.plan.nfilters; ++f) {
        std::snprintf(buf, sizeof(buf), "%lld:%lld;", static_cast<long long>(B.plan.filters[f].lo),
                      static_cast<long long>(B.plan.filters[f].hi));
        mix(buf);
      }
    }
  }
  std::snprintf(buf, sizeof(buf), "%016llx", static_cast<unsigned long long>(h));
  return buf;
}

struct Explorer {
  hawk_ctx* ctx;
  hawk_query* const* W;
  int32_t k;
  const hawk_explore_opts* opts;
  Space space;
  std::map<std::string, double> memo;
  int64_t evaluated = 0, pruned = 0, reused = 0;
  FILE* db = nullptr;
  std::string sig;
  hawk_status fatal = HAWK_OK;  // an error other than pruning or infeasibility stops the search

  double workload_time(const hawk_variant& v) {
    if (fatal) return kInf;
    const std::string key = vkey(v);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
    double total = 0;
    bool bad = false;
    for (int32_t i = 0; i < k && !bad; ++i) {
      double ms = 0;
      hawk_status st = hawk_time_variant(ctx, W[i], &v, opts->reps > 0 ? opts->reps : 3, opts->limit_ms, &ms);
      if (st != HAWK_OK && st != HAWK_E_TIMEOUT && st != HAWK_E_INFEASIBLE) {
        fatal = st;  // the context keeps the message
        return kInf;
      }
      float f[12];
      query_features(W[i], &v, ctx->num_cus, f);
      if (db) {
        std::fprintf(db, "%s\t%d", sig.c_str(), i);
        for (float x : f) std::fprintf(db, "\t%.6g", x);
        std::fprintf(db, "\t%s\t%.6f\t%d\n", key.c_str(), st == HAWK_OK ? ms : -1.0, st);
        std::fflush(db);
      }
      if (st != HAWK_OK) bad = true;
      else total += ms;
    }
    ++evaluated;
    if (bad) {
      ++pruned;
      total = kInf;
      ctx->err.clear();
    }
    memo[key] = total;
    return total;
  }

  // Reads the measurements of this workload from an earlier log: a variant
  // whose k per-query lines are all there enters the memo (any pruned or
  // infeasible query makes it +inf).
  void resume(const char* path) {
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    std::map<std::string, std::map<int32_t, double>> seen;  // variant -> query -> ms (inf: pruned)
    char line[1024];
    while (std::fgets(line, sizeof(line), f)) {
      if (line[0] == '#') continue;
      std::vector<std::string> tok;
      std::string cur;
      for (const char* p = line; *p && *p != '\n'; ++p) {
        if (*p == '\t') { tok.push_back(cur); cur.clear(); }
        else cur += *p;
      }
      tok.push_back(cur);
      if (tok.size() != 17 || tok[0] != sig) continue;  // sig, query, 12 features, variant, ms, status
      const int32_t qi = std::atoi(tok[1].c_str());
      const int st = std::atoi(tok[16].c_str());
      if (qi < 0 || qi >= k) continue;
      seen[tok[14]][qi] = st == HAWK_OK ? std::atof(tok[15].c_str()) : kInf;
    }
    std::fclose(f);
    for (const auto& kv : seen) {
      if (static_cast<int32_t>(kv.second.size()) != k || memo.count(kv.first)) continue;
      double total = 0;
      for (const auto& qt : kv.second) total += qt.second;
      memo[kv.first] = total;
      ++reused;
    }
  }
};

double explorer_cost(const int32_t* cfg, int32_t ndims, void* user) {
  Explorer* E = static_cast<Explorer*>(user);
  std::vector<int32_t> c(cfg, cfg + ndims);
  return E->workload_time(E->space.at(c));
}

}  // namespace

extern "C" hawk_status hawk_explore(hawk_ctx* ctx, hawk_query* const* W, int32_t k, int32_t mode,
                                    const hawk_explore_opts* opts, hawk_variant* best, hawk_explore_report* rep) {
  if (!ctx) return HAWK_E_ARG;
  if (!W || k < 1 || !opts || !best) return set_error(ctx, HAWK_E_ARG, "null argument");
  const auto t0 = std::chrono::steady_clock::now();
  Explorer E{ctx, W, k, opts, {}, {}, 0, 0, 0, nullptr, {}, HAWK_OK};
  E.space.kind = W[0]->kind;
  E.space.table = false;
  for (int32_t i = 0; i < k; ++i) {
    if (!W[i] || W[i]->ctx != ctx) return set_error(ctx, HAWK_E_ARG, "query of another context");
    if (W[i]->kind != E.space.kind) return set_error(ctx, HAWK_E_ARG, "workload mixes pipeline kinds");
    E.space.table = E.space.table || W[i]->has_table;
  }
  if (E.space.kind == 1) E.space.sizes = {2, 7, 2, 2};
  else E.space.sizes = {2, 7, 7, 2, 2};
  // the context's extra dimensions (hawk_ctx_set_variant_dims): a third
  // table kind for joins, unrolling and the SIMD filter for projections
  // (values that do not apply to a query make it infeasible: +inf)
  if (E.space.table) {
    E.space.sizes.push_back(ctx->variant_dims & HAWK_DIM_ROBIN_HOOD ? 3 : 2);
    E.space.sizes.push_back(2);
  }
  if (E.space.kind == 1 && (ctx->variant_dims & HAWK_DIM_UNROLL)) {
    E.space.iu = static_cast<int>(E.space.sizes.size());
    E.space.sizes.push_back(3);
  }
  if (E.space.kind == 1 && (ctx->variant_dims & HAWK_DIM_SIMD_FILTER)) {
    E.space.isimd = static_cast<int>(E.space.sizes.size());
    E.space.sizes.push_back(2);
  }
  E.sig = workload_signature(W, k, ctx->num_cus);
  if (opts->timing_db && opts->resume) E.resume(opts->timing_db);
  if (opts->timing_db) {
    E.db = std::fopen(opts->timing_db, "a");
    if (!E.db) return set_error(ctx, HAWK_E_ARG, std::string("cannot open the timing log ") + opts->timing_db);
    std::fprintf(E.db, "#workload\t%s\t%d\tmode=%d\n", E.sig.c_str(), k, mode);
    std::fflush(E.db);
  }
  std::vector<int32_t> cfg(E.space.sizes.size(), 0);
  hawk_status st = HAWK_OK;
  if (mode == HAWK_EXPLORE_FEATURE_WISE) {
    int64_t calls = 0;
    st = hawk_learn_feature_wise(E.space.sizes.data(), static_cast<int32_t>(E.space.sizes.size()), nullptr,
                                 opts->max_iters > 0 ? opts->max_iters : 5, explorer_cost, &E, cfg.data(), &calls);
  } else if (mode == HAWK_EXPLORE_EXHAUSTIVE) {
    double bt = kInf;
    std::vector<int32_t> c(E.space.sizes.size(), 0);
    for (;;) {
      const double t = E.workload_time(E.space.at(c));
      if (t < bt) {
        bt = t;
        cfg = c;
      }
      size_t d = c.size();
      while (d > 0) {
        --d;
        if (++c[d] < E.space.sizes[d]) break;
        c[d] = 0;
        if (d == 0) { d = c.size() + 1; break; }
      }
      if (d == c.size() + 1) break;
    }
  } else {
    st = set_error(ctx, HAWK_E_ARG, "unknown exploration mode");
  }
  if (E.db) std::fclose(E.db);
  if (st) return st;
  if (E.fatal) return E.fatal;
  *best = E.space.at(cfg);
  if (rep) {
    rep->evaluated = E.evaluated;
    rep->pruned = E.pruned;
    rep->reused = E.reused;
    rep->best_ms = E.workload_time(*best);
    rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return HAWK_OK;
}
