// CPU oracle for pipeline programs: TEST INFRASTRUCTURE ONLY (see oracle.h).
//
// Column-at-a-time interpretation of the operations of the paper's pipeline
// program table (Section 3.1, Table 1):
//   LOOP           -> selection vector of all row ids, ascending
//   FILTER         -> keep ids whose attribute lies in [lo, hi] (conjunction,
//                     one predicate after the other)
//   CROSS_JOIN     -> every surviving id paired with every row of the second
//                     table (row-major: the second table's rows vary fastest);
//                     later operations see pairs (FILTER again on either side)
//   HASH_PUT       -> build pipeline: filter the dimension, then an ordered
//                     map key -> payload (a repeated key is an error)
//   HASH_PROBE     -> inner equi-join: keep ids whose key is in the map and
//                     remember the payload
//   ARITHMETIC     -> binary +, -, * over attributes/constants, 64-bit two's
//                     complement
//   AGGREGATE / HASH_AGGREGATE -> fold COUNT/SUM/MIN/MAX/AVG per group in an
//                     ordered map; sums are exact 128-bit, narrow sums are the
//                     low 64 bits of that
//   PROJECT        -> the attributes of the surviving ids, in row order
// The result is the plain relational answer; every variant of the paper's
// variant space must reproduce it (Section 3.4: variations are orthogonal and
// do not change the pipeline's semantics).
#include "oracle.h"

#include <climits>
#include <cstring>
#include <map>
#include <thread>
#include <vector>

namespace {

typedef __int128 i128;

struct Result {
  int kind = 0;
  int64_t rows = 0;
  std::vector<std::vector<int64_t>> proj;      // [col][row]
  std::vector<std::vector<int64_t>> keys;      // [g][row]
  std::vector<int64_t> count;                  // [row]
  std::vector<std::vector<i128>> vals;         // [agg][row]
  std::vector<int> fns;
};

int64_t load(const orc_col& c, int64_t i) {
  switch (c.dtype) {
    case ORC_I8: return static_cast<const int8_t*>(c.data)[i];
    case ORC_I32: return static_cast<const int32_t*>(c.data)[i];
    default: return static_cast<const int64_t*>(c.data)[i];
  }
}

// LOOP over rows [r0, r1), then FILTER: refine the selection vector, one
// conjunct at a time.
std::vector<int64_t> select(int64_t r0, int64_t r1, const orc_col* cols, int32_t nf, const orc_filter* f) {
  std::vector<int64_t> sv(static_cast<size_t>(r1 - r0));
  for (int64_t i = r0; i < r1; ++i) sv[i - r0] = i;
  for (int32_t k = 0; k < nf; ++k) {
    std::vector<int64_t> next;
    next.reserve(sv.size());
    const orc_col& c = cols[f[k].col];
    for (int64_t i : sv) {
      int64_t x = load(c, i);
      if (x >= f[k].lo && x <= f[k].hi) next.push_back(i);
    }
    sv.swap(next);
  }
  return sv;
}

int64_t wrap(uint64_t v) { int64_t r; std::memcpy(&r, &v, 8); return r; }

typedef std::vector<std::map<int64_t, int64_t>> BuildTables;

// build pipelines: LOOP, FILTER, HASH_PUT
int32_t run_builds(const orc_build* builds, int32_t nbuilds, BuildTables& tables) {
  tables.assign(static_cast<size_t>(nbuilds), std::map<int64_t, int64_t>());
  for (int32_t b = 0; b < nbuilds; ++b) {
    const orc_build& B = builds[b];
    std::vector<int64_t> sv = select(0, B.nrows, B.cols, B.nfilters, B.filters);
    for (int64_t i : sv) {
      int64_t key = load(B.cols[B.key_col], i);
      int64_t pay = load(B.cols[B.payload_col], i);
      if (!tables[b].emplace(key, pay).second) return ORC_E_DUPKEY;
    }
  }
  return ORC_OK;
}

// running aggregates of one group: the row count and, per aggregate, the
// exact value (sum, minimum or maximum)
struct Acc { int64_t count = 0; std::vector<i128> v; };
typedef std::map<std::vector<int64_t>, Acc> Groups;

// the main pipeline over rows [r0, r1): projected rows in row order, or the groups
struct Part {
  std::vector<std::vector<int64_t>> proj;
  Groups groups;
};

std::vector<i128> agg_init(const orc_main* m) {
  std::vector<i128> init(static_cast<size_t>(m->naggs));
  for (int32_t a = 0; a < m->naggs; ++a)
    init[a] = m->aggs[a].fn == ORC_MIN ? i128(INT64_MAX) : m->aggs[a].fn == ORC_MAX ? i128(INT64_MIN) : 0;
  return init;
}

int32_t run_main(const BuildTables& tables, int32_t nbuilds, const orc_main* m, int64_t r0, int64_t r1, Part& out) {
  std::vector<int64_t> sv = select(r0, r1, m->cols, m->nfilters, m->filters);
  // row of the looped table and (CROSS_JOIN) of the second table, per tuple
  std::vector<int64_t> po, pi;
  if (m->ninner > 0) {
    for (int64_t i : sv)
      for (int64_t j = 0; j < m->inner_nrows; ++j) {
        po.push_back(i);
        pi.push_back(j);
      }
    // FILTERs after the CROSS_JOIN, one conjunct at a time over the pairs
    for (int32_t k = 0; k < m->nfilters2; ++k) {
      const orc_filter& F = m->filters2[k];
      std::vector<int64_t> no, ni;
      for (size_t t = 0; t < po.size(); ++t) {
        const int64_t x = F.col < m->ncols ? load(m->cols[F.col], po[t]) : load(m->inner_cols[F.col - m->ncols], pi[t]);
        if (x >= F.lo && x <= F.hi) {
          no.push_back(po[t]);
          ni.push_back(pi[t]);
        }
      }
      po.swap(no);
      pi.swap(ni);
    }
  } else {
    po.swap(sv);
  }
  const int32_t ntab = m->ncols + m->ninner;  // table attributes
  const int32_t nattr = ntab + m->nprobes + m->narith;
  auto tab = [&](int32_t a, size_t j) -> int64_t {
    return a < m->ncols ? load(m->cols[a], po[j]) : load(m->inner_cols[a - m->ncols], pi[j]);
  };
  // computed attributes, materialised over the tuples
  std::vector<std::vector<int64_t>> comp(static_cast<size_t>(m->nprobes + m->narith));
  for (int32_t p = 0; p < m->nprobes; ++p) {
    const orc_probe& P = m->probes[p];
    if (P.build < 0 || P.build >= nbuilds || P.fk_col < 0 || P.fk_col >= ntab) return ORC_E_ARG;
    const auto& T = tables[P.build];
    std::vector<size_t> pos;
    std::vector<int64_t> pay;
    for (size_t j = 0; j < po.size(); ++j) {
      auto it = T.find(tab(P.fk_col, j));
      if (it != T.end()) { pos.push_back(j); pay.push_back(it->second); }
    }
    // the tuples and earlier payloads follow the shrinking selection
    std::vector<int64_t> no(pos.size()), ni(m->ninner > 0 ? pos.size() : 0);
    for (size_t j = 0; j < pos.size(); ++j) {
      no[j] = po[pos[j]];
      if (m->ninner > 0) ni[j] = pi[pos[j]];
    }
    po.swap(no);
    pi.swap(ni);
    for (int32_t q = 0; q < p; ++q) {
      std::vector<int64_t> v(pos.size());
      for (size_t j = 0; j < pos.size(); ++j) v[j] = comp[q][pos[j]];
      comp[q].swap(v);
    }
    comp[p].swap(pay);
  }
  auto attr = [&](int32_t a, size_t j) -> int64_t {
    if (a < ntab) return tab(a, j);
    return comp[a - ntab][j];
  };
  for (int32_t k = 0; k < m->narith; ++k) {
    const orc_arith& A = m->arith[k];
    std::vector<int64_t>& dst = comp[m->nprobes + k];
    dst.resize(po.size());
    for (size_t j = 0; j < po.size(); ++j) {
      uint64_t x = static_cast<uint64_t>(A.x_const ? A.xc : attr(A.x, j));
      uint64_t y = static_cast<uint64_t>(A.y_const ? A.yc : attr(A.y, j));
      uint64_t r = A.op == ORC_ADD ? x + y : A.op == ORC_SUB ? x - y : x * y;
      dst[j] = wrap(r);
    }
  }
  if (m->kind == ORC_PROJECT) {
    out.proj.resize(static_cast<size_t>(m->nproj));
    for (int32_t c = 0; c < m->nproj; ++c) {
      if (m->proj[c] < 0 || m->proj[c] >= nattr) return ORC_E_ARG;
      out.proj[c].resize(po.size());
      for (size_t j = 0; j < po.size(); ++j) out.proj[c][j] = attr(m->proj[c], j);
    }
  } else {
    Groups& groups = out.groups;
    const std::vector<i128> init = agg_init(m);
    if (m->ngroup == 0) groups[std::vector<int64_t>()].v = init;  // AGGREGATE: one row even when empty
    std::vector<int64_t> key(static_cast<size_t>(m->ngroup));
    for (size_t j = 0; j < po.size(); ++j) {
      for (int32_t g = 0; g < m->ngroup; ++g) key[g] = attr(m->group[g], j);
      auto it = groups.find(key);
      if (it == groups.end()) { it = groups.emplace(key, Acc()).first; it->second.v = init; }
      Acc& acc = it->second;
      acc.count += 1;
      for (int32_t a = 0; a < m->naggs; ++a) {
        const orc_agg& A = m->aggs[a];
        if (A.fn == ORC_COUNT) continue;
        int64_t x = attr(A.attr, j);
        if (A.fn == ORC_SUM || A.fn == ORC_AVG) acc.v[a] += x;
        else if (A.fn == ORC_MIN) { if (x < acc.v[a]) acc.v[a] = x; }
        else if (A.fn == ORC_MAX) { if (x > acc.v[a]) acc.v[a] = x; }
      }
    }
  }
  return ORC_OK;
}

// the result of the main pipeline from its (merged) part
Result finish(const orc_main* m, Part& part) {
  Result res;
  res.kind = m->kind;
  if (m->kind == ORC_PROJECT) {
    res.rows = m->nproj > 0 ? static_cast<int64_t>(part.proj[0].size()) : 0;
    res.proj.swap(part.proj);
  } else {
    const Groups& groups = part.groups;
    res.rows = static_cast<int64_t>(groups.size());
    res.keys.assign(static_cast<size_t>(m->ngroup), std::vector<int64_t>());
    res.vals.assign(static_cast<size_t>(m->naggs), std::vector<i128>());
    for (int32_t a = 0; a < m->naggs; ++a) res.fns.push_back(m->aggs[a].fn);
    for (auto& kv : groups) {
      for (int32_t g = 0; g < m->ngroup; ++g) res.keys[g].push_back(kv.first[g]);
      res.count.push_back(kv.second.count);
      for (int32_t a = 0; a < m->naggs; ++a) {
        const orc_agg& A = m->aggs[a];
        i128 v = A.fn == ORC_COUNT ? i128(kv.second.count) : kv.second.v[a];
        // a narrow SUM keeps the low 64 bits (two's complement), as 64-bit hardware does
        if (A.fn == ORC_SUM && !A.wide) v = i128(wrap(static_cast<uint64_t>(v)));
        res.vals[a].push_back(v);
      }
    }
  }
  return res;
}

// folds the groups of `from` into `into` (row counts and sums add, minima and
// maxima combine): the groups of rows [a, b) and of rows [b, c) give those of
// rows [a, c)
void merge_groups(const orc_main* m, Groups& into, const Groups& from) {
  for (const auto& kv : from) {
    auto it = into.find(kv.first);
    if (it == into.end()) {
      into.emplace(kv.first, kv.second);
      continue;
    }
    Acc& acc = it->second;
    acc.count += kv.second.count;
    for (int32_t a = 0; a < m->naggs; ++a) {
      const int fn = m->aggs[a].fn;
      const i128 x = kv.second.v[a];
      if (fn == ORC_SUM || fn == ORC_AVG) acc.v[a] += x;
      else if (fn == ORC_MIN) { if (x < acc.v[a]) acc.v[a] = x; }
      else if (fn == ORC_MAX) { if (x > acc.v[a]) acc.v[a] = x; }
    }
  }
}

}  // namespace

struct orc_result : Result {};

extern "C" int32_t orc_run(const orc_build* builds, int32_t nbuilds, const orc_main* m,
                           orc_result** out) {
  if (!m || !out || m->nrows < 0) return ORC_E_ARG;
  BuildTables tables;
  int32_t st = run_builds(builds, nbuilds, tables);
  if (st != ORC_OK) return st;
  Part part;
  st = run_main(tables, nbuilds, m, 0, m->nrows, part);
  if (st != ORC_OK) return st;
  orc_result* r = new orc_result();
  static_cast<Result&>(*r) = finish(m, part);
  *out = r;
  return ORC_OK;
}

// The same query with the main pipeline's rows split into nthreads
// contiguous ranges, each interpreted as above on its own thread; the
// ranges' projected rows are concatenated in range order and their groups
// merged. Used to time the oracle on all host cores.
extern "C" int32_t orc_run_parallel(const orc_build* builds, int32_t nbuilds, const orc_main* m, int32_t nthreads,
                                    orc_result** out) {
  if (!m || !out || m->nrows < 0 || nthreads < 1) return ORC_E_ARG;
  BuildTables tables;
  int32_t st = run_builds(builds, nbuilds, tables);
  if (st != ORC_OK) return st;
  const int64_t n = m->nrows;
  std::vector<Part> parts(static_cast<size_t>(nthreads));
  std::vector<int32_t> sts(static_cast<size_t>(nthreads), ORC_OK);
  std::vector<std::thread> th;
  for (int32_t t = 0; t < nthreads; ++t) {
    const int64_t r0 = n * t / nthreads, r1 = n * (t + 1) / nthreads;
    th.emplace_back([&, t, r0, r1] { sts[t] = run_main(tables, nbuilds, m, r0, r1, parts[t]); });
  }
  for (auto& x : th) x.join();
  for (int32_t t = 0; t < nthreads; ++t)
    if (sts[t] != ORC_OK) return sts[t];
  Part& all = parts[0];
  for (int32_t t = 1; t < nthreads; ++t) {
    if (m->kind == ORC_PROJECT) {
      for (int32_t c = 0; c < m->nproj; ++c)
        all.proj[c].insert(all.proj[c].end(), parts[t].proj[c].begin(), parts[t].proj[c].end());
    } else {
      merge_groups(m, all.groups, parts[t].groups);
    }
    Part().proj.swap(parts[t].proj);
    Groups().swap(parts[t].groups);
  }
  orc_result* r = new orc_result();
  static_cast<Result&>(*r) = finish(m, all);
  *out = r;
  return ORC_OK;
}

extern "C" void orc_free(orc_result* r) { delete r; }
extern "C" int64_t orc_rows(const orc_result* r) { return r->rows; }

extern "C" void orc_project_column(const orc_result* r, int32_t c, int64_t* dst) {
  if (!r->proj[c].empty()) std::memcpy(dst, r->proj[c].data(), r->proj[c].size() * 8);
}
extern "C" void orc_group_key(const orc_result* r, int32_t g, int64_t* dst) {
  if (!r->keys[g].empty()) std::memcpy(dst, r->keys[g].data(), r->keys[g].size() * 8);
}
extern "C" void orc_group_count(const orc_result* r, int64_t* dst) {
  if (!r->count.empty()) std::memcpy(dst, r->count.data(), r->count.size() * 8);
}
extern "C" void orc_agg_value(const orc_result* r, int32_t a, uint64_t* lo, int64_t* hi) {
  for (size_t j = 0; j < r->vals[a].size(); ++j) {
    i128 v = r->vals[a][j];
    lo[j] = static_cast<uint64_t>(v);
    hi[j] = static_cast<int64_t>(v >> 64);
  }
}
// AVG: the exact sum converted to double (round to nearest), divided by the count.
extern "C" void orc_agg_avg(const orc_result* r, int32_t a, double* dst) {
  for (size_t j = 0; j < r->vals[a].size(); ++j)
    dst[j] = static_cast<double>(r->vals[a][j]) / static_cast<double>(r->count[j]);
}
