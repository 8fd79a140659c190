// Relational plans -> pipeline programs by the produce/consume model
// (Section 2.1): `produce` walks the operator tree from the root; a hash
// join's build side is a pipeline breaker and gets a pipeline of its own
// ending in HASH_PUT; every other operator `consume`s into the pipeline of
// the tuples that reach it (FILTER, ARITHMETIC, HASH_PROBE, CROSS_JOIN), and
// the root ends the probe pipeline with its sink (Table 2). The pipelines are
// then validated and lowered like any other query.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "hawk.h"
#include "hawk_internal.h"

namespace {

hawk_op blank() {
  hawk_op o;
  std::memset(&o, 0, sizeof(o));
  return o;
}

struct Planner {
  hawk_ctx* ctx;
  const hawk_rel* nodes;
  int32_t n;
  std::vector<std::vector<hawk_op>> builds;  // one pipeline per hash-join build side
  int32_t next_ht = 0;
  int32_t depth = 0;

  hawk_status fail(hawk_status st, const std::string& m) { return set_error(ctx, st, m); }

  bool valid(int32_t id) const { return id >= 0 && id < n; }

  // the operations that yield node id's tuples, appended to `ops`
  hawk_status produce(int32_t id, std::vector<hawk_op>& ops) {
    if (!valid(id)) return fail(HAWK_E_ARG, "plan node index out of range");
    if (++depth > n) return fail(HAWK_E_PLAN, "the plan is not a tree (a node reaches itself)");
    const hawk_rel& r = nodes[id];
    hawk_status st = HAWK_OK;
    switch (r.kind) {
      case HAWK_REL_SCAN: {
        hawk_op o = blank();
        o.kind = HAWK_LOOP;
        o.table = r.table;
        ops.push_back(o);
        break;
      }
      case HAWK_REL_SELECT: {
        if ((st = produce(r.input, ops))) break;
        hawk_op o = blank();
        o.kind = HAWK_FILTER;
        o.a = r.a;
        o.lo = r.lo;
        o.hi = r.hi;
        ops.push_back(o);
        break;
      }
      case HAWK_REL_MAP: {
        if ((st = produce(r.input, ops))) break;
        hawk_op o = blank();
        o.kind = HAWK_ARITHMETIC;
        o.a = r.a;
        o.b = r.b;
        o.c = r.c;
        o.arith_op = r.arith_op;
        o.lo = r.lo;
        o.hi = r.hi;
        ops.push_back(o);
        break;
      }
      case HAWK_REL_HASH_JOIN: {
        // pipeline breaker: the build side fills a hash table in a pipeline of its own
        std::vector<hawk_op> b;
        if ((st = produce(r.right, b))) break;
        for (size_t k = 1; k < b.size(); ++k)
          if (b[k].kind != HAWK_FILTER)
            return fail(HAWK_E_PLAN, "a hash join's build side is a scan under selections");
        const int32_t ht = next_ht++;
        hawk_op put = blank();
        put.kind = HAWK_HASH_PUT;
        put.a = r.b;  // build key
        put.b = r.c;  // payload: the build attribute the join passes on
        put.ht = ht;
        b.push_back(put);
        builds.push_back(b);
        // the probe side continues the current pipeline
        if ((st = produce(r.input, ops))) break;
        hawk_op probe = blank();
        probe.kind = HAWK_HASH_PROBE;
        probe.a = r.a;
        probe.b = r.c;
        probe.ht = ht;
        ops.push_back(probe);
        break;
      }
      case HAWK_REL_CROSS_JOIN: {
        if ((st = produce(r.input, ops))) break;
        // the second input is a scan, possibly under selections: its rows are
        // looped over inside the pipeline, its selections follow the join
        std::vector<hawk_op> inner;
        if ((st = produce(r.right, inner))) break;
        for (size_t k = 1; k < inner.size(); ++k)
          if (inner[k].kind != HAWK_FILTER)
            return fail(HAWK_E_PLAN, "a cross join's second input is a scan under selections");
        hawk_op o = blank();
        o.kind = HAWK_CROSS_JOIN;
        o.table = inner[0].table;
        ops.push_back(o);
        ops.insert(ops.end(), inner.begin() + 1, inner.end());
        break;
      }
      case HAWK_REL_GROUP_BY:
      case HAWK_REL_PROJECT:
        st = fail(HAWK_E_PLAN, "aggregation or projection below the root (a query has one sink)");
        break;
      default:
        st = fail(HAWK_E_ARG, "unknown plan operator");
    }
    --depth;
    return st;
  }
};

// True when `name` is a column of table t (an id of ctx's registry).
bool has_col(const hawk_ctx* ctx, int32_t t, const char* name) {
  if (!name || t < 0 || t >= static_cast<int32_t>(ctx->tables.size())) return false;
  for (const auto& c : ctx->tables[t].cols)
    if (c.name == name) return true;
  return false;
}

}  // namespace

extern "C" hawk_status hawk_query_from_plan(hawk_ctx* ctx, const hawk_rel* nodes, int32_t n, int32_t root,
                                            hawk_query** out) {
  if (!ctx) return HAWK_E_ARG;
  if (!nodes || n < 1 || !out || root < 0 || root >= n) return set_error(ctx, HAWK_E_ARG, "bad plan arguments");
  *out = nullptr;
  const hawk_rel& sink = nodes[root];
  if (sink.kind != HAWK_REL_GROUP_BY && sink.kind != HAWK_REL_PROJECT)
    return set_error(ctx, HAWK_E_PLAN, "the plan's root is a group-by or a projection");
  Planner pl{ctx, nodes, n};
  std::vector<hawk_op> main;
  hawk_status st = pl.produce(sink.input, main);
  if (st) return st;
  // The probe pipeline in the order its operations take effect: selections on
  // the looped table's columns first, then the cross join and the selections
  // that read its table, then the probes, then the arithmetic. Selections
  // commute with inner joins and with arithmetic (which only adds
  // attributes), so moving them down keeps the answer; a selection on a
  // join's payload or a computed attribute cannot move and is rejected.
  const int32_t loop_t = main[0].table;
  int32_t cross_t = -1;
  for (const auto& o : main)
    if (o.kind == HAWK_CROSS_JOIN) cross_t = o.table;
  std::vector<hawk_op> ordered{main[0]}, filters2, probes, arith;
  hawk_op cross = blank();
  for (size_t k = 1; k < main.size(); ++k) {
    const hawk_op& o = main[k];
    if (o.kind == HAWK_FILTER) {
      if (has_col(ctx, loop_t, o.a)) ordered.push_back(o);
      else if (has_col(ctx, cross_t, o.a)) filters2.push_back(o);
      else return set_error(ctx, HAWK_E_PLAN, std::string("selection on a join payload or computed attribute: ") +
                                                  (o.a ? o.a : "(null)"));
    } else if (o.kind == HAWK_CROSS_JOIN) {
      cross = o;
    } else if (o.kind == HAWK_HASH_PROBE) {
      probes.push_back(o);
    } else {
      arith.push_back(o);
    }
  }
  if (cross.kind == HAWK_CROSS_JOIN) ordered.push_back(cross);
  ordered.insert(ordered.end(), filters2.begin(), filters2.end());
  ordered.insert(ordered.end(), probes.begin(), probes.end());
  ordered.insert(ordered.end(), arith.begin(), arith.end());
  hawk_op s = blank();
  s.attrs = sink.attrs;
  s.nattrs = sink.nattrs;
  if (sink.kind == HAWK_REL_PROJECT) {
    s.kind = HAWK_PROJECT;
  } else {
    s.kind = sink.nattrs > 0 ? HAWK_HASH_AGGREGATE : HAWK_AGGREGATE;
    s.aggs = sink.aggs;
    s.naggs = sink.naggs;
    s.groups_hint = sink.groups_hint;
  }
  ordered.push_back(s);
  std::vector<hawk_pipeline> pipes;
  for (const auto& b : pl.builds) pipes.push_back({b.data(), static_cast<int32_t>(b.size())});
  pipes.push_back({ordered.data(), static_cast<int32_t>(ordered.size())});
  return hawk_query_create(ctx, pipes.data(), static_cast<int32_t>(pipes.size()), out);
}
