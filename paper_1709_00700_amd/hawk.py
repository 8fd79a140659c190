"""ctypes binding of libhawk.so (include/hawk.h), same names as the C ABI.

Argument marshalling only: every step of a pipeline runs in the library's
gfx950 kernels. There is no CPU fallback: if the shared library is missing
or a call fails, an exception is raised.

Besides the raw entry points (``L().hawk_*``) this module offers thin helpers:
``Context`` (context + table registration from torch tensors), ``build_query``
(neutral query description -> hawk_op arrays), ``variant`` / ``variant_space``
and ``Result`` (copy-out of result columns to numpy).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# HAWK_LIBRARY names another build of the library to load (the host tests
# load one built with sanitizers this way)
LIB_PATH = os.environ.get("HAWK_LIBRARY") or os.path.join(HERE, "libhawk.so")

# status codes
HAWK_OK, HAWK_E_ARG, HAWK_E_NOTFOUND, HAWK_E_TYPE, HAWK_E_PLAN = 0, -1, -2, -3, -4
HAWK_E_INFEASIBLE, HAWK_E_CAPACITY, HAWK_E_DUPKEY, HAWK_E_DEVICE, HAWK_E_OOM, HAWK_E_TIMEOUT = -5, -6, -7, -8, -9, -10
HAWK_I8, HAWK_I32, HAWK_I64 = 1, 2, 3
HAWK_RES_I64, HAWK_RES_I128, HAWK_RES_F64 = 3, 4, 5
(HAWK_LOOP, HAWK_FILTER, HAWK_HASH_PUT, HAWK_HASH_PROBE, HAWK_ARITHMETIC, HAWK_AGGREGATE,
 HAWK_HASH_AGGREGATE, HAWK_PROJECT, HAWK_CROSS_JOIN) = range(1, 10)
ARITH = {"add": 1, "sub": 2, "mul": 3}
AGG_FN = {"count": 1, "sum": 2, "min": 3, "max": 4, "avg": 5}
HAWK_EXPLORE_EXHAUSTIVE, HAWK_EXPLORE_FEATURE_WISE = 0, 1
HAWK_LINEAR_PROBING, HAWK_CUCKOO, HAWK_ROBIN_HOOD = 0, 1, 2
HAWK_DIM_ROBIN_HOOD, HAWK_DIM_UNROLL, HAWK_DIM_SIMD_FILTER = 1, 2, 4

# every symbol include/hawk.h declares
EXPORTS = [
    "hawk_ctx_create", "hawk_ctx_destroy", "hawk_last_error", "hawk_device_info",
    "hawk_table_register", "hawk_table_unregister",
    "hawk_query_create", "hawk_query_free", "hawk_query_kind", "hawk_query_from_plan", "hawk_query_program",
    "hawk_variant_space", "hawk_variant_format",
    "hawk_execute", "hawk_execute_async", "hawk_execute_noalloc",
    "hawk_result_info", "hawk_result_column", "hawk_result_copy_column", "hawk_result_free",
    "hawk_time_variant", "hawk_learn_feature_wise", "hawk_explore",
    "hawk_query_set_stats", "hawk_features",
    "hawk_profile_enable", "hawk_profile_read",
    "hawk_model_create", "hawk_model_free", "hawk_model_set_params", "hawk_model_get_params",
    "hawk_model_train", "hawk_model_predict", "hawk_mlp_forward_dev", "hawk_mlp_grad_dev", "hawk_model_pick",
    "hawk_model_pick_ensemble",
    "hawk_batch_create", "hawk_batch_free", "hawk_batch_run", "hawk_batch_time", "hawk_batch_autotune",
    "hawk_batch_opts_get", "hawk_batch_result", "hawk_ctx_set_jit", "hawk_jit_stats", "hawk_jit_compile_check",
    "hawk_ctx_set_variant_dims",
]


class HawkError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        super().__init__(f"hawk status {code}: {msg}")
        self.code = code


class hawk_column(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("dtype", ctypes.c_int32), ("scale", ctypes.c_int32),
                ("dev_ptr", ctypes.c_void_p)]


class hawk_agg(ctypes.Structure):
    _fields_ = [("fn", ctypes.c_int32), ("wide", ctypes.c_int32), ("attr", ctypes.c_char_p)]


class hawk_op(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("table", ctypes.c_int32),
                ("a", ctypes.c_char_p), ("b", ctypes.c_char_p), ("c", ctypes.c_char_p),
                ("arith_op", ctypes.c_int32), ("ht", ctypes.c_int32),
                ("lo", ctypes.c_int64), ("hi", ctypes.c_int64),
                ("attrs", ctypes.POINTER(ctypes.c_char_p)), ("nattrs", ctypes.c_int32),
                ("naggs", ctypes.c_int32), ("aggs", ctypes.POINTER(hawk_agg)),
                ("groups_hint", ctypes.c_int64)]


class hawk_pipeline(ctypes.Structure):
    _fields_ = [("ops", ctypes.POINTER(hawk_op)), ("nops", ctypes.c_int32)]


class hawk_rel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("input", ctypes.c_int32), ("right", ctypes.c_int32),
                ("table", ctypes.c_int32), ("a", ctypes.c_char_p), ("b", ctypes.c_char_p), ("c", ctypes.c_char_p),
                ("arith_op", ctypes.c_int32), ("nattrs", ctypes.c_int32), ("lo", ctypes.c_int64),
                ("hi", ctypes.c_int64), ("attrs", ctypes.POINTER(ctypes.c_char_p)),
                ("aggs", ctypes.POINTER(hawk_agg)), ("naggs", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("groups_hint", ctypes.c_int64)]


class hawk_variant(ctypes.Structure):
    _fields_ = [("proj_strategy", ctypes.c_uint8), ("mem", ctypes.c_uint8), ("pred", ctypes.c_uint8),
                ("ht", ctypes.c_uint8), ("hash", ctypes.c_uint8), ("agg_strategy", ctypes.c_uint8),
                ("unroll", ctypes.c_uint8), ("filter_mode", ctypes.c_uint8),
                ("thread_mult", ctypes.c_uint32), ("wg_size", ctypes.c_uint32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_ if not f.startswith("reserved")}

    def __repr__(self):
        return format_variant(self)


class hawk_explore_opts(ctypes.Structure):
    _fields_ = [("reps", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("limit_ms", ctypes.c_double),
                ("timing_db", ctypes.c_char_p), ("resume", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class hawk_train_opts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


class hawk_batch_opts(ctypes.Structure):
    _fields_ = [("tile_rows_log2", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32), ("order", ctypes.c_int32),
                ("separate", ctypes.c_int32)]

    def as_dict(self):
        return {"tile_rows_log2": self.tile_rows_log2, "wgs_per_cu": self.wgs_per_cu, "order": self.order,
                "separate": self.separate}


class hawk_explore_report(ctypes.Structure):
    _fields_ = [("evaluated", ctypes.c_int64), ("pruned", ctypes.c_int64), ("best_ms", ctypes.c_double),
                ("seconds", ctypes.c_double), ("reused", ctypes.c_int64)]


COST_FN = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_void_p)

_lib = None


def L():
    """The loaded libhawk.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1709_00700_amd/build.py")
        lib = ctypes.CDLL(LIB_PATH)
        P, i32, i64, vp = ctypes.POINTER, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        sig = {
            "hawk_ctx_create": ([i32, vp, P(vp)], i32),
            "hawk_ctx_destroy": ([vp], None),
            "hawk_last_error": ([vp], ctypes.c_char_p),
            "hawk_device_info": ([vp, P(i32), P(i64)], i32),
            "hawk_table_register": ([vp, ctypes.c_char_p, i64, P(hawk_column), i32, P(i32)], i32),
            "hawk_table_unregister": ([vp, i32], i32),
            "hawk_query_create": ([vp, P(hawk_pipeline), i32, P(vp)], i32),
            "hawk_query_free": ([vp], None),
            "hawk_query_kind": ([vp, P(i32)], i32),
            "hawk_query_from_plan": ([vp, P(hawk_rel), i32, i32, P(vp)], i32),
            "hawk_query_program": ([vp, ctypes.c_char_p, i64, P(i64)], i32),
            "hawk_variant_space": ([vp, P(hawk_variant), i64, P(i64)], i32),
            "hawk_variant_format": ([P(hawk_variant), ctypes.c_char_p, i32], i32),
            "hawk_execute": ([vp, vp, P(hawk_variant), P(vp)], i32),
            "hawk_execute_async": ([vp, vp, P(hawk_variant), P(vp)], i32),
            "hawk_execute_noalloc": ([vp, vp, P(hawk_variant), P(vp), i32, i64, P(i64)], i32),
            "hawk_result_info": ([vp, P(i64), P(i32)], i32),
            "hawk_result_column": ([vp, i32, P(i32), P(vp)], i32),
            "hawk_result_copy_column": ([vp, i32, vp, i64], i32),
            "hawk_result_free": ([vp], None),
            "hawk_time_variant": ([vp, vp, P(hawk_variant), i32, ctypes.c_double, P(ctypes.c_double)], i32),
            "hawk_learn_feature_wise": ([P(i32), i32, P(i32), i32, COST_FN, vp, P(i32), P(i64)], i32),
            "hawk_explore": ([vp, P(vp), i32, i32, P(hawk_explore_opts), P(hawk_variant),
                              P(hawk_explore_report)], i32),
            "hawk_query_set_stats": ([vp, ctypes.c_double], i32),
            "hawk_features": ([vp, P(hawk_variant), P(ctypes.c_float)], i32),
            "hawk_model_create": ([vp, ctypes.c_uint64, P(vp)], i32),
            "hawk_model_free": ([vp], None),
            "hawk_model_set_params": ([vp, P(ctypes.c_float), P(ctypes.c_float), P(ctypes.c_float)], i32),
            "hawk_model_get_params": ([vp, P(ctypes.c_float), P(ctypes.c_float), P(ctypes.c_float)], i32),
            "hawk_model_train": ([vp, P(ctypes.c_float), P(ctypes.c_float), i64, P(hawk_train_opts),
                                  P(ctypes.c_float)], i32),
            "hawk_model_predict": ([vp, P(ctypes.c_float), i64, P(ctypes.c_float)], i32),
            "hawk_mlp_forward_dev": ([vp, vp, i64, vp], i32),
            "hawk_mlp_grad_dev": ([vp, vp, vp, i64, vp, vp], i32),
            "hawk_model_pick": ([vp, P(vp), i32, P(hawk_variant), P(ctypes.c_float)], i32),
            "hawk_model_pick_ensemble": ([P(vp), i32, ctypes.c_float, P(vp), i32, P(hawk_variant),
                                          P(ctypes.c_float)], i32),
            "hawk_profile_enable": ([vp, i32], i32),
            "hawk_profile_read": ([vp, ctypes.c_char_p, P(ctypes.c_double), P(i64)], i32),
            "hawk_batch_create": ([vp, P(vp), i32, P(hawk_variant), P(hawk_batch_opts), P(vp)], i32),
            "hawk_batch_free": ([vp], None),
            "hawk_batch_run": ([vp], i32),
            "hawk_batch_time": ([vp, i32, P(ctypes.c_double)], i32),
            "hawk_batch_autotune": ([vp, i32, P(hawk_batch_opts), P(ctypes.c_double)], i32),
            "hawk_batch_opts_get": ([vp, P(hawk_batch_opts)], i32),
            "hawk_batch_result": ([vp, i32, P(vp)], i32),
            "hawk_ctx_set_jit": ([vp, i32], i32),
            "hawk_ctx_set_variant_dims": ([vp, ctypes.c_uint32], i32),
            "hawk_jit_stats": ([vp, P(i64), P(ctypes.c_double)], i32),
            "hawk_jit_compile_check": ([vp, vp, P(hawk_variant)], i32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def check(st: int, ctx=None):
    if st != HAWK_OK:
        msg = L().hawk_last_error(ctx).decode() if ctx else ""
        raise HawkError(st, msg)


# ---------------------------------------------------------------- variants
def variant(proj_strategy=1, mem=1, pred=0, ht=0, hash=0, agg_strategy=0, thread_mult=1024, wg_size=256, unroll=0,
            filter_mode=0):
    return hawk_variant(proj_strategy, mem, pred, ht, hash, agg_strategy, unroll, filter_mode, thread_mult, wg_size)


def format_variant(v: hawk_variant) -> str:
    buf = ctypes.create_string_buffer(160)
    L().hawk_variant_format(ctypes.byref(v), buf, 160)
    return buf.value.decode()


def variant_space(query) -> list:
    n = ctypes.c_int64()
    check(L().hawk_variant_space(query.handle, None, 0, ctypes.byref(n)))
    arr = (hawk_variant * n.value)()
    check(L().hawk_variant_space(query.handle, arr, n.value, ctypes.byref(n)))
    return list(arr)


# ---------------------------------------------------------------- context / tables / queries
_DT = {1: HAWK_I8, 4: HAWK_I32, 8: HAWK_I64}


class Context:
    """A library context on `device`, ordered on torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        torch.cuda.set_device(device)
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        check(L().hawk_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        self.tables = {}      # name -> table id
        self._keep = []       # tensors kept alive while registered

    def close(self):
        if self.handle:
            L().hawk_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_jit(self, on: bool = True):
        """Run-time compiled aggregation kernels for each plan structure (see hawk.h)."""
        check(L().hawk_ctx_set_jit(self.handle, int(on)), self.handle)
        self.jit = bool(on)

    def set_variant_dims(self, dims: int):
        """Extra variant dimensions (HAWK_DIM_*; 0 = the paper's space)."""
        check(L().hawk_ctx_set_variant_dims(self.handle, int(dims)), self.handle)

    def jit_stats(self):
        """(kernels compiled, total compile milliseconds)."""
        n, ms = ctypes.c_int64(), ctypes.c_double()
        check(L().hawk_jit_stats(self.handle, ctypes.byref(n), ctypes.byref(ms)), self.handle)
        return n.value, ms.value

    def device_info(self):
        n, lds = ctypes.c_int32(), ctypes.c_int64()
        check(L().hawk_device_info(self.handle, ctypes.byref(n), ctypes.byref(lds)), self.handle)
        return n.value, lds.value

    def register(self, name: str, columns: dict) -> int:
        """Registers a table of torch device tensors (int8/int32/int64)."""
        names = list(columns.keys())
        tens = [columns[c].contiguous() for c in names]
        self._keep.extend(tens)
        nrows = int(tens[0].numel()) if tens else 0
        arr = (hawk_column * len(names))(*[
            hawk_column(c.encode(), _DT[t.element_size()], 0, ctypes.c_void_p(t.data_ptr())) for c, t in zip(names, tens)])
        tid = ctypes.c_int32()
        check(L().hawk_table_register(self.handle, name.encode(), nrows, arr, len(names), ctypes.byref(tid)), self.handle)
        self.tables[name] = tid.value
        return tid.value

    def register_numpy(self, tables: dict, device: str = "cuda"):
        """Copies numpy tables to the device and registers them; returns the tensors."""
        import torch
        out = {}
        for tname, cols in tables.items():
            tc = {c: torch.from_numpy(np.ascontiguousarray(a)).to(device) for c, a in cols.items()}
            self.register(tname, tc)
            out[tname] = tc
        return out


class PlanningContext(Context):
    """A device-less context (device -1): plans, variant spaces and features only.
    Tables are registered with placeholder addresses; nothing can execute."""

    def __init__(self):
        h = ctypes.c_void_p()
        check(L().hawk_ctx_create(-1, None, ctypes.byref(h)))
        self.handle = h
        self.tables = {}
        self._keep = []

    def register_shapes(self, tables: dict):
        """tables: name -> {column: numpy array or (dtype, nrows)}; registers placeholders."""
        for tname, cols in tables.items():
            names = list(cols.keys())
            arr = []
            nrows = 0
            for c in names:
                a = cols[c]
                dt, nrows = (np.dtype(a[0]), int(a[1])) if isinstance(a, tuple) else (a.dtype, len(a))
                arr.append(hawk_column(c.encode(), _DT[dt.itemsize], 0, ctypes.c_void_p(0x1000)))
            carr = (hawk_column * len(arr))(*arr)
            tid = ctypes.c_int32()
            check(L().hawk_table_register(self.handle, tname.encode(), nrows, carr, len(arr), ctypes.byref(tid)),
                  self.handle)
            self.tables[tname] = tid.value


class Query:
    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.handle = handle

    def __del__(self):
        try:
            if self.handle:
                L().hawk_query_free(self.handle)
                self.handle = None
        except Exception:
            pass

    @property
    def kind(self) -> int:
        k = ctypes.c_int32()
        check(L().hawk_query_kind(self.handle, ctypes.byref(k)))
        return k.value

    def program(self) -> str:
        """The pipeline programs as text (hawk_query_program)."""
        n = ctypes.c_int64()
        check(L().hawk_query_program(self.handle, None, 0, ctypes.byref(n)), self.ctx.handle)
        buf = ctypes.create_string_buffer(n.value + 1)
        check(L().hawk_query_program(self.handle, buf, n.value + 1, ctypes.byref(n)), self.ctx.handle)
        return buf.value.decode()

    def set_stats(self, selectivity: float):
        check(L().hawk_query_set_stats(self.handle, float(selectivity)))

    def features(self, v: hawk_variant) -> np.ndarray:
        f = (ctypes.c_float * 12)()
        check(L().hawk_features(self.handle, ctypes.byref(v), f))
        return np.frombuffer(f, dtype=np.float32).copy()


def _op(**kw) -> hawk_op:
    op = hawk_op()
    for k, v in kw.items():
        setattr(op, k, v)
    return op


def build_query(ctx: Context, spec: dict) -> Query:
    """Marshals a neutral query description (see paper_1709_00700_amd.datagen)
    into hawk pipelines and creates the query."""
    keep = []

    def cs(s):
        return s.encode() if s is not None else None

    pipes = []
    for i, b in enumerate(spec.get("builds", [])):
        ops = [_op(kind=HAWK_LOOP, table=ctx.tables[b["table"]])]
        for c, lo, hi in b.get("filters", []):
            ops.append(_op(kind=HAWK_FILTER, a=cs(c), lo=int(lo), hi=int(hi)))
        ops.append(_op(kind=HAWK_HASH_PUT, a=cs(b["key"]), b=cs(b["payload"]), ht=i))
        arr = (hawk_op * len(ops))(*ops)
        keep.append(arr)
        pipes.append(hawk_pipeline(arr, len(ops)))
    m = spec["main"]
    ops = [_op(kind=HAWK_LOOP, table=ctx.tables[m["table"]])]
    for c, lo, hi in m.get("filters", []):
        ops.append(_op(kind=HAWK_FILTER, a=cs(c), lo=int(lo), hi=int(hi)))
    if m.get("cross"):
        ops.append(_op(kind=HAWK_CROSS_JOIN, table=ctx.tables[m["cross"]]))
        for c, lo, hi in m.get("cross_filters", []):
            ops.append(_op(kind=HAWK_FILTER, a=cs(c), lo=int(lo), hi=int(hi)))
    for fk, bi, pname in m.get("probes", []):
        ops.append(_op(kind=HAWK_HASH_PROBE, a=cs(fk), b=cs(pname), ht=int(bi)))
    for out, opn, x, y in m.get("arith", []):
        xa, ya = isinstance(x, str), isinstance(y, str)
        ops.append(_op(kind=HAWK_ARITHMETIC, a=cs(out), b=cs(x) if xa else None, c=cs(y) if ya else None,
                       arith_op=ARITH[opn], lo=0 if xa else int(x), hi=0 if ya else int(y)))
    if "project" in m:
        names = (ctypes.c_char_p * len(m["project"]))(*[cs(a) for a in m["project"]])
        keep.append(names)
        ops.append(_op(kind=HAWK_PROJECT, attrs=names, nattrs=len(m["project"])))
    else:
        aggs = (hawk_agg * len(m["aggs"]))(*[hawk_agg(AGG_FN[f], int(bool(w)), cs(a)) for f, a, w in m["aggs"]])
        keep.append(aggs)
        gb = m.get("group_by", [])
        if gb:
            names = (ctypes.c_char_p * len(gb))(*[cs(a) for a in gb])
            keep.append(names)
            ops.append(_op(kind=HAWK_HASH_AGGREGATE, attrs=names, nattrs=len(gb), aggs=aggs, naggs=len(m["aggs"]),
                           groups_hint=int(m.get("groups_hint", 1))))
        else:
            ops.append(_op(kind=HAWK_AGGREGATE, aggs=aggs, naggs=len(m["aggs"])))
    arr = (hawk_op * len(ops))(*ops)
    keep.append(arr)
    pipes.append(hawk_pipeline(arr, len(ops)))
    parr = (hawk_pipeline * len(pipes))(*pipes)
    h = ctypes.c_void_p()
    check(L().hawk_query_create(ctx.handle, parr, len(pipes), ctypes.byref(h)), ctx.handle)
    return Query(ctx, h)


REL = {"scan": 1, "select": 2, "map": 3, "hash_join": 4, "cross_join": 5, "group_by": 6, "project": 7}


def query_from_plan(ctx: Context, plan: dict) -> Query:
    """Marshals a relational plan ({"root": k, "nodes": [...]}, the format
    oracle.relalg documents) into hawk_rel nodes and compiles it
    (hawk_query_from_plan)."""
    keep = []

    def cs(s):
        return s.encode() if isinstance(s, str) else None

    nodes = []
    for nd in plan["nodes"]:
        r = hawk_rel()
        r.kind = REL[nd["op"]]
        r.input = nd.get("input", -1)
        r.right = nd.get("build", nd.get("right", -1))
        op = nd["op"]
        if op == "scan":
            r.table = ctx.tables[nd["table"]]
        elif op == "select":
            r.a, r.lo, r.hi = cs(nd["attr"]), int(nd["lo"]), int(nd["hi"])
        elif op == "map":
            x, y = nd["x"], nd["y"]
            r.a, r.arith_op = cs(nd["out"]), ARITH[nd["fn"]]
            r.b, r.lo = (cs(x), 0) if isinstance(x, str) else (None, int(x))
            r.c, r.hi = (cs(y), 0) if isinstance(y, str) else (None, int(y))
        elif op == "hash_join":
            r.a, r.b, r.c = cs(nd["probe_key"]), cs(nd["build_key"]), cs(nd["payload"])
        elif op in ("group_by", "project"):
            names = nd["keys"] if op == "group_by" else nd["attrs"]
            arr = (ctypes.c_char_p * max(1, len(names)))(*[cs(a) for a in names])
            keep.append(arr)
            r.attrs, r.nattrs = arr, len(names)
            if op == "group_by":
                aggs = (hawk_agg * len(nd["aggs"]))(*[hawk_agg(AGG_FN[f], int(bool(w)), cs(a))
                                                      for f, a, w in nd["aggs"]])
                keep.append(aggs)
                r.aggs, r.naggs, r.groups_hint = aggs, len(nd["aggs"]), int(nd.get("groups_hint", 1))
        nodes.append(r)
    arr = (hawk_rel * len(nodes))(*nodes)
    h = ctypes.c_void_p()
    check(L().hawk_query_from_plan(ctx.handle, arr, len(nodes), int(plan["root"]), ctypes.byref(h)), ctx.handle)
    return Query(ctx, h)


# ---------------------------------------------------------------- results
class Result:
    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.handle = handle

    def free(self):
        if self.handle:
            L().hawk_result_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def info(self):
        n, c = ctypes.c_int64(), ctypes.c_int32()
        check(L().hawk_result_info(self.handle, ctypes.byref(n), ctypes.byref(c)), self.ctx.handle)
        return n.value, c.value

    def column(self, col: int):
        n, _ = self.info()
        kind = ctypes.c_int32()
        ptr = ctypes.c_void_p()
        check(L().hawk_result_column(self.handle, col, ctypes.byref(kind), ctypes.byref(ptr)), self.ctx.handle)
        if kind.value == HAWK_RES_I128:
            raw = np.empty(2 * n, dtype=np.uint64)
            check(L().hawk_result_copy_column(self.handle, col, raw.ctypes.data, raw.nbytes), self.ctx.handle)
            lo, hi = raw[0::2], raw[1::2].view(np.int64)
            return np.array([(int(h) << 64) | int(l) for l, h in zip(lo, hi)], dtype=object)
        dt = np.float64 if kind.value == HAWK_RES_F64 else np.int64
        out = np.empty(n, dtype=dt)
        check(L().hawk_result_copy_column(self.handle, col, out.ctypes.data, out.nbytes), self.ctx.handle)
        return out

    def to_numpy(self, spec: dict) -> dict:
        """Same layout as the oracle's answer; group rows sorted by key."""
        n, ncols = self.info()
        m = spec["main"]
        if "project" in m:
            return {"kind": "project", "rows": n, "cols": [self.column(c) for c in range(ncols)]}
        ng = len(m.get("group_by", []))
        cols = [self.column(c) for c in range(ncols)]
        keys, aggs, cnt = cols[:ng], cols[ng:-1], cols[-1]
        order = np.lexsort(tuple(reversed(keys))) if ng else np.arange(n)
        return {"kind": "aggregate", "rows": n, "keys": [k[order] for k in keys], "count": cnt[order],
                "aggs": [a[order] for a in aggs]}


def profile_enable(ctx: Context, on: bool = True):
    check(L().hawk_profile_enable(ctx.handle, int(on)), ctx.handle)


def profile_read(ctx: Context, kernel: str):
    """(total milliseconds, launches) of a kernel family since profiling was enabled."""
    t, n = ctypes.c_double(), ctypes.c_int64()
    check(L().hawk_profile_read(ctx.handle, kernel.encode(), ctypes.byref(t), ctypes.byref(n)), ctx.handle)
    return t.value, n.value


def execute(ctx: Context, query: Query, v: hawk_variant, sync: bool = True) -> Result:
    h = ctypes.c_void_p()
    fn = L().hawk_execute if sync else L().hawk_execute_async
    check(fn(ctx.handle, query.handle, ctypes.byref(v), ctypes.byref(h)), ctx.handle)
    return Result(ctx, h)


def execute_noalloc(ctx: Context, query: Query, v: hawk_variant, cols=None, cap_rows: int = 0) -> int:
    """hawk_execute_noalloc: `cols` are device addresses (ints) of the result
    columns, each of cap_rows elements; None asks for the cap_rows the
    execution needs. Returns the result rows (or that capacity)."""
    n = ctypes.c_int64()
    if cols is None:
        check(L().hawk_execute_noalloc(ctx.handle, query.handle, ctypes.byref(v), None, 0, 0, ctypes.byref(n)),
              ctx.handle)
        return n.value
    arr = (ctypes.c_void_p * len(cols))(*cols)
    check(L().hawk_execute_noalloc(ctx.handle, query.handle, ctypes.byref(v), arr, len(cols), cap_rows,
                                   ctypes.byref(n)), ctx.handle)
    return n.value


def jit_compile_check(ctx: Context, query: Query, v: hawk_variant):
    """Compiles the run-time kernels of (query, v) without a device; raises HawkError with the compiler log."""
    check(L().hawk_jit_compile_check(ctx.handle, query.handle, ctypes.byref(v)), ctx.handle)


def time_variant(ctx: Context, query: Query, v: hawk_variant, reps=5, limit_ms=0.0) -> float:
    ms = ctypes.c_double()
    check(L().hawk_time_variant(ctx.handle, query.handle, ctypes.byref(v), reps, limit_ms, ctypes.byref(ms)), ctx.handle)
    return ms.value


def learn_feature_wise(dim_sizes, cost, q=5, order=None):
    """Algorithm 1 over abstract dimensions with a Python cost function(cfg tuple) -> float."""
    nd = len(dim_sizes)
    sizes = (ctypes.c_int32 * nd)(*dim_sizes)
    ordp = (ctypes.c_int32 * nd)(*order) if order is not None else None
    best = (ctypes.c_int32 * nd)()
    calls = ctypes.c_int64()

    def cb(cfg, n, user):
        return float(cost(tuple(cfg[i] for i in range(n))))

    fn = COST_FN(cb)
    check(L().hawk_learn_feature_wise(sizes, nd, ordp, q, fn, None, best, ctypes.byref(calls)))
    return tuple(best), calls.value


def explore(ctx: Context, queries: list, mode: int, reps=3, max_iters=5, limit_ms=1000.0, timing_db=None,
            resume=False):
    W = (ctypes.c_void_p * len(queries))(*[q.handle.value for q in queries])
    opts = hawk_explore_opts(reps, max_iters, limit_ms, timing_db.encode() if timing_db else None, int(resume), 0)
    best = hawk_variant()
    rep = hawk_explore_report()
    check(L().hawk_explore(ctx.handle, W, len(queries), mode, ctypes.byref(opts), ctypes.byref(best),
                           ctypes.byref(rep)), ctx.handle)
    return best, {"evaluated": rep.evaluated, "pruned": rep.pruned, "best_ms": rep.best_ms, "seconds": rep.seconds,
                  "reused": rep.reused}


# ---------------------------------------------------------------- learned cost model
MLP_NPARAMS = 5057


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Model:
    """The FP32 cost model on the device (see hawk.h, learned cost model)."""

    def __init__(self, ctx: Context, seed: int = 0):
        self.ctx = ctx
        h = ctypes.c_void_p()
        check(L().hawk_model_create(ctx.handle, seed, ctypes.byref(h)), ctx.handle)
        self.handle = h

    def free(self):
        if self.handle:
            L().hawk_model_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def set_params(self, params, mu, sd):
        p, m, s = (np.ascontiguousarray(a, dtype=np.float32) for a in (params, mu, sd))
        check(L().hawk_model_set_params(self.handle, _fptr(p), _fptr(m), _fptr(s)), self.ctx.handle)

    def get_params(self):
        p, m, s = np.empty(MLP_NPARAMS, np.float32), np.empty(12, np.float32), np.empty(12, np.float32)
        check(L().hawk_model_get_params(self.handle, _fptr(p), _fptr(m), _fptr(s)), self.ctx.handle)
        return p, m, s

    def train(self, X, y, epochs=200, batch=512, lr=3e-3, seed=0) -> float:
        X = np.ascontiguousarray(X, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        o = hawk_train_opts(epochs, batch, lr, seed)
        loss = ctypes.c_float()
        check(L().hawk_model_train(self.handle, _fptr(X), _fptr(y), len(y), ctypes.byref(o), ctypes.byref(loss)),
              self.ctx.handle)
        return loss.value

    def predict(self, X) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float32)
        out = np.empty(len(X), np.float32)
        check(L().hawk_model_predict(self.handle, _fptr(X), len(X), _fptr(out)), self.ctx.handle)
        return out

    def pick(self, queries: list):
        W = (ctypes.c_void_p * len(queries))(*[q.handle.value for q in queries])
        out = (hawk_variant * len(queries))()
        pred = np.empty(len(queries), np.float32)
        check(L().hawk_model_pick(self.handle, W, len(queries), out, _fptr(pred)), self.ctx.handle)
        return list(out), pred


def model_pick_ensemble(models: list, penalty: float, queries: list):
    """hawk_model_pick_ensemble: per query the variant with the lowest mean + penalty * sd
    of the models' predicted ln(ms); returns (variants, predicted ms)."""
    M = (ctypes.c_void_p * len(models))(*[m.handle.value for m in models])
    W = (ctypes.c_void_p * len(queries))(*[q.handle.value for q in queries])
    out = (hawk_variant * len(queries))()
    pred = np.empty(len(queries), np.float32)
    check(L().hawk_model_pick_ensemble(M, len(models), float(penalty), W, len(queries), out, _fptr(pred)),
          models[0].ctx.handle)
    return list(out), pred


# ---------------------------------------------------------------- batched execution
TILE = hawk_variant(0, 0, 0, 0, 0, 0, 0, 0, 0, 0)  # in a batch: the query runs in the tile kernels


class Batch:
    """Many queries replayed as one captured graph (see hawk.h, batched execution).
    variants: None, or one hawk_variant per query (TILE: the tile kernels)."""

    def __init__(self, ctx: Context, queries: list, tile_rows_log2=16, wgs_per_cu=2, order=1, separate=1,
                 variants=None):
        self.ctx = ctx
        self.queries = list(queries)  # the batch borrows them
        W = (ctypes.c_void_p * len(queries))(*[q.handle.value for q in queries])
        V = None if variants is None else (hawk_variant * len(queries))(*variants)
        o = hawk_batch_opts(tile_rows_log2, wgs_per_cu, order, separate)
        h = ctypes.c_void_p()
        check(L().hawk_batch_create(ctx.handle, W, len(queries), V, ctypes.byref(o), ctypes.byref(h)), ctx.handle)
        self.handle = h

    def free(self):
        if self.handle:
            L().hawk_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def run(self):
        check(L().hawk_batch_run(self.handle), self.ctx.handle)

    def time(self, reps=5) -> float:
        ms = ctypes.c_double()
        check(L().hawk_batch_time(self.handle, reps, ctypes.byref(ms)), self.ctx.handle)
        return ms.value

    def autotune(self, reps=3):
        o, ms = hawk_batch_opts(), ctypes.c_double()
        check(L().hawk_batch_autotune(self.handle, reps, ctypes.byref(o), ctypes.byref(ms)), self.ctx.handle)
        return o.as_dict(), ms.value

    def opts(self) -> dict:
        o = hawk_batch_opts()
        check(L().hawk_batch_opts_get(self.handle, ctypes.byref(o)), self.ctx.handle)
        return o.as_dict()

    def result(self, i: int) -> Result:
        h = ctypes.c_void_p()
        check(L().hawk_batch_result(self.handle, i, ctypes.byref(h)), self.ctx.handle)
        return Result(self.ctx, h)
