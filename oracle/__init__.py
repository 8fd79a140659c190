"""CPU oracle for pipeline programs: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never calls it and
shares no code with it.

``run(tables, spec)`` interprets one query (its build pipelines plus the main
pipeline) column at a time in ``hawk_oracle.cpp`` and returns the plain
relational answer (Section 3.1, Table 1 semantics; the readings taken where
the paper is silent are listed in the module docstring of ``hawk_oracle.cpp``
and in the design notes):

* projection: ``{"kind": "project", "rows": n, "cols": [int64 arrays]}``,
  rows in ascending input order (with a CROSS_JOIN, ``spec["main"]["cross"]``:
  ascending (row, second-table row) pairs);
* aggregation: ``{"kind": "aggregate", "rows": g, "keys": [int64 arrays],
  "count": int64 array, "aggs": [array per aggregate]}`` sorted by group key;
  SUM/COUNT/MIN/MAX are int64 arrays (wide SUMs: Python ``int`` object
  arrays, exact), AVG is float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_SANITIZED=1 loads a build with AddressSanitizer and
# UndefinedBehaviorSanitizer (for a process started with the ASan runtime
# preloaded; see tests/test_oracle_sanitized.py)
_SANITIZED = os.environ.get("ORACLE_SANITIZED") == "1"
_SO = os.path.join(_HERE, "liboracle_san.so" if _SANITIZED else "liboracle.so")
_lib = None

ORC_I8, ORC_I32, ORC_I64 = 1, 2, 3
_ARITH = {"add": 1, "sub": 2, "mul": 3}
_FN = {"count": 1, "sum": 2, "min": 3, "max": 4, "avg": 5}
ORC_E_DUPKEY = -7


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


class _Col(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _Filter(ctypes.Structure):
    _fields_ = [("col", ctypes.c_int32), ("pad", ctypes.c_int32), ("lo", ctypes.c_int64), ("hi", ctypes.c_int64)]


class _Build(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("cols", ctypes.POINTER(_Col)), ("ncols", ctypes.c_int32),
                ("nfilters", ctypes.c_int32), ("filters", ctypes.POINTER(_Filter)),
                ("key_col", ctypes.c_int32), ("payload_col", ctypes.c_int32)]


class _Probe(ctypes.Structure):
    _fields_ = [("fk_col", ctypes.c_int32), ("build", ctypes.c_int32)]


class _Arith(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("x_const", ctypes.c_int32), ("y_const", ctypes.c_int32),
                ("x", ctypes.c_int32), ("y", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("xc", ctypes.c_int64), ("yc", ctypes.c_int64)]


class _Agg(ctypes.Structure):
    _fields_ = [("fn", ctypes.c_int32), ("attr", ctypes.c_int32), ("wide", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _Main(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("cols", ctypes.POINTER(_Col)), ("ncols", ctypes.c_int32),
                ("nfilters", ctypes.c_int32), ("filters", ctypes.POINTER(_Filter)),
                ("inner_nrows", ctypes.c_int64), ("inner_cols", ctypes.POINTER(_Col)), ("ninner", ctypes.c_int32),
                ("nfilters2", ctypes.c_int32), ("filters2", ctypes.POINTER(_Filter)),
                ("nprobes", ctypes.c_int32), ("probes", ctypes.POINTER(_Probe)),
                ("narith", ctypes.c_int32), ("arith", ctypes.POINTER(_Arith)),
                ("kind", ctypes.c_int32),
                ("nproj", ctypes.c_int32), ("proj", ctypes.POINTER(ctypes.c_int32)),
                ("ngroup", ctypes.c_int32), ("group", ctypes.POINTER(ctypes.c_int32)),
                ("naggs", ctypes.c_int32), ("aggs", ctypes.POINTER(_Agg))]


def build(force: bool = True, sanitized: bool | None = None) -> str:
    """Compile the oracle with g++ (plain host code); sanitized: with
    AddressSanitizer and UndefinedBehaviorSanitizer (any report aborts)."""
    san = _SANITIZED if sanitized is None else sanitized
    so = os.path.join(_HERE, "liboracle_san.so" if san else "liboracle.so")
    if force or not os.path.exists(so):
        flags = ["-O2"]
        if san:
            flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                     "-fno-sanitize-recover=undefined"]
        subprocess.check_call(["g++"] + flags + ["-std=c++17", "-shared", "-fPIC", "-pthread", "-o", so + ".tmp",
                                                 os.path.join(_HERE, "hawk_oracle.cpp")])
        os.replace(so + ".tmp", so)
    return so


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        L.orc_run.argtypes = [ctypes.POINTER(_Build), ctypes.c_int32, ctypes.POINTER(_Main),
                              ctypes.POINTER(ctypes.c_void_p)]
        L.orc_run.restype = ctypes.c_int32
        L.orc_run_parallel.argtypes = [ctypes.POINTER(_Build), ctypes.c_int32, ctypes.POINTER(_Main), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_void_p)]
        L.orc_run_parallel.restype = ctypes.c_int32
        L.orc_free.argtypes = [ctypes.c_void_p]
        L.orc_rows.argtypes = [ctypes.c_void_p]
        L.orc_rows.restype = ctypes.c_int64
        for nm in ("orc_project_column", "orc_group_key"):
            getattr(L, nm).argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
        L.orc_group_count.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.orc_agg_value.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_agg_avg.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
        _lib = L
    return _lib


def _dtype_code(a: np.ndarray) -> int:
    return {1: ORC_I8, 4: ORC_I32, 8: ORC_I64}[a.dtype.itemsize]


def _cols(table: dict, keep: list):
    names = list(table.keys())
    arrs = [np.ascontiguousarray(table[c]) for c in names]
    keep.extend(arrs)
    cols = (_Col * max(1, len(arrs)))(*[_Col(a.ctypes.data, _dtype_code(a), 0) for a in arrs])
    nrows = len(arrs[0]) if arrs else 0
    return names, cols, nrows


def _filters(flist, names):
    fs = (_Filter * max(1, len(flist)))(*[_Filter(names.index(c), 0, int(lo), int(hi)) for c, lo, hi in flist])
    return fs


def run(tables: dict, spec: dict, threads: int = 1) -> dict:
    """Interpret the query described by ``spec`` over ``tables`` (numpy columns).
    threads > 1: the main pipeline's rows in that many contiguous ranges on as
    many threads (same answer)."""
    L = _load()
    keep = []
    builds = []
    for b in spec.get("builds", []):
        names, cols, nrows = _cols(tables[b["table"]], keep)
        keep.append(cols)
        fs = _filters(b.get("filters", []), names)
        keep.append(fs)
        builds.append(_Build(nrows, cols, len(names), len(b.get("filters", [])), fs,
                             names.index(b["key"]), names.index(b["payload"])))
    barr = (_Build * max(1, len(builds)))(*builds)
    m = spec["main"]
    names, cols, nrows = _cols(tables[m["table"]], keep)
    attrs = list(names)
    # CROSS_JOIN: the second table's columns follow the looped table's
    inner_names, inner_cols, inner_n = [], (_Col * 1)(), 0
    if m.get("cross"):
        inner_names, inner_cols, inner_n = _cols(tables[m["cross"]], keep)
        attrs += inner_names
    keep.append(inner_cols)
    f2 = m.get("cross_filters", [])
    fs2 = (_Filter * max(1, len(f2)))(*[_Filter(attrs.index(c), 0, int(lo), int(hi)) for c, lo, hi in f2])
    keep.append(fs2)
    probes = []
    for fk, bi, pname in m.get("probes", []):
        probes.append(_Probe(attrs.index(fk), bi))
        attrs.append(pname)
    ariths = []
    for out, op, x, y in m.get("arith", []):
        xc, yc = not isinstance(x, str), not isinstance(y, str)
        ariths.append(_Arith(_ARITH[op], int(xc), int(yc),
                             0 if xc else attrs.index(x), 0 if yc else attrs.index(y), 0,
                             int(x) if xc else 0, int(y) if yc else 0))
        attrs.append(out)
    fl = m.get("filters", [])
    fs = _filters(fl, names)
    parr = (_Probe * max(1, len(probes)))(*probes)
    aarr = (_Arith * max(1, len(ariths)))(*ariths)
    is_proj = "project" in m
    proj = [attrs.index(a) for a in m.get("project", [])]
    group = [attrs.index(a) for a in m.get("group_by", [])]
    aggs = [(_FN[fn], attrs.index(a) if a is not None else 0, int(bool(w))) for fn, a, w in m.get("aggs", [])]
    projarr = (ctypes.c_int32 * max(1, len(proj)))(*proj)
    grparr = (ctypes.c_int32 * max(1, len(group)))(*group)
    aggarr = (_Agg * max(1, len(aggs)))(*[_Agg(f, a, w, 0) for f, a, w in aggs])
    main = _Main(nrows, cols, len(names), len(fl), fs, inner_n, inner_cols, len(inner_names), len(f2), fs2,
                 len(probes), parr, len(ariths), aarr,
                 1 if is_proj else 2, len(proj), projarr, len(group), grparr, len(aggs), aggarr)
    h = ctypes.c_void_p()
    if threads > 1:
        st = L.orc_run_parallel(barr, len(builds), ctypes.byref(main), int(threads), ctypes.byref(h))
    else:
        st = L.orc_run(barr, len(builds), ctypes.byref(main), ctypes.byref(h))
    if st != 0:
        raise OracleError(st)
    try:
        n = L.orc_rows(h)
        if is_proj:
            outs = []
            for c in range(len(proj)):
                a = np.empty(n, dtype=np.int64)
                L.orc_project_column(h, c, a.ctypes.data)
                outs.append(a)
            return {"kind": "project", "rows": int(n), "cols": outs}
        keys = []
        for g in range(len(group)):
            a = np.empty(n, dtype=np.int64)
            L.orc_group_key(h, g, a.ctypes.data)
            keys.append(a)
        cnt = np.empty(n, dtype=np.int64)
        L.orc_group_count(h, cnt.ctypes.data)
        vals = []
        for j, (fn, _, wide) in enumerate(aggs):
            if fn == _FN["avg"]:
                a = np.empty(n, dtype=np.float64)
                L.orc_agg_avg(h, j, a.ctypes.data)
                vals.append(a)
                continue
            lo = np.empty(n, dtype=np.uint64)
            hi = np.empty(n, dtype=np.int64)
            L.orc_agg_value(h, j, lo.ctypes.data, hi.ctypes.data)
            if wide:
                vals.append(np.array([(int(h_) << 64) | int(l_) for l_, h_ in zip(lo, hi)], dtype=object))
            else:
                vals.append(lo.view(np.int64).copy())
        return {"kind": "aggregate", "rows": int(n), "keys": keys, "count": cnt, "aggs": vals}
    finally:
        L.orc_free(h)
