"""Streaming CPU oracle ("tier B") for full-size inputs: the plain definition
of every query of a batch, computed by enumerating the natural join D tuple by
tuple (nested loops along the join tree, through per-edge indexes) without
materialising it, on all host cores (``tierb.c``, C with OpenMP).

TEST INFRASTRUCTURE ONLY (same rules as the ``oracle`` package): used by the
tests, the golden-file scripts under ``tests/golden/`` and the cpu_baseline
leg of ``bench.py``.  It shares no code with the GPU library.

Results have the format of ``oracle.evaluate``: per query ``keys`` (int64,
groups x |G|, lexicographic), ``count`` (int64), ``sum`` (FP64 of a
Neumaier-compensated sum) and ``abs`` (sum of |term|).  It is pinned against
the tier-A oracle (which materialises D and sums in 80-bit precision) on small
inputs in ``tests/test_oracle_tierb.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tierb.c")
LIB = os.path.join(HERE, "libtierb.so")

_DT = {"i32": 0, "f32": 1, "f64": 2}
_OPS = {"<=": 0, "<": 1, ">": 2, ">=": 3, "==": 4, "!=": 5}


def build() -> str:
    """Compiles ``tierb.c`` into ``libtierb.so`` (gcc, OpenMP).  x86-64-v3
    keeps the library loadable on any AVX2 host."""
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Werror",
                    "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


class _Problem(C.Structure):
    _fields_ = [("n_rels", C.c_int32), ("n_rows", C.c_void_p), ("parent", C.c_void_p),
                ("col_off", C.c_void_p), ("col_attr", C.c_void_p), ("col_dtype", C.c_void_p),
                ("col_ptr", C.c_void_p), ("n_attrs", C.c_int32), ("attr_dom", C.c_void_p),
                ("n_queries", C.c_int32), ("gb_off", C.c_void_p), ("gb_attr", C.c_void_p),
                ("cond_off", C.c_void_p), ("cond_attr", C.c_void_p), ("cond_op", C.c_void_p),
                ("cond_c", C.c_void_p), ("agg_off", C.c_void_p), ("agg_f_off", C.c_void_p),
                ("f_attr", C.c_void_p), ("f_pow", C.c_void_p)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = C.CDLL(LIB)
        lib.tb_run.argtypes = [C.POINTER(_Problem), C.c_int, C.c_int64]
        lib.tb_run.restype = C.c_void_p
        lib.tb_groups.argtypes = [C.c_void_p, C.c_int]
        lib.tb_groups.restype = C.c_int64
        lib.tb_seconds.argtypes = [C.c_void_p]
        lib.tb_seconds.restype = C.c_double
        lib.tb_index_seconds.argtypes = [C.c_void_p]
        lib.tb_index_seconds.restype = C.c_double
        lib.tb_threads.argtypes = [C.c_void_p]
        lib.tb_threads.restype = C.c_int
        lib.tb_copy.argtypes = [C.c_void_p, C.c_int] + [C.c_void_p] * 4
        lib.tb_copy.restype = None
        lib.tb_free.argtypes = [C.c_void_p]
        lib.tb_free.restype = None
        _lib = lib
    return _lib


def _bfs(problem, root):
    n = len(problem["schema"])
    adj = {i: [] for i in range(n)}
    for a, b in problem["tree"]:
        adj[a].append(b)
        adj[b].append(a)
    order, parent, queue = [root], {root: -1}, [root]
    while queue:
        u = queue.pop(0)
        for v in sorted(adj[u]):
            if v not in parent:
                parent[v] = u
                order.append(v)
                queue.append(v)
    if len(order) != n:
        raise ValueError("join tree does not connect every relation")
    return order, parent


def evaluate(problem: dict, queries=None, threads: int = 0, root_rows: int = -1, root=None, stats=None) -> list:
    """Every query of the batch (or the listed indices), as ``oracle.evaluate``.

    ``root`` names the relation whose rows drive the enumeration (default:
    the largest); ``root_rows`` >= 0 enumerates only the tuples of D that
    extend that relation's first ``root_rows`` rows (a bounded sample).
    ``threads`` = 0 uses every core OpenMP sees.  ``stats`` (a dict) receives
    the evaluation time, the index-building part of it and the thread count."""
    lib = _load()
    schema = problem["schema"]
    names = [r["name"] for r in schema]
    if root is None:
        root = max(range(len(schema)), key=lambda i: schema[i]["n_rows"])
    elif isinstance(root, str):
        root = names.index(root)
    order, parent = _bfs(problem, root)
    pos = {r: i for i, r in enumerate(order)}
    attr_id, attr_dom = {}, []
    keep = []
    col_off, col_attr, col_dtype, col_ptr = [0], [], [], []
    for r in order:
        rel = schema[r]
        for a in rel["attrs"]:
            name = a["name"]
            if name not in attr_id:
                attr_id[name] = len(attr_id)
                attr_dom.append(0)
            dom = int(a.get("domain", 0) or 0)
            if a["dtype"] == "i32":
                v = np.ascontiguousarray(problem["data"][rel["name"]][name], dtype=np.int32)
                if not dom and len(v):
                    dom = int(v.max()) + 1
            else:
                v = np.ascontiguousarray(problem["data"][rel["name"]][name],
                                         dtype=np.float32 if a["dtype"] == "f32" else np.float64)
            attr_dom[attr_id[name]] = max(attr_dom[attr_id[name]], dom)
            keep.append(v)
            col_attr.append(attr_id[name])
            col_dtype.append(_DT[a["dtype"]])
            col_ptr.append(v.ctypes.data)
        col_off.append(len(col_attr))
    batch = problem["batch"]
    idx = list(range(len(batch))) if queries is None else list(queries)
    gb_off, gb_attr = [0], []
    cond_off, cond_attr, cond_op, cond_c = [0], [], [], []
    agg_off, agg_f_off, f_attr, f_pow = [0], [0], [], []
    for qi in idx:
        q = batch[qi]
        for g in q.get("groupby", []):
            gb_attr.append(attr_id[g])
        gb_off.append(len(gb_attr))
        for a, op, c in q.get("where", []):
            cond_attr.append(attr_id[a])
            cond_op.append(_OPS[op])
            cond_c.append(float(c))
        cond_off.append(len(cond_attr))
        for f in q["aggs"]:
            for a, p in f:
                f_attr.append(attr_id[a])
                f_pow.append(int(p))
            agg_f_off.append(len(f_attr))
        agg_off.append(len(agg_f_off) - 1)

    def arr(x, dt):
        a = np.ascontiguousarray(np.asarray(x, dtype=dt))
        if a.size == 0:
            a = np.zeros(1, dtype=dt)
        keep.append(a)
        return a.ctypes.data

    P = _Problem()
    P.n_rels = len(order)
    P.n_rows = arr([schema[r]["n_rows"] for r in order], np.int64)
    P.parent = arr([-1 if parent[r] < 0 else pos[parent[r]] for r in order], np.int32)
    P.col_off = arr(col_off, np.int32)
    P.col_attr = arr(col_attr, np.int32)
    P.col_dtype = arr(col_dtype, np.int32)
    P.col_ptr = arr(col_ptr, np.uint64)
    P.n_attrs = len(attr_id)
    P.attr_dom = arr(attr_dom, np.int64)
    P.n_queries = len(idx)
    P.gb_off, P.gb_attr = arr(gb_off, np.int32), arr(gb_attr, np.int32)
    P.cond_off, P.cond_attr = arr(cond_off, np.int32), arr(cond_attr, np.int32)
    P.cond_op, P.cond_c = arr(cond_op, np.int32), arr(cond_c, np.float64)
    P.agg_off, P.agg_f_off = arr(agg_off, np.int32), arr(agg_f_off, np.int32)
    P.f_attr, P.f_pow = arr(f_attr, np.int32), arr(f_pow, np.int32)
    h = lib.tb_run(C.byref(P), int(threads), int(root_rows))
    if not h:
        raise RuntimeError("tier-B oracle rejected the problem (more than 64 relations)")
    try:
        out = []
        for k, qi in enumerate(idx):
            q = batch[qi]
            n = lib.tb_groups(h, k)
            na = len(q["aggs"])
            cell = np.zeros(max(n, 1), np.int64)
            cnt = np.zeros(max(n, 1), np.int64)
            s = np.zeros(max(n * na, 1), np.float64)
            ab = np.zeros(max(n * na, 1), np.float64)
            lib.tb_copy(h, k, cell.ctypes.data, cnt.ctypes.data, s.ctypes.data, ab.ctypes.data)
            G = q.get("groupby", [])
            keys = np.zeros((n, len(G)), np.int64)
            rem = cell[:n].copy()
            for j in range(len(G) - 1, -1, -1):
                d = max(1, attr_dom[attr_id[G[j]]])
                keys[:, j] = rem % d
                rem //= d
            out.append({"keys": keys, "count": cnt[:n], "sum": s[:n * na].reshape(n, na),
                        "abs": ab[:n * na].reshape(n, na)})
        if stats is not None:
            stats.update(seconds=lib.tb_seconds(h), index_seconds=lib.tb_index_seconds(h),
                         threads=lib.tb_threads(h))
        return out
    finally:
        lib.tb_free(h)
