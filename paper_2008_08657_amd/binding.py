"""ctypes binding of ``liblmfao.so`` (argument marshalling only).

The functions mirror the C ABI in ``include/lmfao.h``; every step of the
evaluation runs in the library's HIP kernels.  PyTorch only provides device
memory for the input columns and the stream handle.  The library must have
been built (``python -m paper_2008_08657_amd.build``); loading fails loudly
otherwise -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblmfao.so")

I32, F32, F64 = 0, 1, 2
PREC_F64, PREC_F32, PREC_BF16X3, PREC_BF16X2 = 0, 1, 2, 3
FORM_FUSED, FORM_PER_VIEW = 0, 1
ROOT_GROUPBY, ROOT_FACT, ROOT_COST = 0, 1, 2
OPS = {"<=": 0, "<": 1, ">": 2, ">=": 3, "==": 4, "!=": 5}
_DTYPES = {"i32": I32, "f32": F32, "f64": F64}
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "EUNSUPPORTED", 5: "EOVERFLOW"}


class lmfao_attr(C.Structure):
    _fields_ = [("name", C.c_char_p), ("dtype", C.c_int32), ("domain", C.c_int64), ("is_key", C.c_int32)]


class lmfao_relation(C.Structure):
    _fields_ = [("name", C.c_char_p), ("n_rows", C.c_int64), ("n_attrs", C.c_int32),
                ("attrs", C.POINTER(lmfao_attr))]


class lmfao_schema(C.Structure):
    _fields_ = [("n_relations", C.c_int32), ("relations", C.POINTER(lmfao_relation))]


class lmfao_edge(C.Structure):
    _fields_ = [("a", C.c_int32), ("b", C.c_int32)]


class lmfao_join_tree(C.Structure):
    _fields_ = [("n_edges", C.c_int32), ("edges", C.POINTER(lmfao_edge))]


class lmfao_factor(C.Structure):
    _fields_ = [("attr", C.c_char_p), ("power", C.c_int32)]


class lmfao_aggregate(C.Structure):
    _fields_ = [("n_factors", C.c_int32), ("factors", C.POINTER(lmfao_factor))]


class lmfao_condition(C.Structure):
    _fields_ = [("attr", C.c_char_p), ("op", C.c_int32), ("constant", C.c_double)]


class lmfao_query(C.Structure):
    _fields_ = [("n_groupby", C.c_int32), ("groupby", C.POINTER(C.c_char_p)),
                ("n_conditions", C.c_int32), ("conditions", C.POINTER(lmfao_condition)),
                ("n_aggregates", C.c_int32), ("aggregates", C.POINTER(lmfao_aggregate)),
                ("root", C.c_int32)]


class lmfao_function(C.Structure):
    _fields_ = [("name", C.c_char_p), ("attr", C.c_char_p), ("n_values", C.c_int64),
                ("values", C.POINTER(C.c_double))]


class lmfao_batch(C.Structure):
    _fields_ = [("n_queries", C.c_int32), ("queries", C.POINTER(lmfao_query)),
                ("n_functions", C.c_int32), ("functions", C.POINTER(lmfao_function))]


class lmfao_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("form", C.c_int32), ("root_policy", C.c_int32),
                ("n_order", C.POINTER(C.c_int32)), ("order", C.POINTER(C.POINTER(C.c_char_p))),
                ("min_segment", C.c_int32), ("row_piece_max", C.c_int64),
                ("contraction", C.c_int32), ("codegen", C.c_int32), ("hash_slots", C.c_int64),
                ("sizing", C.c_int32), ("estimator", C.POINTER(C.c_float)), ("estimator_len", C.c_int64),
                ("graph", C.c_int32), ("one_hot_max", C.c_int32), ("scan_blocks", C.c_int32),
                ("partition", C.c_int32), ("contract_splits", C.c_int32), ("row_weights", C.c_uint32)]


class lmfao_output(C.Structure):
    _fields_ = [("n_groups", C.c_int64), ("n_keys", C.c_int32), ("n_aggs", C.c_int32), ("keys", C.c_void_p),
                ("counts", C.c_void_p), ("values", C.c_void_p)]


class lmfao_grid_dim(C.Structure):
    _fields_ = [("attr", C.c_char_p), ("codes", C.c_void_p), ("cluster", C.c_void_p), ("n_codes", C.c_int64)]


class lmfao_column_condition(C.Structure):
    _fields_ = [("column", C.c_void_p), ("dtype", C.c_int32), ("op", C.c_int32), ("constant", C.c_double)]


class lmfao_cart_candidate(C.Structure):
    _fields_ = [("attr", C.c_char_p), ("kind", C.c_int32), ("value", C.c_double), ("query", C.c_int32),
                ("group", C.c_int64)]


class lmfao_cart_spec(C.Structure):
    _fields_ = [("n_candidates", C.c_int32), ("candidates", C.POINTER(lmfao_cart_candidate)),
                ("total_query", C.c_int32), ("max_depth", C.c_int32), ("min_leaf", C.c_int64),
                ("tie_eps", C.c_double)]


class lmfao_cart_split(C.Structure):
    _fields_ = [("best", C.c_int32), ("pad", C.c_int32), ("n", C.c_int64), ("n_left", C.c_int64),
                ("n_right", C.c_int64), ("sum_y", C.c_double), ("sum_y2", C.c_double),
                ("sum_y_left", C.c_double), ("sum_y2_left", C.c_double), ("cost", C.c_double)]


class lmfao_cart_node(C.Structure):
    _fields_ = [("parent", C.c_int32), ("depth", C.c_int32), ("split", C.c_int32), ("left", C.c_int32),
                ("right", C.c_int32), ("pad", C.c_int32), ("n", C.c_int64), ("sum_y", C.c_double),
                ("sum_y2", C.c_double), ("cost", C.c_double)]


class LmfaoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads the engine library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2008_08657_amd.build`")
    # PyTorch ships its own HIP runtime with the same soname; load it first so
    # the process holds one runtime, shared by torch's tensors and this library
    import torch  # noqa: F401
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.lmfao_default_options.argtypes = [C.POINTER(lmfao_options)]
    lib.lmfao_default_options.restype = None
    lib.lmfao_plan.argtypes = [C.POINTER(lmfao_schema), C.POINTER(lmfao_join_tree), C.POINTER(lmfao_batch),
                               C.POINTER(lmfao_options), C.POINTER(vp)]
    lib.lmfao_plan.restype = C.c_int32
    lib.lmfao_plan_describe.argtypes = [vp, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]
    lib.lmfao_plan_describe.restype = C.c_int32
    lib.lmfao_plan_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    lib.lmfao_plan_workspace_bytes.restype = C.c_int32
    lib.lmfao_prepare.argtypes = [vp, C.POINTER(C.POINTER(vp)), vp, C.POINTER(vp)]
    lib.lmfao_prepare.restype = C.c_int32
    lib.lmfao_run.argtypes = [vp, vp, vp, C.c_int32]
    lib.lmfao_run.restype = C.c_int32
    lib.lmfao_result_shape.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32)]
    lib.lmfao_result_shape.restype = C.c_int32
    lib.lmfao_result_copy.argtypes = [vp, C.c_int32, vp, vp, vp]
    lib.lmfao_result_copy.restype = C.c_int32
    lib.lmfao_view_shape.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32)]
    lib.lmfao_view_shape.restype = C.c_int32
    lib.lmfao_view_copy.argtypes = [vp, C.c_int32, vp, vp, vp]
    lib.lmfao_view_copy.restype = C.c_int32
    lib.lmfao_set_timing.argtypes = [vp, C.c_int32]
    lib.lmfao_set_timing.restype = C.c_int32
    lib.lmfao_run_timing.argtypes = [vp, C.c_int32, C.POINTER(C.c_char_p), C.POINTER(C.c_float),
                                     C.POINTER(C.c_int32)]
    lib.lmfao_run_timing.restype = C.c_int32
    lib.lmfao_prepared_describe.argtypes = [vp, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]
    lib.lmfao_prepared_describe.restype = C.c_int32
    lib.lmfao_plan_free.argtypes = [vp]
    lib.lmfao_plan_free.restype = None
    lib.lmfao_prepared_free.argtypes = [vp]
    lib.lmfao_prepared_free.restype = None
    lib.lmfao_last_error.argtypes = []
    lib.lmfao_last_error.restype = C.c_char_p
    lib.lmfao_tune.argtypes = [C.POINTER(lmfao_schema), C.POINTER(lmfao_join_tree), C.POINTER(lmfao_batch),
                               C.POINTER(lmfao_options), C.POINTER(C.POINTER(vp)), C.c_char_p, C.c_int32,
                               C.POINTER(C.c_double), C.POINTER(C.c_double), vp]
    lib.lmfao_tune.restype = C.c_int32
    lib.lmfao_prepare_in.argtypes = [vp, C.POINTER(C.POINTER(vp)), vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.lmfao_prepare_in.restype = C.c_int32
    lib.lmfao_prepared_workspace_bytes.argtypes = [vp, C.c_int32, C.POINTER(C.c_size_t)]
    lib.lmfao_prepared_workspace_bytes.restype = C.c_int32
    lib.lmfao_result_device.argtypes = [vp, C.c_int32, C.POINTER(lmfao_output), vp]
    lib.lmfao_result_device.restype = C.c_int32
    lib.lmfao_kmeans_1d.argtypes = [C.c_int32, C.POINTER(C.c_int64), vp, vp, C.c_int32, C.c_int32, vp, vp,
                                    C.POINTER(C.c_int32), vp]
    lib.lmfao_kmeans_1d.restype = C.c_int32
    lib.lmfao_grid_coreset.argtypes = [vp, vp, C.POINTER(C.POINTER(vp)), C.c_int32, C.POINTER(lmfao_grid_dim),
                                       C.c_int32, C.POINTER(lmfao_output), vp]
    lib.lmfao_grid_coreset.restype = C.c_int32
    lib.lmfao_row_weights.argtypes = [vp, C.c_int32, C.POINTER(vp)]
    lib.lmfao_row_weights.restype = C.c_int32
    lib.lmfao_eval_conditions.argtypes = [C.c_int64, C.c_int32, C.POINTER(lmfao_column_condition), vp, vp]
    lib.lmfao_eval_conditions.restype = C.c_int32
    lib.lmfao_cart_best_split.argtypes = [vp, C.POINTER(lmfao_cart_spec), C.POINTER(lmfao_cart_split), vp, vp]
    lib.lmfao_cart_best_split.restype = C.c_int32
    lib.lmfao_cart_grow.argtypes = [vp, vp, C.POINTER(C.POINTER(vp)), C.POINTER(lmfao_cart_spec),
                                    C.POINTER(lmfao_cart_node), C.c_int32, C.POINTER(C.c_int32), vp]
    lib.lmfao_cart_grow.restype = C.c_int32
    _lib = lib
    return lib


def _check(lib, st):
    if st != 0:
        raise LmfaoError(st, lib.lmfao_last_error().decode(errors="replace"))


class _DeviceArray:
    """A device array the library owns, described to torch without a copy."""

    def __init__(self, ptr, shape, typestr):
        self.__cuda_array_interface__ = {"shape": tuple(int(x) for x in shape), "typestr": typestr,
                                         "data": (int(ptr), False), "version": 2, "strides": None}


class _Keep:
    """Owns the ctypes buffers passed to one call."""

    def __init__(self):
        self.refs = []

    def s(self, x: str):
        b = x.encode()
        self.refs.append(b)
        return b

    def arr(self, ctype, items):
        a = (ctype * max(1, len(items)))(*items)
        self.refs.append(a)
        return a


def marshal_problem(problem, keep: _Keep):
    """schema / tree / batch dicts -> ctypes structs (host pointers)."""
    rels = []
    names = [r["name"] for r in problem["schema"]]
    for r in problem["schema"]:
        attrs = [lmfao_attr(keep.s(a["name"]), _DTYPES[a["dtype"]], int(a.get("domain", 0)),
                            1 if a.get("key") else 0) for a in r["attrs"]]
        arr = keep.arr(lmfao_attr, attrs)
        rels.append(lmfao_relation(keep.s(r["name"]), int(r["n_rows"]), len(attrs), arr))
    schema = lmfao_schema(len(rels), keep.arr(lmfao_relation, rels))
    edges = [lmfao_edge(int(a), int(b)) for a, b in problem["tree"]]
    tree = lmfao_join_tree(len(edges), keep.arr(lmfao_edge, edges))
    queries = []
    for q in problem["batch"]:
        gb = keep.arr(C.c_char_p, [keep.s(g) for g in q.get("groupby", [])])
        conds = keep.arr(lmfao_condition, [lmfao_condition(keep.s(a), OPS[op], float(c))
                                           for a, op, c in q.get("where", [])])
        aggs = []
        for f in q["aggs"]:
            fs = keep.arr(lmfao_factor, [lmfao_factor(keep.s(a), int(p)) for a, p in f])
            aggs.append(lmfao_aggregate(len(f), fs))
        root = q.get("root")
        root_i = -1 if root is None else (names.index(root) if isinstance(root, str) else int(root))
        queries.append(lmfao_query(len(q.get("groupby", [])), gb, len(q.get("where", [])), conds,
                                   len(aggs), keep.arr(lmfao_aggregate, aggs), root_i))
    funcs = []
    for name, f in problem.get("functions", {}).items():
        vals = [float(x) for x in f["values"]]
        funcs.append(lmfao_function(keep.s(name), keep.s(f["attr"]), len(vals), keep.arr(C.c_double, vals)))
    batch = lmfao_batch(len(queries), keep.arr(lmfao_query, queries), len(funcs), keep.arr(lmfao_function, funcs))
    keep.refs += [schema, tree, batch]
    return schema, tree, batch


def build_options(problem, keep, precision="f64", policy=None, form="fused", order=None,
                  min_segment=0, row_piece_max=0, contraction="mfma", codegen=True, hash_slots=0,
                  sizing="bound", estimator=None, graph=False, one_hot_max=0, scan_blocks=0,
                  contract_splits=0, partition=True, row_weights=(), lib=None):
    """Keyword options -> ``lmfao_options`` (buffers it points to kept in
    ``keep``); ``lib`` is the library whose ``lmfao_default_options`` fills
    the defaults (this package's by default)."""
    lib = lib if lib is not None else load_library()
    opts = lmfao_options()
    lib.lmfao_default_options(C.byref(opts))
    if precision not in ("f64", "f32", "bf16x3", "bf16x2"):
        raise ValueError(f"precision must be 'f64', 'f32', 'bf16x3' or 'bf16x2', not {precision!r}")
    opts.precision = {"f64": PREC_F64, "f32": PREC_F32, "bf16x3": PREC_BF16X3,
                      "bf16x2": PREC_BF16X2}[precision]
    opts.form = FORM_FUSED if form == "fused" else FORM_PER_VIEW
    pol = policy if policy is not None else problem.get("policy", "groupby")
    if pol not in ("fact", "groupby", "cost"):
        raise ValueError(f"policy must be 'fact', 'groupby' or 'cost', not {pol!r}")
    opts.root_policy = {"fact": ROOT_FACT, "groupby": ROOT_GROUPBY, "cost": ROOT_COST}[pol]
    opts.min_segment = int(min_segment)
    opts.row_piece_max = int(row_piece_max)
    if contraction not in ("mfma", "valu"):
        raise ValueError(f"contraction must be 'mfma' or 'valu', not {contraction!r}")
    opts.contraction = 0 if contraction == "mfma" else 1
    opts.codegen = 0 if codegen else 1
    opts.hash_slots = int(hash_slots)
    opts.graph = 1 if graph else 0
    opts.one_hot_max = int(one_hot_max)
    opts.scan_blocks = int(scan_blocks)
    opts.contract_splits = int(contract_splits)
    opts.partition = 0 if partition else 1
    rel_names = [r["name"] for r in problem["schema"]]
    opts.row_weights = sum(1 << rel_names.index(r) for r in row_weights)
    if sizing not in ("bound", "learned", "exact"):
        raise ValueError(f"sizing must be 'bound', 'learned' or 'exact', not {sizing!r}")
    opts.sizing = {"bound": 0, "learned": 1, "exact": 2}[sizing]
    if sizing == "learned" and estimator is None:
        from . import estimator as _est
        estimator = _est.load()
    if estimator is not None:
        import numpy as np
        blob = np.ascontiguousarray(estimator, dtype=np.float32)
        keep.refs.append(blob)
        opts.estimator = blob.ctypes.data_as(C.POINTER(C.c_float))
        opts.estimator_len = int(blob.size)
    if order:
        names = [r["name"] for r in problem["schema"]]
        n_order = [len(order.get(n, [])) for n in names]
        lists = [keep.arr(C.c_char_p, [keep.s(a) for a in order.get(n, [])]) for n in names]
        opts.n_order = keep.arr(C.c_int32, n_order)
        ptrs = keep.arr(C.POINTER(C.c_char_p), [C.cast(l, C.POINTER(C.c_char_p)) for l in lists])
        opts.order = C.cast(ptrs, C.POINTER(C.POINTER(C.c_char_p)))
    keep.refs.append(opts)
    return opts


def _column_table(problem, columns, keep):
    per_rel = []
    for r in problem["schema"]:
        ptrs = [C.c_void_p(int(columns[r["name"]][a["name"]].data_ptr())) for a in r["attrs"]]
        per_rel.append(C.cast(keep.arr(C.c_void_p, ptrs), C.POINTER(C.c_void_p)))
    return keep.arr(C.POINTER(C.c_void_p), per_rel)


def tune(problem, columns, cache_path=None, runs=5, stream=None, **plan_kw) -> dict:
    """Launch shapes tuned for this batch, relations and device
    (``lmfao_tune``): the plan keyword options with scan_blocks,
    contract_splits and one_hot_max replaced, plus the step times of the
    tuned and base options ("tuned_ms", "base_ms")."""
    lib = load_library()
    keep = _Keep()
    schema, tree, batch = marshal_problem(problem, keep)
    opts = build_options(problem, keep, **plan_kw)
    cols = _column_table(problem, columns, keep)
    best, base = C.c_double(), C.c_double()
    path = keep.s(cache_path) if cache_path else None
    _check(lib, lib.lmfao_tune(C.byref(schema), C.byref(tree), C.byref(batch), C.byref(opts), cols, path,
                               int(runs), C.byref(best), C.byref(base), C.c_void_p(stream) if stream else None))
    out = dict(plan_kw, scan_blocks=opts.scan_blocks, contract_splits=opts.contract_splits,
               one_hot_max=opts.one_hot_max)
    return {"options": out, "tuned_ms": best.value, "base_ms": base.value}


class Plan:
    """A plan handle (``lmfao_plan``)."""

    def __init__(self, problem, **kw):
        self.lib = load_library()
        self.problem = problem
        keep = _Keep()
        schema, tree, batch = marshal_problem(problem, keep)
        opts = build_options(problem, keep, **kw)
        precision = kw.get("precision", "f64")
        h = C.c_void_p()
        _check(self.lib, self.lib.lmfao_plan(C.byref(schema), C.byref(tree), C.byref(batch),
                                             C.byref(opts), C.byref(h)))
        self.handle = h
        self.precision = precision

    def describe(self) -> dict:
        need = C.c_size_t()
        _check(self.lib, self.lib.lmfao_plan_describe(self.handle, None, 0, C.byref(need)))
        buf = C.create_string_buffer(need.value)
        _check(self.lib, self.lib.lmfao_plan_describe(self.handle, buf, need.value, C.byref(need)))
        return json.loads(buf.value.decode())

    def workspace_bytes(self) -> int:
        b = C.c_size_t()
        _check(self.lib, self.lib.lmfao_plan_workspace_bytes(self.handle, C.byref(b)))
        return b.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.lmfao_plan_free(h)
            self.handle = None


class Prepared:
    """Sorted relations, pieces and buffers for one plan (``lmfao_prepare``).

    ``columns`` maps relation name -> attribute name -> device tensor (torch,
    contiguous, int32 / float32 / float64 as declared).  The plan must outlive
    this object."""

    def __init__(self, plan: Plan, columns: dict, stream=None, workspace=None):
        self.plan = plan
        self.lib = plan.lib
        keep = _Keep()
        cols = _column_table(plan.problem, columns, keep)
        self.stream = C.c_void_p(stream) if stream else C.c_void_p()
        h = C.c_void_p()
        if workspace is None:
            _check(self.lib, self.lib.lmfao_prepare(plan.handle, cols, self.stream, C.byref(h)))
        else:
            # a caller (torch) allocation holds every device buffer of the handle
            self.workspace = workspace
            _check(self.lib, self.lib.lmfao_prepare_in(plan.handle, cols, C.c_void_p(workspace.data_ptr()),
                                                       workspace.numel() * workspace.element_size(),
                                                       self.stream, C.byref(h)))
        self.handle = h

    def workspace_bytes(self, with_results=True) -> int:
        """Bytes a workspace must hold for this plan and these inputs
        (``lmfao_prepared_workspace_bytes``)."""
        b = C.c_size_t()
        _check(self.lib, self.lib.lmfao_prepared_workspace_bytes(self.handle, 1 if with_results else 0,
                                                                 C.byref(b)))
        return int(b.value)

    def result_device(self, q: int) -> dict:
        """Query q's result compacted on the GPU (``lmfao_result_device``):
        torch tensors over the library's device arrays (no copy), valid until
        the next run."""
        import torch
        o = lmfao_output()
        _check(self.lib, self.lib.lmfao_result_device(self.handle, int(q), C.byref(o), self.stream))
        n = int(o.n_groups)

        def view(ptr, shape, typestr, dtype):
            if n == 0 or not ptr:
                return torch.empty(shape, dtype=dtype, device="cuda")
            return torch.as_tensor(_DeviceArray(ptr, shape, typestr), device="cuda")

        return {"keys": view(o.keys, (n, o.n_keys), "<i8", torch.int64),
                "count": view(o.counts, (n,), "<i8", torch.int64),
                "sum": view(o.values, (n, o.n_aggs), "<f8", torch.float64)}

    def run(self, sync=True, stream=None):
        s = C.c_void_p(stream) if stream is not None else self.stream
        _check(self.lib, self.lib.lmfao_run(self.plan.handle, self.handle, s, 1 if sync else 0))

    def set_timing(self, on=True):
        _check(self.lib, self.lib.lmfao_set_timing(self.handle, 1 if on else 0))

    def describe(self) -> dict:
        need = C.c_size_t()
        _check(self.lib, self.lib.lmfao_prepared_describe(self.handle, None, 0, C.byref(need)))
        buf = C.create_string_buffer(need.value)
        _check(self.lib, self.lib.lmfao_prepared_describe(self.handle, buf, need.value, C.byref(need)))
        return json.loads(buf.value.decode())

    def features(self, q: int):
        """Estimator features of query q (``lmfao_prepared_features``), or None
        for a query without group-by attributes."""
        f = (C.c_float * 26)()
        st = self.lib.lmfao_prepared_features(self.handle, int(q), f)
        if st != 0:
            return None
        return list(f)

    def timing(self):
        n = C.c_int32()
        _check(self.lib, self.lib.lmfao_run_timing(self.handle, 0, None, None, C.byref(n)))
        names = (C.c_char_p * max(1, n.value))()
        ms = (C.c_float * max(1, n.value))()
        _check(self.lib, self.lib.lmfao_run_timing(self.handle, n.value, names, ms, C.byref(n)))
        return [(names[i].decode(), ms[i]) for i in range(n.value)]

    def result(self, q: int) -> dict:
        import numpy as np
        ng, nk, na = C.c_int64(), C.c_int32(), C.c_int32()
        _check(self.lib, self.lib.lmfao_result_shape(self.handle, q, C.byref(ng), C.byref(nk), C.byref(na)))
        keys = np.zeros((ng.value, nk.value), dtype=np.int64)
        cnt = np.zeros(ng.value, dtype=np.int64)
        vals = np.zeros((ng.value, na.value), dtype=np.float64)
        _check(self.lib, self.lib.lmfao_result_copy(
            self.handle, q, keys.ctypes.data_as(C.c_void_p), cnt.ctypes.data_as(C.c_void_p),
            vals.ctypes.data_as(C.c_void_p)))
        return {"keys": keys, "count": cnt, "sum": vals}

    def view(self, v: int) -> dict:
        """Dense contents of intermediate view v: counts, values, codes per key."""
        import numpy as np
        nk, nv, nc = C.c_int64(), C.c_int32(), C.c_int32()
        _check(self.lib, self.lib.lmfao_view_shape(self.handle, v, C.byref(nk), C.byref(nv), C.byref(nc)))
        cnt = np.zeros(nk.value, dtype=np.int64)
        vals = np.zeros((nk.value, nv.value), dtype=np.float64)
        codes = np.zeros((nk.value, nc.value), dtype=np.int32)
        _check(self.lib, self.lib.lmfao_view_copy(self.handle, v, cnt.ctypes.data_as(C.c_void_p),
                                                  vals.ctypes.data_as(C.c_void_p),
                                                  codes.ctypes.data_as(C.c_void_p)))
        return {"count": cnt, "values": vals, "codes": codes}

    def results(self):
        return [self.result(q) for q in range(len(self.plan.problem["batch"]))]

    def kernel_sources(self):
        """Sources of the scan kernels generated for this plan."""
        out = []
        for i in range(self.describe().get("generated_scans", 0)):
            need = C.c_size_t()
            _check(self.lib, self.lib.lmfao_prepared_kernel_source(self.handle, i, None, 0, C.byref(need)))
            buf = C.create_string_buffer(need.value)
            _check(self.lib, self.lib.lmfao_prepared_kernel_source(self.handle, i, buf, need.value, C.byref(need)))
            out.append(buf.value.decode())
        return out

    def _cart_spec(self, keep, spec):
        cands = [lmfao_cart_candidate(keep.s(c["attr"]), {"<=": 0, "==": 1}[c["op"]], float(c["value"]),
                                      int(c["query"]), int(c.get("group", 0))) for c in spec["candidates"]]
        arr = keep.arr(lmfao_cart_candidate, cands)
        sp = lmfao_cart_spec(len(cands), arr, int(spec["total_query"]), int(spec.get("max_depth", 0)),
                             int(spec.get("min_leaf", 1)), float(spec.get("tie_eps", 1e-9)))
        keep.refs.append(sp)
        return sp

    def cart_best_split(self, spec, costs=None) -> dict:
        """The node's best split from the last run's results, chosen on the
        GPU (``lmfao_cart_best_split``); ``costs`` an optional float64 device
        tensor receiving every candidate's cost."""
        keep = _Keep()
        sp = self._cart_spec(keep, spec)
        out = lmfao_cart_split()
        cp = C.c_void_p(costs.data_ptr()) if costs is not None else None
        _check(self.lib, self.lib.lmfao_cart_best_split(self.handle, C.byref(sp), C.byref(out), cp, self.stream))
        return {f: getattr(out, f) for f, _ in lmfao_cart_split._fields_ if f != "pad"}

    def cart_grow(self, spec, columns) -> list:
        """Grows the regression tree on the GPU (``lmfao_cart_grow``);
        ``columns`` are the device tensors given to the constructor (they
        must still be alive).  Returns the nodes as dicts."""
        keep = _Keep()
        cols = _column_table(self.plan.problem, columns, keep)
        sp = self._cart_spec(keep, spec)
        cap = (1 << (int(spec.get("max_depth", 0)) + 1)) - 1
        nodes = (lmfao_cart_node * cap)()
        n = C.c_int32()
        _check(self.lib, self.lib.lmfao_cart_grow(self.plan.handle, self.handle, cols, C.byref(sp), nodes, cap,
                                                  C.byref(n), self.stream))
        return [{f: getattr(nodes[i], f) for f, _ in lmfao_cart_node._fields_ if f != "pad"} for i in range(n.value)]

    def grid_coreset(self, columns, dims, k: int) -> dict:
        """Rk-means step 3 (``lmfao_grid_coreset``): ``dims`` lists (attr,
        codes, cluster) with int64 and int32 device tensors; returns the grid
        points' cluster ids and weights as device tensors (no copy)."""
        import torch
        keep = _Keep()
        cols = _column_table(self.plan.problem, columns, keep)
        ds = keep.arr(lmfao_grid_dim, [lmfao_grid_dim(keep.s(a), C.c_void_p(c.data_ptr()), C.c_void_p(cl.data_ptr()),
                                                      int(c.numel())) for a, c, cl in dims])
        o = lmfao_output()
        _check(self.lib, self.lib.lmfao_grid_coreset(self.plan.handle, self.handle, cols, len(dims), ds, int(k),
                                                     C.byref(o), self.stream))
        n = int(o.n_groups)
        if n == 0:
            return {"keys": torch.empty((0, len(dims)), dtype=torch.int64, device="cuda"),
                    "count": torch.empty(0, dtype=torch.int64, device="cuda")}
        return {"keys": torch.as_tensor(_DeviceArray(o.keys, (n, len(dims)), "<i8"), device="cuda"),
                "count": torch.as_tensor(_DeviceArray(o.counts, (n,), "<i8"), device="cuda")}

    def ridge_sigma(self, continuous, categorical=()):
        """Sigma = sum over D of x x^T assembled on the device from the last
        run's results (``lmfao_ridge_sigma``); a (dim, dim) FP64 torch tensor."""
        import torch
        keep = _Keep()
        cont = keep.arr(C.c_char_p, [keep.s(a) for a in continuous])
        cats = keep.arr(C.c_char_p, [keep.s(a) for a in categorical])
        dim = C.c_int32()
        _check(self.lib, self.lib.lmfao_ridge_sigma(self.handle, len(continuous), cont, len(categorical), cats,
                                                    None, C.byref(dim), self.stream))
        sig = torch.empty((dim.value, dim.value), dtype=torch.float64, device="cuda")
        _check(self.lib, self.lib.lmfao_ridge_sigma(self.handle, len(continuous), cont, len(categorical), cats,
                                                    C.c_void_p(sig.data_ptr()), C.byref(dim), self.stream))
        return sig

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.lmfao_prepared_free(h)
            self.handle = None


def ridge_bgd(sigma, label: int, lam: float, eta: float = 0.0, max_iter: int = 20_000, tol: float = 1e-10,
              stream=None):
    """Batch gradient descent for ridge regression on a device Sigma
    (``lmfao_ridge_bgd``).  Returns (theta tensor, steps, ||grad||, eta)."""
    import torch
    lib = load_library()
    dim = int(sigma.shape[0])
    theta = torch.empty(dim, dtype=torch.float64, device=sigma.device)
    stats = (C.c_double * 3)()
    _check(lib, lib.lmfao_ridge_bgd(C.c_void_p(sigma.data_ptr()), dim, int(label), C.c_double(lam),
                                    C.c_double(eta), int(max_iter), C.c_double(tol),
                                    C.c_void_p(theta.data_ptr()), stats, C.c_void_p(stream) if stream else None))
    return theta, int(stats[0]), float(stats[1]), float(stats[2])


def kmeans_1d(sets, k: int, max_iter: int = 100, stream=None):
    """Rk-means step 2 (``lmfao_kmeans_1d``): ``sets`` lists (values,
    weights) pairs of int64 device tensors (ascending values).  Returns
    (centroids n_sets x k float64 tensor, per-set cluster tensors, update
    steps per set)."""
    import torch
    lib = load_library()
    sizes = [int(v.numel()) for v, _ in sets]
    offsets = [0]
    for m in sizes:
        offsets.append(offsets[-1] + m)
    values = torch.cat([v.reshape(-1) for v, _ in sets]) if sets else torch.empty(0, dtype=torch.int64, device="cuda")
    weights = torch.cat([w.reshape(-1) for _, w in sets]) if sets else torch.empty(0, dtype=torch.int64, device="cuda")
    cent = torch.empty((len(sets), k), dtype=torch.float64, device="cuda")
    assign = torch.empty(max(1, offsets[-1]), dtype=torch.int32, device="cuda")
    steps = (C.c_int32 * max(1, len(sets)))()
    off = (C.c_int64 * len(offsets))(*offsets)
    _check(lib, lib.lmfao_kmeans_1d(len(sets), off, C.c_void_p(values.data_ptr()), C.c_void_p(weights.data_ptr()),
                                    int(k), int(max_iter), C.c_void_p(cent.data_ptr()),
                                    C.c_void_p(assign.data_ptr()), steps, _stream_arg(stream)))
    parts = [assign[offsets[i]:offsets[i + 1]] for i in range(len(sets))]
    return cent, parts, [steps[i] for i in range(len(sets))]


def _stream_arg(stream):
    return C.c_void_p(stream) if stream else None


def mlp_size(d: int, h: int) -> int:
    """Number of FP32 parameters of the estimator network (``lmfao_mlp_size``)."""
    lib = load_library()
    n = C.c_int64()
    _check(lib, lib.lmfao_mlp_size(int(d), int(h), C.byref(n)))
    return int(n.value)


def _f32_dev(x, name):
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    return C.c_void_p(x.data_ptr())


def mlp_grad(params, X, t, h: int, stream=None):
    """Gradient and loss of the mean squared error on device tensors
    (``lmfao_mlp_grad``).  Returns (grad tensor, loss)."""
    import torch
    lib = load_library()
    n, d = int(X.shape[0]), int(X.shape[1])
    grad = torch.empty_like(params)
    loss = C.c_float()
    _check(lib, lib.lmfao_mlp_grad(d, int(h), _f32_dev(params, "params"), _f32_dev(X, "X"), _f32_dev(t, "t"), n,
                                   _f32_dev(grad, "grad"), C.byref(loss), _stream_arg(stream)))
    return grad, float(loss.value)


def mlp_grad_noalloc(params, X, t, h: int, stream=None):
    """``lmfao_mlp_grad_noalloc``: the gradient and loss with the library's
    fixed device scratch instead of allocations.  Returns (grad, loss)."""
    import torch
    lib = load_library()
    n, d = int(X.shape[0]), int(X.shape[1])
    grad = torch.empty_like(params)
    loss = C.c_float()
    _check(lib, lib.lmfao_mlp_grad_noalloc(d, int(h), _f32_dev(params, "params"), _f32_dev(X, "X"),
                                           _f32_dev(t, "t"), n, _f32_dev(grad, "grad"), C.byref(loss),
                                           _stream_arg(stream)))
    return grad, float(loss.value)


def mlp_predict(params, X, h: int, stream=None):
    """Network outputs for the rows of X (``lmfao_mlp_predict``)."""
    import torch
    lib = load_library()
    n, d = int(X.shape[0]), int(X.shape[1])
    y = torch.empty(n, dtype=torch.float32, device=X.device)
    _check(lib, lib.lmfao_mlp_predict(d, int(h), _f32_dev(params, "params"), _f32_dev(X, "X"), n,
                                      _f32_dev(y, "y"), _stream_arg(stream)))
    return y


def mlp_train(params, X, t, order, batch: int, h: int, lr: float = 1e-3, stream=None):
    """Adam steps in place on ``params`` (``lmfao_mlp_train``); ``order`` is an
    int32 device tensor of n_steps*batch row indices.  Returns the per-step
    batch losses."""
    import torch
    lib = load_library()
    n, d = int(X.shape[0]), int(X.shape[1])
    if not (order.is_cuda and order.dtype == torch.int32 and order.is_contiguous()):
        raise TypeError("order must be a contiguous int32 CUDA tensor")
    steps = int(order.numel()) // int(batch)
    trace = (C.c_float * max(steps, 1))()
    _check(lib, lib.lmfao_mlp_train(d, int(h), _f32_dev(params, "params"), _f32_dev(X, "X"), _f32_dev(t, "t"), n,
                                    C.c_void_p(order.data_ptr()), steps, int(batch), C.c_float(lr), trace,
                                    _stream_arg(stream)))
    return list(trace)[:steps]


def device_columns(problem, device="cuda:0"):
    """Copies every generated column to the device as a torch tensor."""
    import numpy as np
    import torch
    out = {}
    for r in problem["schema"]:
        cols = {}
        for a in r["attrs"]:
            v = problem["data"][r["name"]][a["name"]]
            dt = {"i32": np.int32, "f32": np.float32, "f64": np.float64}[a["dtype"]]
            cols[a["name"]] = torch.from_numpy(np.ascontiguousarray(v, dtype=dt)).to(device)
        out[r["name"]] = cols
    return out
