"""The host planner built on its own with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, every warning an error), planning the batch
shapes the planner is used on: the worked example (section 2, Figure 2), the
tiny star, the retail-shaped snowflake in both forms, the grocery star, the
CART node and tree batches (section 3, decision trees), the Rk-means chain
with learned sizing (section 3, Rk-means), user-defined factors, the tagged
star, random acyclic schemas under every root policy, and invalid inputs.

The sanitized library holds only ``planner.cpp`` and the plan ABI
(``plan_abi.cpp``), which run no GPU code.  It runs in a child process with
the sanitizer runtime preloaded; any report aborts the child.  Every plan it
returns must equal the one the library built with hipcc returns for the same
input, and every rejected input must be rejected with the same status.
"""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2008_08657_amd", "csrc")

# (name, generator call, plan options); generators are small and seeded
CASES = [
    ("worked_example", "W.favorita_example()", {"policy": "groupby"}),
    ("tiny_star_fact", "W.tiny_star(seed=0, n_fact=2000)", {"policy": "fact"}),
    ("tiny_star_cost", "W.tiny_star(seed=1, n_fact=2000)", {"policy": "cost"}),
    ("retail_f32", "W.retail_snowflake(seed=0, n_inv=3000, n_locn=40, n_ksn=200, n_weather_dates=130)",
     {"precision": "f32", "policy": "fact"}),
    ("retail_per_view", "W.retail_snowflake(seed=0, n_inv=3000, n_locn=40, n_ksn=200, n_weather_dates=130)",
     {"precision": "f32", "policy": "fact", "form": "per_view"}),
    ("grocery_bf16x3", "W.grocery_star(seed=0, n_sales=3000)", {"precision": "bf16x3", "policy": "fact"}),
    ("cart_node", "W.cart_node(seed=0, n_inv=3000, n_thr=6, n_locn=40, n_ksn=200, n_weather_dates=130)",
     {"precision": "f32", "policy": "fact"}),
    ("cart_tree", "W.cart_tree(seed=0, n_inv=3000, n_thr=4, n_locn=40, n_ksn=200, n_weather_dates=130)",
     {"precision": "f32", "policy": "fact", "row_weights": ("Inv",)}),
    ("rkmeans_learned", "W.rkmeans_chain(seed=0, n1=3000, n2=500, n3=60, n_x=12, n_y=8, n_z=6, max_dom=100000)",
     {"policy": "fact", "sizing": "learned"}),
    ("udf", "W.udf_grocery(seed=0, n_sales=3000)", {"policy": "fact"}),
    ("tagged_star", "W.tagged_star(seed=0, n_fact=3000)", {"policy": "fact"}),
] + [(f"random_{s}_{pol}", f"W.random_acyclic({s}, n_rel={3 + s % 3})", {"policy": pol})
     for s in range(12) for pol in ("groupby", "fact", "cost")]

# invalid inputs: (name, generator call, mutation applied to the problem)
BAD = [
    ("cycle", "W.tiny_star(seed=0, n_fact=500)", "p['tree'] = p['tree'] + [(1, 2)]"),
    ("missing_attr", "W.tiny_star(seed=0, n_fact=500)", "p['batch'][1]['aggs'][0] = [('nope', 1)]"),
    ("bad_root", "W.tiny_star(seed=0, n_fact=500)", "p['batch'][0]['root'] = 9"),
]

DRIVER = r'''
import ctypes as C, json, sys
sys.path.insert(0, ROOT)
from paper_2008_08657_amd import binding as B
import workloads as W

def plan_all(lib, cases, bad):
    out = {}
    for name, gen, kw in cases:
        p = eval(gen)
        out[name] = plan_one(lib, p, kw)
    for name, gen, mut in bad:
        p = eval(gen)
        exec(mut)
        out[name] = plan_one(lib, p, {})
    return out

def plan_one(lib, p, kw):
    keep = B._Keep()
    schema, tree, batch = B.marshal_problem(p, keep)
    opts = B.build_options(p, keep, lib=lib, **kw)
    h = C.c_void_p()
    st = lib.lmfao_plan(C.byref(schema), C.byref(tree), C.byref(batch), C.byref(opts), C.byref(h))
    if st != 0:
        return {"status": st}
    need = C.c_size_t()
    lib.lmfao_plan_describe(h, None, 0, C.byref(need))
    buf = C.create_string_buffer(need.value)
    lib.lmfao_plan_describe(h, buf, need.value, C.byref(need))
    lib.lmfao_plan_free(h)
    return {"status": 0, "plan": json.loads(buf.value.decode())}

def bind(lib):
    vp = C.c_void_p
    lib.lmfao_default_options.argtypes = [C.POINTER(B.lmfao_options)]
    lib.lmfao_default_options.restype = None
    lib.lmfao_plan.argtypes = [C.POINTER(B.lmfao_schema), C.POINTER(B.lmfao_join_tree), C.POINTER(B.lmfao_batch),
                               C.POINTER(B.lmfao_options), C.POINTER(vp)]
    lib.lmfao_plan.restype = C.c_int32
    lib.lmfao_plan_describe.argtypes = [vp, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]
    lib.lmfao_plan_describe.restype = C.c_int32
    lib.lmfao_plan_free.argtypes = [vp]
    lib.lmfao_plan_free.restype = None
    return lib
'''


def _build(tmp):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not installed")
    out = os.path.join(tmp, "libplan_asan.so")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wall", "-Werror", "-Wno-unused-function", "-Wno-unused-variable",
           "-shared", "-fPIC", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(CSRC, "planner.cpp"), os.path.join(CSRC, "plan_abi.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    # the sanitizer runtime first, then the C++ runtime whose exceptions it
    # intercepts (the interpreter itself does not load it)
    pre = [subprocess.run([gxx, f"-print-file-name={n}"], capture_output=True, text=True).stdout.strip()
           for n in ("libasan.so", "libstdc++.so.6")]
    return out, " ".join(pre)


def test_sanitized_planner_matches_and_reports_nothing(tmp_path):
    lib_path, asan = _build(str(tmp_path))
    script = (f"ROOT = {ROOT!r}\n" + DRIVER +
              f"\nlib = bind(C.CDLL({lib_path!r}))\nres = plan_all(lib, {CASES!r}, {BAD!r})\n"
              "sys.stdout.write(json.dumps(res))\n")
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-6000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
    got = json.loads(r.stdout)
    # the same inputs through the library built with hipcc, in this process
    import paper_2008_08657_amd as E
    ns = {"ROOT": ROOT}
    exec(DRIVER, ns)
    ref = ns["plan_all"](E.load_library(), CASES, BAD)
    assert set(got) == set(ref)
    for name in ref:
        assert got[name] == ref[name], name
    assert all(got[n]["status"] == 0 for n, _, _ in CASES[:11]), {n: got[n]["status"] for n, _, _ in CASES}
    assert all(got[n]["status"] != 0 for n, _, _ in BAD)
