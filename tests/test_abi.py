"""The C-ABI library loads and exports every function ``include/lmfao.h``
declares; host-side argument checks return status codes (no device work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lmfao.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lmfao_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("lmfao_plan", "lmfao_prepare", "lmfao_run", "lmfao_result_copy",
                     "lmfao_plan_describe", "lmfao_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2008_08657_amd as E
    lib = E.load_library()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_default_options():
    import paper_2008_08657_amd as E
    from paper_2008_08657_amd.binding import lmfao_options
    lib = E.load_library()
    o = lmfao_options()
    lib.lmfao_default_options(ctypes.byref(o))
    assert (o.precision, o.form, o.root_policy, o.min_segment, o.row_piece_max, o.contraction) == (0, 0, 0, 0, 0, 0)


def test_null_arguments_are_rejected_before_device_work():
    import paper_2008_08657_amd as E
    lib = E.load_library()
    h = ctypes.c_void_p()
    assert lib.lmfao_plan(None, None, None, None, ctypes.byref(h)) == 1
    assert lib.lmfao_last_error()
    assert lib.lmfao_prepare(None, None, None, ctypes.byref(h)) == 1
    assert lib.lmfao_run(None, None, None, 0) == 1


def test_describe_buffer_convention():
    import paper_2008_08657_amd as E
    import workloads as W
    pl = E.Plan(W.tiny_star(n_fact=50), policy="fact")
    need = ctypes.c_size_t()
    assert pl.lib.lmfao_plan_describe(pl.handle, None, 0, ctypes.byref(need)) == 0
    small = ctypes.create_string_buffer(8)
    assert pl.lib.lmfao_plan_describe(pl.handle, small, 8, ctypes.byref(need)) == 0
    assert len(small.value) == 7 and need.value > 8


def test_struct_layouts_match_header(tmp_path):
    # every struct the binding mirrors has the size and field offsets the C
    # compiler gives the header's declaration
    import shutil
    import subprocess
    from paper_2008_08657_amd import binding as B
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    names = ["lmfao_attr", "lmfao_relation", "lmfao_schema", "lmfao_edge", "lmfao_join_tree", "lmfao_factor",
             "lmfao_aggregate", "lmfao_condition", "lmfao_query", "lmfao_function", "lmfao_batch", "lmfao_options",
             "lmfao_output", "lmfao_grid_dim", "lmfao_column_condition", "lmfao_cart_candidate", "lmfao_cart_spec", "lmfao_cart_split",
             "lmfao_cart_node"]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lmfao.h"', "int main(void) {"]
    for n in names:
        lines.append(f'  printf("{n} size %zu\\n", sizeof({n}));')
        for fname, _ in getattr(B, n)._fields_:
            lines.append(f'  printf("{n} {fname} %zu\\n", offsetof({n}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    c_side = {}
    for ln in out:
        if ln:
            parts = ln.split()
            c_side[(parts[0], parts[1])] = int(parts[2])
    for n in names:
        st = getattr(B, n)
        assert c_side[(n, "size")] == ctypes.sizeof(st), n
        for fname, _ in st._fields_:
            assert c_side[(n, fname)] == getattr(st, fname).offset, f"{n}.{fname}"
