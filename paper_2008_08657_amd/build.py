"""Builds the engine's shared library ``liblmfao.so`` for gfx950 with hipcc.

The library holds the planner (C++), the runtime and C ABI, and the HIP
kernels; it is loaded by the ctypes binding in this package.  Usage:
``python -m paper_2008_08657_amd.build``.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "liblmfao.so")

SOURCES = ["planner.cpp", "plan_abi.cpp", "runtime.hip", "kernels.hip", "codegen.hip", "mlp.hip", "rkmeans.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def _flags(src):
    flags = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}", "-Wall",
             "-Wno-unused-function", "-Wno-unused-variable"]
    if src.endswith(".hip"):
        # keep the compiler from emitting packed FP32 instructions (v_pk_*_f32)
        flags += ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
                  "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics"]
    else:
        # host-only C++ (the planner and the plan ABI): warnings are errors
        flags += ["-x", "c++", "-Werror"]
    return flags


def build(verbose: bool = True) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(objdir, s + ".o")
        cmd = [HIPCC] + _flags(s) + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = False
    for cmd, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed = True
            print(text, file=sys.stderr)
        elif verbose and text.strip():
            # host pass warns about the GPU-only target feature; keep other output
            lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l]
            if lines:
                print("\n".join(lines))
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
