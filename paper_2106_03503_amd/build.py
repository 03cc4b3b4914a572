"""Build libedt.so (HIP for gfx950) in-tree.

Every translation unit is compiled by hipcc for gfx950 only.  The shared
library is linked against the HIP runtime that PyTorch ships (NEEDED
``libamdhip64.so``, found through an rpath to torch/lib, then /opt/rocm/lib),
so that a process which has imported torch holds ONE HIP runtime and the
streams and device pointers torch hands over are valid inside the library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libedt.so")
BUILD = os.path.join(HERE, "_build")

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANGXX = os.path.join(ROCM, "llvm", "bin", "clang++")

SOURCES = ["edt_api.hip", "edt_column.hip", "edt_row.hip", "edt_batch.hip", "edt_profile.hip",
           "edt_serve.hip", "edt_row_lanes.hip", "edt_regions.hip",
           "edt_danielsson.hip", "edt_transpose.hip"]

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # no packed-fp32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def torch_lib_dir() -> str | None:
    """Directory of the libamdhip64.so that torch loads (without importing
    torch, which is slow on a cold image)."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        return None
    d = os.path.join(list(spec.submodule_search_locations)[0], "lib")
    return d if os.path.exists(os.path.join(d, "libamdhip64.so")) else None


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        cmd = [HIPCC, "-c", os.path.join(CSRC, src), "-o", obj] + HIP_FLAGS
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tdir = torch_lib_dir()
    link = [CLANGXX, "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if tdir:
        link += ["-L", tdir, "-l:libamdhip64.so", "-Wl,-rpath," + tdir]
    else:
        link += ["-L", os.path.join(ROCM, "lib"), "-l:libamdhip64.so"]
    link += ["-Wl,-rpath," + os.path.join(ROCM, "lib"), "-Wl,--no-undefined",
             "-lstdc++", "-lm"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def clean() -> None:
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
