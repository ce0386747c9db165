"""Build the gfx950 HIP library ``libinpc_raster.so`` in place with hipcc."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libinpc_raster.so")
SOURCES = ["k_project.hip", "k_sort.hip", "k_blend_fwd.hip", "k_blend_bwd.hip", "k_reduce.hip",
           "k_appearance.hip", "k_sampling.hip", "k_tile.hip", "api.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC", "-Wall",
    # no packed-FP32 instruction generation: every float operation stays scalar
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-rdc",
]


def build(verbose: bool = False, jobs: int = 6, objdir: str = None, lib_path: str = None,
          extra_flags=(), link_flags=()) -> str:
    """Compiles every source and links the library (``lib_path``, default
    the in-tree libinpc_raster.so); ``extra_flags`` / ``link_flags`` are added
    to the compile / link lines (the sanitizer test builds a variant)."""
    objdir = objdir or os.path.join(HERE, "_build")
    lib_path = lib_path or LIB
    extra = list(extra_flags)
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = [HIPCC] + FLAGS + extra + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        if len(procs) >= jobs:
            if procs.pop(0).wait() != 0:
                raise RuntimeError("hipcc failed")
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + list(link_flags) + ["-o", lib_path + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib_path + ".tmp", lib_path)
    return lib_path


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
