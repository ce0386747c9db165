"""Build the CPU oracle (``oracle/liborc.so``) with gcc.

TEST INFRASTRUCTURE ONLY.  -ffp-contract=off keeps the float32 projection
free of fused multiply-adds, so every float32 operation rounds exactly as
written in oracle.c.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liborc.so")


def build(verbose: bool = False, lib_path: str = None, opt_flags=("-O2",)) -> str:
    """Builds ``lib_path`` (default the in-tree liborc.so); ``opt_flags``
    replace -O2 (the sanitizer test builds a variant)."""
    out = lib_path or LIB
    cmd = ["gcc"] + list(opt_flags) + ["-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                                       "-fPIC", "-shared", "-Wall", "-Wextra", "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
