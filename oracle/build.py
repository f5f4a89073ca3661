"""Compile the C oracle into oracle/liborc_mdlg.so with the host compiler.

Test infrastructure: the library it builds is loaded only by the tests, the
smoke check and the CPU-baseline leg of the bench.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mdlg_oracle.c")
LIB = os.path.join(HERE, "liborc_mdlg.so")


def build(verbose: bool = False) -> str:
    cc = os.environ.get("CC", "gcc")
    tmp = LIB + ".tmp"
    # -ffp-contract=off keeps every multiply and add a separately rounded
    # double-precision operation, so the oracle is exactly the scalar code.
    cmd = [cc, "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
