"""Compile the C oracle into ``oracle/liboracle.so`` (gcc, FP64, OpenMP).

Test infrastructure only: the HIP library never links or loads the result.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = True, sanitize: bool = False) -> str:
    """Build liboracle.so; with ``force=False`` reuse an up-to-date build."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    out = LIB if not sanitize else os.path.join(HERE, "liboracle_san.so")
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-D_GNU_SOURCE",
           "-Wall", "-Wno-unused-function", SRC, "-o", out + ".tmp", "-lm"]
    if sanitize:
        cmd[3:3] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(force=True, sanitize="--sanitize" in sys.argv))
