"""Compile the FP64 CPU oracle into ``oracle/liboracle.so`` (test infrastructure).

No FMA contraction and no fast-math: every floating-point operation of the
oracle is one IEEE-754 round-to-nearest step in the order the source states.
"""
from __future__ import annotations

import os
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "obk_oracle.c")
OUT = os.path.join(_HERE, "liboracle.so")

CMD = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-Wall", "-Wextra",
       "-shared", "-fPIC", "-o", OUT, SRC, "-lm"]


def build(force: bool = True) -> str:
    if force or not os.path.exists(OUT) or os.path.getmtime(OUT) < os.path.getmtime(SRC):
        tmp = OUT + ".tmp"
        cmd = CMD[:]
        cmd[cmd.index(OUT)] = tmp
        subprocess.run(cmd, check=True)
        os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(force="--lazy" not in sys.argv))
