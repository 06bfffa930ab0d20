"""Compile the oracle's C estimator into ``oracle/_pw_oracle.so`` with gcc.

Test infrastructure only (see ``oracle/__init__.py``).
"""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pw_oracle.c")
LIB = os.path.join(HERE, "_pw_oracle.so")

CMD = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
       "-fno-fast-math", "-Wall", "-o", LIB, SRC, "-lpthread", "-lm"]


def build() -> str:
    tmp = LIB + ".tmp"
    cmd = CMD[:]
    cmd[cmd.index(LIB)] = tmp
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
