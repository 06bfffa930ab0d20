"""Compile the native graph generator (``clgen.cpp``) into ``synth/_clgen.so``.

    python -m synth.build
"""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "clgen.cpp")
LIB = os.path.join(HERE, "_clgen.so")


def build() -> str:
    tmp = LIB + ".tmp"
    subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-Wall", "-o", tmp, SRC],
                   check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
