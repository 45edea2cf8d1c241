"""Compile the oracle's plain C core with gcc (test infrastructure only)."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build() -> str:
    src = os.path.join(_HERE, "core.c")
    out = os.path.join(_HERE, "_core.so")
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, src])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
