"""Builds the oracle's shared object with gcc (test infrastructure only)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB points the tests at another build (the mutation tests use it).
LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "sso_oracle.c")]
CFLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared", "-Wall", "-Wextra"]


def build(out: str = LIB_PATH, extra=(), sources=None) -> str:
    """Compile sso_oracle.c (or `sources`) into `out`; `extra` appends flags."""
    tmp = out + ".tmp"
    srcs = list(sources) if sources else SOURCES
    cmd = ["gcc", *CFLAGS, *extra, "-I", HERE, "-o", tmp, *srcs, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
