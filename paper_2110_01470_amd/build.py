"""Builds libsso.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import glob
import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB_PATH = os.path.join(PKG, "libsso.so")
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")

HIPCC_FLAGS = [
    "-std=c++17", "-O3", "-fPIC", "--offload-arch=gfx950",
    # No packed-FP32 instructions in generated code.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(out: str = LIB_PATH, extra=(), jobs: int | None = None) -> str:
    """Compiles every source to an object (in parallel), then links."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    jobs = jobs or max(1, min(8, os.cpu_count() or 1))
    with tempfile.TemporaryDirectory(prefix="sso_build_") as work:
        def compile_one(src):
            obj = os.path.join(work, os.path.basename(src) + ".o")
            subprocess.run([hipcc, *HIPCC_FLAGS, *extra, "-I", INCLUDE, "-I", CSRC, "-c", src,
                            "-o", obj], check=True)
            return obj

        with ThreadPoolExecutor(jobs) as pool:
            objs = list(pool.map(compile_one, sources()))
        subprocess.run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp],
                       check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
