"""Build libpsst.so (HIP, gfx950) in-tree with hipcc.

Flags: -O3, gfx950 only, no fast-math, FMA contraction only within one source
expression (so every kernel variant rounds the same), packed-FP32 instructions
disabled.  Each source compiles to its own object in parallel (kernels are
launched through host stubs, so no relocatable device code is needed), then
the objects link into the shared library.
"""
import os
import subprocess
import sys
import tempfile
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpsst.so")
SOURCES = ["psst_api.cpp", "streaming.cpp", "rk4_wg.hip", "stage.hip", "adjoint.hip", "network.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
         "-ffp-contract=on", "-fno-fast-math",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
         "-Wno-unused-result", "-Wno-unused-value"]


def _compile(src, obj):
    cmd = [HIPCC] + FLAGS + ["-c", "-o", obj, os.path.join(CSRC, src)]
    return subprocess.run(cmd, capture_output=True, text=True)


def build(verbose: bool = False) -> str:
    srcs = list(SOURCES)
    t = time.time()
    with tempfile.TemporaryDirectory(prefix="psst_build_") as tmpd:
        objs = [os.path.join(tmpd, s + ".o") for s in srcs]
        jobs = min(len(srcs), max(1, min(os.cpu_count() or 1, 8)))
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(_compile, srcs, objs))
        for s, r in zip(srcs, results):
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError(f"hipcc failed compiling {s}")
            if verbose and "warning:" in r.stderr:
                sys.stderr.write(r.stderr)
        tmp = LIB + ".tmp"
        r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs,
                           capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed linking libpsst.so")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t:.1f}s")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
