"""Build the in-tree HIP library librlbm.so for gfx950 (hipcc, no torch extension).

Every source under csrc/ is compiled to an object of its own, in parallel,
then linked into one shared library."""
from __future__ import annotations

import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librlbm.so")
OBJDIR = os.path.join(os.path.dirname(HERE), "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # packed FP32 instructions stay off (the compiler must not form them)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _compile(hipcc: str, src: str, obj: str, extra, verbose: bool):
    cmd = [hipcc, *HIPCC_FLAGS, *extra, "-I", os.path.join(os.path.dirname(HERE), "include"), "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.run(cmd, capture_output=True, text=True)


def build(verbose: bool = False, jobs: int = 0, extra_flags=(), lib: str = LIB) -> str:
    """Compile every HIP/C++ source under csrc/ (always recompiles) and link
    librlbm.so.  extra_flags go to every compile line."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sources()
    tag = "%d" % os.getpid()
    objs = [os.path.join(OBJDIR, os.path.basename(s) + "." + tag + ".o") for s in srcs]
    jobs = jobs or min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    try:
        with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(lambda so: _compile(hipcc, so[0], so[1], list(extra_flags), verbose),
                                  zip(srcs, objs)))
        failed = [(s, r) for s, r in zip(srcs, results) if r.returncode != 0]
        for s, r in failed:
            sys.stderr.write(f"--- {os.path.basename(s)}\n{r.stdout}{r.stderr}")
        if failed:
            raise RuntimeError("hipcc failed building librlbm.so")
        tmp = lib + ".tmp" + tag
        link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(link), flush=True)
        res = subprocess.run(link, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("linking librlbm.so failed")
        os.replace(tmp, lib)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
