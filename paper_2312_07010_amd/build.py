"""Builds libace.so (the HIP library behind include/ace.h) for gfx950.

Each source in csrc/ is compiled to an object in parallel (into _build/,
next to this file), and the objects are linked into one shared library
in-tree.  Device code is FP64 with no implicit FMA contraction (the kernels
write their FMAs explicitly, so every kernel variant rounds the same way) and
without packed FP32 instructions.
"""
import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libace.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", INCLUDE]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def compile_command(src, obj):
    return [HIPCC] + FLAGS + ["-c", src, "-o", obj]


def link_command(objs, out=LIB):
    return [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out] + objs


def _stale(src, obj, deps):
    """True if obj is missing or older than src or any header in deps."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(p) > t for p in [src] + deps)


def build(verbose: bool = False, jobs: int = 0, incremental: bool = False) -> str:
    """Compiles every source (incremental: only sources newer than their
    object or changed headers) and links libace.so."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(OBJ, os.path.basename(s)[:-4] + ".o") for s in srcs]
    headers = glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(INCLUDE, "*.h"))
    pairs = [(s, o) for s, o in zip(srcs, objs) if not incremental or _stale(s, o, headers)]
    cmds = [compile_command(s, o) for s, o in pairs]
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    jobs = jobs or max(1, min(len(cmds), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        results = list(pool.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
    for c, r in zip(cmds, results):
        if r.stderr and verbose:
            print(r.stderr, end="", flush=True)
        if r.returncode != 0:
            raise RuntimeError(f"{' '.join(c)} failed:\n{r.stderr}")
    tmp = LIB + ".tmp"
    link = link_command(objs, tmp)
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build(verbose=True, incremental="--incremental" in sys.argv))
