"""Build libgpw.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgpw.so")
SOURCES = ["gpw_api.hip", "gpw_partition.hip", "gpw_eval.hip", "gpw_poisson.hip"]
# the class kernels: gpw_class.hip once per (l_a, l_b) class
NCLASS = 15
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _newer(obj: str, src: str) -> bool:
    """obj exists and is newer than src and every header of the sources."""
    if not os.path.exists(obj):
        return False
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    deps.append(os.path.join(os.path.dirname(HERE), "include", "gpw.h"))
    t = os.path.getmtime(obj)
    return all(os.path.getmtime(d) < t for d in deps)


def _compile(job, objdir: str, incremental: bool = False) -> str:
    src, defs = job if isinstance(job, tuple) else (job, [])
    tag = "".join("_" + d.split("=")[1] for d in defs)
    obj = os.path.join(objdir, os.path.splitext(src)[0] + tag + ".o")
    if incremental and _newer(obj, os.path.join(CSRC, src)):
        return obj
    cmd = [HIPCC, *FLAGS, *("-D" + d for d in defs), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every HIP source for gfx950 and link libgpw.so next to this file
    (with ``incremental``, objects newer than their sources and headers are kept)."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    # the class objects first: they take longest
    jobs = [("gpw_class.hip", [f"GPW_CLS={c}"]) for c in range(NCLASS)] + list(SOURCES)
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(lambda j: _compile(j, objdir, incremental), jobs))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-lhipfft"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
