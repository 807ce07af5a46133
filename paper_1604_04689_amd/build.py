"""Build the HIP library libmeshnbr.so in-tree for gfx950 with hipcc.

Run ``python -m paper_1604_04689_amd.build`` (or call ``build()``).  Each
source is compiled to an object in ``_build/`` (in parallel), then the objects
are linked; the library is written next to this file so that it travels with
the source tree.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libmeshnbr.so")
SOURCES = ["api.hip", "node_path.hip", "elem_path.hip", "elem_rows.hip", "mixed_path.hip", "batch_path.hip",
           "graph.hip", "timing.hip", "noalloc.hip", "chunk_path.hip"]
ARCH = os.environ.get("MESHNBR_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libmeshnbr.so)")


def compile_flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            # no packed FP32 instructions in any kernel: the device pass honours
            # this feature flag (the host pass warns that it does not know it)
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def command(out: str = LIB):
    """One hipcc line compiling and linking every source (for reference)."""
    return [hipcc(), *compile_flags(), "-shared", *[os.path.join(CSRC, s) for s in SOURCES], "-o", out]


def _headers_mtime() -> float:
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    hdrs += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    return max(os.path.getmtime(h) for h in hdrs)


def _compile(src: str, skip_newer_than: float = -1.0) -> tuple:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *compile_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
    if skip_newer_than >= 0 and os.path.exists(obj) and \
            os.path.getmtime(obj) > max(skip_newer_than, os.path.getmtime(os.path.join(CSRC, src))):
        return src, obj, subprocess.CompletedProcess(cmd, 0, "", ""), ["# up to date:", *cmd]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, obj, r, cmd


def build(verbose: bool = False, jobs: int = 0, incremental: bool = False) -> str:
    """Compile every source and link.  incremental=True (a development
    convenience) reuses objects newer than their source and every header."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))
    objs = []
    skip = _headers_mtime() if incremental else -1.0
    with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
        for src, obj, r, cmd in pool.map(lambda x: _compile(x, skip), SOURCES):
            if verbose:
                print(" ".join(cmd), flush=True)
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError(f"hipcc failed on {src}")
            objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libmeshnbr.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
