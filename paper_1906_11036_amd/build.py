"""Compile libdugks.so for gfx950 with hipcc (in-tree, no JIT cache).

Each source is compiled to its own object in parallel, then the objects are
linked into one shared library.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdugks.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = [os.path.join(CSRC, "dugks_kernels.hip"), os.path.join(CSRC, "dugks_host.cpp"),
           os.path.join(CSRC, "dugks3d_kernels.hip"), os.path.join(CSRC, "dugks3d_host.cpp"),
           os.path.join(CSRC, "dugks1d.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # no packed binary32 instructions in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]
NOISE = "is not a recognized feature for this target"


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if NOISE not in l)
    return res.returncode, err


def _stale(src, obj, headers):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in [src] + headers)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (incremental=True: only those whose object is older
    than the source or any header) and link libdugks.so."""
    os.makedirs(OBJ, exist_ok=True)
    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    headers += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    jobs = []
    for src in SOURCES:
        obj = os.path.join(OBJ, os.path.basename(src) + ".o")
        if incremental and not _stale(src, obj, headers):
            jobs.append((src, obj, None))
            continue
        jobs.append((src, obj, [HIPCC] + FLAGS + ["-c", src, "-o", obj]))
    if verbose:
        for _, _, cmd in jobs:
            if cmd:
                print(" ".join(cmd), flush=True)
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(lambda j: _run(j[2]) if j[2] else (0, ""), jobs))
    for (src, _, _), (rc, err) in zip(jobs, results):
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {os.path.basename(src)} ({rc}):\n{err}")
        if verbose and err.strip():
            print(err)
    tmp = LIB + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + [o for _, o, _ in jobs] + ["-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    rc, err = _run(link)
    if rc != 0:
        raise RuntimeError(f"link failed ({rc}):\n{err}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build(verbose=True, incremental="--incremental" in sys.argv))
