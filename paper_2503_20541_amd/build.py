"""Builds libmdx.so (gfx950) in-tree with hipcc.

    python -m paper_2503_20541_amd.build

Each HIP source is compiled to an object file in parallel (under ``_build/``
next to this file) and the objects are linked into ``libmdx.so``. The binding
(``mdx.py``) calls :func:`ensure_built` on import, so a fresh checkout builds
the library the first time it is used; a failed build raises, there is no
fallback.
"""
from __future__ import annotations

import concurrent.futures
import fcntl
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmdx.so")
OBJDIR = os.path.join(HERE, "_build")
LOCK = os.path.join(HERE, ".libmdx.lock")
SOURCES = ["runtime.hip", "nl.hip", "nonbonded.hip", "pme.hip", "integrate.hip",
           "ewald_direct.hip", "adjoint.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # packed FP32 instructions stay disabled
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _sources() -> list[str]:
    return [os.path.join(CSRC, s) for s in SOURCES]


def _inputs() -> list[str]:
    """Every file whose change makes the built library stale."""
    out = [os.path.abspath(__file__)]
    for d in (CSRC, INCLUDE):
        for name in sorted(os.listdir(d)):
            if name.endswith((".hip", ".h", ".hpp", ".cpp")):
                out.append(os.path.join(d, name))
    return out


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    built = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > built for p in _inputs())


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)}")
    return obj


def _build_locked(verbose: bool) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = _sources()
    workers = max(1, min(len(srcs), len(os.sched_getaffinity(0)), 16))
    with concurrent.futures.ThreadPoolExecutor(workers) as pool:
        objs = list(pool.map(lambda s: _compile(s, verbose), srcs))
    tmp = f"{LIB}.tmp{os.getpid()}"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libmdx.so")
    os.replace(tmp, LIB)
    return LIB


def build(verbose: bool = False) -> str:
    """Compiles and links libmdx.so unconditionally (serialised by a file lock)."""
    with open(LOCK, "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        try:
            return _build_locked(verbose)
        finally:
            fcntl.flock(lk, fcntl.LOCK_UN)


def ensure_built(verbose: bool = False) -> str:
    """Builds libmdx.so when it is missing or older than any of its sources."""
    if not is_stale():
        return LIB
    with open(LOCK, "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        try:
            if is_stale():          # another process may have built it meanwhile
                print(f"[mdx] building {LIB} with hipcc (gfx950)", file=sys.stderr, flush=True)
                _build_locked(verbose)
        finally:
            fcntl.flock(lk, fcntl.LOCK_UN)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
