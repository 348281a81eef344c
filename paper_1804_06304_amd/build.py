"""Build libsnk.so (HIP, gfx950) in-tree with hipcc.

Each csrc/*.hip file is compiled to an object under _build/ (in parallel), then the objects are
linked into paper_1804_06304_amd/libsnk.so. build() recompiles every source; build(incremental=True)
recompiles only sources older than their object or than a header they may include.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsnk.so")
OBJ_DIR = os.path.join(ROOT, "_build", "snk")

HIPFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-result",
]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def headers():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.h")) + glob.glob(os.path.join(ROOT, "include", "*.h")))


def _compile(src: str, obj: str):
    cmd = [hipcc()] + HIPFLAGS + ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
                                  "-c", src, "-o", obj + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    os.replace(obj + ".tmp", obj)
    return res.stdout + res.stderr


def build(verbose: bool = False, incremental: bool = False, jobs: int = 8) -> str:
    """Compile the HIP sources into paper_1804_06304_amd/libsnk.so (every source unless incremental)."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    newest_header = max((os.path.getmtime(h) for h in headers()), default=0.0)
    todo, objs = [], []
    for src in sources():
        obj = os.path.join(OBJ_DIR, os.path.basename(src) + ".o")
        objs.append(obj)
        stale = (not os.path.exists(obj) or os.path.getmtime(obj) < os.path.getmtime(src)
                 or os.path.getmtime(obj) < newest_header)
        if not incremental or stale:
            todo.append((src, obj))
    # the largest translation units first, so they do not start last
    todo.sort(key=lambda so: -os.path.getsize(so[0]))
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        logs = list(ex.map(lambda so: _compile(*so), todo))
    if verbose:
        for (src, _), out in zip(todo, logs):
            if out:
                print(os.path.basename(src) + ":\n" + out)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build(verbose=True, incremental="--incremental" in sys.argv))
