"""Build libhqr.so (HIP, gfx950) in-tree with hipcc.

The library is several translation units (the host dispatch and one per
kernel family), compiled in parallel and linked into one shared object.
build() always recompiles everything; build(incremental=True) reuses an
object whose source, headers and flags are unchanged (objects are kept in
_build/ next to the package).
"""
from __future__ import annotations

import concurrent.futures
import glob
import hashlib
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libhqr.so")
OBJDIR = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    "--offload-arch=gfx950",
    # no packed-FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _local_includes(path, seen):
    """Paths of the project headers `path` includes, recursively."""
    import re
    with open(path) as f:
        names = re.findall(r'^#include "([^"]+)"', f.read(), flags=re.M)
    for nm in names:
        for d in (CSRC, INCLUDE):
            p = os.path.join(d, nm)
            if os.path.exists(p) and p not in seen:
                seen.add(p)
                _local_includes(p, seen)
    return seen


def _digest(src):
    h = hashlib.sha256(" ".join(FLAGS).encode())
    for p in [src] + sorted(_local_includes(src, set())):
        h.update(p.encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _filter(out):
    return "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l or "error" in l)


def _compile(src, obj, verbose):
    cmd = [HIPCC] + FLAGS + ["-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (os.path.basename(src), _filter(res.stdout)))
    os.replace(obj + ".tmp", obj)
    return _filter(res.stdout)


def build(verbose: bool = False, incremental: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = []
    objs = []
    for src in sources():
        key = _digest(src)
        obj = os.path.join(OBJDIR, os.path.basename(src)[:-4] + "." + key + ".o")
        objs.append(obj)
        if not (incremental and os.path.exists(obj)):
            jobs.append((src, obj))
    with concurrent.futures.ThreadPoolExecutor(max_workers=max(1, min(len(jobs), os.cpu_count() or 4))) as ex:
        for out in ex.map(lambda j: _compile(j[0], j[1], verbose), jobs):
            if verbose and out.strip():
                print(out)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950"] + objs + ["-o", tmp]
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + "\n")
        raise RuntimeError("linking libhqr.so failed")
    os.replace(tmp, LIB)
    # keep only the objects of this build
    for p in glob.glob(os.path.join(OBJDIR, "*.o")):
        if p not in objs:
            os.remove(p)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))
