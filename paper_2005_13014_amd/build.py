"""Builds libstencil.so (HIP, gfx950) from csrc/ with hipcc.

Each translation unit is compiled in its own process (the column kernels
unroll their level loops fully and take a while), then everything is linked
into a shared library inside the package directory.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libstencil.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
    "-Wall", "-Wno-unused-result",
    # Packed FP32 instructions stay off (they have produced wrong results on
    # these machines); the host pass warns that it does not know the feature.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # The column kernels unroll their k loop completely so that the Thomas
    # coefficients live in registers; lift the unroller's size limit.
    "-mllvm", "-pragma-unroll-threshold=1000000",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _needs(obj, src):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".hpp")]
    deps.append(os.path.join(ROOT, "include", "stencil.h"))
    return any(os.path.getmtime(d) > t for d in deps)


def _compile(src, obj):
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode == 0:
        os.replace(obj + ".tmp", obj)
    return src, r.returncode, r.stdout


def build(force: bool = True, jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every translation unit (all of them when force, else only the
    out-of-date ones) and link libstencil.so.  Returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    objs, todo = [], []
    for s in sources():
        src, obj = os.path.join(CSRC, s), os.path.join(BUILD, s + ".o")
        objs.append(obj)
        if force or _needs(obj, src):
            todo.append((src, obj))
    t0 = time.time()
    failed = []
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as pool:
        for src, rc, out in pool.map(lambda a: _compile(*a), todo):
            if rc != 0:
                failed.append((src, out))
            elif verbose:
                print("built %s (%.0fs)" % (os.path.basename(src), time.time() - t0), flush=True)
    if failed:
        msg = "\n".join("== %s\n%s" % (s, o[-4000:]) for s, o in failed)
        raise RuntimeError("HIP build failed:\n" + msg)
    if todo or not os.path.exists(LIB):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lhiprtc"]
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + r.stdout[-4000:])
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    force = "--force" in sys.argv
    print(build(force=force, verbose=True))
