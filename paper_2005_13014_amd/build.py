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


_RESOURCE_KEYS = ("VGPRs", "AGPRs", "TotalSGPRs", "ScratchSize [bytes/lane]", "VGPRs Spill", "SGPRs Spill",
                  "LDS Size [bytes/block]", "Occupancy [waves/SIMD]")


def _demangle(names):
    for tool in ("/opt/rocm/llvm/bin/llvm-cxxfilt", "c++filt"):
        try:
            r = subprocess.run([tool], input="\n".join(names), capture_output=True, text=True)
        except OSError:
            continue
        if r.returncode == 0:
            return r.stdout.split("\n")[:len(names)]
    return list(names)


def resources(jobs: int | None = None) -> list:
    """Per-kernel register, LDS and occupancy figures from the compiler's
    resource-usage remarks (device-only compiles of every source with the
    library's flags): one dict per kernel with the source file, the
    demangled name and the keys of _RESOURCE_KEYS."""
    import re
    import tempfile
    jobs = jobs or min(16, os.cpu_count() or 4)
    srcs = [s for s in sources() if s.endswith(".hip")]

    def one(src):
        with tempfile.TemporaryDirectory() as d:
            cmd = [HIPCC] + FLAGS + ["--offload-device-only", "-Rpass-analysis=kernel-resource-usage", "-c",
                                     os.path.join(CSRC, src), "-o", os.path.join(d, "k.o")]
            r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if r.returncode != 0:
            raise RuntimeError("resource compile of %s failed:\n%s" % (src, r.stdout[-4000:]))
        rows, cur = [], None
        for line in r.stdout.split("\n"):
            m = re.search(r"remark: .*Function Name: (\S+)", line)
            if m:
                cur = {"source": src, "mangled": m.group(1)}
                rows.append(cur)
                continue
            m = re.search(r"remark: .*?\s([A-Za-z][A-Za-z ]*(?:\[[^]]*\])?): (\d+)", line)
            if m and cur is not None and m.group(1) in _RESOURCE_KEYS:
                cur[m.group(1)] = int(m.group(2))
        return rows

    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as pool:
        rows = [r for part in pool.map(one, srcs) for r in part]
    for r, n in zip(rows, _demangle([r["mangled"] for r in rows])):
        r["kernel"] = n
    return rows


# Kernels that the benchmark's default workloads launch (the library's
# default variants), marked in the report.
MEASURED = {
    "k_column_pipe<float, 4, 4, 40, 2, true, true, false, 64>": "fused FP32 512x512x80 (headline), 256x256x80",
    "k_column_pipe<double, 4, 2, 40, 1, true, true, false, 64>": "fused FP64 512x512x80, 256x256x80",
    "k_column_batch_pipe<float, 1, 2, 4, 45, 2>": "timestep 6x8, KH 45",
    "k_column_batch_pipe<float, 1, 2, 4, 40, 2>": "timestep 6x8, KH 40",
    "k_column_batch_pipe<float, 1, 2, 4, 32, 2>": "timestep 6x8, KH 32",
    "k_hgrad_strip<float, 8, 4>": "timestep 6x8, hgrad",
    "k_vadv_adjoint<float, 2, 2, 40, false, true, 16>": "reverse FP32 256x256x80",
    "k_hdiff_adjoint_dpp<float, 12, 1>": "reverse FP32 256x256x80",
    "k_vadv_adjoint<double, 2, 4, 40, false, false, 4>": "reverse FP64 256x256x80",
    "k_hdiff_adjoint_dpp<double, 4, 1>": "reverse FP64 256x256x80",
    "k_jvp<float, 4, 2, 40, 1, true>": "forward FP32 256x256x80",
    "k_jvp<double, 2, 2, 40, 1, true>": "forward FP64 256x256x80",
}


def resources_markdown(rows) -> str:
    cmd = "python -m paper_2005_13014_amd.build --resources profiles/kernel_resources.md"
    out = ["# Kernel resources (gfx950)", "",
           "Registers, spills, LDS and occupancy of every kernel the library compiles, from the compiler's",
           "resource-usage remarks (`-Rpass-analysis=kernel-resource-usage`, device-only compiles with the",
           "library's own flags).  Made by, from the repository root:", "", "```", cmd, "```", "",
           "Occupancy is the compiler's waves per SIMD (a SIMD holds up to 8; 512 VGPRs per lane and SIMD",
           "give 2 waves at 256 VGPRs, 3 at 168, 4 at 128, 5 at 96).  Scratch and VGPR spills are per lane.", "",
           "| source | kernel | measured workload | VGPRs | AGPRs | SGPRs | VGPR spill | SGPR spill | scratch B "
           "| LDS B | waves/SIMD |",
           "|---|---|---|---|---|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: (r["source"], r["kernel"])):
        name = r["kernel"].split("(")[0].replace("stl::", "").replace("void ", "")
        out.append("| %s | `%s` | %s | %s | %s | %s | %s | %s | %s | %s | %s |" % (
            r["source"], name, MEASURED.get(name, ""), r.get("VGPRs", "-"), r.get("AGPRs", "-"),
            r.get("TotalSGPRs", "-"),
            r.get("VGPRs Spill", "-"), r.get("SGPRs Spill", "-"), r.get("ScratchSize [bytes/lane]", "-"),
            r.get("LDS Size [bytes/block]", "-"), r.get("Occupancy [waves/SIMD]", "-")))
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    if "--resources" in sys.argv:
        path = sys.argv[sys.argv.index("--resources") + 1]
        with open(path, "w") as fh:
            fh.write(resources_markdown(resources()))
        print(path)
    else:
        force = "--force" in sys.argv
        print(build(force=force, verbose=True))
