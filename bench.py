"""Benchmark of the fused hdiff + vadv stencil program on one MI355X.

One step = one call of the fused program (Laplacian -> limited fluxes ->
update -> flux-form right-hand side -> Thomas elimination and
back-substitution) over a 512 x 512 x 80 grid with FP32 storage and stencil
arithmetic and the FP64 Thomas solve, inputs resident in HBM.  Several input
sets are rotated so that no step finds its inputs in the 256 MB Infinity
Cache left by the previous one.

Prints ONE JSON line on stdout; progress goes to stderr.  Beside the headline
it reports the FP64 and bf16 variants, the unfused "original" FP64 path, the
hdiff optimisation levels, the batched timestep, the adjoint, the copy-probe
ceiling and the CPU oracle on the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fused hdiff+vadv Gpoints/s & % peak HBM GB/s, FP32 vs FP64 at stated error"
PEAK_HBM_GBS = 8000.0
DT = 10.0
SEED = 200513014
ES = {"f32": 4, "f64": 8, "bf16": 2}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_column_f32_512x512x80.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2005_13014_amd", "csrc", n)
                  for n in ("column.hpp", "common.hpp", "column_f32.hip")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def u_cells(ni, nj, nk):
    """Cells of u a fused call must read: the interior plus the part of its
    2-cell ring that the 13-point diamond reaches."""
    return (ni * nj + 4 * (ni + nj) + 4) * nk


def fused_bytes(ni, nj, nk, es):
    """Algorithmic bytes of one fused call: u, five more inputs and the output."""
    return es * (u_cells(ni, nj, nk) + 6 * ni * nj * nk)


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the headline kernel from the committed counter
    summary, or None if it is missing or was taken for other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sources_sha256_16") != kernel_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def make_set(ni, nj, nk, dtype, seed):
    from paper_2005_13014_amd import binding as B
    from paper_2005_13014_amd import inputs
    f = inputs.fields(ni, nj, nk, 2, seed=seed, storage=dtype)
    g = {n: B.Field.from_numpy(f[n], 2, dtype) for n in ("u", "coeff", "wcon", "a", "b", "c")}
    g["x"] = B.Field.empty(ni, nj, nk, 2, dtype, fill=0.0)
    return f, g


def n_sets_for(nbytes):
    return max(2, min(8, math.ceil(3 * 256e6 / nbytes) + 1))


def time_calls(fn, sets, steps, warmup):
    """Runs fn(set) over rotating sets.  Returns (wall ms per step, mean ms of
    one call from HIP events on the current stream)."""
    import torch
    stream = torch.cuda.current_stream()
    for s in range(warmup):
        fn(sets[s % len(sets)])
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for s in range(steps):
        ev[s][0].record(stream)
        fn(sets[s % len(sets)])
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return wall, float(np.mean([a.elapsed_time(b) for a, b in ev]))


def fused(cfg=None):
    from paper_2005_13014_amd import binding as B

    def fn(g):
        B.stencil_hdiff_vadv(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, g["x"],
                             cfg=cfg)
    return fn


def gpu_output(f, x):
    """One GPU result kept on the host for the CPU leg to check: the inputs it
    was computed from and its interior."""
    return {"f": f, "x": x.to_numpy(interior=True)}


def copy_probe():
    import torch
    from paper_2005_13014_amd import binding as B
    nb = 1 << 30
    src = torch.empty(nb // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        B.stencil_probe_copy(src, dst, nb)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        B.stencil_probe_copy(src, dst, nb)
    e1.record()
    torch.cuda.synchronize()
    return 2 * nb / (e0.elapsed_time(e1) / 10 * 1e-3) / 1e9


def read_probe():
    """Achievable HBM read rate (GB/s): the read-only probe over 1 GiB."""
    import torch
    from paper_2005_13014_amd import binding as B
    nb = 1 << 30
    src = torch.empty(nb // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    sink = torch.zeros(4, dtype=torch.int32, device="cuda")
    # key 1: all-equal vectors give checksum 0, so the sink is never written
    for _ in range(3):
        B.stencil_probe_read(src, nb, 1, sink)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        B.stencil_probe_read(src, nb, 1, sink)
    e1.record()
    torch.cuda.synchronize()
    return nb / (e0.elapsed_time(e1) / 10 * 1e-3) / 1e9


def streams_probe(ni=512, nj=512, nk=80):
    """HBM rate (GB/s) of the fused kernel's traffic mix at the headline size:
    six field-sized arrays read and one written, streamed element by element."""
    import torch
    from paper_2005_13014_amd import binding as B
    n = ni * nj * nk
    srcs = [torch.empty(n, dtype=torch.float32, device="cuda").fill_(float(q)) for q in range(6)]
    dst = torch.empty(n, dtype=torch.float32, device="cuda")
    for _ in range(3):
        B.stencil_probe_streams(srcs, dst, 4 * n)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        B.stencil_probe_streams(srcs, dst, 4 * n)
    e1.record()
    torch.cuda.synchronize()
    return 7 * 4 * n / (e0.elapsed_time(e1) / 20 * 1e-3) / 1e9


def variant_column(ni, nj, nk, dtype, level):
    """Fused (level 0) or unfused 'original' (level 1) program in dtype."""
    import torch
    from paper_2005_13014_amd import binding as B
    es = ES[dtype]
    sets = [make_set(ni, nj, nk, dtype, SEED + 3 + 1000 * q)
            for q in range(n_sets_for(fused_bytes(ni, nj, nk, es)))]
    cfg = B.config(level=level)
    w, k = time_calls(fused(cfg), [s[1] for s in sets], 20, 3)
    fused(cfg)(sets[0][1])
    torch.cuda.synchronize()
    ab = fused_bytes(ni, nj, nk, es)
    out = {"Gpoints_s": ni * nj * nk / (w * 1e-3) / 1e9, "ms": w,
           "algorithmic_GBs": ab / (k * 1e-3) / 1e9,
           "frac_hbm_peak": ab / (k * 1e-3) / 1e9 / PEAK_HBM_GBS}
    return out, gpu_output(sets[0][0], sets[0][1]["x"])


def variant_hdiff_levels(ni, nj, nk):
    """hdiff alone in FP32 at the paper's optimisation levels (Sec. VII-C)."""
    from paper_2005_13014_amd import binding as B
    from paper_2005_13014_amd import inputs
    nb = 4 * (u_cells(ni, nj, nk) + 2 * ni * nj * nk)
    sets = []
    for q in range(n_sets_for(nb)):
        f = inputs.fields(ni, nj, nk, 2, seed=SEED + 1 + q, storage="f32", vadv=False)
        sets.append({"u": B.Field.from_numpy(f["u"], 2, "f32"),
                     "coeff": B.Field.from_numpy(f["coeff"], 2, "f32"),
                     "x": B.Field.empty(ni, nj, nk, 2, "f32", fill=0.0)})
    out = {}
    for label, cfg in (("original", B.config(level=1)), ("inline", B.config(unroll=1)),
                       ("inline_unroll2", B.config(unroll=2)), ("inline_unroll4", B.config(unroll=4))):
        def fn(g, cfg=cfg):
            B.stencil_hdiff(g["u"], g["coeff"], g["x"], cfg=cfg)
        w, k = time_calls(fn, sets, 20, 3)
        out[label] = {"ms": w, "algorithmic_GBs": nb / (k * 1e-3) / 1e9}
    return out


def variant_program(implicit=False):
    """The batched timestep: hdiff -> vadv -> vdiff -> hgrad on 8 fields over
    6 uneven subdomains, FP32, hipGraph + autotuned variant; implicit takes
    the implicit vertical diffusion (a second tridiagonal solve per column)."""
    import torch
    from paper_2005_13014_amd import binding as B
    from paper_2005_13014_amd import inputs
    data = inputs.batched(storage="f32")
    subs = []
    pts = 0
    nbytes = 0
    for d in data:
        ni, nj, nk = d["shape"]
        h = d["halo"]
        s = {n: B.Field.from_numpy(d[n], h, "f32") for n in ("coeff", "wcon", "a", "b", "c")}
        s["u"] = [B.Field.from_numpy(u, h, "f32") for u in d["u"]]
        s["z"] = [B.Field.empty(ni, nj, nk, h, "f32", fill=0.0) for _ in d["u"]]
        subs.append(s)
        nf = len(d["u"])
        pts += ni * nj * nk * nf
        # per field: u (3-ring diamond of the grown domain ~ interior) + z; shared coefficients once
        nbytes += 4 * (nf * 2 * ni * nj * nk + 5 * ni * nj * nk)
    stages = B.STAGE_HDIFF | B.STAGE_VADV | B.STAGE_HGRAD | (
        B.STAGE_VDIFF_IMPLICIT if implicit else B.STAGE_VDIFF)
    spec = B.ProgramSpec(subs, stages=stages, dt=DT, flags=B.PROGRAM_GRAPH | B.PROGRAM_AUTOTUNE)
    w, k = time_calls(lambda _: B.stencil_program_run(spec), [None], 20, 3)
    del subs
    torch.cuda.empty_cache()
    return {"ms": w, "Gfieldpoints_s": pts / (w * 1e-3) / 1e9,
            "algorithmic_GBs_lower_bound": nbytes / (k * 1e-3) / 1e9, "field_points": pts}


def variant_adjoint(n=256, nk=80):
    from paper_2005_13014_amd import binding as B
    from paper_2005_13014_amd import inputs
    out = {}
    for dtype in ("f32", "f64"):
        f = inputs.fields(n, n, nk, 2, seed=SEED + 5, storage=dtype, loss=True)
        g = {k: B.Field.from_numpy(f[k], 2, dtype) for k in ("u", "coeff", "wcon", "a", "b", "c", "w")}
        gs = [g["u"].like(fill=0.0) for _ in range(3)]

        def fn(_):
            B.stencil_hdiff_vadv_adjoint(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT,
                                         g["w"], *gs)
        w, k = time_calls(fn, [None], 20, 3)
        # u with its ring, coeff, wcon, a, b, c, w in; gu (interior and ring),
        # gcoeff, gwcon out
        ab = ES[dtype] * (2 * u_cells(n, n, nk) + 8 * n * n * nk)
        out[dtype] = {"ms": w, "Gpoints_s": n * n * nk / (w * 1e-3) / 1e9,
                      "algorithmic_GBs": ab / (k * 1e-3) / 1e9}
    return out


def variant_frontend(ni=512, nj=512, nk=80):
    """hdiff written as a stencil program, inlined, unrolled and compiled at
    run time by the front end (FP32), beside the hand-written hdiff kernel."""
    from paper_2005_13014_amd import binding as B
    from paper_2005_13014_amd import frontend as F
    from paper_2005_13014_amd import inputs
    nb = 4 * (u_cells(ni, nj, nk) + 2 * ni * nj * nk)
    sets = []
    for q in range(n_sets_for(nb)):
        f = inputs.fields(ni, nj, nk, 2, seed=SEED + 1 + q, storage="f32", vadv=False)
        sets.append({"u": B.Field.from_numpy(f["u"], 2, "f32"),
                     "coeff": B.Field.from_numpy(f["coeff"], 2, "f32"),
                     "x": B.Field.empty(ni, nj, nk, 2, "f32", fill=0.0)})
    out = {}
    for tiled in (False, True):
        for unroll in (1, 2, 4):
            k = F.compile_program(F.hdiff_program(), "f32", like=sets[0]["u"], unroll=unroll, tiled=tiled)

            def fn(g, k=k):
                k({"u": g["u"], "coeff": g["coeff"]}, {"out": g["x"]})
            w, kt = time_calls(fn, sets, 20, 3)
            k.close()
            out["generated%s_unroll%d" % ("_tiled" if tiled else "", unroll)] = {
                "ms": w, "algorithmic_GBs": nb / (kt * 1e-3) / 1e9}

    def hand(g):
        B.stencil_hdiff(g["u"], g["coeff"], g["x"])
    w, kt = time_calls(hand, sets, 20, 3)
    out["hand_written_inline"] = {"ms": w, "algorithmic_GBs": nb / (kt * 1e-3) / 1e9}
    return out


def variant_jvp(n=256, nk=80):
    """Forward mode (tangent in all six inputs) at the reverse mode's size."""
    import numpy as np
    from paper_2005_13014_amd import binding as B
    from paper_2005_13014_amd import inputs
    out = {}
    names = ("u", "coeff", "wcon", "a", "b", "c")
    for dtype in ("f32", "f64"):
        f = inputs.fields(n, n, nk, 2, seed=SEED + 6, storage=dtype)
        rng = np.random.default_rng(SEED + 7)
        g = {k: B.Field.from_numpy(f[k], 2, dtype) for k in names}
        t = {k: B.Field.from_numpy(inputs.round_to(rng.standard_normal(f[k].shape), dtype), 2, dtype)
             for k in names}
        x = g["u"].like(fill=0.0)
        B.stencil_hdiff_vadv(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, x)
        dx = g["u"].like(fill=0.0)

        def fn(_):
            B.stencil_hdiff_vadv_jvp(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, dx, x=x,
                                     du=t["u"], dcoeff=t["coeff"], dwcon=t["wcon"], da=t["a"], db=t["b"],
                                     dc=t["c"])
        w, k = time_calls(fn, [None], 20, 3)
        es = ES[dtype]
        # 13 streams in (u, du with their ring; 11 column fields incl. x), 1 out
        ab = es * (2 * u_cells(n, n, nk) + 12 * n * n * nk)
        out[dtype] = {"ms": w, "Gpoints_s": n * n * nk / (w * 1e-3) / 1e9,
                      "algorithmic_GBs": ab / (k * 1e-3) / 1e9}
    return out


def relative_errors(got, ref):
    return {"normwise": float(np.abs(got - ref).max() / np.abs(ref).max()),
            "rms": float(np.sqrt(np.mean((got - ref) ** 2)) / np.sqrt(np.mean(ref ** 2)))}


def cpu_baseline(ni, nj, nk, checks, budget_s=10.0):
    """The host leg: times the FP64 oracle on the workload, then uses it to
    check the GPU outputs in checks (label -> gpu_output); returns the
    baseline record and the errors per label."""
    import oracle
    from paper_2005_13014_amd import inputs

    def run(f):
        return oracle.hdiff_vadv(f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2, f["b"], 2, f["c"],
                                 2, DT)
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 3, storage="f32")
    reps, t0 = 0, time.perf_counter()
    while True:
        run(f)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 20:
            break
    base = {"value": reps * ni * nj * nk / el / 1e9, "unit": "Gpoints/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d full calls of the FP64 oracle on the %dx%dx%d workload (%.1f s, one thread)"
                      % (reps, ni, nj, nk, el)}
    errs = {}
    for label, c in checks.items():
        errs[label] = relative_errors(c["x"], run(c["f"]))
    return base, errs


# Profiling commands (run from the repository root $R on the MI355X machine,
# writing under the directory $OUT) whose
# output --summarize-profiles turns into the committed summaries.
TRACE_CMD = ("cd /tmp && TMPDIR=/tmp rocprofv3 --kernel-trace --stats --output-format csv "
             "-d $OUT/prof_trace -o trace -- python $R/bench.py --quick --with-copy "
             "--steps 20 --warmup 2")
PMC_CMD = ("cd /tmp && TMPDIR=/tmp timeout -s KILL 120 rocprofv3 --pmc {c} --output-format csv "
           "-d $OUT/prof_{t} -o {t} -- python $R/bench.py --quick --with-copy "
           "--steps 4 --warmup 1")
COPY_PROBE_BYTES = 1 << 30


def summarize_profiles(outdir):
    """Writes profiles/k_column_f32_512x512x80_trace.md from the kernel trace
    under outdir/prof_trace and, if the FETCH_SIZE / WRITE_SIZE runs are
    there, the calibrated traffic summary (JSON + Markdown)."""
    import csv
    import glob

    def one(pattern):
        hits = sorted(glob.glob(os.path.join(outdir, pattern), recursive=True))
        return hits[0] if hits else None

    def short(name):
        return name.split("(")[0][:100]

    rows = list(csv.DictReader(open(one("prof_trace/**/*kernel_stats.csv"))))
    cols = [r for r in rows if "k_column" in r["Name"]]
    col = max(cols, key=lambda r: float(r["TotalDurationNs"]))
    kname = short(col["Name"])
    avg_us = float(col["AverageNs"]) / 1e3
    ab = fused_bytes(512, 512, 80, 4)
    out = ["# Kernel trace: fused hdiff+vadv, FP32 512x512x80 (%s)" % kname.split("<")[0].split()[-1],
           "", "Command (from the repository root `$R` on the MI355X machine, output under `$OUT`):", "", "```", TRACE_CMD, "```", "",
           "| kernel | calls | average (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    for r in rows:
        out.append("| `%s` | %s | %.2f | %.2f | %.2f | %.1f%% |" % (
            short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    out += ["", "Headline kernel `%s`: algorithmic bytes per launch %d; at the traced average "
            "duration %.2f us that is %.1f GB/s (%.1f%% of 8 TB/s).  Kernel sources hash %s." % (
                kname, ab, avg_us, ab / (avg_us * 1e-6) / 1e9, 100 * ab / (avg_us * 1e-6) / 8e12,
                kernel_hash())]
    with open(os.path.join(ROOT, "profiles", "k_column_f32_512x512x80_trace.md"), "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("\n".join(out))

    def counter(tag, cname):
        f = one("prof_%s/**/*counter_collection.csv" % tag)
        per = {}
        for r in csv.DictReader(open(f)) if f else []:
            if r.get("Counter_Name") == cname:
                per.setdefault(short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
        return {k: (sum(v) / len(v), len(v)) for k, v in per.items()}

    fetch, write = counter("fetch", "FETCH_SIZE"), counter("write", "WRITE_SIZE")
    probe = [k for k in fetch if "k_copy16" in k]
    if kname not in fetch or kname not in write or not probe:
        print("no matching counter runs; traffic summary not written")
        return
    (cf, ncf), (cw, ncw) = fetch[kname], write[kname]
    pf, pw = fetch[probe[0]][0], write[probe[0]][0]
    f_fac, w_fac = pf * 1024 / COPY_PROBE_BYTES, pw * 1024 / COPY_PROBE_BYTES
    fetch_b, write_b = cf * 1024 / f_fac, cw * 1024 / w_fac
    tot = fetch_b + write_b
    t = {"kernel": kname, "workload": "fused hdiff+vadv f32 512x512x80 halo 2",
         "kernel_sources_sha256_16": kernel_hash(),
         "fetch_kib_per_dispatch": cf, "write_kib_per_dispatch": cw, "dispatches": [ncf, ncw],
         "copy_probe_fetch_kib": pf, "copy_probe_write_kib": pw,
         "copy_probe_bytes_each_way": COPY_PROBE_BYTES,
         "fetch_calibration": f_fac, "write_calibration": w_fac,
         "hbm_fetch_bytes_per_launch": fetch_b, "hbm_write_bytes_per_launch": write_b,
         "hbm_bytes_per_launch": tot, "algorithmic_bytes_per_launch": ab,
         "traffic_over_algorithmic": tot / ab,
         "commands": [PMC_CMD.format(c="FETCH_SIZE", t="fetch"), PMC_CMD.format(c="WRITE_SIZE", t="write")]}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(t, fh, indent=1)
    md = ["# HBM traffic of the fused kernel (FP32, 512x512x80, halo 2)", "",
          "Two counter runs (one counter each), from the repository root `$R` on the MI355X machine, output under `$OUT`:", "",
          "```"] + t["commands"] + ["```", "",
          "`--with-copy` also runs the 1 GiB copy probe (`k_copy16`), which calibrates the counters:", "",
          "| kernel | FETCH_SIZE (KiB/dispatch) | WRITE_SIZE (KiB/dispatch) |", "|---|---|---|",
          "| `k_copy16` (1 GiB read, 1 GiB written) | %.0f | %.0f |" % (pf, pw),
          "| `%s` | %.0f | %.0f |" % (kname, cf, cw), "",
          "Calibration: FETCH_SIZE reads %.3f of the bytes the copy truly reads, WRITE_SIZE %.3f of the "
          "bytes it writes.  Scaled, one fused launch moves %.1f MB in and %.1f MB out = %.1f MB against "
          "%.1f MB algorithmic (u with the ring its stencil reaches, five more inputs, the output): "
          "**%.3fx**.  Kernel sources hash %s (`bench.py` reports `traffic` only while the sources "
          "match)." % (f_fac, w_fac, fetch_b / 1e6, write_b / 1e6, tot / 1e6, ab / 1e6, tot / ab,
                       kernel_hash())]
    with open(TRAFFIC_FILE[:-5] + ".md", "w") as fh:
        fh.write("\n".join(md) + "\n")
    print("\n".join(md))


VARIANT_TRACE_CMD = ("cd /tmp && TMPDIR=/tmp rocprofv3 --kernel-trace --stats --output-format csv "
                     "-d $OUT/v_{v}_trace -o t -- python $R/bench.py --only {v}")
VARIANT_PMC_CMD = ("cd /tmp && TMPDIR=/tmp timeout -s KILL 120 rocprofv3 --pmc {c} --output-format csv "
                   "-d $OUT/v_{v}_{t} -o t -- python $R/bench.py --only {v}")


def summarize_variant(outdir, name, fetch_calibration):
    """Writes profiles/variant_<name>.md: per-kernel times of bench.py --only
    <name> from its kernel trace, with the FETCH_SIZE / WRITE_SIZE counts of the
    matching counter runs when present (FETCH scaled by the copy-probe
    calibration of the headline traffic summary)."""
    import csv
    import glob

    def one(pattern):
        hits = sorted(glob.glob(os.path.join(outdir, pattern), recursive=True))
        return hits[0] if hits else None

    def per_kernel(tag, cname):
        f = one("v_%s_%s/**/*counter_collection.csv" % (name, tag))
        out = {}
        for r in csv.DictReader(open(f)) if f else []:
            if r.get("Counter_Name") == cname:
                out.setdefault(r["Kernel_Name"].split("(")[0], []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in out.items()}

    rows = list(csv.DictReader(open(one("v_%s_trace/**/*kernel_stats.csv" % name))))
    fe, wr = per_kernel("fetch", "FETCH_SIZE"), per_kernel("write", "WRITE_SIZE")
    md = ["# Kernel trace: `bench.py --only %s`" % name, "",
          "Commands (from the repository root `$R` on the MI355X machine, output under `$OUT`):", "", "```",
          VARIANT_TRACE_CMD.format(v=name)]
    if fe:
        md += [VARIANT_PMC_CMD.format(c="FETCH_SIZE", v=name, t="fetch"),
               VARIANT_PMC_CMD.format(c="WRITE_SIZE", v=name, t="write")]
    md += ["```", "", "| kernel | calls | average (us) | HBM read (MB) | HBM write (MB) | GB/s |",
           "|---|---|---|---|---|---|"]
    for r in rows:
        n = r["Name"].split("(")[0]
        if "stl::" not in n:
            continue
        us = float(r["AverageNs"]) / 1e3
        rb = fe[n] * 1024 / fetch_calibration if n in fe else None
        wb = wr[n] * 1024 if n in wr else None
        gbs = (rb + wb) / (us * 1e-6) / 1e9 if rb is not None and wb is not None else None
        md.append("| `%s` | %s | %.1f | %s | %s | %s |" % (
            n, r["Calls"], us, "%.1f" % (rb / 1e6) if rb is not None else "-",
            "%.1f" % (wb / 1e6) if wb is not None else "-", "%.0f" % gbs if gbs else "-"))
    md += ["", "HBM read = FETCH_SIZE / %.3f (the copy-probe calibration), write = WRITE_SIZE; both per "
           "dispatch.  Library sources hash %s." % (fetch_calibration, library_hash())]
    path = os.path.join(ROOT, "profiles", "variant_%s.md" % name)
    with open(path, "w") as fh:
        fh.write("\n".join(md) + "\n")
    print("\n".join(md))


def library_hash():
    import glob
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2005_13014_amd", "csrc", "*"))):
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, nargs=3, default=[512, 512, 80])
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64", "bf16"])
    ap.add_argument("--tile-j", type=int, default=0)
    ap.add_argument("--prefetch", type=int, default=0)
    ap.add_argument("--nontemporal", type=int, default=0, help="1 on, -1 off, 0 library choice")
    ap.add_argument("--schedule", type=int, default=0, help="1 staged, 2 pipelined, 0 library choice")
    ap.add_argument("--quick", action="store_true",
                    help="only the headline measurement (no variants, no CPU baseline)")
    ap.add_argument("--with-copy", action="store_true",
                    help="with --quick: also run the copy probe (counter calibration)")
    ap.add_argument("--only", choices=["timestep", "timestep_implicit", "adjoint", "jvp", "frontend"],
                    help="run only this variant and print its figures (for profiling)")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="write the profile summaries under profiles/ from rocprofv3 output in DIR "
                         "(no GPU needed)")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles)
        cal = 0.5
        try:
            with open(TRAFFIC_FILE) as fh:
                cal = json.load(fh)["fetch_calibration"]
        except (OSError, ValueError, KeyError):
            pass
        for v in ("timestep", "timestep_implicit", "adjoint", "jvp"):
            import glob
            if glob.glob(os.path.join(args.summarize_profiles, "v_%s_trace" % v, "**", "*kernel_stats.csv"),
                         recursive=True):
                summarize_variant(args.summarize_profiles, v, cal)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the stencil path runs on a single MI355X (its "
              "horizontal decomposition and halo exchange are emulated on that one device); run it "
              "with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2005_13014_amd import binding as B
    torch.cuda.init()
    dev = torch.cuda.get_device_properties(0)
    log("device:", dev.name, "CUs:", dev.multi_processor_count)
    if args.only:
        fn = {"timestep": variant_program, "timestep_implicit": lambda: variant_program(implicit=True),
              "adjoint": variant_adjoint, "jvp": variant_jvp, "frontend": variant_frontend}[args.only]
        print(json.dumps({"variant": args.only, "result": fn()}), flush=True)
        return

    ni, nj, nk = args.size
    dtype = args.dtype
    es = ES[dtype]
    cfg = B.config(tile_j=args.tile_j, prefetch=args.prefetch, nontemporal=args.nontemporal,
                   schedule=args.schedule)
    abytes = fused_bytes(ni, nj, nk, es)
    nsets = n_sets_for(abytes)
    log("generating %d input sets %dx%dx%d %s" % (nsets, ni, nj, nk, dtype))
    sets = [make_set(ni, nj, nk, dtype, SEED + 3 + 1000 * q) for q in range(nsets)]
    log("timing %d steps after %d warmup" % (args.steps, args.warmup))
    wall, kern = time_calls(fused(cfg), [s[1] for s in sets], args.steps, args.warmup)
    pts = ni * nj * nk
    achieved = abytes / (kern * 1e-3) / 1e9
    log("wall %.4f ms/step, kernel %.4f ms, %.1f GB/s algorithmic" % (wall, kern, achieved))
    headline = ((ni, nj, nk, dtype) == (512, 512, 80, "f32")
                and not (args.tile_j or args.prefetch or args.nontemporal or args.schedule))
    traffic = measured_traffic() if headline else None

    result = {
        "metric": METRIC,
        "value": pts / (wall * 1e-3) / 1e9,
        "unit": "Gpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic: seeded fields shaped like the paper's domains (u, wcon ~ U(-1,1), "
                "coeff ~ U(0,0.1), a, c ~ U(-0.4,0), b diagonally dominant)",
        "config": {"workload": "fused hdiff+vadv %dx%dx%d halo 2, %s storage and stencil "
                               "arithmetic, FP64 Thomas solve" % (ni, nj, nk, dtype),
                   "ni": ni, "nj": nj, "nk": nk, "input_sets_rotated": nsets,
                   "kernel": "k_column (fused)", "kernel_sources_sha256_16": kernel_hash()},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": abytes, "kernel_ms": kern},
    }
    if args.quick:
        if args.with_copy:
            log("copy probe %.1f GB/s, read probe %.1f GB/s, 6-in 1-out probe %.1f GB/s"
                % (copy_probe(), read_probe(), streams_probe(ni, nj, nk)))
        print(json.dumps(result), flush=True)
        return

    fused(cfg)(sets[0][1])
    torch.cuda.synchronize()
    checks = {"headline": gpu_output(sets[0][0], sets[0][1]["x"])}
    del sets
    torch.cuda.empty_cache()
    variants = {"copy_probe_GBs": copy_probe(), "read_probe_GBs": read_probe(),
                "streams_6in_1out_probe_GBs": streams_probe(ni, nj, nk)}
    torch.cuda.empty_cache()
    for label, dt_, level in (("fused_f64", "f64", 0), ("original_f64", "f64", 1),
                              ("fused_bf16", "bf16", 0)):
        log("variant", label)
        variants[label], checks[label] = variant_column(ni, nj, nk, dt_, level)
        torch.cuda.empty_cache()
    for dt_ in ("f32", "f64"):  # the configuration's other size
        log("variant fused_%s_256x256x80" % dt_)
        label = "fused_%s_256x256x80" % dt_
        variants[label], checks[label] = variant_column(256, 256, 80, dt_, 0)
        torch.cuda.empty_cache()
    variants["speedup_fused_f32_over_original_f64"] = variants["original_f64"]["ms"] / wall
    log("variant hdiff optimisation levels")
    variants["hdiff_f32_levels"] = variant_hdiff_levels(ni, nj, nk)
    torch.cuda.empty_cache()
    log("variant batched timestep")
    variants["timestep_6x8_f32"] = variant_program()
    torch.cuda.empty_cache()
    log("variant batched timestep, implicit vertical diffusion")
    variants["timestep_6x8_f32_implicit_vdiff"] = variant_program(implicit=True)
    torch.cuda.empty_cache()
    log("variant adjoint 256x256x80")
    variants["adjoint_256x256x80"] = variant_adjoint()
    torch.cuda.empty_cache()
    log("variant forward mode 256x256x80")
    variants["jvp_256x256x80"] = variant_jvp()
    torch.cuda.empty_cache()
    log("variant front end: generated hdiff 512x512x80")
    variants["frontend_hdiff_f32_512x512x80"] = variant_frontend()
    result["variants"] = variants
    log("cpu baseline (oracle): timing, then checking the GPU outputs against it")
    result["cpu_baseline"], errs = cpu_baseline(ni, nj, nk, checks)
    result["error_vs_fp64_oracle"] = errs.pop("headline")
    for label, e in errs.items():
        variants[label]["error_vs_fp64_oracle"] = e
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
