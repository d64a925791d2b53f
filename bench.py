"""Benchmark of the fused hdiff + vadv stencil program on one MI355X.

One step = one call of the fused program (Laplacian -> limited fluxes ->
update -> flux-form right-hand side -> Thomas elimination and
back-substitution) over a 512 x 512 x 80 grid with FP32 storage and
arithmetic and the FP64 Thomas solve, inputs resident in HBM.  Several input
sets are rotated so that no step finds its inputs in the 256 MB Infinity
Cache left by the previous one.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(ni, nj, nk, es, fields_in=6, fields_out=1):
    """Bytes a fused call must move: u over the interior plus the part of its
    2-cell ring the 13-point diamond reaches (ni nj + 4 (ni + nj) + 4 cells per
    level), the other inputs and the output on the interior."""
    u_cells = (ni * nj + 4 * (ni + nj) + 4) * nk
    other = (fields_in - 1 + fields_out) * ni * nj * nk
    return es * (u_cells + other)


def make_set(ni, nj, nk, dtype, seed):
    from paper_2005_13014_amd import binding as B
    from paper_2005_13014_amd import inputs
    f = inputs.fields(ni, nj, nk, 2, seed=seed, storage=dtype)
    g = {n: B.Field.from_numpy(f[n], 2, dtype) for n in ("u", "coeff", "wcon", "a", "b", "c")}
    g["x"] = B.Field.empty(ni, nj, nk, 2, dtype, fill=0.0)
    return f, g


def run_call(g, cfg=None):
    from paper_2005_13014_amd import binding as B
    B.stencil_hdiff_vadv(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, g["x"], cfg=cfg)


def time_calls(sets, steps, warmup, cfg=None):
    """Returns (wall ms per step, mean kernel ms from HIP events, list of ms)."""
    import torch
    stream = torch.cuda.current_stream()
    for s in range(warmup):
        run_call(sets[s % len(sets)], cfg)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for s in range(steps):
        ev[s][0].record(stream)
        run_call(sets[s % len(sets)], cfg)
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    ms = [a.elapsed_time(b) for a, b in ev]
    return wall, float(np.mean(ms)), ms


def errors(f, g):
    import oracle
    ref = oracle.hdiff_vadv(f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2, f["b"], 2, f["c"], 2,
                            DT)
    got = g["x"].to_numpy(interior=True)
    return {"normwise": float(np.abs(got - ref).max() / np.abs(ref).max()),
            "rms": float(np.sqrt(np.mean((got - ref) ** 2)) / np.sqrt(np.mean(ref ** 2)))}


def n_sets_for(ni, nj, nk, es):
    foot = algorithmic_bytes(ni, nj, nk, es)
    return max(2, min(8, math.ceil(3 * 256e6 / foot) + 1))


def cpu_baseline(ni, nj, nk, budget_s=10.0):
    import oracle
    from paper_2005_13014_amd import inputs
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 3, storage="f32")
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.hdiff_vadv(f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2, f["b"], 2, f["c"], 2, DT)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 20:
            break
    return {"value": reps * ni * nj * nk / el / 1e9, "unit": "Gpoints/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d full calls of the FP64 oracle on the %dx%dx%d workload (%.1f s, one thread)"
                      % (reps, ni, nj, nk, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, nargs=3, default=[512, 512, 80])
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64", "bf16"])
    ap.add_argument("--tile-j", type=int, default=0)
    ap.add_argument("--prefetch", type=int, default=0)
    ap.add_argument("--quick", action="store_true",
                    help="only the headline measurement (no variants, no CPU baseline)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the stencil path runs on a single MI355X; "
              "multi-GPU halo exchange is not built (pass --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2005_13014_amd import binding as B
    torch.cuda.init()
    dev = torch.cuda.get_device_properties(0)
    log("device:", dev.name, "CUs:", dev.multi_processor_count)

    ni, nj, nk = args.size
    dtype = args.dtype
    es = {"f32": 4, "f64": 8, "bf16": 2}[dtype]
    cfg = B.config(tile_j=args.tile_j, prefetch=args.prefetch)
    nsets = n_sets_for(ni, nj, nk, es)
    log("generating %d input sets %dx%dx%d %s" % (nsets, ni, nj, nk, dtype))
    sets, host = [], None
    for q in range(nsets):
        f, g = make_set(ni, nj, nk, dtype, SEED + 3 + 1000 * q)
        if q == 0:
            host = f
        sets.append(g)
    log("timing %d steps after %d warmup" % (args.steps, args.warmup))
    wall, kern, _ = time_calls(sets, args.steps, args.warmup, cfg)
    pts = ni * nj * nk
    abytes = algorithmic_bytes(ni, nj, nk, es)
    achieved = abytes / (kern * 1e-3) / 1e9
    log("wall %.4f ms/step, kernel %.4f ms, %.1f GB/s algorithmic" % (wall, kern, achieved))

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
                   "kernel": "k_hdiff_vadv"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": abytes, "kernel_ms": kern},
    }
    if not args.quick:
        log("checking errors against the oracle")
        run_call(sets[0], cfg)
        torch.cuda.synchronize()
        result["error_vs_fp64_oracle"] = errors(host, sets[0])
        variants = {}
        # Copy ceiling from the bandwidth probe (1 GiB each way).
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
        variants["copy_probe_GBs"] = 2 * nb / (e0.elapsed_time(e1) / 10 * 1e-3) / 1e9
        del src, dst
        # The unfused FP64 path ("original" level) on the same grid: the speedup denominator.
        del sets
        torch.cuda.empty_cache()
        log("unfused fp64 and fused fp64 / bf16 variants")
        for label, dt_, level in (("fused_f64", "f64", 0), ("original_f64", "f64", 1),
                                  ("fused_bf16", "bf16", 0)):
            es_ = {"f32": 4, "f64": 8, "bf16": 2}[dt_]
            n_ = n_sets_for(ni, nj, nk, es_)
            vs = [make_set(ni, nj, nk, dt_, SEED + 3 + 1000 * q) for q in range(n_)]
            w_, k_, _ = time_calls([v[1] for v in vs], 20, 3, B.config(level=level))
            run_call(vs[0][1], B.config(level=level))
            torch.cuda.synchronize()
            err = errors(vs[0][0], vs[0][1])
            ab = algorithmic_bytes(ni, nj, nk, es_)
            variants[label] = {"Gpoints_s": pts / (w_ * 1e-3) / 1e9, "ms": w_,
                               "algorithmic_GBs": ab / (k_ * 1e-3) / 1e9,
                               "frac_hbm_peak": ab / (k_ * 1e-3) / 1e9 / PEAK_HBM_GBS,
                               "error_vs_fp64_oracle": err}
            del vs
            torch.cuda.empty_cache()
        variants["speedup_fused_f32_over_original_f64"] = (
            variants["original_f64"]["ms"] / wall)
        result["variants"] = variants
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(ni, nj, nk)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
