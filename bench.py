"""Benchmark of the fused hdiff + vadv stencil program on one MI355X.

One step = one call of the fused program (Laplacian -> limited fluxes ->
update -> flux-form right-hand side -> Thomas elimination and
back-substitution) over a 512 x 512 x 80 grid with FP32 storage and stencil
arithmetic and the FP64 Thomas solve, inputs resident in HBM.  Several input
sets are rotated so that no step finds its inputs in the 256 MB Infinity
Cache left by the previous one.

Prints ONE JSON line on stdout; progress goes to stderr.  Times follow the
paper's protocol (Sec. VII-A): the first calls are not timed (a quarter second
of sustained load, so that the GPU's clocks have settled, then the warmup
calls), then the median and quartiles of 100 calls timed with HIP events.  Beside the headline it
reports every workload of the configuration table (hdiff alone in FP64 at
64x64x60; the fused program in FP64 at 128x128x80; FP32, FP64 and bf16 at
256x256x80 and 512x512x80; the unfused "original" FP64 path; the paper's own
domains 128x128x60 and 256x256x60), the hdiff optimisation levels, the
batched timestep, the reverse and forward modes, the front end's generated
hdiff, the grid split into per-GPU shares with its halo exchange, the
bandwidth probes, and the CPU oracle on the same workload (one thread and
all host cores), which also checks every GPU result (max and RMS error).
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
KAPPA, BETA_H, BETA_V = 0.1, 0.05, 0.01
SEED = 200513014
ES = {"f32": 4, "f64": 8, "bf16": 2}
RUNS = 100          # timed calls per variant (the paper's median of 100)
WARM = 5
# Untimed sustained load before the warmup calls of every measurement: the
# GPU's clocks and power state ramp up under load, and a bandwidth-bound
# kernel runs up to 17% slower for its first ~50 ms (the headline kernel:
# 0.115 ms per call at first, 0.0985 ms after ~500 calls).  Times are taken
# in the settled state, as in a long-running timestep loop.
SETTLE_S = 0.25
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_column_f32_512x512x80.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2005_13014_amd", "csrc", n)
                  for n in ("column.hpp", "common.hpp", "column_f32.hip")]
NAMES = ("u", "coeff", "wcon", "a", "b", "c")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def u_cells(ni, nj, nk):
    """Cells of u a fused call must read: the interior plus the part of its
    2-cell ring that the 13-point diamond reaches."""
    return (ni * nj + 4 * (ni + nj) + 4) * nk


def fused_bytes(ni, nj, nk, es):
    """Algorithmic bytes of one fused call: u, five more inputs and the output."""
    return es * (u_cells(ni, nj, nk) + 6 * ni * nj * nk)


def hdiff_bytes(ni, nj, nk, es):
    """Algorithmic bytes of hdiff alone: u with its ring, coeff, the output."""
    return es * (u_cells(ni, nj, nk) + 2 * ni * nj * nk)


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


def make_set(ni, nj, nk, dtype, seed, vadv=True):
    from paper_2005_13014_amd import binding as B
    from paper_2005_13014_amd import inputs
    f = inputs.fields(ni, nj, nk, 2, seed=seed, storage=dtype, vadv=vadv)
    g = {n: B.Field.from_numpy(f[n], 2, dtype) for n in f}
    g["x"] = B.Field.empty(ni, nj, nk, 2, dtype, fill=0.0)
    return f, g


def n_sets_for(nbytes):
    """Input sets to rotate so that their footprint exceeds three times the
    256 MB Infinity Cache."""
    return max(2, min(8, math.ceil(3 * 256e6 / nbytes) + 1))


def settle(fn, sets, seconds=SETTLE_S):
    """Runs fn(set) over rotating sets, untimed, for `seconds` of wall time."""
    import torch
    t0, n = time.perf_counter(), 0
    while time.perf_counter() - t0 < seconds:
        for _ in range(8):
            fn(sets[n % len(sets)])
            n += 1
        torch.cuda.synchronize()
    return n


def time_calls(fn, sets, steps, warmup):
    """Runs fn(set) over rotating sets: SETTLE_S seconds of untimed load,
    warmup untimed calls, then `steps` timed ones.  Returns (wall ms per
    step, list of per-call ms from HIP events on the current stream, which
    the library launches on)."""
    import torch
    stream = torch.cuda.current_stream()
    settle(fn, sets)
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
    return wall, [a.elapsed_time(b) for a, b in ev]


def stats(ms):
    """Median, quartiles and mean of per-call times (ms)."""
    a = np.asarray(ms, dtype=float)
    q1, med, q3 = np.percentile(a, [25, 50, 75])
    return {"median_ms": float(med), "q1_ms": float(q1), "q3_ms": float(q3), "iqr_ms": float(q3 - q1),
            "mean_ms": float(a.mean()), "runs": int(a.size)}


def record(wall, ms, points, nbytes, bytes_key="algorithmic_GBs"):
    """Timing record of a workload: statistics, and the rates at the median."""
    r = stats(ms)
    med = r["median_ms"] * 1e-3
    r["wall_ms"] = wall
    r["Gpoints_s"] = points / med / 1e9
    if nbytes:
        r[bytes_key] = nbytes / med / 1e9
        r["frac_hbm_peak"] = nbytes / med / 1e9 / PEAK_HBM_GBS
    return r


def fused(cfg=None):
    from paper_2005_13014_amd import binding as B

    def fn(g):
        B.stencil_hdiff_vadv(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, g["x"],
                             cfg=cfg)
    return fn


def to_host(field, interior=True):
    return field.to_numpy(interior=interior)


# ---------------------------------------------------------------------------
# Probes
# ---------------------------------------------------------------------------

def _probe_rate(fn, nbytes, reps):
    import torch
    settle(lambda _: fn(), [None])
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9


def copy_probe():
    import torch
    from paper_2005_13014_amd import binding as B
    nb = 1 << 30
    src = torch.empty(nb // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    return _probe_rate(lambda: B.stencil_probe_copy(src, dst, nb), 2 * nb, 10)


def read_probe():
    """Achievable HBM read rate (GB/s): the read-only probe over 1 GiB."""
    import torch
    from paper_2005_13014_amd import binding as B
    nb = 1 << 30
    src = torch.empty(nb // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    sink = torch.zeros(4, dtype=torch.int32, device="cuda")
    # key 1: all-equal vectors give checksum 0, so the sink is never written
    return _probe_rate(lambda: B.stencil_probe_read(src, nb, 1, sink), nb, 10)


def streams_probe(ni=512, nj=512, nk=80):
    """HBM rate (GB/s) of the fused kernel's traffic mix at the headline size:
    six field-sized arrays read and one written, streamed element by element."""
    import torch
    from paper_2005_13014_amd import binding as B
    n = ni * nj * nk
    srcs = [torch.empty(n, dtype=torch.float32, device="cuda").fill_(float(q)) for q in range(6)]
    dst = torch.empty(n, dtype=torch.float32, device="cuda")
    return _probe_rate(lambda: B.stencil_probe_streams(srcs, dst, 4 * n), 7 * 4 * n, 20)


# ---------------------------------------------------------------------------
# Workloads.  Each returns (record, checks): checks is a list of (kind, data)
# for the record itself, or (key, kind, data) for record[key], that the CPU
# leg compares with the oracle.
# ---------------------------------------------------------------------------

def variant_column(ni, nj, nk, dtype, level):
    """Fused (level 0) or unfused 'original' (level 1) program in dtype."""
    import torch
    from paper_2005_13014_amd import binding as B
    es = ES[dtype]
    fb = fused_bytes(ni, nj, nk, es)
    sets = [make_set(ni, nj, nk, dtype, SEED + 3 + 1000 * q) for q in range(n_sets_for(fb))]
    cfg = B.config(level=level)
    w, ms = time_calls(fused(cfg), [s[1] for s in sets], RUNS, WARM)
    fused(cfg)(sets[0][1])
    torch.cuda.synchronize()
    # the unfused path's rate is given on the fused program's bytes (what
    # the same result costs when fused), not on its own temporaries
    r = record(w, ms, ni * nj * nk, fb,
               bytes_key="algorithmic_GBs" if level == 0 else "fused_equivalent_GBs")
    return r, [("hdiff_vadv", {"f": sets[0][0], "x": to_host(sets[0][1]["x"])})]


def variant_hdiff(ni, nj, nk, dtype):
    """hdiff alone (inlined, level 1 of Sec. VII-C) in dtype."""
    import torch
    from paper_2005_13014_amd import binding as B
    hb = hdiff_bytes(ni, nj, nk, ES[dtype])
    sets = [make_set(ni, nj, nk, dtype, SEED + 1 + q, vadv=False) for q in range(n_sets_for(hb))]

    def fn(g):
        B.stencil_hdiff(g["u"], g["coeff"], g["x"])
    w, ms = time_calls(fn, [s[1] for s in sets], RUNS, WARM)
    fn(sets[0][1])
    torch.cuda.synchronize()
    return record(w, ms, ni * nj * nk, hb), [("hdiff", {"f": sets[0][0], "x": to_host(sets[0][1]["x"])})]


def variant_hdiff_levels(ni, nj, nk):
    """hdiff alone in FP32 at the paper's optimisation levels (Sec. VII-C)."""
    from paper_2005_13014_amd import binding as B
    nb = hdiff_bytes(ni, nj, nk, 4)
    sets = [make_set(ni, nj, nk, "f32", SEED + 1 + q, vadv=False)[1] for q in range(n_sets_for(nb))]
    out = {}
    for label, cfg in (("original", B.config(level=1)), ("inline", B.config(unroll=1)),
                       ("inline_unroll2", B.config(unroll=2)), ("inline_unroll4", B.config(unroll=4))):
        def fn(g, cfg=cfg):
            B.stencil_hdiff(g["u"], g["coeff"], g["x"], cfg=cfg)
        w, ms = time_calls(fn, sets, RUNS, WARM)
        out[label] = record(w, ms, ni * nj * nk, nb)
    return out, []


def variant_program(implicit=False, check=True):
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
        # lower bound: per field u in and z out, the five shared coefficient
        # fields read once per subdomain
        nbytes += 4 * (nf * 2 * ni * nj * nk + 5 * ni * nj * nk)
    stages = B.STAGE_HDIFF | B.STAGE_VADV | B.STAGE_HGRAD | (
        B.STAGE_VDIFF_IMPLICIT if implicit else B.STAGE_VDIFF)
    spec = B.ProgramSpec(subs, stages=stages, dt=DT, kappa=KAPPA, beta_h=BETA_H, beta_v=BETA_V,
                         flags=B.PROGRAM_GRAPH | B.PROGRAM_AUTOTUNE)
    w, ms = time_calls(lambda _: B.stencil_program_run(spec), [None], RUNS, WARM)
    torch.cuda.synchronize()
    r = record(w, ms, pts, nbytes, bytes_key="lower_bound_GBs")
    r["Gfieldpoints_s"] = r.pop("Gpoints_s")
    r["field_points"] = pts
    checks = []
    if check:
        z = [[to_host(f) for f in s["z"]] for s in subs]
        checks.append(("timestep", {"data": data, "z": z, "implicit": implicit}))
    del subs
    torch.cuda.empty_cache()
    return r, checks


def variant_adjoint(n=256, nk=80):
    from paper_2005_13014_amd import binding as B
    from paper_2005_13014_amd import inputs
    out, checks = {}, []
    for dtype in ("f32", "f64"):
        f = inputs.fields(n, n, nk, 2, seed=SEED + 5, storage=dtype, loss=True)
        g = {k: B.Field.from_numpy(f[k], 2, dtype) for k in NAMES + ("w",)}
        gs = [g["u"].like(fill=0.0) for _ in range(3)]

        def fn(_):
            B.stencil_hdiff_vadv_adjoint(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT,
                                         g["w"], *gs)
        w, ms = time_calls(fn, [None], RUNS, WARM)
        # u with its ring, coeff, wcon, a, b, c, w in; gu (interior and ring),
        # gcoeff, gwcon out
        ab = ES[dtype] * (2 * u_cells(n, n, nk) + 8 * n * n * nk)
        out[dtype] = record(w, ms, n * n * nk, ab)
        lds = B.config(schedule=1)   # the hdiff adjoint on LDS-staged tiles, for comparison
        w2, ms2 = time_calls(lambda _: B.stencil_hdiff_vadv_adjoint(
            g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, g["w"], *gs, cfg=lds), [None], RUNS, WARM)
        out[dtype]["lds_tiles_median_ms"] = stats(ms2)["median_ms"]
        fn(None)
        checks.append((dtype, "adjoint", {
            "f": f, "gu": to_host(gs[0], interior=False), "gcoeff": to_host(gs[1]), "gwcon": to_host(gs[2])}))
    return out, checks


def variant_jvp(n=256, nk=80):
    """Forward mode (tangent in all six inputs) at the reverse mode's size."""
    from paper_2005_13014_amd import binding as B
    from paper_2005_13014_amd import inputs
    out, checks = {}, []
    for dtype in ("f32", "f64"):
        f = inputs.fields(n, n, nk, 2, seed=SEED + 6, storage=dtype)
        rng = np.random.default_rng(SEED + 7)
        t = {k: inputs.round_to(rng.standard_normal(f[k].shape), dtype) for k in NAMES}
        g = {k: B.Field.from_numpy(f[k], 2, dtype) for k in NAMES}
        gt = {k: B.Field.from_numpy(t[k], 2, dtype) for k in NAMES}
        x = g["u"].like(fill=0.0)
        B.stencil_hdiff_vadv(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, x)
        dx = g["u"].like(fill=0.0)

        def fn(_):
            B.stencil_hdiff_vadv_jvp(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, dx, x=x,
                                     du=gt["u"], dcoeff=gt["coeff"], dwcon=gt["wcon"], da=gt["a"],
                                     db=gt["b"], dc=gt["c"])
        w, ms = time_calls(fn, [None], RUNS, WARM)
        es = ES[dtype]
        # 13 streams in (u, du with their ring; 11 column fields incl. x), 1 out
        ab = es * (2 * u_cells(n, n, nk) + 12 * n * n * nk)
        out[dtype] = record(w, ms, n * n * nk, ab)
        checks.append((dtype, "jvp", {"f": f, "t": t, "dx": to_host(dx)}))
    return out, checks


def variant_frontend(ni=512, nj=512, nk=80):
    """hdiff written as a stencil program, inlined, unrolled and compiled at
    run time by the front end (FP32), beside the hand-written hdiff kernel."""
    import torch
    from paper_2005_13014_amd import binding as B
    from paper_2005_13014_amd import frontend as F
    nb = hdiff_bytes(ni, nj, nk, 4)
    sets = [make_set(ni, nj, nk, "f32", SEED + 1 + q, vadv=False) for q in range(n_sets_for(nb))]
    out, checks = {}, []
    for tiled in (False, True):
        for unroll in (1, 2, 4):
            k = F.compile_program(F.hdiff_program(), "f32", like=sets[0][1]["u"], unroll=unroll, tiled=tiled)

            def fn(g, k=k):
                k({"u": g["u"], "coeff": g["coeff"]}, {"out": g["x"]})
            w, ms = time_calls(fn, [s[1] for s in sets], RUNS, WARM)
            label = "generated%s_unroll%d" % ("_tiled" if tiled else "", unroll)
            out[label] = record(w, ms, ni * nj * nk, nb)
            if unroll == 4:
                fn(sets[0][1])
                torch.cuda.synchronize()
                checks.append((label, "hdiff", {"f": sets[0][0], "x": to_host(sets[0][1]["x"])}))
            k.close()

    def hand(g):
        B.stencil_hdiff(g["u"], g["coeff"], g["x"])
    w, ms = time_calls(hand, [s[1] for s in sets], RUNS, WARM)
    out["hand_written_inline"] = record(w, ms, ni * nj * nk, nb)
    return out, checks


def variant_decomposed(nis=(128,) * 4, njs=(256,) * 2, nk=80, dtype="f32"):
    """512 x 512 x 80 split into 4 x 2 shares of 128 x 256 (what eight GPUs
    would each own), held as separate halo-padded fields on this device: the
    halo exchange of u, the fused kernel on one share at its real shape, and
    the whole decomposed step (exchange, then the eight shares)."""
    import torch
    from paper_2005_13014_amd import binding as B
    from paper_2005_13014_amd import inputs
    px, py, h = len(nis), len(njs), 2
    ni, nj = sum(nis), sum(njs)
    i0 = np.concatenate([[0], np.cumsum(nis)]).astype(int)
    j0 = np.concatenate([[0], np.cumsum(njs)]).astype(int)
    f = inputs.fields(ni, nj, nk, h, seed=SEED + 9, storage=dtype)
    shares = []
    for q in range(py):
        for p in range(px):
            win = {n: f[n][:, j0[q]:j0[q] + njs[q] + 2 * h, i0[p]:i0[p] + nis[p] + 2 * h] for n in NAMES}
            g = {n: B.Field.from_numpy(win[n], h, dtype) for n in NAMES}
            g["x"] = g["u"].like(fill=0.0)
            shares.append(g)
    us = [s["u"] for s in shares]
    # halo strips moved per exchange (read from a neighbour, written here)
    cells = 0
    for q in range(py):
        for p in range(px):
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    if (dx, dy) == (0, 0) or not (0 <= p + dx < px and 0 <= q + dy < py):
                        continue
                    wi = h if dx else nis[p] + (h if p == 0 else 0) + (h if p == px - 1 else 0)
                    wj = h if dy else njs[q] + (h if q == 0 else 0) + (h if q == py - 1 else 0)
                    cells += wi * wj * nk
    xb = 2 * ES[dtype] * cells
    w, ms = time_calls(lambda _: B.stencil_halo_exchange(us, px, py, h), [None], RUNS, WARM)
    exch = record(w, ms, 0, xb, bytes_key="strip_GBs")
    exch.pop("Gpoints_s")
    exch["halo_bytes_moved"] = xb
    one = shares[px + 1] if px * py > 1 else shares[0]
    w, ms = time_calls(fused(), [one], RUNS, WARM)
    share = record(w, ms, nis[1 % px] * njs[1 % py] * nk, fused_bytes(nis[1 % px], njs[1 % py], nk, ES[dtype]))

    def step(_):
        B.stencil_halo_exchange(us, px, py, h)
        for s in shares:
            fused()(s)
    w, ms = time_calls(step, [None], RUNS, WARM)
    whole = record(w, ms, ni * nj * nk, sum(fused_bytes(a, b, nk, ES[dtype]) for b in njs for a in nis))
    step(None)
    torch.cuda.synchronize()
    x = np.empty((nk, nj, ni))
    for n, s in enumerate(shares):
        p, q = n % px, n // px
        x[:, j0[q]:j0[q + 1], i0[p]:i0[p + 1]] = to_host(s["x"])
    r = {"split": "%dx%d shares of %dx%d" % (px, py, nis[0], njs[0]), "halo_exchange": exch,
         "one_share_fused": share, "decomposed_step": whole}
    return r, [("hdiff_vadv", {"f": f, "x": x})]


# ---------------------------------------------------------------------------
# CPU leg
# ---------------------------------------------------------------------------

def relative_errors(got, ref):
    den = np.abs(ref).max()
    rms = np.sqrt(np.mean(ref ** 2))
    return {"normwise": float(np.abs(got - ref).max() / den) if den > 0 else float(np.abs(got - ref).max()),
            "rms": float(np.sqrt(np.mean((got - ref) ** 2)) / rms) if rms > 0 else 0.0}


def host_identity():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_count": os.cpu_count(), "model": model}


def oracle_result(kind, d):
    """The FP64 oracle's result for a check of the given kind, and the GPU's."""
    import oracle
    if kind == "hdiff_vadv":
        f = d["f"]
        return [(d["x"], oracle.hdiff_vadv(f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2, f["b"], 2,
                                           f["c"], 2, DT))]
    if kind == "hdiff":
        f = d["f"]
        return [(d["x"], oracle.hdiff(f["u"], 2, f["coeff"], 2))]
    if kind == "adjoint":
        f = d["f"]
        gu, gc, gw = oracle.hdiff_vadv_adjoint(f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2, f["b"], 2,
                                               f["c"], 2, DT, oracle.interior(f["w"], 2), 0)
        return [(d["gu"], gu), (d["gcoeff"], gc), (d["gwcon"], gw)]
    if kind == "jvp":
        f, t = d["f"], d["t"]
        dx = oracle.hdiff_vadv_jvp(f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2, f["b"], 2, f["c"], 2, DT,
                                   du=t["u"], hdu=2, dcoeff=t["coeff"], hdcf=2, dw=t["wcon"], hdw=2, da=t["a"],
                                   db=t["b"], dc=t["c"], hdm=2)
        return [(d["dx"], dx)]
    if kind == "timestep":
        pairs = []
        for s, zs in zip(d["data"], d["z"]):
            h = s["halo"]
            for u, z in zip(s["u"], zs):
                ref = oracle.timestep(u, h, s["coeff"], h, s["wcon"], h, s["a"], h, s["b"], h, s["c"], h, DT,
                                      KAPPA, BETA_H, BETA_V, implicit=d["implicit"])
                pairs.append((z, ref))
        return pairs
    raise ValueError(kind)


def pooled_errors(pairs):
    """Errors over all pairs together: max |err| / max |ref|, RMS err / RMS ref."""
    num_max = max(float(np.abs(g - r).max()) for g, r in pairs)
    den_max = max(float(np.abs(r).max()) for _, r in pairs)
    n = sum(r.size for _, r in pairs)
    num_sq = sum(float(np.sum((g - r) ** 2)) for g, r in pairs)
    den_sq = sum(float(np.sum(r ** 2)) for _, r in pairs)
    return {"normwise": num_max / den_max if den_max > 0 else num_max,
            "rms": math.sqrt(num_sq / n) / math.sqrt(den_sq / n) if den_sq > 0 else 0.0}


def cpu_baseline(ni, nj, nk, checks, budget_s=8.0):
    """The host leg: times the FP64 oracle on the workload on one thread and
    on all host cores (bitwise the same results), then uses it to check every
    GPU output in checks; returns the baseline record and errors by label."""
    import oracle
    from paper_2005_13014_amd import inputs

    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 3, storage="f32")

    def run():
        return oracle.hdiff_vadv(f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2, f["b"], 2, f["c"],
                                 2, DT)

    def timed():
        reps, t0 = 0, time.perf_counter()
        while True:
            run()
            reps += 1
            el = time.perf_counter() - t0
            if el >= budget_s or reps >= 40:
                return reps, el
    r1, e1 = timed()
    with oracle.parallel():
        rn, en = timed()
    nthreads = oracle.threads()
    pts = ni * nj * nk
    base = {"value": rn * pts / en / 1e9, "unit": "Gpoints/s", "cores": nthreads, "kind": "oracle",
            "sample": "%d full calls of the FP64 oracle on the %dx%dx%d workload on %d threads (%.1f s); "
                      "one thread: %d calls (%.1f s)" % (rn, ni, nj, nk, nthreads, en, r1, e1),
            "single_thread_value": r1 * pts / e1 / 1e9,
            "algorithmic_GBs_all_cores": rn * fused_bytes(ni, nj, nk, 4) / en / 1e9,
            "host": host_identity()}
    errs = {}
    with oracle.parallel():
        for label, kind, d in checks:
            log("  checking", label)
            errs[label] = pooled_errors(oracle_result(kind, d))
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


def kernel_name(name):
    """A traced kernel's name without its parameter list."""
    return name.replace("(anonymous namespace)::", "").split("(")[0]


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
        return kernel_name(name)[:100]

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
                out.setdefault(kernel_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
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
        n = kernel_name(r["Name"])
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
    ap.add_argument("--tile-i", type=int, default=0)
    ap.add_argument("--tile-j", type=int, default=0)
    ap.add_argument("--prefetch", type=int, default=0)
    ap.add_argument("--nontemporal", type=int, default=0, help="1 on, -1 off, 0 library choice")
    ap.add_argument("--schedule", type=int, default=0, help="1 staged, 2 pipelined, 0 library choice")
    ap.add_argument("--quick", action="store_true",
                    help="only the headline measurement (no variants, no CPU baseline)")
    ap.add_argument("--with-copy", action="store_true",
                    help="with --quick: also run the copy probe (counter calibration)")
    ap.add_argument("--only", choices=["timestep", "timestep_implicit", "adjoint", "jvp", "frontend",
                                       "decomposed"],
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
        for v in ("timestep", "timestep_implicit", "adjoint", "jvp", "decomposed"):
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
        fn = {"timestep": lambda: variant_program(check=False),
              "timestep_implicit": lambda: variant_program(implicit=True, check=False),
              "adjoint": variant_adjoint, "jvp": variant_jvp, "frontend": variant_frontend,
              "decomposed": variant_decomposed}[args.only]
        print(json.dumps({"variant": args.only, "result": fn()[0]}), flush=True)
        return

    ni, nj, nk = args.size
    dtype = args.dtype
    es = ES[dtype]
    cfg = B.config(tile_j=args.tile_j, prefetch=args.prefetch, nontemporal=args.nontemporal,
                   schedule=args.schedule, tile_i=args.tile_i)
    abytes = fused_bytes(ni, nj, nk, es)
    nsets = n_sets_for(abytes)
    log("generating %d input sets %dx%dx%d %s" % (nsets, ni, nj, nk, dtype))
    sets = [make_set(ni, nj, nk, dtype, SEED + 3 + 1000 * q) for q in range(nsets)]
    log("timing %d steps after %d warmup" % (args.steps, args.warmup))
    wall, ms = time_calls(fused(cfg), [s[1] for s in sets], args.steps, args.warmup)
    st = stats(ms)
    kern = st["mean_ms"]
    pts = ni * nj * nk
    achieved = abytes / (kern * 1e-3) / 1e9
    log("wall %.4f ms/step, kernel mean %.4f ms, median %.4f ms (IQR %.4f), %.1f GB/s algorithmic"
        % (wall, kern, st["median_ms"], st["iqr_ms"], achieved))
    headline = ((ni, nj, nk, dtype) == (512, 512, 80, "f32")
                and not (args.tile_i or args.tile_j or args.prefetch or args.nontemporal or args.schedule))
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
                   "untimed_settle_s_before_warmup": SETTLE_S,
                   "kernel": "k_column (fused)", "kernel_sources_sha256_16": kernel_hash()},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": abytes, "kernel_ms": kern},
        "timing": dict(st, wall_ms=wall, Gpoints_s_at_median=pts / (st["median_ms"] * 1e-3) / 1e9,
                       frac_hbm_peak_at_median=abytes / (st["median_ms"] * 1e-3) / 1e9 / PEAK_HBM_GBS),
    }
    if args.quick:
        if args.with_copy:
            log("copy probe %.1f GB/s, read probe %.1f GB/s, 6-in 1-out probe %.1f GB/s"
                % (copy_probe(), read_probe(), streams_probe(ni, nj, nk)))
        print(json.dumps(result), flush=True)
        return

    fused(cfg)(sets[0][1])
    torch.cuda.synchronize()
    checks = [("headline", "hdiff_vadv", {"f": sets[0][0], "x": to_host(sets[0][1]["x"])})]
    del sets
    torch.cuda.empty_cache()
    variants = {"copy_probe_GBs": copy_probe(), "read_probe_GBs": read_probe(),
                "streams_6in_1out_probe_GBs": streams_probe(ni, nj, nk)}
    torch.cuda.empty_cache()

    def run(label, fn, *a, **kw):
        log("variant", label)
        rec, cks = fn(*a, **kw)
        variants[label] = rec
        for c in cks:
            checks.append((label,) + tuple(c) if len(c) == 2 else (label + "/" + c[0],) + tuple(c[1:]))
        torch.cuda.empty_cache()

    run("C1_hdiff_f64_64x64x60", variant_hdiff, 64, 64, 60, "f64")
    run("C2_fused_f64_128x128x80", variant_column, 128, 128, 80, "f64", 0)
    for n in (256, 512):
        for dt_ in ("f32", "f64", "bf16"):
            if (n, dt_) == (512, "f32"):
                continue  # the headline
            run("fused_%s_%dx%dx80" % (dt_, n, n), variant_column, n, n, 80, dt_, 0)
        run("original_f64_%dx%dx80" % (n, n), variant_column, n, n, 80, "f64", 1)
    for n in (128, 256):  # the paper's two domains (Sec. VII-A), K = 60
        for dt_ in ("f32", "f64"):
            run("fused_%s_%dx%dx60" % (dt_, n, n), variant_column, n, n, 60, dt_, 0)
            run("hdiff_%s_%dx%dx60" % (dt_, n, n), variant_hdiff, n, n, 60, dt_)
    variants["speedup_fused_f32_over_original_f64"] = (
        variants["original_f64_512x512x80"]["median_ms"] / st["median_ms"])
    run("hdiff_f32_levels_512x512x80", variant_hdiff_levels, ni, nj, nk)
    run("timestep_6x8_f32", variant_program)
    run("timestep_6x8_f32_implicit_vdiff", variant_program, implicit=True)
    run("adjoint_256x256x80", variant_adjoint)
    run("jvp_256x256x80", variant_jvp)
    run("frontend_hdiff_f32_512x512x80", variant_frontend)
    run("decomposed_f32_512x512x80", variant_decomposed)
    result["variants"] = variants
    log("cpu baseline (oracle): timing, then checking the GPU outputs against it")
    result["cpu_baseline"], errs = cpu_baseline(ni, nj, nk, checks)
    result["error_vs_fp64_oracle"] = errs.pop("headline")
    for label, e in errs.items():
        top, _, sub = label.partition("/")
        (variants[top][sub] if sub else variants[top])["error_vs_fp64_oracle"] = e
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
