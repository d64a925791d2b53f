"""The batched timestep program on the GPU: every stage prefix against the
oracle, the 6-subdomain x 8-field configuration, graph replay, autotuning
and table chunking (GPU only)."""
import numpy as np
import pytest

import oracle
from helpers import DT, TOL, halo_untouched, normwise
from paper_2005_13014_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2005_13014_amd import binding as B  # noqa: E402

KAPPA, BH, BV = 0.1, 0.05, 0.01
FULL = B.STAGE_HDIFF | B.STAGE_VADV | B.STAGE_VDIFF | B.STAGE_HGRAD
FULL_IMPLICIT = B.STAGE_HDIFF | B.STAGE_VADV | B.STAGE_VDIFF_IMPLICIT | B.STAGE_HGRAD


def note(*a):
    print(*a, flush=True)


def device_program(data, dtype, canary=-7.0):
    subs = []
    for d in data:
        h = d["halo"]
        s = {n: B.Field.from_numpy(d[n], h, dtype) for n in ("coeff", "wcon", "a", "b", "c")}
        s["u"] = [B.Field.from_numpy(u, h, dtype) for u in d["u"]]
        ni, nj, nk = d["shape"]
        s["z"] = [B.Field.empty(ni, nj, nk, h, dtype, fill=canary) for _ in d["u"]]
        subs.append(s)
    return subs


def reference(d, f, stages):
    h = d["halo"]
    args = (d["u"][f], h, d["coeff"], h, d["wcon"], h, d["a"], h, d["b"], h, d["c"], h, DT)
    if stages in (FULL, FULL_IMPLICIT):
        return oracle.timestep(*args, KAPPA, BH, BV, implicit=stages == FULL_IMPLICIT)
    x = oracle.hdiff_vadv(*args)
    if stages & B.STAGE_VDIFF:
        x = oracle.vdiff(x, 0, KAPPA)
    if stages & B.STAGE_VDIFF_IMPLICIT:
        x = oracle.vdiff_implicit(x, 0, KAPPA)
    return x


def run(subs, stages, flags=0):
    spec = B.ProgramSpec(subs, stages=stages, dt=DT, kappa=KAPPA, beta_h=BH, beta_v=BV, flags=flags)
    B.stencil_program_run(spec)
    torch.cuda.synchronize()


def small_data(dtype, nfields=3, shapes=((70, 13, 9), (40, 33, 17), (5, 3, 1), (64, 8, 40))):
    return inputs.batched(storage=dtype, subdomains=shapes, nfields=nfields)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("stages", [B.STAGE_HDIFF | B.STAGE_VADV,
                                    B.STAGE_HDIFF | B.STAGE_VADV | B.STAGE_VDIFF, FULL,
                                    B.STAGE_HDIFF | B.STAGE_VADV | B.STAGE_VDIFF_IMPLICIT,
                                    FULL_IMPLICIT])
def test_program_stage_chains(dtype, stages):
    data = small_data(dtype)
    subs = device_program(data, dtype)
    run(subs, stages)
    worst = 0.0
    for d, s in zip(data, subs):
        for f in range(len(d["u"])):
            got = s["z"][f].to_numpy(interior=True)
            worst = max(worst, normwise(got, reference(d, f, stages)))
    note("program %s stages %d worst normwise %.2e" % (dtype, stages, worst))
    # z is rounded once more per intermediate kept in storage precision.
    tol = {"f64": 1e-12, "f32": 1e-5, "bf16": 2.0 ** -7}[dtype]
    assert worst <= tol


def test_config4_six_subdomains_eight_fields():
    """hdiff -> vadv -> vdiff -> hgrad on 8 fields over the 6 uneven
    subdomains (96x96x60 .. 384x256x90), FP32, graph + autotune; every field
    of every subdomain against the oracle."""
    data = inputs.batched(storage="f32")
    subs = device_program(data, "f32")
    run(subs, FULL, flags=B.PROGRAM_GRAPH | B.PROGRAM_AUTOTUNE)
    worst = 0.0
    for s_idx, (d, s) in enumerate(zip(data, subs)):
        for f in range(8):
            got = s["z"][f].to_numpy(interior=True)
            e = normwise(got, reference(d, f, FULL))
            worst = max(worst, e)
    note("C4 worst normwise %.2e" % worst)
    assert worst <= TOL["f32"]


def test_implicit_vertical_diffusion_six_subdomains():
    """The timestep with the implicit vertical diffusion on the 6 uneven
    subdomains (60 .. 90 levels, every register bucket), FP32 and FP64."""
    for dtype in ("f64", "f32"):
        data = inputs.batched(storage=dtype, nfields=2)
        subs = device_program(data, dtype)
        run(subs, FULL_IMPLICIT, flags=B.PROGRAM_AUTOTUNE)
        worst = 0.0
        for d, s in zip(data, subs):
            for f in range(len(d["u"])):
                worst = max(worst, normwise(s["z"][f].to_numpy(interior=True), reference(d, f, FULL_IMPLICIT)))
        note("implicit timestep %s worst normwise %.2e" % (dtype, worst))
        assert worst <= TOL[dtype]


def test_graph_replays_match_eager():
    data = small_data("f32")
    subs = device_program(data, "f32")
    run(subs, FULL)
    eager = [[z.to_numpy() for z in s["z"]] for s in subs]
    spec = B.ProgramSpec(subs, stages=FULL, dt=DT, kappa=KAPPA, beta_h=BH, beta_v=BV,
                         flags=B.PROGRAM_GRAPH)
    for rep in range(4):
        for s in subs:
            for z in s["z"]:
                z.buf.fill_(-7.0)
        # eager work of the program's own between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        B.stencil_program_run(spec)
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for s, ref in zip(subs, eager):
            for z, r in zip(s["z"], ref):
                assert np.array_equal(z.to_numpy(), r), rep


def test_autotune_does_not_change_results():
    data = small_data("f32", nfields=2)
    subs = device_program(data, "f32")
    run(subs, FULL)
    ref = [[z.to_numpy() for z in s["z"]] for s in subs]
    run(subs, FULL, flags=B.PROGRAM_AUTOTUNE)
    for s, r in zip(subs, ref):
        for z, rr in zip(s["z"], r):
            assert np.array_equal(z.to_numpy(), rr)


@pytest.mark.parametrize("stages", [B.STAGE_HDIFF | B.STAGE_VADV, B.STAGE_HDIFF | B.STAGE_VADV | B.STAGE_VDIFF,
                                    FULL, FULL_IMPLICIT])
def test_pipelined_and_staged_column_stages_agree(stages):
    """The column stages with the software-pipelined level loop (the default)
    and with the staged one (STENCIL_PROGRAM_STAGED) give the same bits, in
    every register bucket (1 .. 96 levels, ragged tiles)."""
    shapes = ((70, 13, 9), (40, 33, 17), (5, 3, 1), (64, 8, 40), (40, 9, 70), (20, 5, 90), (130, 7, 84),
              (33, 6, 91), (17, 4, 96))
    data = small_data("f32", nfields=3, shapes=shapes)
    subs = device_program(data, "f32")
    run(subs, stages)
    pipe = [[z.to_numpy() for z in s["z"]] for s in subs]
    run(subs, stages, flags=B.PROGRAM_STAGED)
    for s, r in zip(subs, pipe):
        for z, rr in zip(s["z"], r):
            assert np.array_equal(z.to_numpy(), rr)
    worst = 0.0
    for d, s in zip(data, subs):
        for f in range(len(d["u"])):
            worst = max(worst, normwise(s["z"][f].to_numpy(interior=True), reference(d, f, stages)))
    assert worst <= TOL["f32"]


def shifted(field, by):
    """The same field in a fresh buffer whose interior origin sits `by`
    elements later (so it no longer starts on a 128-byte line)."""
    buf = torch.full((field.buf.numel() + 64,), -9.0, dtype=field.buf.dtype, device=field.buf.device)
    buf[by:by + field.buf.numel()] = field.buf
    return B.Field(buf, field.origin + by, field.ni, field.nj, field.nk, field.hi, field.hj, field.sj,
                   field.sk, field.dtype)


@pytest.mark.parametrize("dtype", ["f32", "f64", "bf16"])
def test_column_tiles_follow_the_field_alignment(dtype):
    """The column tiles start on 128-byte lines of the coefficient fields when
    that takes no extra tile; fields whose origins sit elsewhere in a line give
    bitwise the results of line-aligned ones (each column is computed the same
    way whichever tile holds it), with and without the horizontal stage."""
    shapes = ((320, 9, 84), (70, 13, 9), (128, 6, 40), (5, 3, 1))
    data = small_data(dtype, nfields=2, shapes=shapes)
    for stages in (FULL, B.STAGE_HDIFF | B.STAGE_VADV | B.STAGE_VDIFF):
        subs = device_program(data, dtype)
        run(subs, stages)
        ref = [[z.to_numpy() for z in s["z"]] for s in subs]
        for by in (1, 3, 17):
            moved = [{n: (shifted(v, by) if n not in ("u", "z") else [shifted(f, by) for f in v])
                      for n, v in s.items()} for s in subs]
            for s in moved:
                for z in s["z"]:
                    z.buf.fill_(-7.0)
            run(moved, stages)
            for s, r in zip(moved, ref):
                for z, rr in zip(s["z"], r):
                    assert np.array_equal(z.to_numpy(), rr), (stages, by)
                    assert halo_untouched(z)


def test_tables_split_over_many_subdomains_and_fields():
    # 10 subdomains (more than one table) and 11 fields (more than one entry).
    shapes = tuple((17 + 3 * q, 6 + q, 5 + q) for q in range(10))
    data = inputs.batched(storage="f32", subdomains=shapes, nfields=11, halo_u=3, halo_coef=3)
    data[3]["u"] = data[3]["u"][:0]  # a subdomain without fields
    subs = device_program(data, "f32")
    run(subs, FULL)
    worst = 0.0
    for d, s in zip(data, subs):
        for f in range(len(d["u"])):
            worst = max(worst, normwise(s["z"][f].to_numpy(interior=True), reference(d, f, FULL)))
    assert worst <= TOL["f32"]


def test_program_outputs_leave_halos_alone():
    data = small_data("f32", nfields=1)
    subs = device_program(data, "f32")
    run(subs, FULL)
    for s in subs:
        assert halo_untouched(s["z"][0])


def test_program_cache_is_bounded_and_shares_scratch():
    """Forty programs that differ only in their output pointers: the cache
    keeps the 16 most recent, they share one scratch buffer, and a program
    that was evicted runs again with the same result."""
    data = small_data("f32", nfields=2, shapes=((70, 13, 9), (40, 33, 17)))
    subs = device_program(data, "f32")
    B.stencil_shutdown()
    assert B.stencil_held_memory() == (0, 0)
    run(subs, FULL)
    ref = [[z.to_numpy() for z in s["z"]] for s in subs]
    held1, n1 = B.stencil_held_memory()
    assert n1 == 1 and held1 > 0
    outs = []
    for q in range(40):
        z = [[B.Field.empty(*d["shape"], d["halo"], "f32", fill=-7.0) for _ in d["u"]] for d in data]
        alt = [dict(s, z=zz) for s, zz in zip(subs, z)]
        run(alt, FULL, flags=B.PROGRAM_GRAPH if q % 2 else 0)
        outs.append(z)
        held, n = B.stencil_held_memory()
        assert n == min(q + 2, 16) and held == held1, (q, n, held, held1)
    for s in subs:
        for z in s["z"]:
            z.buf.fill_(-7.0)
    run(subs, FULL)  # evicted long ago: planned again
    for s, r in zip(subs, ref):
        for z, rr in zip(s["z"], r):
            assert np.array_equal(z.to_numpy(), rr)
    for z in outs:
        for zz, r in zip(z, ref):
            for a, b in zip(zz, r):
                assert np.array_equal(a.to_numpy(), b)


def test_program_inside_a_captured_graph():
    """A program already run on a stream is enqueued into that stream's
    capture (no allocation, no nested capture); a program never run there is
    refused under capture instead of allocating."""
    data = small_data("f32", nfields=2)
    subs = device_program(data, "f32")
    run(subs, FULL)
    ref = [[z.to_numpy() for z in s["z"]] for s in subs]
    s_cap = torch.cuda.Stream()
    spec = B.ProgramSpec(subs, stages=FULL, dt=DT, kappa=KAPPA, beta_h=BH, beta_v=BV,
                         flags=B.PROGRAM_GRAPH | B.PROGRAM_AUTOTUNE)
    with torch.cuda.stream(s_cap):
        B.stencil_program_run(spec)          # first run on this stream: plans, tunes, allocates
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s_cap):
        B.stencil_program_run(spec)
    for rep in range(4):
        for s in subs:
            for z in s["z"]:
                z.buf.fill_(-7.0)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for s, r in zip(subs, ref):
            for z, rr in zip(s["z"], r):
                assert np.array_equal(z.to_numpy(), rr), rep
    other = B.ProgramSpec(subs, stages=B.STAGE_HDIFF | B.STAGE_VADV | B.STAGE_VDIFF, dt=DT, kappa=KAPPA,
                          beta_h=BH, beta_v=BV)
    g2 = torch.cuda.CUDAGraph()
    with pytest.raises(B.StencilError) as e:
        with torch.cuda.graph(g2, stream=s_cap):
            B.stencil_program_run(other)
    assert e.value.status == "E_UNSUPPORTED"
