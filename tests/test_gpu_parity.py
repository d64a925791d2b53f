"""Parity of the HIP path with the FP64 CPU oracle, element by element on the
same seeded inputs (GPU only).  Sizes span several tiles with ragged tails;
the full-size cases run in the launch configuration the benchmark times."""
import sys

import numpy as np
import pytest

import oracle
from helpers import (DT, SEED, TOL, gpu_fields, halo_untouched, interior, limiter_masks, normwise, out_field,
                     rms_rel)
from paper_2005_13014_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2005_13014_amd import binding as B  # noqa: E402

VADV = ("wcon", "a", "b", "c")


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_hdiff_vadv(f, ni, nj, nk, halo, dtype, cfg=None):
    g = gpu_fields(f, halo, dtype, ("u", "coeff") + VADV)
    x = out_field(ni, nj, nk, halo, dtype)
    B.stencil_hdiff_vadv(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, x, cfg=cfg)
    torch.cuda.synchronize()
    return x


def ref_hdiff_vadv(f, halo):
    return oracle.hdiff_vadv(f["u"], halo, f["coeff"], halo, f["wcon"], halo, f["a"], halo,
                             f["b"], halo, f["c"], halo, DT)


# ---- horizontal diffusion alone ------------------------------------------

@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("shape", [(64, 64, 60), (70, 13, 5), (130, 9, 3), (1, 1, 1)])
@pytest.mark.parametrize("variant", ["u1", "u2", "u4", "original"])
def test_hdiff(dtype, shape, variant):
    ni, nj, nk = shape
    note("hdiff", dtype, shape, variant)
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 1, storage=dtype, vadv=False)
    g = gpu_fields(f, 2, dtype, ("u", "coeff"))
    out = out_field(ni, nj, nk, 2, dtype)
    cfg = B.config(level=1) if variant == "original" else B.config(unroll=int(variant[1]))
    B.stencil_hdiff(g["u"], g["coeff"], out, cfg=cfg)
    torch.cuda.synchronize()
    ref = oracle.hdiff(f["u"], 2, f["coeff"], 2)
    got = out.to_numpy(interior=True)
    assert normwise(got, ref) <= TOL[dtype], normwise(got, ref)
    assert halo_untouched(out)


@pytest.mark.parametrize("variant", ["u1", "u2", "u4", "original"])
def test_hdiff_f32_at_the_benchmarked_size(variant):
    """hdiff alone, FP32, 512 x 512 x 80 at every optimisation level the
    benchmark times: every element against the FP64 oracle taking the FP32
    limiter decisions."""
    ni, nj, nk = 512, 512, 80
    note("hdiff f32 512x512x80", variant)
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 1, storage="f32", vadv=False)
    g = gpu_fields(f, 2, "f32", ("u", "coeff"))
    out = out_field(ni, nj, nk, 2, "f32")
    cfg = B.config(level=1) if variant == "original" else B.config(unroll=int(variant[1]))
    B.stencil_hdiff(g["u"], g["coeff"], out, cfg=cfg)
    torch.cuda.synchronize()
    kx, ky = limiter_masks(f["u"], 2, "f32")
    ref = oracle.hdiff(f["u"], 2, f["coeff"], 2, force_kx=kx, force_ky=ky)
    err = normwise(out.to_numpy(interior=True), ref)
    note("normwise %.2e" % err)
    assert err <= TOL["f32"]
    assert halo_untouched(out)


def test_hdiff_fp64_follows_the_definition_order():
    # FP64: the kernel evaluates the Laplacian and the fluxes in the oracle's
    # order, so the limiter takes identical decisions and only the update's
    # fused multiply-add differs from the oracle's separate product and sum:
    # |fma - oracle| <= ulp(coeff * div) / 2 + ulp(result), also where u and
    # coeff * div cancel.
    ni, nj, nk = 64, 64, 60
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 1, storage="f64", vadv=False)
    g = gpu_fields(f, 2, "f64", ("u", "coeff"))
    out = out_field(ni, nj, nk, 2, "f64")
    B.stencil_hdiff(g["u"], g["coeff"], out)
    torch.cuda.synchronize()
    ref = oracle.hdiff(f["u"], 2, f["coeff"], 2)
    got = out.to_numpy(interior=True)
    cdiv = interior(f["u"], 2) - ref
    assert np.all(np.abs(got - ref) <= np.spacing(np.abs(cdiv)) + np.spacing(np.abs(ref)))


# ---- vertical advection alone --------------------------------------------

@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("nk", [1, 2, 5, 32, 33, 64, 65, 80, 81, 96, 97])
def test_vadv(dtype, nk):
    ni, nj = 67, 9
    note("vadv", dtype, nk)
    f = inputs.fields(ni, nj, nk, 1, seed=SEED + 20 + nk, storage=dtype)
    h = inputs.round_to(np.random.default_rng(nk).uniform(-1, 1, f["u"].shape), dtype)
    f["h"] = h
    g = gpu_fields(f, 1, dtype, ("h",) + VADV)
    x = out_field(ni, nj, nk, 1, dtype)
    B.stencil_vadv(g["h"], g["wcon"], g["a"], g["b"], g["c"], DT, x)
    torch.cuda.synchronize()
    ref = oracle.vadv(h, 1, f["wcon"], 1, f["a"], 1, f["b"], 1, f["c"], 1, DT)
    got = x.to_numpy(interior=True)
    assert normwise(got, ref) <= TOL[dtype], normwise(got, ref)
    assert halo_untouched(x)


# ---- the fused program ---------------------------------------------------

@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("shape", [(64, 64, 60), (131, 70, 33), (65, 5, 80), (3, 2, 1), (70, 9, 96)])
@pytest.mark.parametrize("level", [0, 1])
def test_hdiff_vadv(dtype, shape, level):
    ni, nj, nk = shape
    note("hdiff_vadv", dtype, shape, level)
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 2, storage=dtype)
    x = run_hdiff_vadv(f, ni, nj, nk, 2, dtype, cfg=B.config(level=level))
    ref = ref_hdiff_vadv(f, 2)
    got = x.to_numpy(interior=True)
    assert normwise(got, ref) <= TOL[dtype], normwise(got, ref)
    assert halo_untouched(x)


@pytest.mark.parametrize("n,level", [(512, 0), (512, 1), (256, 0)])
def test_fp64_at_the_benchmarked_size(n, level):
    """FP64 hdiff + vadv on n x n x 80, fused (level 0) and the unfused
    original path (level 1), as the benchmark times them: every element
    within 1e-12 of the oracle."""
    ni, nj, nk = n, n, 80
    note("hdiff_vadv f64 %dx%dx80 level %d" % (n, n, level))
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 3, storage="f64")
    x = run_hdiff_vadv(f, ni, nj, nk, 2, "f64", cfg=B.config(level=level))
    ref = ref_hdiff_vadv(f, 2)
    got = x.to_numpy(interior=True)
    note("normwise %.3e rms %.3e" % (normwise(got, ref), rms_rel(got, ref)))
    assert normwise(got, ref) <= 1e-12 and rms_rel(got, ref) <= 1e-12
    assert halo_untouched(x)


def test_config2_fp64_128x128x80():
    """hdiff + vadv, FP64, 128x128x80: FP64 must match the oracle to 1e-12."""
    ni, nj, nk = 128, 128, 80
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 2, storage="f64")
    x = run_hdiff_vadv(f, ni, nj, nk, 2, "f64")
    ref = ref_hdiff_vadv(f, 2)
    got = x.to_numpy(interior=True)
    note("C2 fp64 normwise %.3e rms %.3e" % (normwise(got, ref), rms_rel(got, ref)))
    assert normwise(got, ref) <= 1e-12
    assert rms_rel(got, ref) <= 1e-12


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("n", [256, 512])
def test_config3_full_size(dtype, n):
    """hdiff + vadv on n x n x 80 in FP32 (bf16 storage variant) with the FP64
    Thomas solve; every element against the FP64 oracle."""
    nk = 80
    f = inputs.fields(n, n, nk, 2, seed=SEED + 3, storage=dtype)
    x = run_hdiff_vadv(f, n, n, nk, 2, dtype)
    ref = ref_hdiff_vadv(f, 2)
    got = x.to_numpy(interior=True)
    e, r = normwise(got, ref), rms_rel(got, ref)
    note("C3 %s %d^2 normwise %.3e rms %.3e" % (dtype, n, e, r))
    assert e <= TOL[dtype] and r <= TOL[dtype]
    assert halo_untouched(x)


@pytest.mark.parametrize("tj,pf,nt,sched", [(2, 4, -1, 1), (4, 4, -1, 1), (2, 2, -1, 1), (2, 8, -1, 1),
                                            (1, 4, -1, 1), (2, 4, 1, 1), (4, 4, 1, 1), (2, 8, 1, 1),
                                            (2, 2, 1, 1), (2, 4, 1, 2), (2, 8, 1, 2), (2, 4, 1, 3),
                                            (4, 4, 1, 2), (1, 4, 1, 2), (2, 2, 1, 2)])
def test_fused_variants_are_bitwise_identical(tj, pf, nt, sched):
    ni, nj, nk = 200, 37, 80
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 4, storage="f32")
    base = run_hdiff_vadv(f, ni, nj, nk, 2, "f32", cfg=B.config(schedule=1)).to_numpy(interior=True)
    cfg = B.config(tile_j=tj, prefetch=pf, nontemporal=nt, schedule=sched)
    got = run_hdiff_vadv(f, ni, nj, nk, 2, "f32", cfg=cfg)
    assert np.array_equal(got.to_numpy(interior=True), base)


@pytest.mark.parametrize("ti,tj,pf,sched", [(128, 1, 4, 2), (128, 2, 4, 2), (256, 1, 4, 2), (64, 4, 2, 2)])
@pytest.mark.parametrize("shape", [(200, 37, 80), (300, 9, 33), (1, 3, 5), (513, 2, 96)])
def test_wide_tiles_are_bitwise_identical(ti, tj, pf, sched, shape):
    """Pipelined tiles 128 or 256 columns wide, or four rows tall (ragged
    last tile in i and j, depths below, at and above the register buckets)
    give the bits of the staged 64 x 2 tile."""
    ni, nj, nk = shape
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 41, storage="f32")
    base = run_hdiff_vadv(f, ni, nj, nk, 2, "f32", cfg=B.config(schedule=1)).to_numpy(interior=True)
    x = run_hdiff_vadv(f, ni, nj, nk, 2, "f32", cfg=B.config(tile_i=ti, tile_j=tj, prefetch=pf, nontemporal=1,
                                                                schedule=sched))
    assert np.array_equal(x.to_numpy(interior=True), base)
    assert halo_untouched(x)


@pytest.mark.parametrize("dtype,tj,pf,nt", [("f64", 2, 2, 1), ("f64", 2, 2, -1), ("f64", 4, 2, 1),
                                             ("bf16", 2, 4, 1), ("bf16", 2, 8, 1), ("bf16", 4, 4, -1),
                                             ("bf16", 4, 4, 1)])
@pytest.mark.parametrize("nk", [7, 80, 90])
def test_other_storage_variants_are_bitwise_identical(dtype, tj, pf, nt, nk):
    """FP64 and bf16 storage: every compiled tile shape, prefetch depth,
    cache policy and schedule gives the same bits as the staged default."""
    ni, nj = 130, 9
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 80 + nk, storage=dtype)
    base = run_hdiff_vadv(f, ni, nj, nk, 2, dtype, cfg=B.config(schedule=1)).to_numpy(interior=True)
    for sched in (1, 2):
        cfg = B.config(tile_j=tj, prefetch=pf, nontemporal=nt, schedule=sched)
        try:
            x = run_hdiff_vadv(f, ni, nj, nk, 2, dtype, cfg=cfg)
        except B.StencilError as e:
            assert e.status == "E_UNSUPPORTED"  # this combination is not compiled
            continue
        assert np.array_equal(x.to_numpy(interior=True), base), sched
        assert halo_untouched(x)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nk", [8, 9, 13, 31, 33, 60, 64, 79, 80, 81, 90, 96])
def test_four_lanes_per_column(dtype, nk):
    """The partitioned solve over four segments per column (schedule 4):
    every depth from the shortest segments (two rows) to the deepest bucket,
    on ragged tiles, against the oracle; halos untouched."""
    ni, nj = 70, 6
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 90 + nk, storage=dtype)
    x = run_hdiff_vadv(f, ni, nj, nk, 2, dtype, cfg=B.config(schedule=4))
    got = x.to_numpy(interior=True)
    ref = ref_hdiff_vadv(f, 2)
    e = normwise(got, ref)
    note("four lanes %s nk=%d normwise %.2e" % (dtype, nk, e))
    assert e <= TOL[dtype] and rms_rel(got, ref) <= TOL[dtype]
    assert halo_untouched(x)


def test_four_lanes_need_eight_levels():
    ni, nj, nk = 64, 4, 7
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 89, storage="f32")
    with pytest.raises(B.StencilError) as ei:
        run_hdiff_vadv(f, ni, nj, nk, 2, "f32", cfg=B.config(schedule=4))
    assert ei.value.status == "E_UNSUPPORTED"
    # the library's own choice falls back to two lanes per column
    x = run_hdiff_vadv(f, ni, nj, nk, 2, "f32")
    assert normwise(x.to_numpy(interior=True), ref_hdiff_vadv(f, 2)) <= TOL["f32"]


@pytest.mark.parametrize("nk", [1, 2, 3, 4, 5, 9, 31, 32, 33, 64, 65, 79, 80, 81, 96])
def test_pipelined_schedule_every_depth(nk):
    """The pipelined level loop has its own prologue and drain; every column
    depth, including those shorter than the pipeline, against the staged loop
    (same arithmetic, so bitwise) and the oracle."""
    ni, nj = 70, 5
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 40 + nk, storage="f32")
    staged = run_hdiff_vadv(f, ni, nj, nk, 2, "f32", cfg=B.config(schedule=1)).to_numpy(interior=True)
    for pf, sched in ((4, 2), (8, 2), (4, 3)):
        x = run_hdiff_vadv(f, ni, nj, nk, 2, "f32", cfg=B.config(prefetch=pf, nontemporal=1, schedule=sched))
        assert np.array_equal(x.to_numpy(interior=True), staged), (pf, sched)
        assert halo_untouched(x)
    assert normwise(staged, ref_hdiff_vadv(f, 2)) <= TOL["f32"]


@pytest.mark.parametrize("nk", [80, 37])
def test_persistent_schedule_walks_several_tiles(nk):
    """More tiles than resident workgroups (4 x 151 = 604 ragged tiles), so
    workgroups of the persistent grid chain tiles: bitwise equal to the
    one-shot staged grid, halos untouched."""
    ni, nj = 200, 301
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 60 + nk, storage="f32")
    staged = run_hdiff_vadv(f, ni, nj, nk, 2, "f32", cfg=B.config(schedule=1)).to_numpy(interior=True)
    x = run_hdiff_vadv(f, ni, nj, nk, 2, "f32", cfg=B.config(prefetch=4, nontemporal=1, schedule=3))
    assert np.array_equal(x.to_numpy(interior=True), staged)
    assert halo_untouched(x)


def test_deterministic_and_wider_halo():
    ni, nj, nk = 96, 40, 64
    f = inputs.fields(ni, nj, nk, 3, seed=SEED + 5, storage="f32")
    a = run_hdiff_vadv(f, ni, nj, nk, 3, "f32").to_numpy(interior=True)
    b = run_hdiff_vadv(f, ni, nj, nk, 3, "f32").to_numpy(interior=True)
    assert np.array_equal(a, b)
    ref = oracle.hdiff_vadv(f["u"], 3, f["coeff"], 3, f["wcon"], 3, f["a"], 3, f["b"], 3, f["c"],
                            3, DT)
    assert normwise(a, ref) <= TOL["f32"]


def test_fp64_beyond_register_columns_falls_back_to_unfused():
    ni, nj, nk = 40, 6, 120
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 6, storage="f64")
    x = run_hdiff_vadv(f, ni, nj, nk, 2, "f64")
    assert normwise(x.to_numpy(interior=True), ref_hdiff_vadv(f, 2)) <= 1e-12
    with pytest.raises(B.StencilError) as ei:
        run_hdiff_vadv(f, ni, nj, nk, 2, "f64", cfg=B.config(level=2))
    assert ei.value.status == "E_UNSUPPORTED"


def test_probe_copy():
    n = 1 << 22
    src = torch.randn(n, device="cuda")
    dst = torch.zeros(n, device="cuda")
    B.stencil_probe_copy(src, dst, n * 4)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    # A ragged size (not a multiple of the 4 x 256 vectors a workgroup moves per trip).
    m = 4 * (1000 * 4 + 3)
    dst2 = torch.zeros(n, device="cuda")
    B.stencil_probe_copy(src, dst2, m * 4)
    torch.cuda.synchronize()
    assert torch.equal(dst2[:m], src[:m]) and not dst2[m:].any()


def test_probe_streams():
    n = (1 << 20) + 12  # ragged: not a multiple of the 4096-vector trip
    srcs = [torch.randint(-2**31, 2**31 - 1, (n,), dtype=torch.int32, device="cuda") for _ in range(6)]
    dst = torch.zeros(n + 4, dtype=torch.int32, device="cuda")
    B.stencil_probe_streams(srcs, dst, n * 4)
    torch.cuda.synchronize()
    ref = srcs[0]
    for t in srcs[1:]:
        ref = torch.bitwise_xor(ref, t)
    assert torch.equal(dst[:n], ref) and not dst[n:].any()


def test_probe_read():
    n = 1 << 22
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    sink = torch.full((4,), 7, dtype=torch.int32, device="cuda")
    # All-equal 16-byte vectors cancel pairwise: every lane's checksum is 0.
    B.stencil_probe_read(src, n * 4, 1, sink)
    torch.cuda.synchronize()
    assert sink.tolist() == [7, 7, 7, 7]
    B.stencil_probe_read(src, n * 4, 0, sink)
    torch.cuda.synchronize()
    assert sink[0].item() == 0 and sink[1:].tolist() == [7, 7, 7]
