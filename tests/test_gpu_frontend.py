"""Programs compiled by the stencil front end, run on the GPU, against the
FP64 oracle (GPU only)."""
import numpy as np
import pytest

import oracle
from helpers import SEED, TOL, halo_untouched, limiter_masks, normwise
from paper_2005_13014_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2005_13014_amd import binding as B  # noqa: E402
from paper_2005_13014_amd import frontend as F  # noqa: E402


def note(*a):
    print(*a, flush=True)


def run_hdiff(f, dtype, unroll, tiled=False):
    u = B.Field.from_numpy(f["u"], 2, dtype)
    coeff = B.Field.from_numpy(f["coeff"], 2, dtype)
    out = u.like(fill=-7.0)
    k = F.compile_program(F.hdiff_program(), dtype, like=u, unroll=unroll, tiled=tiled)
    try:
        k({"u": u, "coeff": coeff}, {"out": out})
        torch.cuda.synchronize()
    finally:
        k.close()
    return out


@pytest.mark.parametrize("tiled", [False, True])
@pytest.mark.parametrize("unroll", [1, 2, 4])
@pytest.mark.parametrize("shape", [(64, 64, 60), (70, 13, 5), (131, 9, 7), (3, 2, 1)])
def test_generated_hdiff_fp64(shape, unroll, tiled):
    ni, nj, nk = shape
    note("front end hdiff f64", shape, unroll, tiled)
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 70, storage="f64", vadv=False)
    out = run_hdiff(f, "f64", unroll, tiled)
    err = normwise(out.to_numpy(interior=True), oracle.hdiff(f["u"], 2, f["coeff"], 2))
    note("normwise %.2e" % err)
    assert err <= TOL["f64"]
    assert halo_untouched(out)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("tiled", [False, True])
@pytest.mark.parametrize("unroll", [1, 4])
def test_generated_hdiff_low_precision_under_its_own_masks(unroll, tiled, dtype):
    ni, nj, nk = 99, 17, 12
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 71, storage=dtype, vadv=False)
    kx, ky = limiter_masks(f["u"], 2, dtype)
    ref = oracle.hdiff(f["u"], 2, f["coeff"], 2, force_kx=kx, force_ky=ky)
    out = run_hdiff(f, dtype, unroll, tiled)
    err = normwise(out.to_numpy(interior=True), ref)
    note("front end hdiff %s normwise %.2e" % (dtype, err))
    assert err <= TOL[dtype]
    assert halo_untouched(out)


@pytest.mark.parametrize("tiled", [False, True])
def test_generated_hdiff_f32_at_the_benchmarked_size(tiled):
    """512 x 512 x 80 FP32, every unroll factor the benchmark times: every
    element against the FP64 oracle under the FP32 limiter decisions."""
    ni, nj, nk = 512, 512, 80
    note("front end hdiff f32 512x512x80 tiled=%s" % tiled)
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 1, storage="f32", vadv=False)
    kx, ky = limiter_masks(f["u"], 2, "f32")
    ref = oracle.hdiff(f["u"], 2, f["coeff"], 2, force_kx=kx, force_ky=ky)
    for unroll in (1, 2, 4):
        out = run_hdiff(f, "f32", unroll, tiled)
        err = normwise(out.to_numpy(interior=True), ref)
        note("unroll %d normwise %.2e" % (unroll, err))
        assert err <= TOL["f32"]
        assert halo_untouched(out)


def test_generated_biharmonic():
    # A program the hand-written kernels do not cover: out = u - c lap(lap(u)).
    p = F.Program()
    u, c = p.input("u"), p.input("c")
    lap = p.apply("lap", 4.0 * u[0, 0] - u[1, 0] - u[-1, 0] - u[0, 1] - u[0, -1])
    lap2 = p.apply("lap2", 4.0 * lap[0, 0] - lap[1, 0] - lap[-1, 0] - lap[0, 1] - lap[0, -1])
    out = p.apply("out", u[0, 0] - c[0, 0] * lap2[0, 0])
    p.output(out)
    assert F.infer_shapes(p)[1]["u"] == (2, 2, 2, 2)
    ni, nj, nk = 77, 21, 6
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 72, storage="f64", vadv=False)
    l1 = oracle.lap(f["u"], 2, e=1)
    l2 = oracle.lap(l1, 1, e=0)
    ref = f["u"][:, 2:-2, 2:-2] - f["coeff"][:, 2:-2, 2:-2] * l2
    ug = B.Field.from_numpy(f["u"], 2, "f64")
    cg = B.Field.from_numpy(f["coeff"], 2, "f64")
    og = ug.like(fill=-7.0)
    for tiled in (False, True):
        og.buf.fill_(-7.0)
        k = F.compile_program(p, "f64", like=ug, unroll=2, tiled=tiled)
        k({"u": ug, "c": cg}, {"out": og})
        torch.cuda.synchronize()
        k.close()
        assert normwise(og.to_numpy(interior=True), ref) <= TOL["f64"]
        assert halo_untouched(og)


def test_halo_and_layout_checks():
    f = inputs.fields(16, 8, 2, 2, seed=SEED + 73, storage="f64", vadv=False)
    u = B.Field.from_numpy(f["u"], 2, "f64")
    coeff = B.Field.from_numpy(f["coeff"], 2, "f64")
    k = F.compile_program(F.hdiff_program(), "f64", like=u)
    try:
        thin = B.Field.from_numpy(f["u"][:, 1:-1, 1:-1], 1, "f64")
        with pytest.raises(ValueError):
            k({"u": thin, "coeff": coeff}, {"out": u.like(fill=0.0)})
        other = B.Field.from_numpy(inputs.fields(17, 8, 2, 2, seed=1, vadv=False)["u"], 2, "f64")
        with pytest.raises(ValueError):
            k({"u": other, "coeff": coeff}, {"out": u.like(fill=0.0)})
    finally:
        k.close()


@pytest.mark.parametrize("tiled", [False, True])
def test_two_outputs(tiled):
    # A program may return several applies: here the Laplacian and the update.
    p = F.hdiff_program()
    lap = next(a for a in p.applies if a.name == "lap")
    p.output(lap)
    assert [o.name for o in p.outputs] == ["out", "lap"]
    ni, nj, nk = 70, 11, 4
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 74, storage="f64", vadv=False)
    u = B.Field.from_numpy(f["u"], 2, "f64")
    coeff = B.Field.from_numpy(f["coeff"], 2, "f64")
    out, lp = u.like(fill=-7.0), u.like(fill=-7.0)
    with F.compile_program(p, "f64", like=u, unroll=2, tiled=tiled) as k:
        k({"u": u, "coeff": coeff}, {"out": out, "lap": lp})
        torch.cuda.synchronize()
    assert normwise(out.to_numpy(interior=True), oracle.hdiff(f["u"], 2, f["coeff"], 2)) <= TOL["f64"]
    assert normwise(lp.to_numpy(interior=True), oracle.lap(f["u"], 2)) <= TOL["f64"]
    assert halo_untouched(out) and halo_untouched(lp)
