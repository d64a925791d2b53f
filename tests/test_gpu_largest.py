"""The largest problems the buffer-addressed kernels take (GPU only): the
deepest register-held column (96 levels) on a field whose addressed span sits
just below the 2 GiB that the kernels' 32-bit buffer offsets reach, for the
fused kernel, hdiff alone, the reverse pass, the forward mode and the batched
timestep.  Inputs are
drawn on the device with a seeded generator, in the distributions of the
shared input module; column blocks at the corners, in the middle and in the
ragged last tile are copied back and checked against the FP64 oracle."""
import sys

import numpy as np
import pytest

import oracle
from helpers import DT, SEED, TOL, normwise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2005_13014_amd import binding as B  # noqa: E402

NK = 96        # deepest column the fused kernel holds in registers
HALO = 2
SPAN_LIMIT = 2 ** 31 - 1  # bytes a column-kernel buffer can address
BLOCK = 12


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def span_bytes(ni, nj, nk, es, halo=HALO, reach=2):
    """Bytes a kernel addresses from cell (-reach, -reach, 0) to the last cell
    its reads reach on the far side (reach - 1 beyond the interior), for the
    layout binding.Field.empty gives (rows padded to 128-byte lines)."""
    row = -(-(ni + 2 * halo) // (128 // es)) * (128 // es)
    plane = row * (nj + 2 * halo)
    return ((ni + 2 * reach - 1) + (nj + 2 * reach - 1) * row + (nk - 1) * plane + 1) * es


def largest_nj(ni, es, halo=HALO, reach=2):
    nj = 1
    while span_bytes(ni, nj + 1, NK, es, halo, reach) < SPAN_LIMIT:
        nj += 1
    return nj


def device_inputs(ni, nj, dtype, seed, extra=(), halo=HALO):
    """u ~ U(-1, 1), coeff ~ U(0, 0.1), wcon ~ U(-1, 1), a, c ~ U(-0.4, 0)
    with a(0) = c(K-1) = 0, b = 1 + |a| + |c| + U(0, 0.2), on every padded cell;
    each name in `extra` (a loss weight or a tangent) ~ N(0, 1)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    names = ("u", "coeff", "wcon", "a", "b", "c") + tuple(extra)
    f = {n: B.Field.empty(ni, nj, NK, halo, dtype, fill=0.0) for n in names}
    f["u"].padded().uniform_(-1.0, 1.0, generator=g)
    f["coeff"].padded().uniform_(0.0, 0.1, generator=g)
    f["wcon"].padded().uniform_(-1.0, 1.0, generator=g)
    f["a"].padded().uniform_(-0.4, 0.0, generator=g)
    f["c"].padded().uniform_(-0.4, 0.0, generator=g)
    f["a"].padded()[0].zero_()
    f["c"].padded()[NK - 1].zero_()
    b = f["b"].padded()
    b.uniform_(0.0, 0.2, generator=g)
    b.add_(f["a"].padded().abs()).add_(f["c"].padded().abs()).add_(1.0)
    for n in extra:
        f[n].padded().normal_(generator=g)
    return f


def edge_shape(dtype, halo=HALO, reach=2):
    es = 4 if dtype == "f32" else 8
    ni = 2357 if dtype == "f32" else 1660
    nj = largest_nj(ni, es, halo, reach)
    span = span_bytes(ni, nj, NK, es, halo, reach)
    assert span < SPAN_LIMIT <= span_bytes(ni, nj + 1, NK, es, halo, reach)
    note("largest field", dtype, (ni, nj, NK), "span %.4f of 2 GiB" % (span / 2.0 ** 31))
    return ni, nj


def block_starts(ni, nj):
    """Corners, middle, and a block in the ragged last tile in i."""
    last_i = (ni - 1) // 64 * 64
    starts = [(0, 0), (ni - BLOCK, nj - BLOCK), (ni // 2, nj // 2), (last_i, nj // 3), (ni - BLOCK, 0),
              (0, nj - BLOCK)]
    return [(min(max(i0, 0), ni - BLOCK), min(max(j0, 0), nj - BLOCK)) for i0, j0 in starts]


def block(field, i0, j0, w, h, ring):
    """Padded float64 copy of interior columns [i0, i0 + w) x [j0, j0 + h)
    with `ring` cells around them."""
    p, o = field.padded(), field.hi
    return p[:, o + j0 - ring:o + j0 + h + ring, o + i0 - ring:o + i0 + w + ring] \
        .detach().to("cpu", torch.float64).numpy().copy()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_fused_on_the_largest_field_its_buffers_address(dtype):
    ni, nj = edge_shape(dtype)
    f = device_inputs(ni, nj, dtype, SEED + 31)
    x = B.Field.empty(ni, nj, NK, HALO, dtype, fill=-7.0)
    # level 2 runs the fused kernel or refuses: no silent detour to the unfused kernels
    B.stencil_hdiff_vadv(f["u"], f["coeff"], f["wcon"], f["a"], f["b"], f["c"], DT, x, cfg=B.config(level=2))
    torch.cuda.synchronize()
    worst = 0.0
    for i0, j0 in block_starts(ni, nj):
        ins = {n: block(f[n], i0, j0, BLOCK, BLOCK, HALO) for n in f}
        ref = oracle.hdiff_vadv(ins["u"], HALO, ins["coeff"], HALO, ins["wcon"], HALO, ins["a"], HALO,
                                ins["b"], HALO, ins["c"], HALO, DT)
        e = normwise(block(x, i0, j0, BLOCK, BLOCK, 0), ref)
        worst = max(worst, e)
        assert e <= TOL[dtype], (i0, j0, e)
    note("  worst normwise %.3e" % worst)
    del f, x
    torch.cuda.empty_cache()


def test_hdiff_on_the_largest_field_its_buffers_address():
    """The inlined hdiff kernel (level 2: it runs or refuses) in FP32."""
    ni, nj = edge_shape("f32")
    f = device_inputs(ni, nj, "f32", SEED + 32)
    out = B.Field.empty(ni, nj, NK, HALO, "f32", fill=-7.0)
    B.stencil_hdiff(f["u"], f["coeff"], out, cfg=B.config(level=2))
    torch.cuda.synchronize()
    worst = 0.0
    for i0, j0 in block_starts(ni, nj):
        ref = oracle.hdiff(block(f["u"], i0, j0, BLOCK, BLOCK, HALO), HALO,
                           block(f["coeff"], i0, j0, BLOCK, BLOCK, HALO), HALO)
        e = normwise(block(out, i0, j0, BLOCK, BLOCK, 0), ref)
        worst = max(worst, e)
        assert e <= TOL["f32"], (i0, j0, e)
    note("  worst normwise %.3e" % worst)
    del f, out
    torch.cuda.empty_cache()


def test_adjoint_on_the_largest_field_its_buffers_address():
    """Reverse pass in FP64 (whose limiter decisions are the oracle's).  The
    gradients on a block depend on the loss weights within 2 columns of it and
    on the inputs within 4 (the limiter decisions of those columns), so the
    oracle runs on the block grown by 4 columns (clipped at the domain) and
    the block itself is compared."""
    ni, nj = edge_shape("f64")
    f = device_inputs(ni, nj, "f64", SEED + 33, extra=("w",))
    out = {n: B.Field.empty(ni, nj, NK, HALO, "f64", fill=0.0) for n in ("gu", "gcoeff", "gwcon")}
    B.stencil_hdiff_vadv_adjoint(f["u"], f["coeff"], f["wcon"], f["a"], f["b"], f["c"], DT, f["w"],
                                 out["gu"], out["gcoeff"], out["gwcon"])
    torch.cuda.synchronize()
    worst = 0.0
    for i0, j0 in block_starts(ni, nj):
        si, sj = max(i0 - 4, 0), max(j0 - 4, 0)
        wi, wj = min(i0 + BLOCK + 4, ni) - si, min(j0 + BLOCK + 4, nj) - sj
        ins = {n: block(f[n], si, sj, wi, wj, HALO) for n in f}
        gu, gc, gw = oracle.hdiff_vadv_adjoint(ins["u"], HALO, ins["coeff"], HALO, ins["wcon"], HALO, ins["a"],
                                               HALO, ins["b"], HALO, ins["c"], HALO, DT,
                                               ins["w"][:, HALO:-HALO, HALO:-HALO], 0)
        oi, oj = i0 - si, j0 - sj  # the block inside the grown one
        pairs = ((block(out["gu"], i0, j0, BLOCK, BLOCK, 0),
                  gu[:, HALO + oj:HALO + oj + BLOCK, HALO + oi:HALO + oi + BLOCK]),
                 (block(out["gcoeff"], i0, j0, BLOCK, BLOCK, 0), gc[:, oj:oj + BLOCK, oi:oi + BLOCK]),
                 (block(out["gwcon"], i0, j0, BLOCK, BLOCK, 0), gw[:, oj:oj + BLOCK, oi:oi + BLOCK]))
        for got, ref in pairs:
            e = normwise(got, ref)
            worst = max(worst, e)
            assert e <= TOL["f64"], (i0, j0, e)
    note("  worst normwise %.3e" % worst)
    del f, out
    torch.cuda.empty_cache()


def test_jvp_on_the_largest_field_its_buffers_address():
    """Forward mode in FP64 in the direction du: the tangent of a column
    depends on u and du within 2 columns of it."""
    ni, nj = edge_shape("f64")
    f = device_inputs(ni, nj, "f64", SEED + 34, extra=("du",))
    dx = B.Field.empty(ni, nj, NK, HALO, "f64", fill=-7.0)
    B.stencil_hdiff_vadv_jvp(f["u"], f["coeff"], f["wcon"], f["a"], f["b"], f["c"], DT, dx, du=f["du"])
    torch.cuda.synchronize()
    worst = 0.0
    for i0, j0 in block_starts(ni, nj):
        ins = {n: block(f[n], i0, j0, BLOCK, BLOCK, HALO) for n in f}
        ref = oracle.hdiff_vadv_jvp(ins["u"], HALO, ins["coeff"], HALO, ins["wcon"], HALO, ins["a"], HALO,
                                    ins["b"], HALO, ins["c"], HALO, DT, du=ins["du"], hdu=HALO)
        e = normwise(block(dx, i0, j0, BLOCK, BLOCK, 0), ref)
        worst = max(worst, e)
        assert e <= TOL["f64"], (i0, j0, e)
    note("  worst normwise %.3e" % worst)
    del f, dx
    torch.cuda.empty_cache()


def test_timestep_on_the_largest_subdomain_its_buffers_address():
    """hdiff -> vadv -> vdiff -> hgrad on one FP32 subdomain whose fields (halo
    3: hgrad's ring plus hdiff's) span just below 2 GiB from the cell the
    program kernels address first, (-3, -3, 0).  z on a block depends on u
    within 3 columns of it."""
    kappa, bh, bv = 0.1, 0.05, 0.01
    ni, nj = edge_shape("f32", halo=3, reach=3)
    f = device_inputs(ni, nj, "f32", SEED + 35, halo=3)
    z = B.Field.empty(ni, nj, NK, 3, "f32", fill=-7.0)
    sub = {n: f[n] for n in ("coeff", "wcon", "a", "b", "c")}
    sub["u"], sub["z"] = [f["u"]], [z]
    stages = B.STAGE_HDIFF | B.STAGE_VADV | B.STAGE_VDIFF | B.STAGE_HGRAD
    B.stencil_program_run(B.ProgramSpec([sub], stages=stages, dt=DT, kappa=kappa, beta_h=bh, beta_v=bv))
    torch.cuda.synchronize()
    worst = 0.0
    for i0, j0 in block_starts(ni, nj):
        ins = {n: block(f[n], i0, j0, BLOCK, BLOCK, 3) for n in f}
        ref = oracle.timestep(ins["u"], 3, ins["coeff"], 3, ins["wcon"], 3, ins["a"], 3, ins["b"], 3, ins["c"], 3,
                              DT, kappa, bh, bv)
        e = normwise(block(z, i0, j0, BLOCK, BLOCK, 0), ref)
        worst = max(worst, e)
        assert e <= TOL["f32"], (i0, j0, e)
    note("  worst normwise %.3e" % worst)
    del f, z, sub
    torch.cuda.empty_cache()
