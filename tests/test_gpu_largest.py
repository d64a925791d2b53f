"""The largest problems the buffer-addressed kernels take (GPU only): the
deepest register-held column (96 levels) on a field whose addressed span sits
just below the 2 GiB that the kernels' 32-bit buffer offsets reach, for the
fused kernel, hdiff alone, the reverse pass and the forward mode.  Inputs are
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


def span_bytes(ni, nj, nk, es):
    """Bytes from u's cell (-2, -2, 0) to its last interior cell, for the
    layout binding.Field.empty gives (rows padded to 128-byte lines)."""
    row = -(-(ni + 2 * HALO) // (128 // es)) * (128 // es)
    plane = row * (nj + 2 * HALO)
    return ((ni + 3) + (nj + 3) * row + (nk - 1) * plane + 1) * es


def largest_nj(ni, es):
    nj = 1
    while span_bytes(ni, nj + 1, NK, es) < SPAN_LIMIT:
        nj += 1
    return nj


def device_inputs(ni, nj, dtype, seed, extra=()):
    """u ~ U(-1, 1), coeff ~ U(0, 0.1), wcon ~ U(-1, 1), a, c ~ U(-0.4, 0)
    with a(0) = c(K-1) = 0, b = 1 + |a| + |c| + U(0, 0.2), on every padded cell;
    each name in `extra` (a loss weight or a tangent) ~ N(0, 1)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    names = ("u", "coeff", "wcon", "a", "b", "c") + tuple(extra)
    f = {n: B.Field.empty(ni, nj, NK, HALO, dtype, fill=0.0) for n in names}
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


def edge_shape(dtype):
    es = 4 if dtype == "f32" else 8
    ni = 2357 if dtype == "f32" else 1660
    nj = largest_nj(ni, es)
    span = span_bytes(ni, nj, NK, es)
    assert span < SPAN_LIMIT <= span_bytes(ni, nj + 1, NK, es)
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
    p = field.padded()
    return p[:, HALO + j0 - ring:HALO + j0 + h + ring, HALO + i0 - ring:HALO + i0 + w + ring] \
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
