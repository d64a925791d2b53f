"""The largest problems the fused kernel takes (GPU only): the deepest
register-held column (96 levels) on a field whose addressed span sits just
below the 2 GiB that the kernel's 32-bit buffer offsets reach.  Inputs are
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


def device_inputs(ni, nj, dtype, seed):
    """u ~ U(-1, 1), coeff ~ U(0, 0.1), wcon ~ U(-1, 1), a, c ~ U(-0.4, 0)
    with a(0) = c(K-1) = 0, b = 1 + |a| + |c| + U(0, 0.2), on every padded cell."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    f = {n: B.Field.empty(ni, nj, NK, HALO, dtype, fill=0.0) for n in ("u", "coeff", "wcon", "a", "b", "c")}
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
    return f


def block(field, i0, j0, w, h, ring):
    """Padded float64 copy of interior columns [i0, i0 + w) x [j0, j0 + h)
    with `ring` cells around them."""
    p = field.padded()
    return p[:, HALO + j0 - ring:HALO + j0 + h + ring, HALO + i0 - ring:HALO + i0 + w + ring] \
        .detach().to("cpu", torch.float64).numpy().copy()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_fused_on_the_largest_field_its_buffers_address(dtype):
    es = 4 if dtype == "f32" else 8
    ni = 2357 if dtype == "f32" else 1660
    nj = largest_nj(ni, es)
    span = span_bytes(ni, nj, NK, es)
    assert span < SPAN_LIMIT <= span_bytes(ni, nj + 1, NK, es)
    note("largest fused field", dtype, (ni, nj, NK), "span %.4f of 2 GiB" % (span / 2.0 ** 31))
    f = device_inputs(ni, nj, dtype, SEED + 31)
    x = B.Field.empty(ni, nj, NK, HALO, dtype, fill=-7.0)
    # level 2 runs the fused kernel or refuses: no silent detour to the unfused kernels
    B.stencil_hdiff_vadv(f["u"], f["coeff"], f["wcon"], f["a"], f["b"], f["c"], DT, x, cfg=B.config(level=2))
    torch.cuda.synchronize()
    last_i = (ni - 1) // 64 * 64  # first column of the ragged last tile in i
    starts = [(0, 0), (ni - BLOCK, nj - BLOCK), (ni // 2, nj // 2), (last_i, nj // 3), (ni - BLOCK, 0),
              (0, nj - BLOCK)]
    worst = 0.0
    for i0, j0 in starts:
        i0, j0 = min(max(i0, 0), ni - BLOCK), min(max(j0, 0), nj - BLOCK)
        ins = {n: block(f[n], i0, j0, BLOCK, BLOCK, HALO) for n in f}
        ref = oracle.hdiff_vadv(ins["u"], HALO, ins["coeff"], HALO, ins["wcon"], HALO, ins["a"], HALO,
                                ins["b"], HALO, ins["c"], HALO, DT)
        got = block(x, i0, j0, BLOCK, BLOCK, 0)
        e = normwise(got, ref)
        worst = max(worst, e)
        assert e <= TOL[dtype], (i0, j0, e)
    note("  worst normwise %.3e over %d blocks" % (worst, len(starts)))
    del f, x
    torch.cuda.empty_cache()
