"""The reverse pass that allocates nothing (stencil_hdiff_vadv_adjoint_noalloc)
against the one that uses library scratch (stencil_hdiff_vadv_adjoint), through
the C ABI: the same kernels on different scratch, so the gradients must agree
bit for bit.  Two calls in a row per storage type, the second smaller (the
fixed array then still holds the first call's larger planes), plus the size
limit of the fixed array (GPU only)."""
import numpy as np
import pytest

import oracle
from helpers import DT, SEED, interior, normwise
from paper_2005_13014_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2005_13014_amd import binding as B  # noqa: E402

NAMES = ("u", "coeff", "wcon", "a", "b", "c", "w")
OUTS = ("gu", "gcoeff", "gwcon", "ga", "gb", "gc")


def note(*a):
    print(*a, flush=True)


def run(entry, g, x):
    out = {n: g["u"].like(fill=-7.0) for n in OUTS}
    entry(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, g["w"], out["gu"], out["gcoeff"],
          out["gwcon"], x=x, ga=out["ga"], gb=out["gb"], gc=out["gc"])
    torch.cuda.synchronize()
    return {n: out[n].to_numpy() for n in OUTS}


def case(ni, nj, nk, dtype, seed):
    f = inputs.fields(ni, nj, nk, 2, seed=seed, storage=dtype, loss=True)
    g = {n: B.Field.from_numpy(f[n], 2, dtype) for n in NAMES}
    x = g["u"].like(fill=0.0)
    B.stencil_hdiff_vadv(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, x)
    return f, g, x


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_noalloc_adjoint_matches_the_scratch_entry_point(dtype):
    big = (256, 256, 80) if dtype == "f64" else (512, 512, 80)
    for n, shape in enumerate((big, (70, 13, 5))):
        note("noalloc adjoint", dtype, shape, "call", n + 1)
        f, g, x = case(*shape, dtype, SEED + 700 + n)
        fixed = run(B.stencil_hdiff_vadv_adjoint_noalloc, g, x)
        ref = run(B.stencil_hdiff_vadv_adjoint, g, x)
        for name in OUTS:
            assert np.array_equal(fixed[name], ref[name]), (dtype, shape, name)
        if dtype == "f64" and n == 1:
            # and both are the oracle's gradient (the small call, on the CPU)
            gu, gc, gw = oracle.hdiff_vadv_adjoint(
                f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2, f["b"], 2, f["c"], 2, DT,
                interior(f["w"], 2), 0)
            assert normwise(fixed["gu"], gu) <= 1e-12
            assert normwise(interior(fixed["gcoeff"], 2), gc) <= 1e-12
            assert normwise(interior(fixed["gwcon"], 2), gw) <= 1e-12


def test_noalloc_adjoint_refuses_more_than_its_fixed_scratch():
    # 512 x 512 x 80 in FP64 needs two planes of about 170 MB each
    f, g, _ = case(512, 512, 80, "f64", SEED + 710)
    out = {n: g["u"].like(fill=0.0) for n in ("gu", "gcoeff", "gwcon")}
    with pytest.raises(B.StencilError, match="fixed scratch"):
        B.stencil_hdiff_vadv_adjoint_noalloc(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, g["w"],
                                             out["gu"], out["gcoeff"], out["gwcon"])
    torch.cuda.synchronize()
    assert np.all(out["gu"].to_numpy() == 0)
