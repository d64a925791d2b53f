"""The method's closed-form cases through the HIP path (GPU only).

* A constant u: every Laplacian and flux is 0, so h = u exactly.
* u = s (i^4 + j^4) (s a power of two): every flux is kept (flx * du < 0 at
  every face) and h = u + 48 s coeff, exact in FP64 for coeff held in 24 bits.
  Its grid is 70 x 70 (still two tiles in i, the second ragged) so that 4u,
  and with it every partial sum of the Laplacian in any evaluation order,
  stays below 2^24 units of s: the stencil arithmetic is then exact in FP32
  too, and only the final update rounds.
* Unit spikes: h follows the hand-derived fixture tests/golden/hdiff_spike.txt
  exactly, including the fluxes that sit on a limiter tie (product exactly 0,
  kept).  Spikes sit on tile seams, at the ragged edges and in the halo.

Each goes through stencil_hdiff at every optimisation level (bitwise where the
closed form is exact in the storage type) and through the fused
stencil_hdiff_vadv against the FP64 oracle (1e-12 FP64, 1e-5 FP32).
"""
import os

import numpy as np
import pytest

import oracle
from helpers import DT, SEED, TOL, halo_untouched, normwise
from paper_2005_13014_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2005_13014_amd import binding as B  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NI, NJ, NK, H = 100, 70, 10, 2         # two 64-wide tiles (the second ragged), ragged rows;
                                        # nk >= 8 for the four-lanes-per-column schedule
LEVELS = {"original": B.config(level=1), "u1": B.config(unroll=1), "u2": B.config(unroll=2),
          "u4": B.config(unroll=4)}
SPIKES = [(0, 0), (NI - 1, NJ - 1), (63, 8), (64, 17), (-2, 30), (NI + 1, 44), (30, -1), (50, NJ + 1),
          (20, 15), (90, 55), (40, 62), (10, 50), (75, 30), (NI - 1, 4)]
SCALE = 2.0 ** -16


def note(*a):
    print(*a, flush=True)


def spike_rows():
    with open(os.path.join(GOLDEN, "hdiff_spike.txt")) as fh:
        return [[int(v) for v in ln.split()] for ln in fh if ln.strip() and not ln.lstrip().startswith("#")]


NI_QUARTIC = 70


def dims(case):
    """Interior extents (ni, nj, nk) of a case."""
    return (NI_QUARTIC if case == "quartic" else NI), NJ, NK


def grid(ni, nj, nk):
    k, j, i = np.meshgrid(np.arange(nk), np.arange(-H, nj + H), np.arange(-H, ni + H), indexing="ij")
    return k, j, i


def case_inputs(case):
    """Padded u and coeff (float64 holding values exact in every storage type)
    and the closed-form h on the interior."""
    ni, nj, nk = dims(case)
    rng = np.random.default_rng(SEED + 900)
    shape = (nk, nj + 2 * H, ni + 2 * H)
    coeff = inputs.round_to(rng.uniform(0.0, 0.1, shape), "bf16")
    if case == "constant":
        u = np.full(shape, 0.375)
        h = u[:, H:-H, H:-H].copy()
    elif case == "quartic":
        _, j, i = grid(ni, nj, nk)
        u = SCALE * ((i - 35.0) ** 4 + (j - 35.0) ** 4)
        assert 4 * u.max() / SCALE < 2 ** 24
        h = (u + 48.0 * SCALE * coeff)[:, H:-H, H:-H]
    else:
        c = 2.0 ** -4
        coeff = np.full(shape, c)
        u = np.zeros(shape)
        h = np.zeros((nk, nj, ni))
        for si, sj in SPIKES:
            u[:, sj + H, si + H] = 1.0
            for di, dj, base, mult in spike_rows():
                i, j = si + di, sj + dj
                if 0 <= i < ni and 0 <= j < nj:
                    h[:, j, i] += base + mult * c
        # the spikes are at least 6 cells apart in i or j: no two diamonds meet
        for p in range(len(SPIKES)):
            for q in range(p):
                assert max(abs(SPIKES[p][0] - SPIKES[q][0]), abs(SPIKES[p][1] - SPIKES[q][1])) >= 6
    return u, coeff, h


def exact_in(x, dtype):
    return np.array_equal(inputs.round_to(x, dtype), x)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("case", ["constant", "quartic", "spikes"])
@pytest.mark.parametrize("level", list(LEVELS))
def test_hdiff_closed_forms(dtype, case, level):
    if case == "quartic" and dtype == "bf16":
        pytest.skip("i^4 + j^4 is not exact in bfloat16")
    note("closed form", case, dtype, level)
    u, coeff, h = case_inputs(case)
    ni, nj, nk = dims(case)
    assert exact_in(u, dtype) and exact_in(coeff, dtype)
    gu = B.Field.from_numpy(u, H, dtype)
    gc = B.Field.from_numpy(coeff, H, dtype)
    out = B.Field.empty(ni, nj, nk, H, dtype, fill=-7.0)
    B.stencil_hdiff(gu, gc, out, cfg=LEVELS[level])
    torch.cuda.synchronize()
    got = out.to_numpy(interior=True)
    if exact_in(h, dtype):
        # constant and spikes everywhere; quartic in FP64
        assert np.array_equal(got, h), np.abs(got - h).max()
    else:
        # quartic in FP32: every Laplacian, flux and coeff * divergence is
        # exact (coeff has 8 significant bits, 48 s two); only u + that
        # product rounds
        ulp = np.spacing(np.abs(h).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(got - h) <= ulp), np.abs((got - h) / ulp).max()
    assert halo_untouched(out)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", ["constant", "quartic", "spikes"])
@pytest.mark.parametrize("schedule", [0, 1, 2, 4])
def test_fused_closed_forms(dtype, case, schedule):
    note("fused closed form", case, dtype, "schedule", schedule)
    u, coeff, h = case_inputs(case)
    ni, nj, nk = dims(case)
    f = inputs.fields(ni, nj, nk, H, seed=SEED + 901, storage=dtype)
    f["u"], f["coeff"] = u, coeff
    g = {n: B.Field.from_numpy(f[n], H, dtype) for n in ("u", "coeff", "wcon", "a", "b", "c")}
    x = B.Field.empty(ni, nj, nk, H, dtype, fill=-7.0)
    cfg = B.config(schedule=schedule) if schedule else None
    B.stencil_hdiff_vadv(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, x, cfg=cfg)
    torch.cuda.synchronize()
    got = x.to_numpy(interior=True)
    ref = oracle.hdiff_vadv(f["u"], H, f["coeff"], H, f["wcon"], H, f["a"], H, f["b"], H, f["c"], H, DT)
    # the oracle's hdiff stage reproduces the closed form (pinned on the CPU)
    assert np.allclose(oracle.hdiff(u, H, coeff, H), h, rtol=0, atol=1e-12 * max(1.0, np.abs(h).max()))
    err = normwise(got, ref)
    note("normwise %.2e" % err)
    assert err <= TOL[dtype]
    assert halo_untouched(x)
