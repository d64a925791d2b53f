"""Horizontal domain decomposition on one device (GPU only): a grid split into
px x py shares, each a separate halo-padded field, with the halo exchange
between them and its transpose for gradients.

* After stencil_halo_exchange every share holds exactly the undivided grid's
  values on its interior and halo (bitwise), edges and corners alike, for
  even and uneven splits and halo widths 1 to 3; blocks on the outer
  boundary keep what they held.
* The fused hdiff + vadv kernel run share by share on exchanged halos gives
  bitwise the undivided run (the arithmetic of a column does not depend on
  where its tile sits), and the FP64 oracle's result to 1e-12.
* Per-share reverse passes followed by stencil_halo_accumulate give the
  undivided gradient: gcoeff and gwcon bitwise, gu (whose ring sums now run
  in another order) to the tolerance of the storage type, and the oracle's
  gradient to 1e-12 in FP64.
"""
import numpy as np
import pytest

import oracle
from helpers import DT, SEED, TOL, interior, normwise
from paper_2005_13014_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2005_13014_amd import binding as B  # noqa: E402

CANARY = 1.0e30
NAMES = ("u", "coeff", "wcon", "a", "b", "c")


def note(*a):
    print(*a, flush=True)


def starts(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(int)


def windows(g, h, nis, njs):
    """Padded windows of the padded global array g for every share, row-major
    (p fastest); halo cells toward a neighbour set to CANARY."""
    i0, j0 = starts(nis), starts(njs)
    px, py = len(nis), len(njs)
    out = []
    for q in range(py):
        for p in range(px):
            w = g[:, j0[q]:j0[q] + njs[q] + 2 * h, i0[p]:i0[p] + nis[p] + 2 * h].copy()
            if p > 0:
                w[:, :, :h] = CANARY
            if p < px - 1:
                w[:, :, -h:] = CANARY
            if q > 0:
                w[:, :h, :] = CANARY
            if q < py - 1:
                w[:, -h:, :] = CANARY
            out.append(w)
    return out


def share_fields(g, h, nis, njs, dtype):
    return [B.Field.from_numpy(w, h, dtype) for w in windows(g, h, nis, njs)]


def gather_interior(shares, nis, njs, nk):
    i0, j0 = starts(nis), starts(njs)
    out = np.empty((nk, j0[-1], i0[-1]))
    for n, f in enumerate(shares):
        p, q = n % len(nis), n // len(nis)
        out[:, j0[q]:j0[q + 1], i0[p]:i0[p + 1]] = f.to_numpy(interior=True)
    return out


def gather_padded(shares, h, nis, njs, nk):
    """The global padded array: interiors from every share, the outer ring
    from the boundary shares' halos."""
    i0, j0 = starts(nis), starts(njs)
    px, py = len(nis), len(njs)
    out = np.full((nk, j0[-1] + 2 * h, i0[-1] + 2 * h), np.nan)
    for n, f in enumerate(shares):
        p, q = n % px, n // px
        w = f.to_numpy()
        ilo = 0 if p == 0 else h
        ihi = w.shape[2] if p == px - 1 else w.shape[2] - h
        jlo = 0 if q == 0 else h
        jhi = w.shape[1] if q == py - 1 else w.shape[1] - h
        out[:, j0[q] + jlo:j0[q] + jhi, i0[p] + ilo:i0[p] + ihi] = w[:, jlo:jhi, ilo:ihi]
    return out


SPLITS = [
    ((40, 30, 30), (37, 33), 10),     # uneven 3 x 2, ragged tiles
    ((64, 36), (70,), 6),             # 2 x 1
    ((100,), (20, 25, 25), 6),        # 1 x 3
    ((25, 25, 25, 25), (35, 35), 4),  # 4 x 2
]


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("width", [1, 2, 3])
@pytest.mark.parametrize("split", range(len(SPLITS)))
def test_exchange_reproduces_the_undivided_grid(dtype, width, split):
    nis, njs, nk = SPLITS[split]
    note("halo exchange", dtype, "width", width, nis, njs, nk)
    g = inputs.round_to(np.random.default_rng(SEED + 800 + split).uniform(-1, 1, (nk, sum(njs) + 2 * width,
                                                                                 sum(nis) + 2 * width)), dtype)
    shares = share_fields(g, width, nis, njs, dtype)
    B.stencil_halo_exchange(shares, len(nis), len(njs), width)
    torch.cuda.synchronize()
    # every cell of every share, halo included, equals the undivided grid's
    # cell at that position (the halo blocks toward neighbours started as
    # CANARY; the outer boundary's halo cells kept the grid's halo data)
    i0, j0 = starts(nis), starts(njs)
    for n, f in enumerate(shares):
        p, q = n % len(nis), n // len(nis)
        ref = g[:, j0[q]:j0[q] + njs[q] + 2 * width, i0[p]:i0[p] + nis[p] + 2 * width]
        assert np.array_equal(f.to_numpy(), ref), (n, p, q)


def test_exchange_at_the_benchmarked_split():
    # 512 x 512 x 80 FP32 split 4 x 2 into 128 x 256 shares, width 2
    nis, njs, nk, h = (128,) * 4, (256,) * 2, 80, 2
    g = inputs.round_to(np.random.default_rng(SEED + 810).uniform(-1, 1, (nk, 512 + 2 * h, 512 + 2 * h)), "f32")
    shares = share_fields(g, h, nis, njs, "f32")
    B.stencil_halo_exchange(shares, 4, 2, h)
    torch.cuda.synchronize()
    i0, j0 = starts(nis), starts(njs)
    for n, f in enumerate(shares):
        p, q = n % 4, n // 4
        assert np.array_equal(f.to_numpy(), g[:, j0[q]:j0[q] + njs[q] + 2 * h, i0[p]:i0[p] + nis[p] + 2 * h])


TWO_LANES = B.config(schedule=2)   # the pipelined two-lanes-per-column kernel at any size


def run_fused(fs, h, dtype, cfg):
    g = {n: B.Field.from_numpy(fs[n], h, dtype) for n in NAMES}
    x = B.Field.empty(g["u"].ni, g["u"].nj, g["u"].nk, h, dtype, fill=0.0)
    B.stencil_hdiff_vadv(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, x, cfg=cfg)
    return x


def decomposed_fused(f, nis, njs, dtype, cfg, h=2):
    """Per-share fields (u exchanged on the device), fused kernel per share."""
    px, py = len(nis), len(njs)
    parts = {n: share_fields(f[n], h, nis, njs, dtype) for n in NAMES}
    B.stencil_halo_exchange(parts["u"], px, py, h)
    xs = []
    for s in range(px * py):
        x = parts["u"][s].like(fill=0.0)
        B.stencil_hdiff_vadv(*[parts[n][s] for n in NAMES], DT, x, cfg=cfg)
        xs.append(x)
    torch.cuda.synchronize()
    return parts, xs


@pytest.mark.parametrize("dtype,nis,njs,nk", [
    ("f64", (40, 30, 30), (37, 33), 20),
    ("f32", (40, 30, 30), (37, 33), 20),
    ("bf16", (64, 36), (20, 25, 25), 12),
    ("f32", (128,) * 4, (256,) * 2, 80),   # 512 x 512 x 80, the benchmarked split
])
def test_fused_per_share_equals_the_undivided_run(dtype, nis, njs, nk):
    note("decomposed fused", dtype, nis, njs, nk)
    ni, nj = sum(nis), sum(njs)
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 820, storage=dtype)
    # one kernel variant for the whole grid and the shares: bitwise equal
    whole = run_fused(f, 2, dtype, TWO_LANES).to_numpy(interior=True)
    _, xs = decomposed_fused(f, nis, njs, dtype, TWO_LANES)
    assert np.array_equal(gather_interior(xs, nis, njs, nk), whole)
    # the library's own choice for each size (small shares take four lanes
    # per column, another order of the same solve)
    _, xs = decomposed_fused(f, nis, njs, dtype, None)
    got = gather_interior(xs, nis, njs, nk)
    if dtype == "f64":
        ref = oracle.hdiff_vadv(f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2, f["b"], 2, f["c"], 2, DT)
        assert normwise(got, ref) <= TOL["f64"]
    else:
        assert normwise(got, whole) <= TOL[dtype]


@pytest.mark.parametrize("dtype,nis,njs,nk", [
    ("f64", (40, 30, 30), (37, 33), 20),
    ("f64", (64, 64), (32, 32, 64), 60),
    ("f32", (128, 128), (128, 128), 80),   # 256 x 256 x 80 in 2 x 2 shares
    ("bf16", (64, 36), (20, 25, 25), 12),
])
def test_adjoint_per_share_with_halo_accumulate(dtype, nis, njs, nk):
    note("decomposed adjoint", dtype, nis, njs, nk)
    px, py = len(nis), len(njs)
    ni, nj = sum(nis), sum(njs)
    f = inputs.fields(ni, nj, nk, 2, seed=SEED + 830, storage=dtype, loss=True)
    # undivided
    g = {n: B.Field.from_numpy(f[n], 2, dtype) for n in NAMES + ("w",)}
    whole = {n: g["u"].like(fill=0.0) for n in ("gu", "gcoeff", "gwcon")}
    B.stencil_hdiff_vadv_adjoint(*[g[n] for n in NAMES], DT, g["w"], whole["gu"], whole["gcoeff"], whole["gwcon"])
    # per share: u exchanged, reverse pass, then the gradient ring folded back
    parts = {n: share_fields(f[n], 2, nis, njs, dtype) for n in NAMES + ("w",)}
    B.stencil_halo_exchange(parts["u"], px, py, 2)
    outs = {n: [] for n in ("gu", "gcoeff", "gwcon")}
    for s in range(px * py):
        o = {n: parts["u"][s].like(fill=0.0) for n in outs}
        B.stencil_hdiff_vadv_adjoint(*[parts[n][s] for n in NAMES], DT, parts["w"][s], o["gu"], o["gcoeff"],
                                     o["gwcon"])
        for n in outs:
            outs[n].append(o[n])
    B.stencil_halo_accumulate(outs["gu"], px, py, 2)
    torch.cuda.synchronize()
    gu = gather_padded(outs["gu"], 2, nis, njs, nk)
    gc = gather_interior(outs["gcoeff"], nis, njs, nk)
    gw = gather_interior(outs["gwcon"], nis, njs, nk)
    assert np.array_equal(gc, whole["gcoeff"].to_numpy(interior=True))
    assert np.array_equal(gw, whole["gwcon"].to_numpy(interior=True))
    ref_gu = whole["gu"].to_numpy()
    err = normwise(gu, ref_gu)
    note("gu normwise vs undivided %.2e" % err)
    assert err <= {"f64": 1e-14, "f32": 1e-6, "bf16": TOL["bf16"]}[dtype]
    if dtype == "f64":
        o_gu, o_gc, o_gw = oracle.hdiff_vadv_adjoint(f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2, f["b"], 2,
                                                     f["c"], 2, DT, interior(f["w"], 2), 0)
        assert normwise(gu, o_gu) <= TOL["f64"]
        assert normwise(gc, o_gc) <= TOL["f64"]
        assert normwise(gw, o_gw) <= TOL["f64"]


def test_accumulate_is_the_transpose_of_the_exchange():
    # <E x, y> = <x, E^T y> over the shares' whole padded arrays, FP64:
    # E copies interior cells into neighbours' halos (and keeps everything
    # else); E^T adds halo cells toward neighbours into the cells they copy.
    nis, njs, nk, h = (7, 9, 8), (6, 10), 3, 2
    rng = np.random.default_rng(SEED + 840)
    px, py = len(nis), len(njs)
    x = [rng.standard_normal((nk, nj + 2 * h, ni + 2 * h)) for nj in njs for ni in nis]
    y = [rng.standard_normal(a.shape) for a in x]
    fx = [B.Field.from_numpy(a, h, "f64") for a in x]
    fy = [B.Field.from_numpy(a, h, "f64") for a in y]
    B.stencil_halo_exchange(fx, px, py, h)
    B.stencil_halo_accumulate(fy, px, py, h)
    torch.cuda.synchronize()
    ex = [f.to_numpy() for f in fx]
    ety = [f.to_numpy() for f in fy]

    # E zeroes nothing: halo cells toward neighbours are overwritten.  As a
    # linear map on the concatenated arrays, E = P + C where C writes the
    # copies; E^T y then keeps y on cells E keeps and folds the halo cells
    # toward neighbours into their sources, with those halo cells themselves
    # contributing nothing (their old values are overwritten by E).
    def toward(p, q):
        m = np.zeros((nk, njs[q] + 2 * h, nis[p] + 2 * h), bool)
        if p > 0:
            m[:, :, :h] = True
        if p < px - 1:
            m[:, :, -h:] = True
        if q > 0:
            m[:, :h, :] = True
        if q < py - 1:
            m[:, -h:, :] = True
        return m

    lhs = sum(float(np.sum(a * b)) for a, b in zip(ex, y))
    rhs = 0.0
    for n, (a, b) in enumerate(zip(x, ety)):
        m = toward(n % px, n // px)
        rhs += float(np.sum(a[~m] * b[~m]))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
