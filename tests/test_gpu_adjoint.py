"""Reverse mode on the GPU: the hand-written adjoint against the FP64 oracle's
gradient, against central finite differences of the GPU forward pass, and
through torch.autograd (GPU only)."""
import sys

import numpy as np
import pytest

import oracle
from helpers import DT, SEED, TOL, interior, limiter_masks, normwise, rms_rel
from paper_2005_13014_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2005_13014_amd import binding as B  # noqa: E402
from paper_2005_13014_amd import autograd as AG  # noqa: E402

NAMES = ("u", "coeff", "wcon", "a", "b", "c", "w")


def note(*a):
    print(*a, flush=True)


def setup(ni, nj, nk, dtype, seed):
    f = inputs.fields(ni, nj, nk, 2, seed=seed, storage=dtype, loss=True)
    g = {n: B.Field.from_numpy(f[n], 2, dtype) for n in NAMES}
    return f, g


def gpu_adjoint(g, dtype):
    out = {n: g["u"].like(fill=0.0) for n in ("gu", "gcoeff", "gwcon")}
    B.stencil_hdiff_vadv_adjoint(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, g["w"],
                                 out["gu"], out["gcoeff"], out["gwcon"])
    torch.cuda.synchronize()
    return out


def oracle_adjoint(f, masks=None):
    kx, ky = masks if masks is not None else (None, None)
    return oracle.hdiff_vadv_adjoint(f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2, f["b"], 2,
                                     f["c"], 2, DT, interior(f["w"], 2), 0, force_kx=kx, force_ky=ky)


def check(out, ref, tol, label):
    gu, gc, gw = ref
    got_u = out["gu"].to_numpy()                    # padded, halo 2
    got_c = out["gcoeff"].to_numpy(interior=True)
    got_w = out["gwcon"].to_numpy(interior=True)
    errs = (normwise(got_u, gu), normwise(got_c, gc), normwise(got_w, gw))
    note(label, "normwise gu %.2e gcoeff %.2e gwcon %.2e" % errs,
         "rms %.2e" % max(rms_rel(got_u, gu), rms_rel(got_c, gc), rms_rel(got_w, gw)))
    assert max(errs) <= tol, errs
    # Nothing outside the interior and the 2-cell ring is written.
    assert np.all(out["gcoeff"].to_numpy()[:, :2] == 0) and np.all(out["gwcon"].to_numpy()[:, :, :2] == 0)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("shape", [(64, 64, 60), (70, 13, 5), (3, 2, 1), (131, 9, 96), (117, 61, 7), (256, 256, 80)])
def test_register_strips_equal_lds_tiles(dtype, shape):
    """The hdiff adjoint on register strips with cross-lane neighbours
    (default) and on LDS-staged tiles (schedule 1) perform the same
    operations: bitwise equal gradients, strip seams and ragged edges
    included."""
    ni, nj, nk = shape
    f, g = setup(ni, nj, nk, dtype, SEED + 55)
    cfgs = [B.config(schedule=1), B.config()]
    cfgs += [B.config(tile_j=tj, prefetch=pf) for tj in ((4,) if dtype == "f64" else (4, 8)) for pf in (1, 2)]
    if dtype != "f64":
        cfgs.append(B.config(tile_j=12, prefetch=1))
    outs = []
    for cfg in cfgs:
        o = {n: g["u"].like(fill=-7.0) for n in ("gu", "gcoeff", "gwcon")}
        B.stencil_hdiff_vadv_adjoint(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, g["w"],
                                     o["gu"], o["gcoeff"], o["gwcon"], cfg=cfg)
        torch.cuda.synchronize()
        outs.append({n: o[n].to_numpy() for n in o})
    for q in range(1, len(outs)):
        for n in ("gu", "gcoeff", "gwcon"):
            assert np.array_equal(outs[q][n], outs[0][n]), (q, n)


@pytest.mark.parametrize("shape", [(64, 64, 60), (70, 13, 5), (3, 2, 1), (131, 9, 96)])
def test_adjoint_fp64_matches_oracle(shape):
    ni, nj, nk = shape
    f, g = setup(ni, nj, nk, "f64", SEED + 50)
    check(gpu_adjoint(g, "f64"), oracle_adjoint(f), 1e-12, "adjoint f64 %s" % (shape,))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("shape", [(64, 64, 60), (99, 17, 33)])
def test_adjoint_low_precision_under_its_own_masks(dtype, shape):
    # The limiter decisions of an FP32 forward pass can differ from FP64 ones
    # where a flux sits within rounding of the switch; the gradient jumps there,
    # so the FP32 adjoint is compared with the oracle's adjoint evaluated under
    # the FP32 decisions.
    ni, nj, nk = shape
    f, g = setup(ni, nj, nk, dtype, SEED + 51)
    masks = limiter_masks(f["u"], 2, dtype)
    _, _, _, kx, ky = oracle.hdiff(f["u"], 2, f["coeff"], 2, fluxes=True)
    flips = int((masks[0] != kx).sum() + (masks[1] != ky).sum())
    note("%s %s: %d limiter decisions differ from FP64" % (dtype, shape, flips))
    tol = 1e-5 if dtype == "f32" else 2.0 ** -7
    check(gpu_adjoint(g, dtype), oracle_adjoint(f, masks), tol, "adjoint %s %s" % (dtype, shape))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_adjoint_config5_256x256x80(dtype):
    """Reverse mode of hdiff + vadv on 256 x 256 x 80 in FP32 and FP64."""
    f, g = setup(256, 256, 80, dtype, SEED + 5)
    masks = None if dtype == "f64" else limiter_masks(f["u"], 2, dtype)
    check(gpu_adjoint(g, dtype), oracle_adjoint(f, masks), TOL[dtype], "C5 adjoint %s" % dtype)


def gpu_matrix_adjoint(g, dtype, x, fill=-7.0):
    out = {n: g["u"].like(fill=fill) for n in ("gu", "gcoeff", "gwcon", "ga", "gb", "gc")}
    B.stencil_hdiff_vadv_adjoint(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, g["w"],
                                 out["gu"], out["gcoeff"], out["gwcon"], x=x, ga=out["ga"],
                                 gb=out["gb"], gc=out["gc"])
    torch.cuda.synchronize()
    return out


def gpu_forward(g):
    x = g["u"].like(fill=0.0)
    B.stencil_hdiff_vadv(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, x)
    torch.cuda.synchronize()
    return x


@pytest.mark.parametrize("dtype,shape", [("f64", (64, 64, 60)), ("f64", (70, 13, 5)), ("f64", (3, 2, 1)),
                                         ("f64", (131, 9, 96)), ("f32", (99, 17, 33)),
                                         ("f32", (256, 256, 80))])
def test_matrix_gradients_match_oracle(dtype, shape):
    """ga, gb, gc from the transposed solve and the forward result, against
    the oracle's (FP32: under the FP32 limiter decisions); the other three
    gradients are unchanged by asking for them."""
    ni, nj, nk = shape
    f, g = setup(ni, nj, nk, dtype, SEED + 55)
    masks = None if dtype == "f64" else limiter_masks(f["u"], 2, dtype)
    kx, ky = masks if masks is not None else (None, None)
    ref = oracle.hdiff_vadv_adjoint(f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2, f["b"], 2,
                                    f["c"], 2, DT, interior(f["w"], 2), 0, matrix=True, force_kx=kx,
                                    force_ky=ky)
    out = gpu_matrix_adjoint(g, dtype, gpu_forward(g))
    errs = [normwise(out[n].to_numpy(interior=True), r) for n, r in zip(("ga", "gb", "gc"), ref[3:])]
    note("matrix gradients %s %s normwise ga %.2e gb %.2e gc %.2e" % (dtype, shape, *errs))
    assert max(errs) <= TOL[dtype], errs
    assert np.all(out["ga"].to_numpy(interior=True)[0] == 0)
    assert np.all(out["gc"].to_numpy(interior=True)[-1] == 0)
    plain = gpu_adjoint(g, dtype)
    for n in ("gu", "gcoeff", "gwcon"):
        got = out[n].to_numpy()
        if n != "gu":
            got = out[n].to_numpy(interior=True)
            assert np.array_equal(got, plain[n].to_numpy(interior=True))
        else:
            assert np.array_equal(got, plain[n].to_numpy())
    # matrix gradients write their interior only
    for n in ("ga", "gb", "gc"):
        full = out[n].to_numpy()
        assert np.all(full[:, :2] == -7.0) and np.all(full[:, :, :2] == -7.0)


@pytest.mark.parametrize("shape", [(96, 40, 80), (256, 256, 80)])
def test_adjoint_against_central_differences(shape):
    # FP64 forward on the GPU, eps = 1e-6: L is piecewise linear in u and
    # linear in coeff and wcon, so central differences are exact up to
    # rounding away from limiter switches; probes that move a decision are
    # skipped.  The loss difference is summed in FP64 over all points (only
    # the few columns a probe touches differ).  256 x 256 x 80 is the
    # reverse-mode workload itself.
    ni, nj, nk = shape
    note("central differences at %dx%dx%d" % shape)
    f, g = setup(ni, nj, nk, "f64", SEED + 52)
    out = gpu_matrix_adjoint(g, "f64", gpu_forward(g))
    grads = {n: out["g" + n].to_numpy() for n in ("u", "coeff", "wcon", "a", "b", "c")}
    wl = interior(f["w"], 2)
    kx0, ky0 = limiter_masks(f["u"], 2, "f64")
    rng = np.random.default_rng(7)
    eps = 1e-6
    x = g["u"].like(fill=0.0)
    checked = 0

    def loss_diff(name, arr_p, arr_m):
        vals = []
        for arr in (arr_p, arr_m):
            fld = B.Field.from_numpy(arr, 2, "f64")
            args = dict(g)
            args[name] = fld
            B.stencil_hdiff_vadv(args["u"], args["coeff"], args["wcon"], args["a"], args["b"],
                                 args["c"], DT, x)
            torch.cuda.synchronize()
            vals.append(x.to_numpy(interior=True))
        return float((wl * (vals[0] - vals[1])).sum())

    for name in ("u", "coeff", "wcon", "a", "b", "c"):
        for _ in range(8):
            k = int(rng.integers(0, nk))
            if name == "a" and k == 0 or name == "c" and k == nk - 1:
                continue  # outside the matrix
            lo = -2 if name == "u" else 0
            j = int(rng.integers(lo, nj - lo))
            i = int(rng.integers(lo, ni - lo))
            plus, minus = f[name].copy(), f[name].copy()
            plus[k, j + 2, i + 2] += eps
            minus[k, j + 2, i + 2] -= eps
            if name == "u":
                mp, mm = limiter_masks(plus, 2, "f64"), limiter_masks(minus, 2, "f64")
                if not all(np.array_equal(a, b) for a, b in zip(mp + mm, (kx0, ky0, kx0, ky0))):
                    continue
            fd = loss_diff(name, plus, minus) / (2 * eps)
            an = grads[name][k, j + 2, i + 2]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, k, j, i, fd, an)
            checked += 1
    note("central differences: %d probes agree" % checked)
    assert checked >= 36


def test_autograd_function_matches_adjoint():
    ni, nj, nk = 70, 12, 40
    f, g = setup(ni, nj, nk, "f64", SEED + 53)
    u = B.Field.from_numpy(f["u"], 2, "f64")
    coeff = B.Field.from_numpy(f["coeff"], 2, "f64")
    wcon = B.Field.from_numpy(f["wcon"], 2, "f64")
    a = B.Field.from_numpy(f["a"], 2, "f64")
    c = B.Field.from_numpy(f["c"], 2, "f64")
    for fld in (u, coeff, wcon, a, c):
        fld.buf.requires_grad_(True)
    x = AG.hdiff_vadv(u, coeff, wcon, a, g["b"], c, DT)
    wbuf = g["w"].buf.detach()
    loss = (x.buf * wbuf).sum()
    loss.backward()
    ref = gpu_matrix_adjoint(g, "f64", gpu_forward(g), fill=0.0)
    assert torch.equal(u.buf.grad, ref["gu"].buf)
    assert torch.equal(coeff.buf.grad, ref["gcoeff"].buf)
    assert torch.equal(wcon.buf.grad, ref["gwcon"].buf)
    # a and c carry gradients on the interior only (the rest of the buffer is 0)
    for fld, n in ((a, "ga"), (c, "gc")):
        got = B.Field(fld.buf.grad, fld.origin, ni, nj, nk, 2, 2, fld.sj, fld.sk, "f64")
        assert np.array_equal(got.to_numpy(interior=True), ref[n].to_numpy(interior=True))
    assert g["b"].buf.grad is None


def test_torch_gradcheck_small():
    # u = i^4 + j^4 keeps every flux far from the limiter switch, so the map
    # is linear in u and torch's finite differences are exact.
    ni, nj, nk = 6, 5, 4
    f, g = setup(ni, nj, nk, "f64", SEED + 54)
    kk, jj, ii = np.meshgrid(np.arange(nk), np.arange(-2, nj + 2), np.arange(-2, ni + 2), indexing="ij")
    uq = ((ii - 3.0) ** 4 + (jj - 2.0) ** 4) / 100.0
    u = B.Field.from_numpy(uq, 2, "f64")
    lay = u

    def fn(ubuf, cbuf, wbuf):
        return AG.HdiffVadv.apply(ubuf, cbuf, wbuf, g["a"].buf, g["b"].buf, g["c"].buf, (lay, DT))

    inputs_ = tuple(t.buf.detach().clone().requires_grad_(True) for t in (u, g["coeff"], g["wcon"]))
    assert torch.autograd.gradcheck(fn, inputs_, eps=1e-6, atol=1e-8, rtol=1e-6, fast_mode=True)


def test_adjoint_inside_a_captured_graph():
    """After one call on a stream has sized its scratch, the reverse pass
    captures into a graph and replays; a larger call under capture, which
    would have to grow the scratch, is refused instead of allocating."""
    ni, nj, nk = 70, 12, 40
    f, g = setup(ni, nj, nk, "f32", SEED + 55)
    s_cap = torch.cuda.Stream()
    ref = gpu_adjoint(g, "f32")
    out = {n: g["u"].like(fill=0.0) for n in ("gu", "gcoeff", "gwcon")}

    def call():
        B.stencil_hdiff_vadv_adjoint(g["u"], g["coeff"], g["wcon"], g["a"], g["b"], g["c"], DT, g["w"],
                                     out["gu"], out["gcoeff"], out["gwcon"])

    with torch.cuda.stream(s_cap):
        call()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s_cap):
        call()
    for rep in range(3):
        for t in out.values():
            t.buf.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for n in out:
            assert np.array_equal(out[n].to_numpy(), ref[n].to_numpy()), (rep, n)
    f2, g2 = setup(2 * ni, 2 * nj, nk, "f32", SEED + 56)
    out2 = {n: g2["u"].like(fill=0.0) for n in ("gu", "gcoeff", "gwcon")}
    graph2 = torch.cuda.CUDAGraph()
    with pytest.raises(B.StencilError) as e:
        with torch.cuda.graph(graph2, stream=s_cap):
            B.stencil_hdiff_vadv_adjoint(g2["u"], g2["coeff"], g2["wcon"], g2["a"], g2["b"], g2["c"], DT,
                                         g2["w"], out2["gu"], out2["gcoeff"], out2["gwcon"])
    assert e.value.status == "E_UNSUPPORTED"
