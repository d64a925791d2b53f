"""Pins of the oracle's reverse mode: every adjoint stage against a Jacobian
built by brute-force probing of the (separately pinned) forward stages, the
whole chain against a dot-product test with frozen limiter decisions, and
against central finite differences (no GPU)."""
import numpy as np
import pytest

import oracle
from paper_2005_13014_amd import inputs

DT = 10.0


def probe_jacobian(fn, shape, base=None):
    """Columns of the Jacobian of an affine map fn at base, by unit probes."""
    x0 = np.zeros(shape) if base is None else base
    f0 = fn(x0)
    cols = []
    for q in range(x0.size):
        x = x0.copy().reshape(-1)
        x[q] += 1.0
        cols.append((fn(x.reshape(shape)) - f0).reshape(-1))
    return np.array(cols).T


def test_rhs_adjoint_equals_transposed_jacobian():
    nk, nj, ni = 6, 2, 2
    rng = np.random.default_rng(1)
    h = rng.uniform(-1, 1, (nk, nj, ni))
    w = rng.uniform(-1, 1, (nk, nj, ni))
    lam = rng.standard_normal((nk, nj, ni))
    gh, gw = oracle.rhs_adjoint(h, 0, w, 0, DT, lam, 0)
    Jh = probe_jacobian(lambda hh: oracle.rhs(hh, 0, w, 0, DT), h.shape)
    Jw = probe_jacobian(lambda ww: oracle.rhs(h, 0, ww, 0, DT), w.shape)
    assert np.abs(gh.reshape(-1) - Jh.T @ lam.reshape(-1)).max() < 1e-12
    assert np.abs(gw.reshape(-1) - Jw.T @ lam.reshape(-1)).max() < 1e-12


def test_hdiff_adjoint_equals_transposed_jacobian():
    ni, nj, nk, h = 5, 4, 2, 2
    f = inputs.fields(ni, nj, nk, h, seed=77, vadv=False)
    u, coeff = f["u"], f["coeff"]
    _, _, _, kx, ky = oracle.hdiff(u, h, coeff, h, fluxes=True)
    gh = np.random.default_rng(2).standard_normal((nk, nj, ni))
    gu, gc = oracle.hdiff_adjoint(u, h, coeff, h, gh, 0)
    # Forward with the limiter decisions frozen is linear in u and in coeff.
    Ju = probe_jacobian(lambda uu: oracle.hdiff(uu, h, coeff, h, force_kx=kx, force_ky=ky),
                        u.shape)
    Jc = probe_jacobian(lambda cc: oracle.hdiff(u, h, cc, h, force_kx=kx, force_ky=ky),
                        coeff.shape)
    assert np.abs(gu.reshape(-1) - Ju.T @ gh.reshape(-1)).max() < 1e-12
    gc_full = Jc.T @ gh.reshape(-1)
    assert np.abs(oracle.interior(gc_full.reshape(coeff.shape), h) - gc).max() < 1e-12
    # Only the interior of coeff is read; its halo gets no gradient.
    mask = np.ones(coeff.shape, bool)
    mask[:, h:-h, h:-h] = False
    assert np.all(gc_full.reshape(coeff.shape)[mask] == 0.0)


def _fields(ni, nj, nk, seed):
    f = inputs.fields(ni, nj, nk, 2, seed=seed, loss=True)
    f["wl"] = oracle.interior(f["w"], 2).copy()
    return f


def _loss(f, u=None, coeff=None, wcon=None, a=None, b=None, c=None, kx=None, ky=None):
    u = f["u"] if u is None else u
    coeff = f["coeff"] if coeff is None else coeff
    wcon = f["wcon"] if wcon is None else wcon
    a = f["a"] if a is None else a
    b = f["b"] if b is None else b
    c = f["c"] if c is None else c
    hh = oracle.hdiff(u, 2, coeff, 2, force_kx=kx, force_ky=ky)
    x = oracle.vadv(hh, 0, wcon, 2, a, 2, b, 2, c, 2, DT)
    return float((f["wl"] * x).sum())


def test_dot_product_with_frozen_limiter():
    # With the limiter decisions frozen, x is linear in u, so
    # <wl, x(u + v) - x(u)> = <grad_u L, v> up to rounding only.
    ni, nj, nk = 6, 5, 7
    f = _fields(ni, nj, nk, seed=88)
    _, _, _, kx, ky = oracle.hdiff(f["u"], 2, f["coeff"], 2, fluxes=True)
    gu, gcoeff, gw = oracle.hdiff_vadv_adjoint(f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2,
                                               f["b"], 2, f["c"], 2, DT, f["wl"], 0)
    rng = np.random.default_rng(3)
    for _ in range(3):
        v = rng.standard_normal(f["u"].shape)
        lhs = _loss(f, u=f["u"] + v, kx=kx, ky=ky) - _loss(f, kx=kx, ky=ky)
        rhs = float((gu * v).sum())
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(rhs))
        vc = rng.standard_normal(f["coeff"].shape)
        lhs = _loss(f, coeff=f["coeff"] + vc, kx=kx, ky=ky) - _loss(f, kx=kx, ky=ky)
        rhs = float((gcoeff * oracle.interior(vc, 2)).sum())
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(rhs))
        vw = rng.standard_normal(f["wcon"].shape)
        lhs = _loss(f, wcon=f["wcon"] + vw) - _loss(f)
        rhs = float((gw * oracle.interior(vw, 2)).sum())
        assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(rhs))


def test_gradient_support():
    # 40 levels: the limiter zeroes ~90% of the fluxes of white noise, so some
    # level keeps a flux through every corner cell that the diamond reaches.
    ni, nj, nk = 6, 5, 40
    f = _fields(ni, nj, nk, seed=89)
    gu, gcoeff, gw = oracle.hdiff_vadv_adjoint(f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2,
                                               f["b"], 2, f["c"], 2, DT, f["wl"], 0)
    # u's gradient reaches the 2-cell ring through the 13-point diamond: of each
    # 2x2 corner block only the cell diagonal to the interior corner is reached.
    for cj, ci, inner in ((0, 0, (1, 1)), (0, -1, (1, -2)), (-1, 0, (-2, 1)), (-1, -1, (-2, -2))):
        sj = 1 if cj == 0 else -1
        si = 1 if ci == 0 else -1
        assert np.all(gu[:, cj, ci] == 0)
        assert np.all(gu[:, cj + sj, ci] == 0) and np.all(gu[:, cj, ci + si] == 0)
        assert np.abs(gu[:, inner[0], inner[1]]).max() > 0
    assert np.abs(gu[:, 0, 2:-2]).max() > 0 and np.abs(gu[:, 2:-2, 0]).max() > 0


@pytest.mark.parametrize("name", ["u", "coeff", "wcon", "a", "b", "c"])
def test_central_finite_differences(name):
    ni, nj, nk = 7, 6, 9
    f = _fields(ni, nj, nk, seed=90)
    gu, gcoeff, gw, ga, gb, gc = oracle.hdiff_vadv_adjoint(
        f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2, f["b"], 2, f["c"], 2, DT, f["wl"], 0,
        matrix=True)
    grads = {"u": gu, "coeff": gcoeff, "wcon": gw, "a": ga, "b": gb, "c": gc}
    _, _, _, kx0, ky0 = oracle.hdiff(f["u"], 2, f["coeff"], 2, fluxes=True)
    rng = np.random.default_rng(4)
    eps = 1e-6
    checked = 0
    for _ in range(25):
        k = int(rng.integers(0, nk))
        if name == "u":
            j, i = int(rng.integers(-2, nj + 2)), int(rng.integers(-2, ni + 2))
        else:
            j, i = int(rng.integers(0, nj)), int(rng.integers(0, ni))
        if name == "a" and k == 0 or name == "c" and k == nk - 1:
            continue
        arr = f[name]
        plus, minus = arr.copy(), arr.copy()
        plus[k, j + 2, i + 2] += eps
        minus[k, j + 2, i + 2] -= eps
        if name == "u":
            # skip probes that move a limiter decision
            _, _, _, kxp, kyp = oracle.hdiff(plus, 2, f["coeff"], 2, fluxes=True)
            _, _, _, kxm, kym = oracle.hdiff(minus, 2, f["coeff"], 2, fluxes=True)
            if not (np.array_equal(kxp, kx0) and np.array_equal(kxm, kx0)
                    and np.array_equal(kyp, ky0) and np.array_equal(kym, ky0)):
                continue
        fd = (_loss(f, **{name: plus}) - _loss(f, **{name: minus})) / (2 * eps)
        g = grads[name]
        an = g[k, j + 2, i + 2] if name == "u" else g[k, j, i]
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, k, j, i, fd, an)
        checked += 1
    assert checked >= 10
