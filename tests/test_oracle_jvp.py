"""Pins of the oracle's forward mode (the tangent dx = J v of the fused
hdiff + vadv program): duality with the separately pinned reverse mode,
central finite differences of the forward oracle, and closed forms for one
tangent input at a time built from the forward stages and dense NumPy solves
(no GPU)."""
import numpy as np
import pytest

import oracle
from paper_2005_13014_amd import inputs

DT = 10.0
NAMES = ("u", "coeff", "wcon", "a", "b", "c")
KW = {"u": "du", "coeff": "dcoeff", "wcon": "dw", "a": "da", "b": "db", "c": "dc"}


def _fields(ni, nj, nk, seed):
    f = inputs.fields(ni, nj, nk, 2, seed=seed, loss=True)
    f["wl"] = oracle.interior(f["w"], 2).copy()
    return f


def _direction(f, seed, names=NAMES):
    rng = np.random.default_rng(seed)
    return {n: rng.standard_normal(f[n].shape) for n in names}


def _jvp(f, v, **kw):
    t = {KW[n]: v[n] for n in v}
    return oracle.hdiff_vadv_jvp(f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2, f["b"], 2, f["c"], 2,
                                 DT, hdu=2, hdcf=2, hdw=2, hdm=2, **t, **kw)


def _forward(f, **over):
    g = dict(f)
    g.update(over)
    return oracle.hdiff_vadv(g["u"], 2, g["coeff"], 2, g["wcon"], 2, g["a"], 2, g["b"], 2, g["c"], 2, DT)


def _masks(u, coeff):
    _, _, _, kx, ky = oracle.hdiff(u, 2, coeff, 2, fluxes=True)
    return kx, ky


def test_duality_with_the_adjoint():
    # <wl, J v> = <J^T wl, v>: the tangent and the reverse-mode gradients are
    # independent code; they agree to rounding for every input direction.
    ni, nj, nk = 7, 6, 11
    f = _fields(ni, nj, nk, seed=301)
    gu, gcoeff, gw, ga, gb, gc = oracle.hdiff_vadv_adjoint(
        f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2, f["b"], 2, f["c"], 2, DT, f["wl"], 0,
        matrix=True)
    grads = {"u": gu, "coeff": gcoeff, "wcon": gw, "a": ga, "b": gb, "c": gc}
    for seed in (1, 2):
        v = _direction(f, seed)
        dx = _jvp(f, v)
        lhs = float((f["wl"] * dx).sum())
        terms = [float((gu * v["u"]).sum())]
        terms += [float((grads[n] * oracle.interior(v[n], 2)).sum()) for n in NAMES[1:]]
        assert abs(lhs - sum(terms)) <= 1e-12 * sum(abs(t) for t in terms)
        # and one input at a time
        for n in NAMES:
            dx1 = _jvp(f, {n: v[n]})
            t = terms[NAMES.index(n)]
            assert abs(float((f["wl"] * dx1).sum()) - t) <= 1e-12 * max(1.0, abs(t)), n


def test_central_finite_differences():
    ni, nj, nk = 6, 5, 9
    f = _fields(ni, nj, nk, seed=302)
    kx0, ky0 = _masks(f["u"], f["coeff"])
    eps = 1e-6
    checked = 0
    for seed in range(10, 20):
        v = _direction(f, seed)
        plus = {n: f[n] + eps * v[n] for n in NAMES}
        minus = {n: f[n] - eps * v[n] for n in NAMES}
        # skip directions that move a limiter decision within +-eps
        if not all(np.array_equal(m, m0) for m, m0 in
                   zip(_masks(plus["u"], plus["coeff"]) + _masks(minus["u"], minus["coeff"]),
                       (kx0, ky0, kx0, ky0))):
            continue
        fd = (_forward(f, **plus) - _forward(f, **minus)) / (2 * eps)
        dx = _jvp(f, v)
        assert np.abs(fd - dx).max() <= 1e-6 * np.abs(dx).max()
        checked += 1
    assert checked >= 5


def _dense_solve_columns(f, rhs):
    """Solves T y = rhs column by column with a dense matrix (numpy.linalg)."""
    a, b, c = (oracle.interior(f[n], 2) for n in ("a", "b", "c"))
    nk, nj, ni = rhs.shape
    y = np.empty_like(rhs)
    for j in range(nj):
        for i in range(ni):
            T = np.diag(b[:, j, i]) + np.diag(a[1:, j, i], -1) + np.diag(c[:-1, j, i], 1)
            y[:, j, i] = np.linalg.solve(T, rhs[:, j, i])
    return y


def test_matrix_tangents_closed_form():
    # T x = d with d fixed: dx = -T^-1 (dT x), dT = tridiag(da, db, dc).
    ni, nj, nk = 4, 3, 12
    f = _fields(ni, nj, nk, seed=303)
    x = _forward(f)
    v = _direction(f, 5, ("a", "b", "c"))
    da, db, dc = (oracle.interior(v[n], 2) for n in ("a", "b", "c"))
    r = db * x
    r[1:] += da[1:] * x[:-1]
    r[:-1] += dc[:-1] * x[1:]
    ref = -_dense_solve_columns(f, r)
    got = _jvp(f, v)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # the entries a(0) and c(nk-1) lie outside T: their tangents do nothing
    v0 = {"a": np.zeros_like(f["a"]), "c": np.zeros_like(f["c"])}
    v0["a"][0] = 1.0
    v0["c"][-1] = 1.0
    assert np.all(_jvp(f, v0) == 0)


def test_u_tangent_without_diffusion():
    # coeff = 0 makes h = u, and the right-hand side is linear in h for fixed
    # w, so the u tangent is the vertical advection of du itself.
    ni, nj, nk = 5, 4, 10
    f = _fields(ni, nj, nk, seed=304)
    f["coeff"] = np.zeros_like(f["coeff"])
    v = _direction(f, 6, ("u",))
    ref = oracle.vadv(oracle.interior(v["u"], 2), 0, f["wcon"], 2, f["a"], 2, f["b"], 2, f["c"], 2, DT)
    got = _jvp(f, v)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_coeff_tangent_from_the_flux_divergence():
    # h = u - coeff * div, so dh = -dcoeff * div with div = u - hdiff(u, 1),
    # and dx is the vertical advection of dh.
    ni, nj, nk = 5, 4, 10
    f = _fields(ni, nj, nk, seed=305)
    div = oracle.interior(f["u"], 2) - oracle.hdiff(f["u"], 2, np.ones_like(f["coeff"]), 2)
    v = _direction(f, 7, ("coeff",))
    dh = -oracle.interior(v["coeff"], 2) * div
    ref = oracle.vadv(dh, 0, f["wcon"], 2, f["a"], 2, f["b"], 2, f["c"], 2, DT)
    got = _jvp(f, v)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


def test_wcon_tangent_from_the_right_hand_side():
    # The right-hand side is linear in w: its tangent is rhs(h, dw) - h.
    ni, nj, nk = 5, 4, 10
    f = _fields(ni, nj, nk, seed=306)
    h = oracle.hdiff(f["u"], 2, f["coeff"], 2)
    v = _direction(f, 8, ("wcon",))
    dd = oracle.rhs(h, 0, oracle.interior(v["wcon"], 2), 0, DT) - h
    ref = _dense_solve_columns(f, dd)
    got = _jvp(f, v)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_linear_in_the_direction_and_zero_without_one():
    ni, nj, nk = 6, 4, 7
    f = _fields(ni, nj, nk, seed=307)
    v1, v2 = _direction(f, 9), _direction(f, 10)
    comb = {n: 2.0 * v1[n] - 0.5 * v2[n] for n in NAMES}
    ref = 2.0 * _jvp(f, v1) - 0.5 * _jvp(f, v2)
    assert np.abs(_jvp(f, comb) - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.all(_jvp(f, {}) == 0)


def test_forced_masks_change_only_the_u_tangent():
    ni, nj, nk = 6, 5, 6
    f = _fields(ni, nj, nk, seed=308)
    kx, ky = _masks(f["u"], f["coeff"])
    v = _direction(f, 11)
    base = _jvp(f, v)
    assert np.array_equal(_jvp(f, v, force_kx=kx, force_ky=ky), base)
    flipped = _jvp(f, {"u": v["u"]}, force_kx=1 - kx, force_ky=ky)
    assert np.abs(flipped - _jvp(f, {"u": v["u"]})).max() > 0


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 2, 1), (2, 3, 2)])
def test_degenerate_shapes(shape):
    ni, nj, nk = shape
    f = _fields(ni, nj, nk, seed=309)
    v = _direction(f, 12)
    eps = 1e-6
    fd = (_forward(f, **{n: f[n] + eps * v[n] for n in NAMES})
          - _forward(f, **{n: f[n] - eps * v[n] for n in NAMES})) / (2 * eps)
    dx = _jvp(f, v)
    assert dx.shape == (nk, nj, ni)
    assert np.abs(fd - dx).max() <= 1e-5 * max(1.0, np.abs(dx).max())
