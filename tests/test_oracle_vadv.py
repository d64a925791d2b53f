"""Pins of the oracle's vertical stages (flux-form right-hand side, Thomas
solve, vertical diffusion, horizontal-gradient update) against dense LAPACK
solves, closed forms and conservation laws (no GPU)."""
import numpy as np
import pytest

import oracle
from paper_2005_13014_amd import inputs


def dense_T(a, b, c):
    """Dense tridiagonal matrix of one column: row k has a(k) at k-1, b(k) at
    k, c(k) at k+1."""
    n = len(b)
    T = np.diag(b.astype(float))
    for k in range(1, n):
        T[k, k - 1] = a[k]
    for k in range(n - 1):
        T[k, k + 1] = c[k]
    return T


def columns(ni, nj, nk, seed):
    f = inputs.fields(ni, nj, nk, 0, seed=seed)
    return f


# ---- Thomas ---------------------------------------------------------------

@pytest.mark.parametrize("nk", [1, 2, 3, 5, 8])
def test_thomas_matches_dense_lu(nk):
    ni, nj = 4, 3
    f = columns(ni, nj, nk, seed=100 + nk)
    rng = np.random.default_rng(nk)
    d = rng.uniform(-1, 1, (nk, nj, ni))
    x = oracle.thomas(f["a"], 0, f["b"], 0, f["c"], 0, d, 0)
    for j in range(nj):
        for i in range(ni):
            T = dense_T(f["a"][:, j, i], f["b"][:, j, i], f["c"][:, j, i])
            ref = np.linalg.solve(T, d[:, j, i])
            assert np.abs(x[:, j, i] - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())


def test_thomas_residual_at_80_levels():
    ni, nj, nk = 6, 5, 80
    f = columns(ni, nj, nk, seed=3)
    d = np.random.default_rng(1).uniform(-1, 1, (nk, nj, ni))
    x = oracle.thomas(f["a"], 0, f["b"], 0, f["c"], 0, d, 0)
    for j in range(nj):
        for i in range(ni):
            T = dense_T(f["a"][:, j, i], f["b"][:, j, i], f["c"][:, j, i])
            r = T @ x[:, j, i] - d[:, j, i]
            assert np.abs(r).max() / np.abs(d[:, j, i]).max() < 1e-12


def test_thomas_manufactured_solution():
    ni, nj, nk = 5, 4, 17
    f = columns(ni, nj, nk, seed=4)
    xs = np.random.default_rng(2).uniform(-2, 2, (nk, nj, ni))
    d = np.empty_like(xs)
    for j in range(nj):
        for i in range(ni):
            d[:, j, i] = dense_T(f["a"][:, j, i], f["b"][:, j, i], f["c"][:, j, i]) @ xs[:, j, i]
    x = oracle.thomas(f["a"], 0, f["b"], 0, f["c"], 0, d, 0)
    assert np.abs(x - xs).max() <= 1e-13


def test_thomas_diagonal_system():
    nk, nj, ni = 9, 2, 3
    rng = np.random.default_rng(5)
    b = rng.uniform(1, 2, (nk, nj, ni))
    d = rng.uniform(-1, 1, (nk, nj, ni))
    z = np.zeros_like(b)
    x = oracle.thomas(z, 0, b, 0, z, 0, d, 0)
    assert np.array_equal(x, d / b)


def test_thomas_ignores_structural_zeros():
    # a(0) and c(nk-1) lie outside the matrix: garbage there changes nothing.
    ni, nj, nk = 3, 2, 6
    f = columns(ni, nj, nk, seed=8)
    d = np.random.default_rng(8).uniform(-1, 1, (nk, nj, ni))
    x0 = oracle.thomas(f["a"], 0, f["b"], 0, f["c"], 0, d, 0)
    a, c = f["a"].copy(), f["c"].copy()
    a[0] = 123.0
    c[-1] = -77.0
    assert np.array_equal(oracle.thomas(a, 0, f["b"], 0, c, 0, d, 0), x0)


def test_thomas_transpose_matches_dense():
    ni, nj, nk = 3, 3, 11
    f = columns(ni, nj, nk, seed=12)
    g = np.random.default_rng(12).uniform(-1, 1, (nk, nj, ni))
    lam = oracle.thomas_transpose(f["a"], 0, f["b"], 0, f["c"], 0, g, 0)
    for j in range(nj):
        for i in range(ni):
            T = dense_T(f["a"][:, j, i], f["b"][:, j, i], f["c"][:, j, i])
            assert np.abs(T.T @ lam[:, j, i] - g[:, j, i]).max() < 1e-13
            assert np.abs(lam[:, j, i] - np.linalg.solve(T.T, g[:, j, i])).max() < 1e-13


# ---- flux-form right-hand side -------------------------------------------

def test_rhs_conserves_column_sum():
    ni, nj, nk = 7, 6, 30
    f = columns(ni, nj, nk, seed=21)
    h = np.random.default_rng(21).uniform(-1, 1, (nk, nj, ni))
    d = oracle.rhs(h, 0, f["wcon"], 0, 10.0)
    assert np.abs(d.sum(axis=0) - h.sum(axis=0)).max() <= 1e-12
    assert np.abs(d - h).max() > 1.0      # the flux terms are not trivially zero


def test_rhs_without_velocity_is_identity():
    h = np.random.default_rng(0).uniform(-1, 1, (9, 4, 5))
    assert np.array_equal(oracle.rhs(h, 0, np.zeros_like(h), 0, 10.0), h)


def test_rhs_constant_fields():
    nk, h0, w0, dt = 7, 0.75, -0.3, 10.0
    h = np.full((nk, 2, 3), h0)
    w = np.full((nk, 2, 3), w0)
    d = oracle.rhs(h, 0, w, 0, dt)
    assert np.allclose(d[0], h0 * (1 - dt * w0), rtol=0, atol=1e-15)
    assert np.allclose(d[-1], h0 * (1 + dt * w0), rtol=0, atol=1e-15)
    assert np.allclose(d[1:-1], h0, rtol=0, atol=1e-15)


def test_rhs_quadratic_profile_uses_face_means():
    # h = k^2, w = w0: face value (k^2 + (k+1)^2)/2 = k^2 + k + 1/2, so
    # F(k+1/2) - F(k-1/2) = 2 k w0 inside the column.
    nk, w0, dt = 9, 0.4, 10.0
    kk = np.arange(nk, dtype=float)
    h = np.broadcast_to((kk ** 2)[:, None, None], (nk, 2, 2)).copy()
    w = np.full_like(h, w0)
    d = oracle.rhs(h, 0, w, 0, dt)
    inner = kk[1:-1]
    assert np.allclose(d[1:-1, 0, 0], inner ** 2 - dt * 2 * inner * w0, rtol=0, atol=1e-12)
    assert np.isclose(d[0, 0, 0], 0.0 - dt * w0 * 0.5, rtol=0, atol=1e-14)
    top = nk - 1
    f_dn = w0 * ((top - 1) ** 2 + top ** 2) / 2
    assert np.isclose(d[-1, 0, 0], top ** 2 + dt * f_dn, rtol=0, atol=1e-12)


def test_rhs_linear_velocity_profile():
    # w = k, h = h0: F(k+1/2) = h0 (k + 1/2); interior d = h0 - dt h0.
    nk, h0, dt = 6, 2.0, 10.0
    kk = np.arange(nk, dtype=float)
    w = np.broadcast_to(kk[:, None, None], (nk, 1, 1)).copy()
    h = np.full_like(w, h0)
    d = oracle.rhs(h, 0, w, 0, dt)
    assert np.allclose(d[1:-1, 0, 0], h0 - dt * h0, rtol=0, atol=1e-12)
    assert np.isclose(d[0, 0, 0], h0 - dt * h0 * 0.5)
    assert np.isclose(d[-1, 0, 0], h0 + dt * h0 * (nk - 1.5))


def test_vadv_solves_the_system_it_builds():
    ni, nj, nk = 5, 4, 20
    f = columns(ni, nj, nk, seed=31)
    h = np.random.default_rng(31).uniform(-1, 1, (nk, nj, ni))
    x = oracle.vadv(h, 0, f["wcon"], 0, f["a"], 0, f["b"], 0, f["c"], 0, 10.0)
    d = oracle.rhs(h, 0, f["wcon"], 0, 10.0)
    for j in range(nj):
        for i in range(ni):
            T = dense_T(f["a"][:, j, i], f["b"][:, j, i], f["c"][:, j, i])
            assert np.abs(T @ x[:, j, i] - d[:, j, i]).max() < 1e-12


def test_hdiff_vadv_is_the_composition():
    ni, nj, nk, hh = 9, 8, 12, 2
    f = inputs.fields(ni, nj, nk, hh, seed=41)
    x = oracle.hdiff_vadv(f["u"], hh, f["coeff"], hh, f["wcon"], hh, f["a"], hh, f["b"], hh,
                          f["c"], hh, 10.0)
    h = oracle.hdiff(f["u"], hh, f["coeff"], hh)
    x2 = oracle.vadv(h, 0, f["wcon"], hh, f["a"], hh, f["b"], hh, f["c"], hh, 10.0)
    assert np.array_equal(x, x2)


# ---- vertical diffusion and horizontal gradient --------------------------

def test_vdiff_invariants():
    nk, kappa = 13, 0.1
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, (nk, 3, 4))
    y = oracle.vdiff(x, 0, kappa)
    assert np.abs(y.sum(axis=0) - x.sum(axis=0)).max() <= 1e-13
    c = np.full((nk, 2, 2), 3.5)
    assert np.array_equal(oracle.vdiff(c, 0, kappa), c)
    kk = np.arange(nk, dtype=float)
    lin = np.broadcast_to((2 * kk - 1)[:, None, None], (nk, 1, 1)).copy()
    yl = oracle.vdiff(lin, 0, kappa)
    assert np.allclose(yl[1:-1], lin[1:-1], rtol=0, atol=1e-14)
    assert np.isclose(yl[0, 0, 0], lin[0, 0, 0] + kappa * 2.0)
    assert np.isclose(yl[-1, 0, 0], lin[-1, 0, 0] - kappa * 2.0)
    quad = np.broadcast_to((kk ** 2)[:, None, None], (nk, 1, 1)).copy()
    yq = oracle.vdiff(quad, 0, kappa)
    assert np.allclose(yq[1:-1], quad[1:-1] + 2 * kappa, rtol=0, atol=1e-12)


@pytest.mark.parametrize("nk", [1, 2, 3, 8, 40])
def test_vdiff_implicit_pins(nk):
    """Backward-Euler vertical diffusion: conserves the column sum (zero-flux
    ends), keeps constants, agrees with a dense solve of the same matrix, and
    the explicit operator applied to its result gives back the input."""
    kappa = 0.1
    rng = np.random.default_rng(40 + nk)
    x = rng.uniform(-1, 1, (nk, 3, 2))
    y = oracle.vdiff_implicit(x, 0, kappa)
    assert np.abs(y.sum(axis=0) - x.sum(axis=0)).max() <= 1e-13 * nk
    c = np.full((nk, 2, 2), -2.25)
    assert np.allclose(oracle.vdiff_implicit(c, 0, kappa), c, rtol=0, atol=1e-14)
    # dense matrix of (I - kappa L), L the zero-flux Laplacian along k
    A = np.eye(nk)
    for k in range(nk):
        if k > 0:
            A[k, k - 1] -= kappa
            A[k, k] += kappa
        if k + 1 < nk:
            A[k, k + 1] -= kappa
            A[k, k] += kappa
    for j in range(3):
        for i in range(2):
            assert np.allclose(y[:, j, i], np.linalg.solve(A, x[:, j, i]), rtol=0, atol=1e-14)
    # y - kappa L y = x: the explicit operator with -kappa undoes the implicit one
    back = oracle.vdiff(y, 0, -kappa)
    assert np.allclose(back, x, rtol=0, atol=1e-14)


def test_timestep_implicit_is_the_chain():
    ni, nj, nk, h = 7, 6, 9, 3
    f = inputs.fields(ni, nj, nk, h, seed=52)
    args = (f["u"], h, f["coeff"], h, f["wcon"], h, f["a"], h, f["b"], h, f["c"], h, 10.0)
    z = oracle.timestep(*args, 0.1, 0.05, 0.01, implicit=True)
    x = oracle.hdiff_vadv(*args, e=1)
    y = oracle.vdiff_implicit(x, 1, 0.1, e=1)
    assert np.array_equal(z, oracle.hgrad(y, 1, 0.05, 0.01))
    assert not np.array_equal(z, oracle.timestep(*args, 0.1, 0.05, 0.01))


@pytest.mark.parametrize("al,be,ga", [(0.5, -1.25, 2.0), (1.0, 0.0, -3.0)])
def test_hgrad_linear_field(al, be, ga):
    ni, nj, nk, bh, bv = 6, 5, 7, 0.05, 0.01
    kk, jj, ii = np.meshgrid(np.arange(nk), np.arange(-1, nj + 1), np.arange(-1, ni + 1),
                             indexing="ij")
    y = al * ii + be * jj + ga * kk + 0.5
    z = oracle.hgrad(y, 1, bh, bv)
    assert np.allclose(z, y[:, 1:-1, 1:-1] - bh * (al + be) - bv * ga, rtol=0, atol=1e-12)


def test_hgrad_constant_and_one_sided_ends():
    ni, nj, nk, bh, bv = 4, 3, 5, 0.05, 0.01
    y = np.full((nk, nj + 2, ni + 2), -1.5)
    assert np.array_equal(oracle.hgrad(y, 1, bh, bv), np.full((nk, nj, ni), -1.5))
    kk = np.arange(nk, dtype=float)
    yq = np.broadcast_to((kk ** 2)[:, None, None], (nk, nj + 2, ni + 2)).copy()
    z = oracle.hgrad(yq, 1, bh, bv)
    assert np.isclose(z[0, 0, 0], 0.0 - bv * 1.0)                      # y(1) - y(0)
    assert np.isclose(z[-1, 0, 0], 16.0 - bv * (16.0 - 9.0))           # y(4) - y(3)
    assert np.isclose(z[2, 0, 0], 4.0 - bv * (9.0 - 1.0) / 2)


def test_timestep_is_the_chain():
    ni, nj, nk, h = 7, 6, 9, 3
    f = inputs.fields(ni, nj, nk, h, seed=51)
    args = (f["u"], h, f["coeff"], h, f["wcon"], h, f["a"], h, f["b"], h, f["c"], h, 10.0)
    z = oracle.timestep(*args, 0.1, 0.05, 0.01)
    x = oracle.hdiff_vadv(*args, e=1)
    y = oracle.vdiff(x, 1, 0.1, e=1)
    assert np.array_equal(z, oracle.hgrad(y, 1, 0.05, 0.01))


def test_openmp_build_is_bitwise_the_serial_one():
    # The all-core build splits the outermost loops of the forward stages over
    # threads without changing any element's arithmetic.
    f = inputs.fields(37, 23, 19, 3, seed=200513074, storage="f64")
    args = (f["u"], 3, f["coeff"], 3, f["wcon"], 3, f["a"], 3, f["b"], 3, f["c"], 3, 10.0)
    x1 = oracle.hdiff_vadv(*args)
    z1 = oracle.timestep(*args, 0.1, 0.05, 0.01)
    with oracle.parallel():
        x2 = oracle.hdiff_vadv(*args)
        z2 = oracle.timestep(*args, 0.1, 0.05, 0.01)
    assert np.array_equal(x1, x2) and np.array_equal(z1, z2)
