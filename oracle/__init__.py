"""NumPy front end of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product package never imports this module
and this module never imports the product package.

Every array is a C-contiguous float64 NumPy array of shape
``(nk, nj + 2h, ni + 2h)`` (k slowest, i fastest) with a halo of ``h`` cells on
both sides in i and j; interior point (i, j, k) is ``arr[k, j + h, i + h]``.
Each function takes the halo of every array explicitly, derives (ni, nj, nk)
from the first array, and returns new arrays.  ``e`` grows the computed domain
by ``e`` cells in i and j (outputs then carry a halo of ``e``).

See ``oracle.c`` for the definitions and the passages of the paper they follow.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# The same source built with OpenMP (its pragmas split the outermost loops of
# the forward stages over threads; results are bitwise the same).  Used only
# to time the oracle on all host cores.
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

_libs = {}
_parallel = False


def _compile(out, openmp):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wextra"] + (["-fopenmp"] if openmp else ["-Wno-unknown-pragmas"]) + ["-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, no FP contraction) and,
    with OpenMP, into liboracle_omp.so."""
    for out, omp in ((_LIB, False), (_LIB_OMP, True)):
        if force or not os.path.exists(out):
            _compile(out, omp)
    return _LIB


class parallel:
    """Context in which the oracle functions run on all the threads OpenMP
    gives them (OMP_NUM_THREADS, else every host core)."""

    def __enter__(self):
        global _parallel
        self._old, _parallel = _parallel, True
        return self

    def __exit__(self, *exc):
        global _parallel
        _parallel = self._old
        return False


def threads():
    """Threads the OpenMP build uses (1 for the plain build)."""
    lib = ctypes.CDLL(_LIB_OMP) if os.path.exists(_LIB_OMP) else None
    if lib is None:
        return 1
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
        return int(gomp.omp_get_max_threads())
    except OSError:
        return 1


def _load():
    path = _LIB_OMP if _parallel else _LIB
    lib = _libs.get(path)
    if lib is None:
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            _compile(path, path == _LIB_OMP)
        lib = _libs[path] = ctypes.CDLL(path)
    return lib


_D = ctypes.POINTER(ctypes.c_double)
_U8 = ctypes.POINTER(ctypes.c_uint8)


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _u8(a):
    if a is None:
        return None
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(_U8)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dims(a, h):
    nk, pj, pi = a.shape
    return pi - 2 * h, pj - 2 * h, nk


def padded(ni, nj, nk, h, dtype=np.float64):
    return np.zeros((nk, nj + 2 * h, ni + 2 * h), dtype=dtype)


def _check(rc, name):
    if rc != 0:
        raise RuntimeError("oracle %s failed with code %d" % (name, rc))


_I = ctypes.c_int
_DBL = ctypes.c_double


def lap(u, hu, e=0):
    """Laplacian stage on the interior grown by e."""
    lib = _load()
    u = _f64(u)
    ni, nj, nk = _dims(u, hu)
    out = padded(ni, nj, nk, e)
    _check(lib.oracle_lap(_I(ni), _I(nj), _I(nk), _dp(u), _I(hu), _dp(out), _I(e), _I(e)), "lap")
    return out


def hdiff(u, hu, coeff, hc, e=0, fluxes=False, force_kx=None, force_ky=None):
    """Horizontal diffusion.  Returns out (halo e), or with fluxes=True a tuple
    (out, flx, fly, kx, ky) where the flux arrays and the 0/1 keep masks carry
    halo e + 1."""
    lib = _load()
    u, coeff = _f64(u), _f64(coeff)
    ni, nj, nk = _dims(u, hu)
    out = padded(ni, nj, nk, e)
    flx = fly = kx = ky = None
    if fluxes:
        flx, fly = padded(ni, nj, nk, e + 1), padded(ni, nj, nk, e + 1)
        kx, ky = padded(ni, nj, nk, e + 1, np.uint8), padded(ni, nj, nk, e + 1, np.uint8)
    fkx = None if force_kx is None else np.ascontiguousarray(force_kx, dtype=np.uint8)
    fky = None if force_ky is None else np.ascontiguousarray(force_ky, dtype=np.uint8)
    rc = lib.oracle_hdiff_ex(_I(ni), _I(nj), _I(nk), _dp(u), _I(hu), _dp(coeff), _I(hc), _dp(out),
                             _I(e), _I(e), _dp(flx), _dp(fly), _u8(kx), _u8(ky), _u8(fkx), _u8(fky))
    _check(rc, "hdiff")
    return (out, flx, fly, kx, ky) if fluxes else out


def rhs(h, hh, w, hw, dt, e=0):
    """Flux-form vertical-advection right-hand side."""
    lib = _load()
    h, w = _f64(h), _f64(w)
    ni, nj, nk = _dims(h, hh)
    d = padded(ni, nj, nk, e)
    _check(lib.oracle_rhs(_I(ni), _I(nj), _I(nk), _dp(h), _I(hh), _dp(w), _I(hw), _DBL(dt), _dp(d),
                          _I(e), _I(e)), "rhs")
    return d


def thomas(a, ha, b, hb, c, hc, d, hd, e=0):
    """Per-column tridiagonal solve T x = d, T = tridiag(a, b, c)."""
    lib = _load()
    a, b, c, d = _f64(a), _f64(b), _f64(c), _f64(d)
    ni, nj, nk = _dims(a, ha)
    x = padded(ni, nj, nk, e)
    _check(lib.oracle_thomas(_I(ni), _I(nj), _I(nk), _dp(a), _I(ha), _dp(b), _I(hb), _dp(c), _I(hc),
                             _dp(d), _I(hd), _dp(x), _I(e), _I(e)), "thomas")
    return x


def thomas_transpose(a, ha, b, hb, c, hc, g, hg, e=0):
    """Per-column transposed solve T^T lam = g."""
    lib = _load()
    a, b, c, g = _f64(a), _f64(b), _f64(c), _f64(g)
    ni, nj, nk = _dims(a, ha)
    lam = padded(ni, nj, nk, e)
    _check(lib.oracle_thomas_transpose(_I(ni), _I(nj), _I(nk), _dp(a), _I(ha), _dp(b), _I(hb),
                                       _dp(c), _I(hc), _dp(g), _I(hg), _dp(lam), _I(e), _I(e)),
           "thomas_transpose")
    return lam


def vadv(h, hh, w, hw, a, ha, b, hb, c, hc, dt, e=0):
    lib = _load()
    h, w, a, b, c = map(_f64, (h, w, a, b, c))
    ni, nj, nk = _dims(h, hh)
    x = padded(ni, nj, nk, e)
    _check(lib.oracle_vadv(_I(ni), _I(nj), _I(nk), _dp(h), _I(hh), _dp(w), _I(hw), _dp(a), _I(ha),
                           _dp(b), _I(hb), _dp(c), _I(hc), _DBL(dt), _dp(x), _I(e), _I(e)), "vadv")
    return x


def hdiff_vadv(u, hu, coeff, hcf, w, hw, a, ha, b, hb, c, hc, dt, e=0):
    """The fused program x = vadv(hdiff(u, coeff), w, a, b, c, dt)."""
    lib = _load()
    u, coeff, w, a, b, c = map(_f64, (u, coeff, w, a, b, c))
    ni, nj, nk = _dims(u, hu)
    x = padded(ni, nj, nk, e)
    _check(lib.oracle_hdiff_vadv(_I(ni), _I(nj), _I(nk), _dp(u), _I(hu), _dp(coeff), _I(hcf),
                                 _dp(w), _I(hw), _dp(a), _I(ha), _dp(b), _I(hb), _dp(c), _I(hc),
                                 _DBL(dt), _dp(x), _I(e), _I(e)), "hdiff_vadv")
    return x


def vdiff(x, hx, kappa, e=0):
    lib = _load()
    x = _f64(x)
    ni, nj, nk = _dims(x, hx)
    y = padded(ni, nj, nk, e)
    _check(lib.oracle_vdiff(_I(ni), _I(nj), _I(nk), _dp(x), _I(hx), _DBL(kappa), _dp(y), _I(e),
                            _I(e)), "vdiff")
    return y


def vdiff_implicit(x, hx, kappa, e=0):
    """Implicit vertical diffusion with zero-flux ends (a tridiagonal solve per column)."""
    lib = _load()
    x = _f64(x)
    ni, nj, nk = _dims(x, hx)
    y = padded(ni, nj, nk, e)
    _check(lib.oracle_vdiff_implicit(_I(ni), _I(nj), _I(nk), _dp(x), _I(hx), _DBL(kappa), _dp(y),
                                     _I(e), _I(e)), "vdiff_implicit")
    return y


def hgrad(y, hy, beta_h, beta_v, e=0):
    lib = _load()
    y = _f64(y)
    ni, nj, nk = _dims(y, hy)
    z = padded(ni, nj, nk, e)
    _check(lib.oracle_hgrad(_I(ni), _I(nj), _I(nk), _dp(y), _I(hy), _DBL(beta_h), _DBL(beta_v),
                            _dp(z), _I(e), _I(e)), "hgrad")
    return z


def timestep(u, hu, coeff, hcf, w, hw, a, ha, b, hb, c, hc, dt, kappa, beta_h, beta_v,
             implicit=False):
    """One field of the batched timestep: hdiff -> vadv -> vdiff (explicit or
    implicit) -> hgrad."""
    lib = _load()
    u, coeff, w, a, b, c = map(_f64, (u, coeff, w, a, b, c))
    ni, nj, nk = _dims(u, hu)
    z = padded(ni, nj, nk, 0)
    _check(lib.oracle_timestep_ex(_I(ni), _I(nj), _I(nk), _dp(u), _I(hu), _dp(coeff), _I(hcf),
                                  _dp(w), _I(hw), _dp(a), _I(ha), _dp(b), _I(hb), _dp(c), _I(hc),
                                  _DBL(dt), _DBL(kappa), _DBL(beta_h), _DBL(beta_v),
                                  _I(1 if implicit else 0), _dp(z), _I(0)), "timestep")
    return z


def rhs_adjoint(h, hh, w, hw, dt, lam, hl):
    """Returns (gh, gw) on the interior (halo 0)."""
    lib = _load()
    h, w, lam = _f64(h), _f64(w), _f64(lam)
    ni, nj, nk = _dims(h, hh)
    gh, gw = padded(ni, nj, nk, 0), padded(ni, nj, nk, 0)
    _check(lib.oracle_rhs_adjoint(_I(ni), _I(nj), _I(nk), _dp(h), _I(hh), _dp(w), _I(hw), _DBL(dt),
                                  _dp(lam), _I(hl), _dp(gh), _I(0), _dp(gw), _I(0)), "rhs_adjoint")
    return gh, gw


def hdiff_adjoint(u, hu, coeff, hc, gh, hgh, force_kx=None, force_ky=None):
    """Returns (gu with halo 2, gcoeff with halo 0)."""
    lib = _load()
    u, coeff, gh = _f64(u), _f64(coeff), _f64(gh)
    ni, nj, nk = _dims(u, hu)
    gu, gcoeff = padded(ni, nj, nk, 2), padded(ni, nj, nk, 0)
    fkx = None if force_kx is None else np.ascontiguousarray(force_kx, dtype=np.uint8)
    fky = None if force_ky is None else np.ascontiguousarray(force_ky, dtype=np.uint8)
    _check(lib.oracle_hdiff_adjoint(_I(ni), _I(nj), _I(nk), _dp(u), _I(hu), _dp(coeff), _I(hc),
                                    _dp(gh), _I(hgh), _dp(gu), _I(2), _dp(gcoeff), _I(0), _u8(fkx),
                                    _u8(fky)), "hdiff_adjoint")
    return gu, gcoeff


def hdiff_vadv_adjoint(u, hu, coeff, hcf, w, hw, a, ha, b, hb, c, hc, dt, wl, hwl,
                       matrix=False, force_kx=None, force_ky=None):
    """Gradient of sum(wl * x) over the interior, x = hdiff_vadv(...).
    Returns (gu [halo 2], gcoeff, gwcon) and with matrix=True also (ga, gb, gc),
    all but gu on the interior (halo 0)."""
    lib = _load()
    u, coeff, w, a, b, c, wl = map(_f64, (u, coeff, w, a, b, c, wl))
    ni, nj, nk = _dims(u, hu)
    gu = padded(ni, nj, nk, 2)
    gcoeff, gw = padded(ni, nj, nk, 0), padded(ni, nj, nk, 0)
    ga = gb = gc = None
    if matrix:
        ga, gb, gc = padded(ni, nj, nk, 0), padded(ni, nj, nk, 0), padded(ni, nj, nk, 0)
    fkx = None if force_kx is None else np.ascontiguousarray(force_kx, dtype=np.uint8)
    fky = None if force_ky is None else np.ascontiguousarray(force_ky, dtype=np.uint8)
    rc = lib.oracle_hdiff_vadv_adjoint(
        _I(ni), _I(nj), _I(nk), _dp(u), _I(hu), _dp(coeff), _I(hcf), _dp(w), _I(hw), _dp(a),
        _I(ha), _dp(b), _I(hb), _dp(c), _I(hc), _DBL(dt), _dp(wl), _I(hwl), _dp(gu), _I(2),
        _dp(gcoeff), _I(0), _dp(gw), _I(0), _dp(ga), _dp(gb), _dp(gc), _I(0), _u8(fkx), _u8(fky))
    _check(rc, "hdiff_vadv_adjoint")
    if matrix:
        return gu, gcoeff, gw, ga, gb, gc
    return gu, gcoeff, gw


def hdiff_vadv_jvp(u, hu, coeff, hcf, w, hw, a, ha, b, hb, c, hc, dt, du=None, hdu=2, dcoeff=None,
                   hdcf=0, dw=None, hdw=0, da=None, db=None, dc=None, hdm=0, force_kx=None,
                   force_ky=None):
    """Forward mode: the tangent dx = J v of x = hdiff_vadv(...) in the
    direction v = (du, dcoeff, dw, da, db, dc), each None for a zero tangent,
    under the forward pass's limiter masks (or the forced ones).  du carries a
    halo hdu >= 2, dcoeff / dw halos hdcf / hdw, da / db / dc the halo hdm.
    Returns dx on the interior (halo 0)."""
    lib = _load()
    u, coeff, w, a, b, c = map(_f64, (u, coeff, w, a, b, c))
    du, dcoeff, dw, da, db, dc = (None if t is None else _f64(t) for t in (du, dcoeff, dw, da, db, dc))
    ni, nj, nk = _dims(u, hu)
    dx = padded(ni, nj, nk, 0)
    fkx = None if force_kx is None else np.ascontiguousarray(force_kx, dtype=np.uint8)
    fky = None if force_ky is None else np.ascontiguousarray(force_ky, dtype=np.uint8)
    rc = lib.oracle_hdiff_vadv_jvp(
        _I(ni), _I(nj), _I(nk), _dp(u), _I(hu), _dp(coeff), _I(hcf), _dp(w), _I(hw), _dp(a), _I(ha),
        _dp(b), _I(hb), _dp(c), _I(hc), _DBL(dt), _dp(du), _I(hdu), _dp(dcoeff), _I(hdcf), _dp(dw),
        _I(hdw), _dp(da), _dp(db), _dp(dc), _I(hdm), _dp(dx), _I(0), _u8(fkx), _u8(fky))
    _check(rc, "hdiff_vadv_jvp")
    return dx


def interior(a, h):
    """View of the interior of a padded array."""
    if h == 0:
        return a
    return a[:, h:-h, h:-h]
