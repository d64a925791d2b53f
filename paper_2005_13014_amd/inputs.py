"""Seeded synthetic inputs for the hdiff + vadv stencil program.

This module holds no arithmetic of the method itself: it only draws random
fields and rounds them to a storage precision.  Both the HIP path and the CPU
oracle are fed from here, so they see bit-identical inputs.

The paper evaluates COSMO/FV3 stencil programs on 128x128x60 and 256x256x60
domains (Sec. VII-A); their data is not available, so seeded synthetic fields
of the same structure stand in for it:

* u     ~ U(-1, 1)   over the whole halo-padded array (the halo is input data)
* coeff ~ U(0, 0.1)  diffusion coefficient per point
* wcon  ~ U(-1, 1)   vertical velocity
* a, c  ~ U(-0.4, 0) sub- and super-diagonal of the vertical system,
          a(k=0) = c(k=nk-1) = 0
* b     = 1 + |a| + |c| + U(0, 0.2)  (strictly diagonally dominant)
* w     ~ N(0, 1)    weights of the scalar loss sum(w * x) (adjoint only)

Every field is drawn over the full padded shape (nk, nj + 2h, ni + 2h) in C
order, in the order listed above, from ``numpy.random.Generator(PCG64(seed))``,
then rounded to the storage dtype (round-to-nearest-even) and returned as
float64 holding the exactly representable stored values.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 200513014

# The batched timestep: six independent subdomains of uneven size (I, J, K).
BATCHED_SUBDOMAINS = (
    (96, 96, 60),
    (128, 96, 64),
    (192, 128, 72),
    (256, 192, 80),
    (320, 256, 84),
    (384, 256, 90),
)
BATCHED_FIELDS = 8


def round_to(x: np.ndarray, storage: str) -> np.ndarray:
    """Round float64 values to the storage dtype and return them as float64.

    f32: IEEE round-to-nearest-even.  bf16: round to f32, then to bf16 by
    round-to-nearest-even on the upper 16 bits of the f32 pattern."""
    if storage == "f64":
        return np.ascontiguousarray(x, dtype=np.float64)
    f = np.ascontiguousarray(x, dtype=np.float32)
    if storage == "f32":
        return f.astype(np.float64)
    if storage == "bf16":
        bits = f.view(np.uint32).astype(np.uint64)
        bits = (bits + 0x7FFF + ((bits >> 16) & 1)) >> 16
        out = (bits.astype(np.uint32) << 16).view(np.float32)
        return out.astype(np.float64)
    raise ValueError("unknown storage dtype %r" % storage)


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """uint16 bit patterns of values that are exactly representable in bf16."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def fields(ni: int, nj: int, nk: int, halo: int, seed: int, storage: str = "f64",
           vadv: bool = True, loss: bool = False) -> dict:
    """Draw one problem instance.  Returns a dict of padded float64 arrays:
    'u', 'coeff' and, with vadv, 'wcon', 'a', 'b', 'c'; with loss, 'w'."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (nk, nj + 2 * halo, ni + 2 * halo)
    out = {}
    out["u"] = round_to(rng.uniform(-1.0, 1.0, shape), storage)
    out["coeff"] = round_to(rng.uniform(0.0, 0.1, shape), storage)
    if vadv:
        out.update(coefficients_vadv(rng, shape, storage))
    if loss:
        out["w"] = round_to(rng.standard_normal(shape), storage)
    return out


def coefficients_vadv(rng, shape, storage):
    wcon = round_to(rng.uniform(-1.0, 1.0, shape), storage)
    a = round_to(rng.uniform(-0.4, 0.0, shape), storage)
    c = round_to(rng.uniform(-0.4, 0.0, shape), storage)
    extra = rng.uniform(0.0, 0.2, shape)
    nk = shape[0]
    if nk > 0:
        a[0] = 0.0
        c[nk - 1] = 0.0
    b = round_to(1.0 + np.abs(a) + np.abs(c) + extra, storage)
    return {"wcon": wcon, "a": a, "b": b, "c": c}


def batched(storage: str = "f32", halo_u: int = 3, halo_coef: int = 3, subdomains=None,
            nfields: int = BATCHED_FIELDS) -> list:
    """Inputs of the batched timestep: for each subdomain s a dict with the
    shared 'coeff', 'wcon', 'a', 'b', 'c' (seed SEED_BASE + 4000 + 10 s + 9) and
    a list 'u' of nfields fields (seed SEED_BASE + 4000 + 10 s + f).  All arrays
    of one subdomain carry the same halo max(halo_u, halo_coef) so that they
    share one layout."""
    subs = BATCHED_SUBDOMAINS if subdomains is None else subdomains
    h = max(halo_u, halo_coef)
    out = []
    for s, (ni, nj, nk) in enumerate(subs):
        shape = (nk, nj + 2 * h, ni + 2 * h)
        rng = np.random.Generator(np.random.PCG64(SEED_BASE + 4000 + 10 * s + 9))
        d = {"shape": (ni, nj, nk), "halo": h}
        d["coeff"] = round_to(rng.uniform(0.0, 0.1, shape), storage)
        d.update(coefficients_vadv(rng, shape, storage))
        us = []
        for f in range(nfields):
            r = np.random.Generator(np.random.PCG64(SEED_BASE + 4000 + 10 * s + f))
            us.append(round_to(r.uniform(-1.0, 1.0, shape), storage))
        d["u"] = us
        out.append(d)
    return out
