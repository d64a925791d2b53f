"""ctypes binding of libstencil.so (the C ABI declared in include/stencil.h).

Argument marshalling only: every function here forwards to the C entry point
of the same name, which validates on the host and enqueues HIP kernels on the
current torch stream.  There is no fallback: without the built library, or
with fields that are not on a GPU, calls raise.

Fields are halo-padded 3D arrays in device memory (``Field``), laid out
i-fastest with row and plane strides padded so that every row's first
interior element is 128-byte aligned and the interior origin 256-byte
aligned.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstencil.so")

F64, F32, BF16 = 0, 1, 2
DTYPE_CODE = {"f64": F64, "f32": F32, "bf16": BF16}
TORCH_DTYPE = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}
ELEM_SIZE = {"f64": 8, "f32": 4, "bf16": 2}

LEVEL_DEFAULT, LEVEL_ORIGINAL, LEVEL_INLINE = 0, 1, 2
STAGE_HDIFF, STAGE_VADV, STAGE_VDIFF, STAGE_HGRAD, STAGE_VDIFF_IMPLICIT = 1, 2, 4, 8, 16
PROGRAM_GRAPH, PROGRAM_AUTOTUNE, PROGRAM_STAGED = 1, 2, 4

STATUS = {0: "OK", 1: "E_NULL", 2: "E_DTYPE", 3: "E_SHAPE", 4: "E_STRIDE", 5: "E_HALO",
          6: "E_ALIAS", 7: "E_UNSUPPORTED", 8: "E_HIP", 9: "E_ARG"}


class StencilError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s: %s" % (STATUS.get(code, code), message))
        self.code = code
        self.status = STATUS.get(code, str(code))


class FieldDesc(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("ni", ctypes.c_int32),
                ("nj", ctypes.c_int32), ("nk", ctypes.c_int32), ("hi", ctypes.c_int32),
                ("hj", ctypes.c_int32), ("sj", ctypes.c_int64), ("sk", ctypes.c_int64)]


class Config(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("unroll", ctypes.c_int32), ("tile_j", ctypes.c_int32),
                ("prefetch", ctypes.c_int32), ("nontemporal", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("tile_i", ctypes.c_int32)]


class Subdomain(ctypes.Structure):
    _fields_ = [("coeff", FieldDesc), ("wcon", FieldDesc), ("a", FieldDesc), ("b", FieldDesc),
                ("c", FieldDesc), ("nfields", ctypes.c_int32), ("u", ctypes.POINTER(FieldDesc)),
                ("z", ctypes.POINTER(FieldDesc))]


class Program(ctypes.Structure):
    _fields_ = [("nsub", ctypes.c_int32), ("sub", ctypes.POINTER(Subdomain)),
                ("stages", ctypes.c_int32), ("flags", ctypes.c_int32), ("dt", ctypes.c_double),
                ("kappa", ctypes.c_double), ("beta_h", ctypes.c_double),
                ("beta_v", ctypes.c_double)]


_P = ctypes.POINTER(FieldDesc)
_C = ctypes.POINTER(Config)
_V = ctypes.c_void_p
_SIGNATURES = {
    "stencil_hdiff": [_P, _P, _P, _C, _V],
    "stencil_vadv": [_P, _P, _P, _P, _P, ctypes.c_double, _P, _C, _V],
    "stencil_hdiff_vadv": [_P, _P, _P, _P, _P, _P, ctypes.c_double, _P, _C, _V],
    "stencil_hdiff_vadv_adjoint": [_P, _P, _P, _P, _P, _P, ctypes.c_double, _P, _P, _P, _P, _P, _P,
                                   _P, _P, _C, _V],
    "stencil_hdiff_vadv_adjoint_noalloc": [_P, _P, _P, _P, _P, _P, ctypes.c_double, _P, _P, _P, _P, _P,
                                           _P, _P, _P, _C, _V],
    "stencil_hdiff_vadv_jvp": [_P, _P, _P, _P, _P, _P, ctypes.c_double, _P, _P, _P, _P, _P, _P, _P, _P,
                               _C, _V],
    "stencil_program_run": [ctypes.POINTER(Program), _V],
    "stencil_halo_exchange": [ctypes.POINTER(FieldDesc), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _V],
    "stencil_halo_accumulate": [ctypes.POINTER(FieldDesc), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _V],
    "stencil_rtc_compile": [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)],
    "stencil_rtc_launch": [_V, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
                           ctypes.POINTER(ctypes.c_void_p), _V],
    "stencil_rtc_release": [_V],
    "stencil_last_error": [],
    "stencil_abi_version": [],
    "stencil_shutdown": [],
    "stencil_held_memory": [ctypes.POINTER(ctypes.c_int32)],
    "stencil_probe_copy": [_V, _V, ctypes.c_int64, _V],
    "stencil_probe_read": [_V, ctypes.c_int64, ctypes.c_uint32, _V, _V],
    "stencil_probe_streams": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, _V, ctypes.c_int64, _V],
}
EXPORTS = tuple(_SIGNATURES)

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libstencil.so is not built (run paper_2005_13014_amd/build.py)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGNATURES.items():
            fn = getattr(handle, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        handle.stencil_last_error.restype = ctypes.c_char_p
        handle.stencil_shutdown.restype = None
        handle.stencil_held_memory.restype = ctypes.c_int64
        _lib = handle
    return _lib


def _check(rc: int):
    if rc != 0:
        raise StencilError(rc, lib().stencil_last_error().decode())


def _round_up(v, a):
    return (v + a - 1) // a * a


class Field:
    """A halo-padded 3D field in device memory.

    ``buf`` is a flat torch tensor; the interior origin is element ``origin``
    of it, element (i, j, k) at ``origin + i + sj*j + sk*k``."""

    def __init__(self, buf, origin, ni, nj, nk, hi, hj, sj, sk, dtype):
        self.buf, self.origin = buf, origin
        self.ni, self.nj, self.nk, self.hi, self.hj = ni, nj, nk, hi, hj
        self.sj, self.sk, self.dtype = sj, sk, dtype

    # -- construction -------------------------------------------------------
    @classmethod
    def empty(cls, ni, nj, nk, halo=2, dtype="f32", device="cuda", hj=None, fill=None):
        hi, hj = halo, halo if hj is None else hj
        es = ELEM_SIZE[dtype]
        sj = _round_up(ni + 2 * hi, 128 // es)
        sk = sj * (nj + 2 * hj)
        origin = _round_up(hi + hj * sj, 256 // es)
        total = origin - hi - hj * sj + max(nk, 1) * sk + 256 // es
        buf = torch.empty(total, dtype=TORCH_DTYPE[dtype], device=device)
        if fill is not None:
            buf.fill_(fill)
        f = cls(buf, origin, ni, nj, nk, hi, hj, sj, sk, dtype)
        assert f.data_ptr() % 256 == 0 or buf.device.type == "cpu"
        return f

    @classmethod
    def from_numpy(cls, arr, halo, dtype="f32", device="cuda", fill_pad=0.0):
        """Field holding a dense padded float64 array of shape
        (nk, nj + 2 halo, ni + 2 halo); values must be representable in dtype."""
        nk, pj, pi = arr.shape
        f = cls.empty(pi - 2 * halo, pj - 2 * halo, nk, halo, dtype, device, fill=fill_pad)
        f.padded().copy_(torch.from_numpy(np.ascontiguousarray(arr)).to(TORCH_DTYPE[dtype]))
        return f

    # -- views --------------------------------------------------------------
    def _block(self):
        start = self.origin - self.hi - self.hj * self.sj
        return self.buf[start:start + self.nk * self.sk].view(self.nk, self.nj + 2 * self.hj,
                                                              self.sj)

    def padded(self):
        """View of shape (nk, nj + 2 hj, ni + 2 hi)."""
        return self._block()[:, :, :self.ni + 2 * self.hi]

    def interior(self):
        """View of shape (nk, nj, ni)."""
        return self.padded()[:, self.hj:self.hj + self.nj, self.hi:self.hi + self.ni]

    def to_numpy(self, interior=False):
        t = self.interior() if interior else self.padded()
        return t.detach().to("cpu", torch.float64).numpy().copy()

    def data_ptr(self):
        return self.buf.data_ptr() + self.origin * ELEM_SIZE[self.dtype]

    def desc(self) -> FieldDesc:
        return FieldDesc(self.data_ptr(), DTYPE_CODE[self.dtype], self.ni, self.nj, self.nk,
                         self.hi, self.hj, self.sj, self.sk)

    def like(self, halo=None, fill=None):
        """A new field of the same extents and dtype: with halo None, the same
        layout exactly (buffer size, origin, halos, strides); otherwise the
        standard layout with that halo."""
        if halo is None:
            buf = torch.empty_like(self.buf)
            if fill is not None:
                buf.fill_(fill)
            return Field(buf, self.origin, self.ni, self.nj, self.nk, self.hi, self.hj, self.sj, self.sk,
                         self.dtype)
        return Field.empty(self.ni, self.nj, self.nk, halo, self.dtype, self.buf.device, fill=fill)

    def layout(self):
        """Everything a descriptor takes from this field besides its buffer."""
        return (self.origin, self.ni, self.nj, self.nk, self.hi, self.hj, self.sj, self.sk, self.dtype,
                self.buf.numel())

    @property
    def shape(self):
        return (self.ni, self.nj, self.nk)


def _desc(f):
    if f is None:
        return None
    if isinstance(f, FieldDesc):
        return ctypes.byref(f)
    if f.buf.device.type != "cuda":
        raise ValueError("fields must live in GPU memory")
    return ctypes.byref(f.desc())


def config(level=0, unroll=0, tile_j=0, prefetch=0, nontemporal=0, schedule=0, tile_i=0):
    return Config(level, unroll, tile_j, prefetch, nontemporal, schedule, tile_i)


def _cfg(cfg):
    if cfg is None:
        return None
    if isinstance(cfg, dict):
        cfg = config(**cfg)
    return ctypes.byref(cfg)


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(stream)


# -- entry points (same names as the C ABI) ---------------------------------

def stencil_hdiff(u, coeff, out, cfg=None, stream=None):
    _check(lib().stencil_hdiff(_desc(u), _desc(coeff), _desc(out), _cfg(cfg), _stream(stream)))


def stencil_vadv(h, wcon, a, b, c, dt, x, cfg=None, stream=None):
    _check(lib().stencil_vadv(_desc(h), _desc(wcon), _desc(a), _desc(b), _desc(c), float(dt),
                              _desc(x), _cfg(cfg), _stream(stream)))


def stencil_hdiff_vadv(u, coeff, wcon, a, b, c, dt, x, cfg=None, stream=None):
    _check(lib().stencil_hdiff_vadv(_desc(u), _desc(coeff), _desc(wcon), _desc(a), _desc(b),
                                    _desc(c), float(dt), _desc(x), _cfg(cfg), _stream(stream)))


def stencil_hdiff_vadv_adjoint(u, coeff, wcon, a, b, c, dt, w, gu, gcoeff, gwcon, x=None, ga=None,
                               gb=None, gc=None, cfg=None, stream=None):
    """Reverse mode of x = vadv(hdiff(u)) for the loss sum(w * x): gu, gcoeff,
    gwcon, and with the forward result x also any of ga, gb, gc."""
    _check(lib().stencil_hdiff_vadv_adjoint(
        _desc(u), _desc(coeff), _desc(wcon), _desc(a), _desc(b), _desc(c), float(dt), _desc(w),
        _desc(gu), _desc(gcoeff), _desc(gwcon), _desc(x), _desc(ga), _desc(gb), _desc(gc), _cfg(cfg),
        _stream(stream)))


def stencil_hdiff_vadv_adjoint_noalloc(u, coeff, wcon, a, b, c, dt, w, gu, gcoeff, gwcon, x=None, ga=None,
                                       gb=None, gc=None, cfg=None, stream=None):
    """stencil_hdiff_vadv_adjoint through the entry point that allocates
    nothing (fixed device scratch of 128 MiB per device)."""
    _check(lib().stencil_hdiff_vadv_adjoint_noalloc(
        _desc(u), _desc(coeff), _desc(wcon), _desc(a), _desc(b), _desc(c), float(dt), _desc(w),
        _desc(gu), _desc(gcoeff), _desc(gwcon), _desc(x), _desc(ga), _desc(gb), _desc(gc), _cfg(cfg),
        _stream(stream)))


def stencil_hdiff_vadv_jvp(u, coeff, wcon, a, b, c, dt, dx, x=None, du=None, dcoeff=None, dwcon=None,
                           da=None, db=None, dc=None, cfg=None, stream=None):
    """Forward mode of x = vadv(hdiff(u)): the tangent dx in the direction
    (du, dcoeff, dwcon, da, db, dc), None tangents being zero; x (the forward
    result) is needed when any of da, db, dc is given."""
    _check(lib().stencil_hdiff_vadv_jvp(
        _desc(u), _desc(coeff), _desc(wcon), _desc(a), _desc(b), _desc(c), float(dt), _desc(x), _desc(du),
        _desc(dcoeff), _desc(dwcon), _desc(da), _desc(db), _desc(dc), _desc(dx), _cfg(cfg), _stream(stream)))


def stencil_rtc_compile(source, kernel_name):
    """Compiles generated HIP source; returns the kernel handle (an int)."""
    h = ctypes.c_void_p()
    _check(lib().stencil_rtc_compile(source.encode(), kernel_name.encode(), ctypes.byref(h)))
    return h.value


def stencil_rtc_launch(handle, grid, block, args, stream=None):
    """args: ctypes scalars / pointers, one per kernel parameter, in order."""
    g = (ctypes.c_uint32 * 3)(*grid)
    b = (ctypes.c_uint32 * 3)(*block)
    ptrs = (ctypes.c_void_p * len(args))(*[ctypes.cast(ctypes.pointer(a), ctypes.c_void_p) for a in args])
    _check(lib().stencil_rtc_launch(ctypes.c_void_p(handle), g, b, ptrs, _stream(stream)))


def stencil_rtc_release(handle):
    _check(lib().stencil_rtc_release(ctypes.c_void_p(handle)))


def stencil_program_run(prog, stream=None):
    if isinstance(prog, ProgramSpec):
        prog = prog.struct
    _check(lib().stencil_program_run(ctypes.byref(prog), _stream(stream)))


def _shares(shares, px, py):
    """The descriptor array of px * py Fields given row-major (p fastest)."""
    if len(shares) != px * py:
        raise ValueError("%d shares for a %d x %d decomposition" % (len(shares), px, py))
    arr = (FieldDesc * len(shares))()
    for n, f in enumerate(shares):
        if isinstance(f, FieldDesc):
            arr[n] = f
        else:
            if f.buf.device.type != "cuda":
                raise ValueError("fields must live in GPU memory")
            arr[n] = f.desc()
    return arr


def stencil_halo_exchange(shares, px, py, width, stream=None):
    """Fills the shares' halos from their neighbours' interiors (shares[p + px*q])."""
    _check(lib().stencil_halo_exchange(_shares(shares, px, py), int(px), int(py), int(width), _stream(stream)))


def stencil_halo_accumulate(shares, px, py, width, stream=None):
    """Adds the shares' halo cells into the neighbours' interior cells they mirror."""
    _check(lib().stencil_halo_accumulate(_shares(shares, px, py), int(px), int(py), int(width),
                                         _stream(stream)))


class ProgramSpec:
    """A stencil_program_t built from Fields; keeps the descriptor arrays alive.

    subdomains: list of dicts with Fields 'coeff', 'wcon', 'a', 'b', 'c' and
    lists of Fields 'u' and 'z' (same length)."""

    def __init__(self, subdomains, stages=STAGE_HDIFF | STAGE_VADV | STAGE_VDIFF | STAGE_HGRAD,
                 dt=10.0, kappa=0.1, beta_h=0.05, beta_v=0.01, flags=0):
        self._keep = []
        subs = (Subdomain * max(1, len(subdomains)))()
        for q, sd in enumerate(subdomains):
            n = len(sd["u"])
            assert len(sd["z"]) == n
            us = (FieldDesc * max(1, n))(*[f.desc() for f in sd["u"]])
            zs = (FieldDesc * max(1, n))(*[f.desc() for f in sd["z"]])
            self._keep += [us, zs]
            subs[q] = Subdomain(sd["coeff"].desc(), sd["wcon"].desc(), sd["a"].desc(), sd["b"].desc(),
                                sd["c"].desc(), n, us, zs)
        self._keep.append(subs)
        self.struct = Program(len(subdomains), subs, stages, flags, dt, kappa, beta_h, beta_v)


def stencil_probe_copy(src, dst, nbytes, stream=None):
    _check(lib().stencil_probe_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                    int(nbytes), _stream(stream)))


def stencil_probe_read(src, nbytes, key, sink, stream=None):
    _check(lib().stencil_probe_read(ctypes.c_void_p(src.data_ptr()), int(nbytes), int(key),
                                    ctypes.c_void_p(sink.data_ptr()), _stream(stream)))


def stencil_probe_streams(srcs, dst, nbytes, stream=None):
    arr = (ctypes.c_void_p * len(srcs))(*[t.data_ptr() for t in srcs])
    _check(lib().stencil_probe_streams(arr, len(srcs), ctypes.c_void_p(dst.data_ptr()), int(nbytes),
                                       _stream(stream)))


def stencil_last_error():
    return lib().stencil_last_error().decode()


def stencil_abi_version():
    return lib().stencil_abi_version()


def stencil_shutdown():
    lib().stencil_shutdown()


def stencil_held_memory():
    """(bytes of device memory the library holds, cached programs)."""
    n = ctypes.c_int32(0)
    b = lib().stencil_held_memory(ctypes.byref(n))
    return int(b), int(n.value)
