"""The C ABI on the CPU: the library loads, exports exactly what the header
declares, and rejects invalid calls on the host with the documented codes
before anything touches a GPU (no compute call is made here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stencil.h")

B = pytest.importorskip("paper_2005_13014_amd.binding")

if not os.path.exists(B.LIB_PATH):
    pytest.skip("libstencil.so not built", allow_module_level=True)

# The validation tests hand the library descriptors with fake device pointers
# and expect a rejection before any launch; where a GPU is visible a call that
# slipped through validation would launch on them, so they run only without one.
_torch = pytest.importorskip("torch")
if _torch.cuda.is_available():
    pytest.skip("host-validation tests use fake device pointers; they run where no GPU is visible",
                allow_module_level=True)


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|void|const char \*)\s*(stencil_\w+)\s*\(", text,
                                 re.M)))


def test_header_declarations_are_exported():
    decl = declared_functions()
    assert len(decl) >= 9
    lib = B.lib()
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(B.EXPORTS) == decl


def test_only_the_abi_is_exported():
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    text_syms = sorted(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert text_syms == declared_functions()


def test_abi_version_matches_header():
    m = re.search(r"#define STENCIL_ABI_VERSION (\d+)", open(HEADER).read())
    assert B.stencil_abi_version() == int(m.group(1))


# ---- validation (host only) ------------------------------------------------

FAKE = 1 << 40          # never dereferenced: validation fails before any launch


def fd(origin=FAKE, dtype=1, ni=16, nj=12, nk=5, hi=2, hj=2, sj=None, sk=None):
    sj = ni + 2 * hi if sj is None else sj
    sk = sj * (nj + 2 * hj) if sk is None else sk
    return B.FieldDesc(origin, dtype, ni, nj, nk, hi, hj, sj, sk)


def spaced(n, **kw):
    """n descriptors with disjoint byte ranges."""
    out = []
    for q in range(n):
        out.append(fd(origin=FAKE + q * (1 << 30), **kw))
    return out


def hdiff(u, coeff, out, cfg=None):
    r = ctypes.byref
    return B.lib().stencil_hdiff(r(u) if u else None, r(coeff) if coeff else None,
                                 r(out) if out else None, r(cfg) if cfg else None, None)


def fused(fs, dt=10.0, cfg=None):
    r = ctypes.byref
    return B.lib().stencil_hdiff_vadv(*[r(f) for f in fs[:6]], dt, r(fs[6]),
                                      r(cfg) if cfg else None, None)


def vadv(fs, dt=10.0):
    r = ctypes.byref
    return B.lib().stencil_vadv(*[r(f) for f in fs[:5]], dt, r(fs[5]), None, None)


def adjoint(fs, x=None, ga=None, gb=None, gc=None, dt=10.0):
    """fs: u, coeff, wcon, a, b, c, w, gu, gcoeff, gwcon."""
    r = ctypes.byref
    opt = lambda f: r(f) if f is not None else None  # noqa: E731
    return B.lib().stencil_hdiff_vadv_adjoint(*[r(f) for f in fs[:6]], dt, *[r(f) for f in fs[6:10]],
                                              opt(x), opt(ga), opt(gb), opt(gc), None, None)


def test_adjoint_matrix_gradient_checks():
    fs = spaced(14)
    base, (x, ga, gb, gc) = fs[:10], fs[10:]
    # the matrix gradients need the forward result
    assert adjoint(base, ga=ga) == 1
    assert "forward result" in B.stencil_last_error()
    # an output overlapping an input, or another output
    bad = fd(origin=fs[3].origin + 64)
    assert adjoint(base, x=x, gb=bad) == 6
    assert adjoint(base, x=x, ga=ga, gc=ga) == 6
    # shape mismatch of an optional field
    assert adjoint(base, x=fd(origin=x.origin, ni=15), gb=gb) == 3
    # an empty interior is a no-op that still validates every field
    empty = spaced(14, nk=0)
    assert adjoint(empty[:10], x=empty[10], ga=empty[11], gb=empty[12], gc=empty[13]) == 0


def adjoint_noalloc(fs, dt=10.0):
    r = ctypes.byref
    return B.lib().stencil_hdiff_vadv_adjoint_noalloc(*[r(f) for f in fs[:6]], dt, *[r(f) for f in fs[6:10]],
                                                      None, None, None, None, None, None)


def test_noalloc_adjoint_limit_is_checked_on_the_host():
    # The fixed scratch holds 128 MiB: FP64 at 512 x 512 x 80 (two planes of
    # about 170 MB) is refused before anything touches a device; the same
    # validation as the scratch entry point comes first.
    sj = 516
    big = [fd(origin=FAKE + q * (1 << 36), dtype=0, ni=512, nj=512, nk=80, sj=sj, sk=sj * 516) for q in range(10)]
    assert adjoint_noalloc(big) == 7
    assert "fixed scratch" in B.stencil_last_error()
    assert adjoint_noalloc(spaced(10, nk=97)) == 7
    assert adjoint_noalloc(spaced(10)[:9] + [fd(origin=FAKE + 64)]) == 6
    assert adjoint_noalloc(spaced(10, nk=0)) == 0


def jvp(fs, x=None, du=None, dcoeff=None, dwcon=None, da=None, db=None, dc=None, dt=10.0):
    """fs: u, coeff, wcon, a, b, c, dx."""
    r = ctypes.byref
    opt = lambda f: r(f) if f is not None else None  # noqa: E731
    return B.lib().stencil_hdiff_vadv_jvp(*[r(f) for f in fs[:6]], dt, opt(x), opt(du), opt(dcoeff),
                                          opt(dwcon), opt(da), opt(db), opt(dc), r(fs[6]), None, None)


def test_jvp_argument_checks():
    fs = spaced(14)
    base, (x, du, dcoeff, dwcon, da, db, dc) = fs[:7], fs[7:]
    # the matrix tangents need the forward result
    assert jvp(base, db=db) == 1
    assert "forward result" in B.stencil_last_error()
    # du needs the 2-cell halo that u has
    assert jvp(base, du=fd(origin=du.origin, hi=1, hj=1, sj=du.sj, sk=du.sk)) == 5
    # the output may not overlap a tangent
    assert jvp(base[:6] + [fd(origin=dcoeff.origin + 64)], dcoeff=dcoeff) == 6
    # shape mismatch of a tangent
    assert jvp(base, dwcon=fd(origin=dwcon.origin, ni=15)) == 3
    # more levels than the kernel's buckets hold
    deep = spaced(7, nk=97)
    assert jvp(deep) == 7
    # an empty interior is a no-op that still validates every field
    empty = spaced(14, nk=0)
    assert jvp(empty[:7], x=empty[7], du=empty[8], dcoeff=empty[9], dwcon=empty[10], da=empty[11],
               db=empty[12], dc=empty[13]) == 0
    assert jvp(base, dt=float("nan")) == 9


def test_size_limits_of_the_column_kernels():
    # 32-bit buffer offsets: fields of 2 GiB or more are refused (the fused
    # level-INLINE call, the adjoint and the forward mode), before any launch.
    sk = 6 * 1024 * 1024              # FP32: 95 * sk * 4 B > 2 GiB at nk = 96
    big = [fd(origin=FAKE + q * (1 << 36), nk=96, sk=sk) for q in range(14)]
    r = ctypes.byref
    cfg = B.config(level=2)
    assert B.lib().stencil_hdiff_vadv(*[r(f) for f in big[:6]], 10.0, r(big[6]), r(cfg), None) == 7
    assert adjoint(big[:10]) == 7
    assert jvp(big[:7]) == 7
    # and more levels than the column buckets hold
    deep = [fd(origin=FAKE + q * (1 << 30), nk=97) for q in range(10)]
    assert adjoint(deep) == 7


def test_null_descriptor_and_origin():
    u, c, o = spaced(3)
    assert hdiff(None, c, o) == 1
    assert "NULL" in B.stencil_last_error()
    u.origin = None
    assert hdiff(u, c, o) == 1


def test_dtype_checks():
    u, c, o = spaced(3)
    c.dtype = 0
    assert hdiff(u, c, o) == 2
    u, c, o = spaced(3, dtype=7)
    assert hdiff(u, c, o) == 2


def test_shape_checks():
    u, c, o = spaced(3)
    o.nj = 11
    o.sk = o.sj * (11 + 4)
    assert hdiff(u, c, o) == 3
    u, c, o = spaced(3)
    u.ni = -1
    assert hdiff(u, c, o) == 3


def test_stride_checks():
    u, c, o = spaced(3)
    u.sj = u.ni + 3        # < ni + 2 hi
    assert hdiff(u, c, o) == 4
    u, c, o = spaced(3)
    u.sk = u.sj * u.nj     # cannot hold the j halo
    assert hdiff(u, c, o) == 4
    u, c, o = spaced(3, sj=40)
    c.sj = 41
    c.sk = 41 * 16
    assert hdiff(u, c, o) == 4


def test_halo_from_shape_inference():
    # hdiff reads a 2-cell halo of u (the 13-point diamond); coeff needs none.
    u, c, o = spaced(3, hi=1, hj=2)
    assert hdiff(u, c, o) == 5
    assert "halo" in B.stencil_last_error()
    fs = spaced(7, hi=1, hj=1)
    assert fused(fs) == 5


def test_alias_checks():
    u, c, o = spaced(3)
    o.origin = u.origin
    assert hdiff(u, c, o) == 6
    u, c, o = spaced(3)
    # out's first row overlaps the last plane of u
    o.origin = u.origin + 4 * (u.sk * (u.nk - 1))
    assert hdiff(u, c, o) == 6
    fs = spaced(7)
    fs[6].origin = fs[3].origin + 4 * 7
    assert fused(fs) == 6


def test_scalar_and_config_checks():
    u, c, o = spaced(3)
    assert hdiff(u, c, o, B.config(unroll=3)) == 9
    assert hdiff(u, c, o, B.config(level=7)) == 9
    assert fused(spaced(7), dt=float("nan")) == 9
    assert vadv(spaced(6), dt=float("inf")) == 9
    assert fused(spaced(7), cfg=B.config(tile_j=3, prefetch=4)) == 7
    assert fused(spaced(7), cfg=B.config(schedule=5)) == 9
    # four lanes per column need nk >= 8 (these fields have 5 levels)
    assert fused(spaced(7), cfg=B.config(schedule=4)) == 7
    assert fused(spaced(7), cfg=B.config(schedule=-1)) == 9
    assert fused(spaced(7), cfg=B.config(nontemporal=2)) == 9
    # a compiled tile shape with a schedule it is not compiled for
    assert fused(spaced(7), cfg=B.config(tile_j=1, prefetch=8, nontemporal=1, schedule=2)) == 7
    assert fused(spaced(7), cfg=B.config(tile_j=2, prefetch=8, nontemporal=1, schedule=3)) == 7


def test_offsets_beyond_32_bits_are_unsupported():
    u, c, o = spaced(3, ni=2000, nj=2000, nk=600)
    assert hdiff(u, c, o) == 7


def test_empty_interior_is_a_noop():
    for dims in ((0, 12, 5), (16, 0, 5), (16, 12, 0)):
        u, c, o = spaced(3, ni=dims[0], nj=dims[1], nk=dims[2])
        assert hdiff(u, c, o) == 0
        assert fused(spaced(7, ni=dims[0], nj=dims[1], nk=dims[2])) == 0


def test_probe_copy_validation():
    lib = B.lib()
    assert lib.stencil_probe_copy(None, ctypes.c_void_p(FAKE), 16, None) == 1
    assert lib.stencil_probe_copy(ctypes.c_void_p(FAKE), ctypes.c_void_p(FAKE + 1024), 17, None) == 9
    assert lib.stencil_probe_copy(ctypes.c_void_p(FAKE), ctypes.c_void_p(FAKE + 16), 64, None) == 6
    V = ctypes.c_void_p
    srcs = (V * 2)(FAKE, FAKE + (1 << 20))
    assert lib.stencil_probe_streams(srcs, 0, V(FAKE + (2 << 20)), 64, None) == 9
    assert lib.stencil_probe_streams(srcs, 9, V(FAKE + (2 << 20)), 64, None) == 9
    assert lib.stencil_probe_streams(srcs, 2, V(FAKE + 32), 64, None) == 6
    assert lib.stencil_probe_streams(srcs, 2, None, 64, None) == 1
    assert lib.stencil_probe_streams(srcs, 2, V(FAKE + (2 << 20)), 24, None) == 9
    assert lib.stencil_probe_read(None, 16, 0, ctypes.c_void_p(FAKE), None) == 1
    assert lib.stencil_probe_read(ctypes.c_void_p(FAKE), 16, 0, None, None) == 1
    assert lib.stencil_probe_read(ctypes.c_void_p(FAKE), 24, 0, ctypes.c_void_p(FAKE), None) == 9
    assert lib.stencil_probe_read(ctypes.c_void_p(FAKE + 8), 16, 0, ctypes.c_void_p(FAKE), None) == 9


# ---- batched program validation --------------------------------------------

FULL = 1 | 2 | 4 | 8


def program(halo_u=3, halo_c=1, stages=FULL, nsub=1, alias=False, nfields=2):
    keep = []
    subs = (B.Subdomain * max(1, nsub))()
    base = FAKE
    for s in range(nsub):
        def nxt(h):
            nonlocal base
            base += 1 << 30
            return fd(origin=base, hi=h, hj=h, sj=40, sk=40 * 40)
        coef = [nxt(halo_c) for _ in range(5)]
        us = (B.FieldDesc * nfields)(*[nxt(halo_u) for _ in range(nfields)])
        zs = (B.FieldDesc * nfields)(*[nxt(0) for _ in range(nfields)])
        if alias:
            zs[1].origin = us[0].origin
        keep += [us, zs]
        subs[s] = B.Subdomain(*coef, nfields, us, zs)
    keep.append(subs)
    return B.Program(nsub, subs, stages, 0, 10.0, 0.1, 0.05, 0.01), keep


def run_program(p):
    return B.lib().stencil_program_run(ctypes.byref(p), None)


def test_program_validation():
    assert B.lib().stencil_program_run(None, None) == 1
    p, keep = program(stages=1 | 4)
    assert run_program(p) == 9
    p, keep = program(stages=1 | 2 | 4 | 16)           # explicit and implicit vdiff together
    assert run_program(p) == 9
    p, keep = program(stages=1 | 2 | 16 | 8, halo_u=2)  # implicit chain with hgrad: u needs 3
    assert run_program(p) == 5
    p, keep = program(halo_u=2)                      # hgrad grows the domain: u needs 3
    assert run_program(p) == 5
    p, keep = program(halo_c=0)                      # coefficients need the 1-cell ring
    assert run_program(p) == 5
    p, keep = program(alias=True)
    assert run_program(p) == 6
    p, keep = program()
    p.dt = float("nan")
    assert run_program(p) == 9
    p, keep = program()
    p.flags = 8                                      # unknown flag
    assert run_program(p) == 9
    p, keep = program(halo_u=2)
    p.flags = 1 | 2 | 4                              # known flags pass, the halo check still runs
    assert run_program(p) == 5
    p, keep = program(nsub=0)
    assert run_program(p) == 0                       # an empty program is a no-op


# ---- spans of 2 GiB and more ---------------------------------------------------

def far(n, **kw):
    """n descriptors 64 GiB apart (room for the largest spans below)."""
    return [fd(origin=FAKE + q * (1 << 36), **kw) for q in range(n)]


@pytest.mark.parametrize("dtype,ni,nj,nk", [
    (0, 1024, 1024, 520),    # FP64, 4.4 GB
    (0, 1400, 1400, 1000),   # FP64, 15.9 GB
    (1, 1024, 1024, 1050),   # FP32, 4.5 GB
    (1, 1400, 1400, 1000),   # FP32, 7.9 GB
    (1, 1024, 1024, 600),    # FP32, 2.6 GB
    (2, 2000, 2000, 300),    # bf16, 2.4 GB
])
def test_hdiff_spans_beyond_the_inline_kernels_buffers(dtype, ni, nj, nk):
    # Element offsets fit in 32 bits, byte offsets do not: the inlined kernel
    # (raw buffers of < 2^31 bytes) must not run.  Asked for explicitly it is
    # refused; by default the unfused kernels take the call, which here (no
    # device) fails in the runtime before any launch rather than in the
    # inlined kernel's launch.
    u, c, o = far(3, dtype=dtype, ni=ni, nj=nj, nk=nk)
    span = ((ni + 3) + (nj + 3) * u.sj + (nk - 1) * u.sk + 1) * (8, 4, 2)[dtype]
    assert (ni + 3) + (nj + 3) * u.sj + (nk - 1) * u.sk < 2 ** 31 <= span
    assert hdiff(u, c, o, B.config(level=2)) == 7
    assert "below 2 GiB" in B.stencil_last_error()
    assert hdiff(u, c, o, B.config(unroll=4, level=2)) == 7
    rc = hdiff(u, c, o)
    assert rc == 8 and "hdiff kernel" not in B.stencil_last_error(), B.stencil_last_error()


def test_fused_spans_beyond_the_column_kernels_buffers():
    fs = far(7, dtype=0, ni=3000, nj=3000, nk=40)   # FP64, 2.9 GB per field
    r = ctypes.byref
    assert B.lib().stencil_hdiff_vadv(*[r(f) for f in fs[:6]], 10.0, r(fs[6]), r(B.config(level=2)),
                                      None) == 7
    assert adjoint_far(far(10, dtype=1, ni=3000, nj=3000, nk=80)) == 7


def adjoint_far(fs):
    r = ctypes.byref
    return B.lib().stencil_hdiff_vadv_adjoint(*[r(f) for f in fs[:6]], 10.0, r(fs[6]), r(fs[7]), r(fs[8]),
                                              r(fs[9]), None, None, None, None, None, None)


def halo(shares, px, py, width, accumulate=False):
    arr = (B.FieldDesc * len(shares))(*shares)
    fn = B.lib().stencil_halo_accumulate if accumulate else B.lib().stencil_halo_exchange
    return fn(arr, px, py, width, None)


@pytest.mark.parametrize("accumulate", [False, True])
def test_halo_exchange_validation(accumulate):
    def shares(nis, njs, **kw):
        out, n = [], 0
        for nj in njs:
            for ni in nis:
                out.append(fd(origin=FAKE + n * (1 << 30), ni=ni, nj=nj, **kw))
                n += 1
        return out

    ok = shares((16, 12, 9), (12, 7))
    assert halo([], 0, 1, 2, accumulate) == 9
    assert halo(shares((4,) * 9, (4,) * 8), 9, 8, 2, accumulate) == 9    # more than 64 shares
    assert halo(ok, 3, 2, 0, accumulate) == 9                              # width < 1
    assert halo(ok, 3, 2, 3, accumulate) == 5                              # halo 2 < width 3
    bad = list(ok)
    bad[4] = fd(origin=bad[4].origin, ni=13, nj=7)                         # ni differs within column 1
    assert halo(bad, 3, 2, 2, accumulate) == 3
    bad = list(ok)
    bad[5] = fd(origin=bad[5].origin, ni=9, nj=8)                          # nj differs within row 1
    assert halo(bad, 3, 2, 2, accumulate) == 3
    bad = list(ok)
    bad[2] = fd(origin=bad[2].origin, ni=9, nj=12, nk=4)                   # nk differs
    assert halo(bad, 3, 2, 2, accumulate) == 3
    bad = list(ok)
    bad[3] = fd(origin=bad[3].origin, dtype=0, ni=16, nj=7)                # dtype differs
    assert halo(bad, 3, 2, 2, accumulate) == 2
    bad = list(ok)
    bad[1] = fd(origin=ok[0].origin + 256, ni=12, nj=12)                   # overlapping shares
    assert halo(bad, 3, 2, 2, accumulate) == 6
    assert halo(shares((1, 12, 9), (12, 7)), 3, 2, 2, accumulate) == 3     # interior narrower than width
    assert halo(shares((16, 12, 9), (12, 7), nk=0), 3, 2, 2, accumulate) == 0   # empty: no-op
    assert halo(shares((16,), (12,)), 1, 1, 2, accumulate) == 0           # one share: nothing to exchange


def test_held_memory_starts_empty():
    n = ctypes.c_int32(-1)
    assert B.lib().stencil_held_memory(ctypes.byref(n)) == 0
    assert n.value == 0
    assert B.lib().stencil_held_memory(None) == 0
