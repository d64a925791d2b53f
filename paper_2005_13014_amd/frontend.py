"""A small stencil-program front end: the paper's method for programs beyond
the hand-written hdiff + vadv kernels.

A program is a sequence of *applies* (Sec. IV-A): each computes one value per
grid point from neighbourhood *accesses* of program inputs or of earlier
applies, with constant offsets in i and j (the paper's ``stencil.access`` with
its offset vector; levels are independent here: no k offsets).  Three passes
then produce one GPU kernel:

* **shape inference** (Sec. V-B): walking back from the outputs, the region
  each apply must be computed on and the halo each input must carry;
* **inlining** (Sec. V-A): every access to an apply is replaced by that
  apply's expression shifted by the access offset, so the kernel keeps no
  temporaries and recomputes instead;
* **unrolling** (Sec. V-A): each thread evaluates ``unroll`` consecutive
  points in j, which exposes the subexpressions they share to the compiler.

Code generation emits HIP source whose extents and strides are compile-time
constants (the paper specialises on static shapes, Sec. IV-B) and compiles it
at run time through the library (``stencil_rtc_compile``).  By default the
generated kernel is the paper's execution model: one thread per point (times
``unroll``), one level per workgroup layer, no synchronisation; ``tiled``
stages the inputs that are read at offsets in LDS over the halo shape
inference derived and marches each workgroup over a run of levels.

Example (horizontal diffusion, the ``hdiffsa`` benchmark)::

    prog = hdiff_program()
    k = compile_program(prog, "f32", like=u_field, unroll=2)
    k({"u": u, "coeff": coeff}, {"out": out})
"""
from __future__ import annotations

import ctypes

from . import binding as B

# ---------------------------------------------------------------------------
# Expressions
# ---------------------------------------------------------------------------


class Expr:
    def _wrap(self, v):
        return v if isinstance(v, Expr) else Num(float(v))

    def __add__(self, o):
        return Bin("+", self, self._wrap(o))

    def __radd__(self, o):
        return Bin("+", self._wrap(o), self)

    def __sub__(self, o):
        return Bin("-", self, self._wrap(o))

    def __rsub__(self, o):
        return Bin("-", self._wrap(o), self)

    def __mul__(self, o):
        return Bin("*", self, self._wrap(o))

    def __rmul__(self, o):
        return Bin("*", self._wrap(o), self)

    def __truediv__(self, o):
        return Bin("/", self, self._wrap(o))

    def __rtruediv__(self, o):
        return Bin("/", self._wrap(o), self)

    def __neg__(self):
        return Neg(self)

    def __gt__(self, o):
        return Cmp(">", self, self._wrap(o))

    def __lt__(self, o):
        return Cmp("<", self, self._wrap(o))

    def __ge__(self, o):
        return Cmp(">=", self, self._wrap(o))

    def __le__(self, o):
        return Cmp("<=", self, self._wrap(o))


class Num(Expr):
    def __init__(self, value):
        self.value = float(value)
        if self.value != self.value or self.value in (float("inf"), float("-inf")):
            raise ValueError("constants must be finite (%r)" % value)


class Acc(Expr):
    """Access of ``src`` (an Input or an Apply) at offset (di, dj)."""

    def __init__(self, src, di, dj):
        self.src, self.di, self.dj = src, int(di), int(dj)


class Bin(Expr):
    def __init__(self, op, a, b):
        self.op, self.a, self.b = op, a, b


class Neg(Expr):
    def __init__(self, a):
        self.a = a


class Cmp(Expr):
    def __init__(self, op, a, b):
        self.op, self.a, self.b = op, a, b


class Sel(Expr):
    def __init__(self, c, a, b):
        self.c, self.a, self.b = c, a, b


def select(cond, a, b):
    """cond ? a : b, evaluated branch-free in the generated code."""
    w = Expr()._wrap
    return Sel(cond, w(a), w(b))


class _Source:
    def __getitem__(self, off):
        di, dj = off
        return Acc(self, di, dj)


class Input(_Source):
    def __init__(self, name):
        self.name = name


class Apply(_Source):
    def __init__(self, name, body):
        self.name, self.body = name, body


class Program:
    """Inputs, applies in definition order (each may read inputs and earlier
    applies) and the applies that are outputs."""

    def __init__(self):
        self.inputs, self.applies, self.outputs = [], [], []

    def input(self, name):
        self._fresh(name)
        f = Input(name)
        self.inputs.append(f)
        return f

    def apply(self, name, body):
        self._fresh(name)
        if not isinstance(body, Expr):
            body = Num(body)
        for a in _accesses(body):
            if a.src not in self.inputs and a.src not in self.applies:
                raise ValueError("apply %r reads %r, which is not defined before it" % (name, a.src.name))
        ap = Apply(name, body)
        self.applies.append(ap)
        return ap

    def output(self, *applies):
        for a in applies:
            if a not in self.applies:
                raise ValueError("outputs must be applies of this program")
            self.outputs.append(a)

    def _fresh(self, name):
        if not name.isidentifier() or any(x.name == name for x in self.inputs + self.applies):
            raise ValueError("names must be fresh identifiers (%r)" % name)


def _children(e):
    if isinstance(e, (Bin, Cmp)):
        return (e.a, e.b)
    if isinstance(e, Neg):
        return (e.a,)
    if isinstance(e, Sel):
        return (e.c, e.a, e.b)
    return ()


def _accesses(e):
    out, stack = [], [e]
    while stack:
        x = stack.pop()
        if isinstance(x, Acc):
            out.append(x)
        stack.extend(_children(x))
    return out


# ---------------------------------------------------------------------------
# Shape inference (Sec. V-B)
# ---------------------------------------------------------------------------


def infer_shapes(prog):
    """Returns (growth, halo): growth[apply name] = (west, east, south, north),
    the cells beyond the interior on each side on which the apply is needed;
    halo[input name] the same for each input, i.e. the halo it must carry."""
    if not prog.outputs:
        raise ValueError("the program has no outputs")
    grow = {a.name: None for a in prog.applies}
    halo = {f.name: (0, 0, 0, 0) for f in prog.inputs}
    for o in prog.outputs:
        grow[o.name] = (0, 0, 0, 0)
    for ap in reversed(prog.applies):
        g = grow[ap.name]
        if g is None:
            continue  # not needed by any output
        for a in _accesses(ap.body):
            w, e, s, n = g
            need = (w - a.di, e + a.di, s - a.dj, n + a.dj)
            tbl = halo if isinstance(a.src, Input) else grow
            old = tbl[a.src.name] or (0, 0, 0, 0)
            tbl[a.src.name] = tuple(max(0, x, y) for x, y in zip(old, need))
    return grow, halo


# ---------------------------------------------------------------------------
# Inlining (Sec. V-A)
# ---------------------------------------------------------------------------


def inline(e, di=0, dj=0):
    """The expression with every access to an apply replaced by that apply's
    expression shifted by the access offset (and the whole shifted by
    (di, dj)): only input accesses remain."""
    if isinstance(e, Acc):
        if isinstance(e.src, Apply):
            return inline(e.src.body, di + e.di, dj + e.dj)
        return Acc(e.src, e.di + di, e.dj + dj)
    if isinstance(e, Num):
        return e
    if isinstance(e, Bin):
        return Bin(e.op, inline(e.a, di, dj), inline(e.b, di, dj))
    if isinstance(e, Cmp):
        return Cmp(e.op, inline(e.a, di, dj), inline(e.b, di, dj))
    if isinstance(e, Neg):
        return Neg(inline(e.a, di, dj))
    if isinstance(e, Sel):
        return Sel(inline(e.c, di, dj), inline(e.a, di, dj), inline(e.b, di, dj))
    raise TypeError(type(e))


# ---------------------------------------------------------------------------
# Code generation
# ---------------------------------------------------------------------------

# storage type -> (element type in memory, compute type, widening load, rounding store)
_TYPES = {
    "f64": ("double", "double", "%s", "%s"),
    "f32": ("float", "float", "%s", "%s"),
    # bfloat16: the upper half of a float; loads are exact, stores round to
    # nearest even (NaN stays NaN)
    "bf16": ("unsigned short", "float", "bf16_load(%s)", "bf16_round(%s)"),
}
_CTYPE = {k: v[1] for k, v in _TYPES.items()}

_BF16_HELPERS = """__device__ __forceinline__ float bf16_load(unsigned short b) {
    return __uint_as_float(static_cast<unsigned>(b) << 16);
}
__device__ __forceinline__ unsigned short bf16_round(float v) {
    const unsigned bits = __float_as_uint(v);
    const unsigned rne = (bits + 0x7fffu + ((bits >> 16) & 1u)) >> 16;
    return static_cast<unsigned short>((bits & 0x7fffffffu) > 0x7f800000u ? ((bits >> 16) | 0x40u) : rne);
}
"""


def _prelude(dtype):
    return _BF16_HELPERS if dtype == "bf16" else ""


def _emit(e, ctype, load):
    if isinstance(e, Num):
        v = repr(e.value)
        return "%s(%s)" % (ctype, v)
    if isinstance(e, Acc):
        return load(e.src.name, e.di, e.dj)
    if isinstance(e, Bin):
        return "(%s %s %s)" % (_emit(e.a, ctype, load), e.op, _emit(e.b, ctype, load))
    if isinstance(e, Cmp):
        return "(%s %s %s)" % (_emit(e.a, ctype, load), e.op, _emit(e.b, ctype, load))
    if isinstance(e, Neg):
        return "(-%s)" % _emit(e.a, ctype, load)
    if isinstance(e, Sel):
        return "(%s ? %s : %s)" % (_emit(e.c, ctype, load), _emit(e.a, ctype, load), _emit(e.b, ctype, load))
    raise TypeError(type(e))


TI, TJ = 64, 4  # threads per workgroup in i and j (256 lanes)


def generate(prog, dtype, ni, nj, nk, sj, sk, unroll=1, name="stencil_program", tiled=False, run=1):
    """HIP source of the inlined, unrolled program specialised on the extents
    (ni, nj, nk) and the strides (sj, sk) every field shares.  Kernel
    parameters: one pointer per input (interior origin), then one per output,
    in program order.  tiled: see generate_tiled."""
    if dtype not in _TYPES:
        raise ValueError("dtype must be f64, f32 or bf16")
    if unroll not in (1, 2, 4, 8):
        raise ValueError("unroll must be 1, 2, 4 or 8")
    if tiled:
        return generate_tiled(prog, dtype, ni, nj, nk, sj, sk, unroll, name, run)
    infer_shapes(prog)
    mt, ct, ld, stf = _TYPES[dtype]
    params = ["const %s *__restrict__ in_%s" % (mt, f.name) for f in prog.inputs]
    params += ["%s *__restrict__ out_%s" % (mt, o.name) for o in prog.outputs]
    lines = [_prelude(dtype) +
        "// Generated by the stencil front end: %d applies inlined into one kernel," % len(prog.applies),
        "// %d point(s) per thread along j; extents and strides are compile-time." % unroll,
        'extern "C" __global__ __launch_bounds__(%d) void %s(%s) {' % (TI * TJ, name, ", ".join(params)),
        "    constexpr int I = %d, J = %d, K = %d;" % (ni, nj, nk),
        "    constexpr long long SJ = %d, SK = %d;" % (sj, sk),
        "    const int i = blockIdx.x * %d + (threadIdx.x & %d);" % (TI, TI - 1),
        "    const int j0 = (blockIdx.y * %d + (threadIdx.x >> %d)) * %d;" % (TJ, TI.bit_length() - 1, unroll),
        "    const int k = blockIdx.z;",
        "    if (i >= I || k >= K) return;",
        "    const long long o0 = i + j0 * SJ + k * SK;",
    ]
    for u in range(unroll):
        def load(fname, di, dj, u=u):
            return ld % ("in_%s[o0 + %d + %d * SJ]" % (fname, di, dj + u))
        lines.append("    if (j0 + %d < J) {" % u)
        for o in prog.outputs:
            lines.append("        out_%s[o0 + %d * SJ] = %s;" % (o.name, u, stf % _emit(inline(o.body), ct, load)))
        lines.append("    }")
    lines.append("}")
    return "\n".join(lines) + "\n"


PF_TILED = 4  # levels in flight in the tiled form (even: the LDS tile alternates)


def generate_tiled(prog, dtype, ni, nj, nk, sj, sk, unroll, name, run):
    """Tiled form: a workgroup owns a 64 x (4 unroll) tile and marches over
    `run` consecutive levels.  Every input that is read at an offset is staged
    in LDS over the tile grown by the halo shape inference derived for it
    (loads outside the input's own halo are clamped onto valid cells: no point
    of the interior reads them); inputs read only at offset 0 are read at the
    thread's points.  The global loads of the next PF_TILED levels sit in a
    register ring, the LDS tile is double buffered, and one barrier closes
    each level."""
    _, halo = infer_shapes(prog)
    mt, ct, ld, stf = _TYPES[dtype]
    rj, nthr = TJ * unroll, TI * TJ
    staged = [f for f in prog.inputs if any(halo[f.name])]
    direct = [f for f in prog.inputs if not any(halo[f.name])]
    params = ["const %s *__restrict__ in_%s" % (mt, f.name) for f in prog.inputs]
    params += ["%s *__restrict__ out_%s" % (mt, o.name) for o in prog.outputs]
    L = [_prelude(dtype) +
        "// Generated by the stencil front end (tiled): %d applies inlined into one kernel," % len(prog.applies),
        "// %d point(s) per thread along j, LDS-staged inputs, %d level(s) per workgroup," % (unroll, run),
        "// loads %d levels ahead." % PF_TILED,
        'extern "C" __global__ __launch_bounds__(%d) void %s(%s) {' % (nthr, name, ", ".join(params)),
        "    constexpr int I = %d, J = %d, K = %d, RUN = %d, PF = %d, UJ = %d;" % (ni, nj, nk, run, PF_TILED, unroll),
        "    constexpr long long SJ = %d, SK = %d;" % (sj, sk),
        "    const int tx = threadIdx.x & %d, ty = threadIdx.x >> %d;" % (TI - 1, TI.bit_length() - 1),
        "    const int i0 = blockIdx.x * %d, jt = blockIdx.y * %d;" % (TI, rj),
        "    const int i = i0 + tx, j0 = jt + ty * UJ;",
        "    const int kbeg = blockIdx.z * RUN, kend = min(K, kbeg + RUN);",
    ]
    for f in staged:
        n_ = f.name
        w, e, s_, n = halo[n_]
        L += [
            "    // %s staged with halo (w %d, e %d, s %d, n %d)" % (n_, w, e, s_, n),
            "    constexpr int PX_%s = %d, PY_%s = %d, W_%s = %d, S_%s = %d;" % (n_, TI + w + e, n_, rj + s_ + n, n_, w, n_, s_),
            "    constexpr int NE_%s = (PX_%s * PY_%s + %d) / %d;" % (n_, n_, n_, nthr - 1, nthr),
            "    __shared__ %s t_%s[2][PX_%s * PY_%s];" % (ct, n_, n_, n_),
            "    long long o_%s[NE_%s];" % (n_, n_),
            "    for (int q = 0; q < NE_%s; ++q) {" % n_,
            "        const int e = min(static_cast<int>(threadIdx.x) + %d * q, PX_%s * PY_%s - 1);" % (nthr, n_, n_),
            "        const int x = min(max(i0 - W_%s + e %% PX_%s, %d), I - 1 + %d);" % (n_, n_, -max(w, e), max(w, e)),
            "        const int y = min(max(jt - S_%s + e / PX_%s, %d), J - 1 + %d);" % (n_, n_, -max(s_, n), max(s_, n)),
            "        o_%s[q] = x + y * SJ;" % n_,
            "    }",
            "    %s r_%s[PF][NE_%s];" % (mt, n_, n_),
        ]
    L += [
        "    long long od[UJ];",
        "    for (int u = 0; u < UJ; ++u) od[u] = min(i, I - 1) + min(j0 + u, J - 1) * SJ;",
    ]
    for f in direct:
        L.append("    %s r_%s[PF][UJ];" % (mt, f.name))
    L.append("    auto load = [&](int q, int k) {")
    L.append("        const long long ko = min(k, kend - 1) * SK;  // past the run: its last level again")
    for f in staged:
        L.append("        for (int n = 0; n < NE_%s; ++n) r_%s[q][n] = in_%s[ko + o_%s[n]];" % ((f.name,) * 4))
    for f in direct:
        L.append("        for (int u = 0; u < UJ; ++u) r_%s[q][u] = in_%s[ko + od[u]];" % (f.name, f.name))
    L += [
        "    };",
        "#pragma unroll",
        "    for (int q = 0; q < PF; ++q) load(q, kbeg + q);",
        "    for (int kk = kbeg; kk < kend; kk += PF) {",
        "#pragma unroll",
        "        for (int q = 0; q < PF; ++q) {",
        "            const int k = kk + q;",
        "            if (k >= kend) break;",
        "            const long long ko = k * SK;",
    ]
    for f in staged:
        n_ = f.name
        L += [
            "            %s *tb_%s = t_%s[q & 1];" % (ct, n_, n_),
            "            for (int n = 0; n < NE_%s; ++n)" % n_,
            "                if (threadIdx.x + %d * n < PX_%s * PY_%s) tb_%s[threadIdx.x + %d * n] = %s;"
            % (nthr, n_, n_, n_, nthr, ld % ("r_%s[q][n]" % n_)),
        ]
    for f in direct:
        L.append("            %s v_%s[UJ];" % (ct, f.name))
        L.append("            for (int u = 0; u < UJ; ++u) v_%s[u] = %s;" % (f.name, ld % ("r_%s[q][u]" % f.name)))
    L += [
        "            load(q, k + PF);",
        "            __syncthreads();",
        "            if (i < I) {",
    ]
    staged_names = [f.name for f in staged]
    for u in range(unroll):
        def load_expr(fname, di, dj, u=u):
            if fname in staged_names:
                return "tb_%s[(ty * UJ + %d + %d + S_%s) * PX_%s + tx + %d + W_%s]" % (
                    fname, u, dj, fname, fname, di, fname)
            return "v_%s[%d]" % (fname, u)
        L.append("                if (j0 + %d < J) {" % u)
        for o in prog.outputs:
            L.append("                    out_%s[ko + i + (j0 + %d) * SJ] = %s;"
                     % (o.name, u, stf % _emit(inline(o.body), ct, load_expr)))
        L.append("                }")
    L += ["            }", "        }", "    }", "}"]
    return "\n".join(L) + "\n"


class CompiledProgram:
    """A program compiled for one shape and storage type; call it with dicts
    of Fields (inputs and outputs by name).  Checks that every field has the
    shape, strides and dtype it was compiled for and that each input carries
    the halo shape inference derived."""

    def __init__(self, prog, dtype, ni, nj, nk, sj, sk, unroll=1, tiled=False):
        # dtype: storage of every field, "f64", "f32" or "bf16" (FP32 arithmetic)
        self.prog, self.dtype, self.unroll, self.tiled = prog, dtype, unroll, tiled
        self.shape, self.strides = (ni, nj, nk), (sj, sk)
        _, self.halo = infer_shapes(prog)
        # Tiled: levels per workgroup so that the launch has about 4096 workgroups.
        tiles = ((ni + TI - 1) // TI) * ((nj + TJ * unroll - 1) // (TJ * unroll))
        self.run = max(1, -(-nk // max(1, 4096 // max(1, tiles)))) if tiled else 1
        self.source = generate(prog, dtype, ni, nj, nk, sj, sk, unroll, tiled=tiled, run=self.run)
        self.handle = B.stencil_rtc_compile(self.source, "stencil_program")

    def __call__(self, inputs, outputs, stream=None):
        if not self.handle:
            raise RuntimeError("the compiled program has been closed")
        ni, nj, nk = self.shape
        args = []
        for f in self.prog.inputs:
            fld = inputs[f.name]
            self._check(fld, f.name)
            w, e, s, n = self.halo[f.name]
            if max(w, e) > fld.hi or max(s, n) > fld.hj:
                raise ValueError("input %s needs halo (%d, %d) in (i, j), has (%d, %d)"
                                 % (f.name, max(w, e), max(s, n), fld.hi, fld.hj))
            args.append(ctypes.c_void_p(fld.data_ptr()))
        for o in self.prog.outputs:
            fld = outputs[o.name]
            self._check(fld, o.name)
            args.append(ctypes.c_void_p(fld.data_ptr()))
        grid = ((ni + TI - 1) // TI, (nj + TJ * self.unroll - 1) // (TJ * self.unroll),
                (nk + self.run - 1) // self.run)
        B.stencil_rtc_launch(self.handle, grid, (TI * TJ, 1, 1), args, stream)

    def _check(self, fld, name):
        if (fld.ni, fld.nj, fld.nk) != self.shape or (fld.sj, fld.sk) != self.strides or fld.dtype != self.dtype:
            raise ValueError("field %s does not match the shape, strides or dtype compiled for" % name)

    def close(self):
        """Unloads the kernel (also on garbage collection and on leaving a
        ``with`` block)."""
        if self.handle:
            B.stencil_rtc_release(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the library may be gone
            pass


def compile_program(prog, dtype, like, unroll=1, tiled=False):
    """Compiles `prog` for fields laid out like the Field `like`; tiled
    selects the LDS-staged, level-marching form (generate_tiled) over the
    one-thread-per-point form."""
    return CompiledProgram(prog, dtype, like.ni, like.nj, like.nk, like.sj, like.sk, unroll, tiled)


def hdiff_program():
    """Horizontal diffusion written as a stencil program: Laplacian, limited
    fluxes in i and j, update (the operator definitions of the fused kernel)."""
    p = Program()
    u, coeff = p.input("u"), p.input("coeff")
    lap = p.apply("lap", 4.0 * u[0, 0] - u[1, 0] - u[-1, 0] - u[0, 1] - u[0, -1])
    fx = lap[1, 0] - lap[0, 0]
    flx = p.apply("flx", select(fx * (u[1, 0] - u[0, 0]) > 0.0, 0.0, fx))
    fy = lap[0, 1] - lap[0, 0]
    fly = p.apply("fly", select(fy * (u[0, 1] - u[0, 0]) > 0.0, 0.0, fy))
    out = p.apply("out", u[0, 0] - coeff[0, 0] * (flx[0, 0] - flx[-1, 0] + fly[0, 0] - fly[0, -1]))
    p.output(out)
    return p
