"""The stencil front end on the CPU: shape inference, inlining (checked by
evaluating the program stage by stage and inlined with NumPy on the same
inputs), the hdiff program against the FP64 oracle, code generation, and
the run-time compiler's error path (no GPU needed)."""
import numpy as np
import pytest

import oracle
from paper_2005_13014_amd import frontend as F
from paper_2005_13014_amd import inputs

H = 4  # common padding of the NumPy evaluation grid


def shift(a, di, dj):
    """out[..., j, i] = a[..., j + dj, i + di], NaN where that leaves the grid."""
    out = np.full_like(a, np.nan)
    nj, ni = a.shape[-2:]
    js, je = max(0, -dj), min(nj, nj - dj)
    is_, ie = max(0, -di), min(ni, ni - di)
    out[..., js:je, is_:ie] = a[..., js + dj:je + dj, is_ + di:ie + di]
    return out


def evaluate(e, env):
    """Pointwise value of expression e on the padded grid (NaN = undefined)."""
    if isinstance(e, F.Num):
        return np.full(next(iter(env.values())).shape, e.value)
    if isinstance(e, F.Acc):
        return shift(env[e.src.name], e.di, e.dj)
    if isinstance(e, F.Neg):
        return -evaluate(e.a, env)
    if isinstance(e, F.Bin):
        a, b = evaluate(e.a, env), evaluate(e.b, env)
        if e.op == "/":
            return a / b
        return a + b if e.op == "+" else a - b if e.op == "-" else a * b
    if isinstance(e, F.Cmp):
        a, b = evaluate(e.a, env), evaluate(e.b, env)
        with np.errstate(invalid="ignore"):
            v = {">": a > b, "<": a < b, ">=": a >= b, "<=": a <= b}[e.op].astype(float)
        v[np.isnan(a) | np.isnan(b)] = np.nan
        return v
    if isinstance(e, F.Sel):
        c, a, b = evaluate(e.c, env), evaluate(e.a, env), evaluate(e.b, env)
        v = np.where(c == 1.0, a, b)
        v[np.isnan(c)] = np.nan
        return v
    raise TypeError(type(e))


def padded_inputs(arrays, halo):
    """Inputs embedded in the common grid; NaN beyond each one's own halo."""
    env = {}
    for name, a in arrays.items():
        g = np.full((a.shape[0], a.shape[1] - 2 * halo[name] + 2 * H, a.shape[2] - 2 * halo[name] + 2 * H), np.nan)
        d = H - halo[name]
        g[:, d:d + a.shape[1], d:d + a.shape[2]] = a
        env[name] = g
    return env


def staged(prog, env):
    """Every apply over the whole grid in definition order (no inlining)."""
    env = dict(env)
    for ap in prog.applies:
        env[ap.name] = evaluate(ap.body, env)
    return env


def interior(a):
    return a[:, H:-H, H:-H]


def test_shape_inference_of_hdiff():
    grow, halo = F.infer_shapes(F.hdiff_program())
    assert halo == {"u": (2, 2, 2, 2), "coeff": (0, 0, 0, 0)}
    assert grow == {"lap": (1, 1, 1, 1), "flx": (1, 0, 0, 0), "fly": (0, 0, 1, 0), "out": (0, 0, 0, 0)}


def test_shape_inference_asymmetric_and_unused():
    p = F.Program()
    a, b = p.input("a"), p.input("b")
    t = p.apply("t", a[2, 0] + a[0, -1])
    p.apply("unused", b[5, 5])
    o = p.apply("o", t[0, 3] - t[-1, 0])
    p.output(o)
    grow, halo = F.infer_shapes(p)
    assert grow["t"] == (1, 0, 0, 3) and grow["unused"] is None
    # a is read at (2, 0) and (0, -1) from t's region [-1, I) x [0, J+3)
    assert halo["a"] == (1, 2, 1, 3) and halo["b"] == (0, 0, 0, 0)


def test_program_validation():
    with pytest.raises(ValueError):
        F.Num(float("nan"))
    with pytest.raises(ValueError):
        F.Program().input("u")[0, 0] * float("inf")
    p = F.Program()
    u = p.input("u")
    with pytest.raises(ValueError):
        p.input("u")
    q = F.Program()
    foreign = q.apply("x", q.input("v")[0, 0])
    with pytest.raises(ValueError):
        p.apply("y", u[0, 0] + foreign[0, 0])
    with pytest.raises(ValueError):
        F.infer_shapes(p)  # no outputs
    with pytest.raises(ValueError):
        p.output(foreign)


@pytest.mark.parametrize("seed", [1, 2])
def test_inlining_preserves_the_program(seed):
    f = inputs.fields(11, 9, 3, 2, seed=seed, vadv=False)
    prog = F.hdiff_program()
    env = padded_inputs({"u": f["u"], "coeff": f["coeff"]}, {"u": 2, "coeff": 2})
    ref = interior(staged(prog, env)["out"])
    got = interior(evaluate(F.inline(prog.outputs[0].body), env))
    assert not np.isnan(ref).any()
    assert np.array_equal(got, ref)


def test_hdiff_program_is_the_oracle_operator():
    f = inputs.fields(13, 10, 4, 2, seed=3, vadv=False)
    prog = F.hdiff_program()
    env = padded_inputs({"u": f["u"], "coeff": f["coeff"]}, {"u": 2, "coeff": 2})
    got = interior(staged(prog, env)["out"])
    ref = oracle.hdiff(f["u"], 2, f["coeff"], 2)
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()


def test_shape_inference_is_sufficient_and_tight():
    # With exactly the inferred halo the output interior is defined; one cell
    # less on any side leaves some of it undefined.
    prog = F.hdiff_program()
    f = inputs.fields(8, 7, 2, 2, seed=4, vadv=False)
    body = F.inline(prog.outputs[0].body)
    env = padded_inputs({"u": f["u"], "coeff": f["coeff"]}, {"u": 2, "coeff": 2})
    assert not np.isnan(interior(evaluate(body, env))).any()
    small = f["u"][:, 1:-1, 1:-1]
    env = padded_inputs({"u": small, "coeff": f["coeff"]}, {"u": 1, "coeff": 2})
    assert np.isnan(interior(evaluate(body, env))).any()


def test_generated_source():
    prog = F.hdiff_program()
    src = F.generate(prog, "f64", 64, 48, 60, 72, 72 * 52, unroll=4)
    assert "constexpr int I = 64, J = 48, K = 60;" in src
    assert "constexpr long long SJ = 72, SK = 3744;" in src
    assert src.count("if (j0 + ") == 4 and src.count("out_out[") == 4
    assert "in_u" in src and "in_coeff" in src and "lap" not in src.split("{", 1)[1]  # no temporaries
    assert "double" in src and "float" not in src
    with pytest.raises(ValueError):
        F.generate(prog, "f16", 8, 8, 1, 12, 144)
    b = F.generate(prog, "bf16", 8, 8, 1, 16, 192)
    assert "unsigned short *__restrict__ out_out" in b and "bf16_round(" in b and "bf16_load(" in b
    with pytest.raises(ValueError):
        F.generate(prog, "f32", 8, 8, 1, 12, 144, unroll=3)


def test_compile_errors_come_back_with_the_log():
    from paper_2005_13014_amd import binding as B
    with pytest.raises(B.StencilError) as ex:
        B.stencil_rtc_compile('extern "C" __global__ void k(float *x) { x[0] = undeclared_name; }', "k")
    assert ex.value.code == 9 and "undeclared_name" in str(ex.value)
