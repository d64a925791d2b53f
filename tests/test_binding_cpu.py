"""Host-side checks of the Python layer that need no GPU: the autograd
wrapper refuses fields whose layouts differ from u's (it describes every
buffer with u's layout), and Field.like reproduces a layout exactly."""
import pytest

torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_2005_13014_amd.binding")
from paper_2005_13014_amd import autograd as AG  # noqa: E402


def fields(**over):
    base = dict(ni=20, nj=9, nk=6, halo=2, dtype="f64")
    out = {}
    for n in ("u", "coeff", "wcon", "a", "b", "c"):
        kw = dict(base)
        kw.update(over.get(n, {}))
        out[n] = B.Field.empty(kw["ni"], kw["nj"], kw["nk"], kw["halo"], kw["dtype"], device="cpu", fill=0.0)
    return out


@pytest.mark.parametrize("name,change", [
    ("coeff", {"halo": 0}),       # narrower halo: smaller buffer, other strides
    ("wcon", {"halo": 3}),
    ("a", {"ni": 19}),
    ("c", {"dtype": "f32"}),
])
def test_autograd_refuses_a_different_layout(name, change):
    f = fields(**{name: change})
    with pytest.raises(ValueError, match=name):
        AG.hdiff_vadv(f["u"], f["coeff"], f["wcon"], f["a"], f["b"], f["c"], 10.0)


def test_autograd_refuses_same_shape_other_origin():
    f = fields()
    g = f["coeff"]
    f["coeff"] = B.Field(g.buf, g.origin + 1, g.ni, g.nj, g.nk, g.hi, g.hj, g.sj, g.sk, g.dtype)
    with pytest.raises(ValueError, match="coeff"):
        AG.hdiff_vadv(f["u"], f["coeff"], f["wcon"], f["a"], f["b"], f["c"], 10.0)


def test_like_keeps_the_layout():
    u = B.Field.empty(20, 9, 6, 2, "f64", device="cpu", hj=3, fill=1.0)
    v = u.like(fill=0.0)
    assert v.layout() == u.layout()
    assert float(v.buf.abs().sum()) == 0.0
    w = u.like(halo=1)
    assert (w.hi, w.hj) == (1, 1)
