"""torch.autograd wrapper of the fused hdiff + vadv program.

The differentiable tensors are the flat device buffers of the fields
(``Field.buf``), so a gradient lands in the same halo-padded layout as its
field: the gradient of u covers the interior and the 2-cell ring that the
13-point diamond reads, those of coeff and wcon the interior; every other
element of a gradient buffer is zero.  The backward pass is the hand-written
adjoint (``stencil_hdiff_vadv_adjoint``) with the limiter decisions of the
forward pass held fixed; the gradients of the matrix a, b, c (interior; the
entries a(0) and c(K-1) outside the matrix get 0) come from the same
transposed solve and the saved forward result.  No gradient flows to dt.

Forward mode (``torch.autograd.forward_ad``) runs the hand-written tangent
kernel (``stencil_hdiff_vadv_jvp``) under the same frozen limiter decisions;
inputs without a tangent cost no loads.
"""
from __future__ import annotations

import torch

from . import binding as B


def _wrap(buf, like):
    return B.Field(buf, like.origin, like.ni, like.nj, like.nk, like.hi, like.hj, like.sj, like.sk,
                   like.dtype)


class HdiffVadv(torch.autograd.Function):
    """x.buf = HdiffVadv.apply(u.buf, coeff.buf, wcon.buf, a.buf, b.buf, c.buf, meta)
    with meta = (layout, dt): a Field whose layout every field of the call
    shares (the output and the gradients are allocated with it)."""

    @staticmethod
    def forward(ctx, u_buf, coeff_buf, wcon_buf, a_buf, b_buf, c_buf, meta):
        lay, dt = meta
        x_lay = lay
        u, coeff, wcon, a, b, c = (_wrap(t, lay) for t in (u_buf, coeff_buf, wcon_buf, a_buf, b_buf,
                                                           c_buf))
        x = x_lay.like(fill=0.0)
        B.stencil_hdiff_vadv(u, coeff, wcon, a, b, c, dt, x)
        ctx.save_for_backward(u_buf, coeff_buf, wcon_buf, a_buf, b_buf, c_buf, x.buf)
        ctx.save_for_forward(u_buf, coeff_buf, wcon_buf, a_buf, b_buf, c_buf, x.buf)
        ctx.set_materialize_grads(False)  # absent tangents / gradients arrive as None
        ctx.meta = meta
        return x.buf

    @staticmethod
    def jvp(ctx, du_buf, dcoeff_buf, dwcon_buf, da_buf, db_buf, dc_buf, _meta):
        lay, dt = ctx.meta
        u, coeff, wcon, a, b, c, x = (_wrap(t, lay) for t in ctx.saved_tensors)
        tan = [None if t is None else _wrap(t.contiguous(), lay)
               for t in (du_buf, dcoeff_buf, dwcon_buf, da_buf, db_buf, dc_buf)]
        dx = lay.like(fill=0.0)
        B.stencil_hdiff_vadv_jvp(u, coeff, wcon, a, b, c, dt, dx,
                                 x=x if any(t is not None for t in tan[3:]) else None,
                                 du=tan[0], dcoeff=tan[1], dwcon=tan[2], da=tan[3], db=tan[4], dc=tan[5])
        return dx.buf

    @staticmethod
    def backward(ctx, gx_buf):
        if gx_buf is None:
            return None, None, None, None, None, None, None
        lay, dt = ctx.meta
        x_lay = lay
        u, coeff, wcon, a, b, c, x = (_wrap(t, lay) for t in ctx.saved_tensors)
        w = _wrap(gx_buf.contiguous(), x_lay)
        gu, gcoeff, gwcon = (lay.like(fill=0.0) for _ in range(3))
        need = ctx.needs_input_grad
        gm = [lay.like(fill=0.0) if need[3 + q] else None for q in range(3)]
        B.stencil_hdiff_vadv_adjoint(u, coeff, wcon, a, b, c, dt, w, gu, gcoeff, gwcon,
                                     x=x if any(g is not None for g in gm) else None,
                                     ga=gm[0], gb=gm[1], gc=gm[2])
        return (gu.buf if need[0] else None, gcoeff.buf if need[1] else None,
                gwcon.buf if need[2] else None, *(g.buf if g is not None else None for g in gm),
                None)


def hdiff_vadv(u, coeff, wcon, a, b, c, dt):
    """Differentiable x = vadv(hdiff(u, coeff), wcon, a, b, c, dt) on Fields;
    returns a Field whose ``buf`` carries the autograd graph.  The function
    passes buffers through autograd and describes every one of them with u's
    layout, so all six fields must share it exactly (ValueError otherwise)."""
    lay = u.layout()
    for name, f in (("coeff", coeff), ("wcon", wcon), ("a", a), ("b", b), ("c", c)):
        if f.layout() != lay:
            raise ValueError("%s has layout %s but u has %s (origin, extents, halos, strides, dtype, "
                             "buffer size must match)" % (name, f.layout(), lay))
    buf = HdiffVadv.apply(u.buf, coeff.buf, wcon.buf, a.buf, b.buf, c.buf, (u, float(dt)))
    return _wrap(buf, u)
