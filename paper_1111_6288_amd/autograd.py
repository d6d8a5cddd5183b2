"""``torch.autograd.Function`` around the HIP sign function and its adjoint.

``sign_apply(ctx, field, U, eta, x, q)`` returns y = s(U, eta) x for one RHS
of background group ``field`` with charge q, holding the group's small space,
the polynomial and the norm fixed (Sec. 2; background field of Sec. 4,
eq. (3)).  The backward calls ``ov_sign_backward`` and returns gradients in
PyTorch's complex convention (grad = dL/dRe + i dL/dIm, so dL = Re<grad, dz>):

* dL/dU for the base links, complex128 (4, V, 3, 3);
* dL/deta, a real 0-dim tensor;
* dL/dx = s g (s is Hermitian).

Each forward uploads U and sets (q, eta) of the group on the context, so
calls with different links or field strengths stay consistent.
"""
from __future__ import annotations

import torch


class SignApply(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ctx, field, U, eta, x, q, ckpt_every, prec):
        ctx.upload_gauge(U.detach().contiguous())
        ctx.set_field_eta(field, q, float(eta))
        y = ctx.sign_apply(x.detach().reshape(1, ctx.V, 4, 3).contiguous(), [field], prec=prec)[0]
        fctx.save_for_backward(U, x)
        fctx.ov = (ctx, field, float(eta), float(q), ckpt_every)
        return y

    @staticmethod
    def backward(fctx, gy):
        U, x = fctx.saved_tensors
        ctx, field, eta, q, ckpt = fctx.ov
        need_U, need_eta, need_x = fctx.needs_input_grad[2], fctx.needs_input_grad[3], fctx.needs_input_grad[4]
        ctx.upload_gauge(U.detach().contiguous())
        ctx.set_field_eta(field, q, eta)
        gU, geta, gx = ctx.sign_backward(field, x.detach().contiguous(), gy.detach().contiguous(), want_U=need_U,
                                         want_eta=need_eta, want_x=need_x, ckpt_every=ckpt)
        ge = torch.tensor(geta, dtype=torch.float64, device=x.device) if need_eta else None
        return None, None, gU, ge, (gx.reshape(x.shape) if need_x else None), None, None, None


def sign_apply(ctx, field, U, eta, x, q, ckpt_every=32, prec="fp64"):
    """y = s(U, eta) x with autograd support (see SignApply)."""
    if not torch.is_tensor(eta):
        eta = torch.tensor(float(eta), dtype=torch.float64)
    return SignApply.apply(ctx, field, U, eta, x, float(q), int(ckpt_every), prec)
