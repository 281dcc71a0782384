"""torch.autograd.Function over the library's log psi and its hand-written backward.

``logpsi(model, params, spins)`` returns log psi(s_b) for every sample; its backward returns
d loss / d params = sum_b (d loss / d log psi_b) * O[b, :], where O are the per-sample
log-derivatives computed by dn_grad_logpsi (the contraction with the incoming gradient runs
in the library's kernels). The spins carry no gradient. The backward differentiates at the
parameters its forward saw: if the model has been given other parameters in between, it sets
the saved ones for the backward and restores the newer ones afterwards.
"""
from __future__ import annotations

import torch

from ._lib import Model


class _LogPsi(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, spins: torch.Tensor, model: Model):
        model.set_params(params.detach().to(torch.float64))
        out = model.logpsi(spins)
        ctx.model = model
        ctx.version = model.param_version
        ctx.params = model.params
        ctx.save_for_backward(spins)
        return out

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (spins,) = ctx.saved_tensors
        model = ctx.model
        newer = model.params if model.param_version != ctx.version else None
        if newer is not None:
            model.set_params(ctx.params)
        try:
            g = grad_out.detach()
            if g.is_complex():
                # complex log psi of real parameters: the incoming gradient is
                # dL/dRe log psi + i dL/dIm log psi, so dL/dtheta = sum_b Re(g_b) dRe O_b + Im(g_b) dIm O_b
                _, _, ws_r = model.grad_logpsi(spins, weights=g.real, want_grads=False)
                _, _, ws_i = model.grad_logpsi(spins, weights=g.imag, want_grads=False)
                wsum = ws_r.real + ws_i.imag
            else:
                _, _, wsum = model.grad_logpsi(spins, weights=g, want_grads=False)
        finally:
            if newer is not None:
                model.set_params(newer)
        return wsum.to(ctx.params.device), None, None


def logpsi(model: Model, params: torch.Tensor, spins: torch.Tensor) -> torch.Tensor:
    """log psi(s) [B] (float64; complex128 for a complex-output model), differentiable with
    respect to the flat (real) parameter vector."""
    return _LogPsi.apply(params, spins, model)
