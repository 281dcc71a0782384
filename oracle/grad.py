"""Per-sample log-derivatives O_theta(s) = d log psi(s) / d theta, FP64 (test infrastructure only).

Reverse-mode automatic differentiation of ``model.forward`` (including the S4 kernel
generation, in complex128) with PyTorch's autograd on the CPU. These are the
log-derivatives that variational Monte Carlo with stochastic reconfiguration consumes
(Sec. VI, training paragraph). Pinned against central finite differences. For a
complex-output network O = d Re(log psi)/d theta + i d Im(log psi)/d theta (complex [B, P]).
"""
from __future__ import annotations

import torch

from .model import DT, forward


def grad_logpsi(desc, theta, spins) -> torch.Tensor:
    """[B, P] matrix of d log psi(s_b) / d theta."""
    theta = torch.as_tensor(theta, dtype=DT).detach()
    s = torch.as_tensor(spins)
    rows = []
    for b in range(s.shape[0]):
        th = theta.clone().requires_grad_(True)
        lp = forward(desc, th, s[b:b + 1])["logpsi"][0]
        if lp.is_complex():
            (gr,) = torch.autograd.grad(lp.real, th, retain_graph=True)
            (gi,) = torch.autograd.grad(lp.imag, th)
            rows.append(torch.complex(gr, gi))
        else:
            (g,) = torch.autograd.grad(lp, th)
            rows.append(g)
    return torch.stack(rows)


def grad_logpsi_batched(desc, theta, spins) -> torch.Tensor:
    """Same as grad_logpsi with one shared kernel generation (one backward per sample)."""
    theta = torch.as_tensor(theta, dtype=DT).detach().clone().requires_grad_(True)
    lp = forward(desc, theta, torch.as_tensor(spins))["logpsi"]
    rows = []
    for b in range(lp.shape[0]):
        keep = b + 1 < lp.shape[0]
        if lp.is_complex():
            (gr,) = torch.autograd.grad(lp[b].real, theta, retain_graph=True)
            (gi,) = torch.autograd.grad(lp[b].imag, theta, retain_graph=keep)
            rows.append(torch.complex(gr, gi))
        else:
            (g,) = torch.autograd.grad(lp[b], theta, retain_graph=keep)
            rows.append(g)
    return torch.stack(rows)
