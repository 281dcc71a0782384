"""Pin of the oracle's per-sample log-derivatives (used by VMC/SR, Sec. VI): reverse-mode
gradients against central finite differences (eps = 1e-6, FP64) on 16 random parameters, for
the Definition block and for phi injected into the h stream (Fig. 1c)."""
import numpy as np
import pytest
import torch

import dn_inputs as di
from oracle.grad import grad_logpsi, grad_logpsi_batched
from oracle.model import ModelDesc, forward


@pytest.mark.parametrize("inj,bc", [(0, "open"), (1, "open"), (1, "periodic")])
def test_gradient_matches_central_differences(inj, bc):
    shape = di.ModelShape(12, 2, 4, 3, bc=bc, act="silu", inject_phi=inj)
    desc = ModelDesc.of(shape)
    th = torch.tensor(di.draw_params(shape, 6005, "stress"))
    sp = torch.tensor(di.uniform_spins(2, 12, 3))
    G = grad_logpsi(desc, th, sp)
    G2 = grad_logpsi_batched(desc, th, sp)
    assert torch.allclose(G, G2, rtol=1e-12, atol=1e-14)
    rng = np.random.Generator(np.random.PCG64(6005))
    idx = rng.choice(th.numel(), size=16, replace=False)
    eps = 1e-6
    for k in idx:
        tp, tm = th.clone(), th.clone()
        tp[k] += eps
        tm[k] -= eps
        fd = (forward(desc, tp, sp)["logpsi"] - forward(desc, tm, sp)["logpsi"]) / (2 * eps)
        scale = max(G[:, k].abs().max().item(), 1e-8)
        assert (fd - G[:, k]).abs().max().item() <= 1e-6 * scale + 1e-10
