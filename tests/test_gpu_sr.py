"""GPU stochastic-reconfiguration update (dn_sr_update, conjugate gradients) against the FP64
oracle's dense solve (Sec. II and VI; App. "Network parameters": standard SR, diagonal shift).

* one update from Monte Carlo samples (uniform or given weights): the oracle computes its own
  log-derivatives and local energies from the same parameters and spins and solves
  (S + shift I) x = F by Cholesky; float64: <= 1e-8 relative, float32 log-derivatives: 1e-4;
* a VMC run with exact enumeration (every configuration, weights |psi|^2 / Z) on the GPU: the
  energy the update reports equals the oracle's exact energy at the same parameters at every
  step, and it approaches the ground-state energy of the dense Hamiltonian, with and without
  phi injected into the h stream.
"""
import sys

import numpy as np
import pytest
import torch

import dn_inputs as di
import oracle as O
from oracle.grad import grad_logpsi_batched
from oracle.model import ModelDesc
from oracle.vmc import all_configs, exact_energy, sr_update
from test_oracle_hamiltonian import dense_h

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2603_11189_amd import _lib
    _lib.lib()
    return _lib


@pytest.mark.parametrize("prec,weighted", [("fp64", False), ("fp64", True), ("fp32", False)])
def test_sr_update_matches_dense_solve(L, prec, weighted):
    shape = di.ModelShape(12, 2, 4, 2, bc="open")
    ham = di.HamSpec("lrtfim", "open", J=-1.0, alpha=2.0, h=-0.8)
    desc = ModelDesc.of(shape)
    th = torch.tensor(di.draw_params(shape, 51, "stress"))
    m = L.Model(shape, prec)
    m.set_params(th)
    B = 48
    sp = di.uniform_spins(B, shape.N, 52)
    spd = torch.tensor(sp, device="cuda")
    _, g, _ = m.grad_logpsi(spd)
    _, _, el = m.eloc(ham, spd, shape.N)
    w = None
    w_ref = torch.full((B,), 1.0 / B, dtype=torch.float64)
    if weighted:
        rng = np.random.Generator(np.random.PCG64(53))
        wr = rng.random(B)
        w_ref = torch.tensor(wr / wr.sum())
        w = w_ref.cuda()
    shift, eta = 1e-2, 0.1
    delta, energy, iters = m.sr_update(g, el, w, shift=shift, eta=eta, max_iter=1000, tol=1e-13)
    ref_O = grad_logpsi_batched(desc, th, sp)
    ref = O.eloc_plain(desc, ham, th, sp, shape.N)
    ref_delta = sr_update(ref_O, ref["eloc"], w_ref, shift, eta)
    e = (delta.cpu() - ref_delta).norm().item() / ref_delta.norm().item()
    e_E = abs(energy.item() - (w_ref * ref["eloc"]).sum().item())
    _say(f"sr {prec} weighted={weighted}: P={ref_O.shape[1]} CG iterations {iters}, rel err of delta {e:.3e}, "
         f"|d E| {e_E:.3e}")
    assert e <= (1e-8 if prec == "fp64" else 1e-4)
    assert e_E <= (1e-12 if prec == "fp64" else 1e-6) * max(1.0, abs(energy.item()))
    m.close()


@pytest.mark.parametrize("inj", [0, 1])
def test_vmc_with_exact_enumeration_approaches_ground_state(L, inj):
    # inj: phi injected into the h stream (the estimator, gradients and SR of that block)
    shape = di.ModelShape(6, 1, 3, 2, act="tanh", bc="open", inject_phi=inj)
    ham = di.HamSpec("lrtfim", "open", J=-1.0, alpha=2.0, h=-0.6)
    desc = ModelDesc.of(shape)
    th = torch.tensor(di.draw_params(shape, 31, "stress")).cuda()
    m = L.Model(shape, "fp64")
    confs = all_configs(shape.N).cuda()
    e0 = float(np.linalg.eigvalsh(dense_h(ham, shape.N)).min())
    hist = []
    for it in range(25):
        m.set_params(th)
        lp, g, _ = m.grad_logpsi(confs)
        _, _, el = m.eloc(ham, confs, shape.N)
        p = torch.exp(2 * (lp - lp.max()))
        w = p / p.sum()
        shift = 1e-2 + (1e-4 - 1e-2) * it / 24
        delta, energy, _ = m.sr_update(g, el, w, shift=shift, eta=0.05, max_iter=500, tol=1e-12)
        E_ref = exact_energy(desc, ham, th.cpu())
        assert abs(energy.item() - E_ref) <= 1e-10 * abs(E_ref)
        hist.append(energy.item())
        th = th + delta
    _say(f"vmc (inject {inj}): E {hist[0]:.6f} -> {hist[-1]:.6f} (ground state {e0:.6f})")
    assert hist[-1] < hist[0]
    assert hist[-1] - e0 <= 0.1 * (hist[0] - e0)
    m.close()
