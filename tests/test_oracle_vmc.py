"""Pins of the oracle's VMC/SR step (Sec. II and VI: variational Monte Carlo with stochastic
reconfiguration; App. "Network parameters": standard SR with a diagonal shift).

* the force is half the energy gradient: 2 F_k equals central differences (eps = 1e-6) of the
  exact variational energy <psi|H|psi>/<psi|psi>, enumerated over all 2^N configurations;
* the SR matrix S is symmetric positive semi-definite, and a small SR step lowers the exact energy;
* repeated SR steps with exact enumeration approach the ground-state energy of the dense
  Hamiltonian (built independently from Pauli bit operations, the same builder the Hamiltonian
  pins use).
"""
import numpy as np
import pytest
import torch

import dn_inputs as di
from oracle.model import ModelDesc
from oracle.vmc import exact_energy, exact_sr_inputs, sr_moments, sr_update
from test_oracle_hamiltonian import dense_h

SHAPE = di.ModelShape(6, 1, 3, 2, act="tanh", bc="open")
HAM = di.HamSpec("lrtfim", "open", J=-1.0, alpha=2.0, h=-0.6)


def test_force_is_half_the_energy_gradient():
    desc = ModelDesc.of(SHAPE)
    th = torch.tensor(di.draw_params(SHAPE, 31, "stress"))
    _, w, O, E = exact_sr_inputs(desc, HAM, th)
    _, F, _ = sr_moments(O, E, w)
    rng = np.random.Generator(np.random.PCG64(9))
    idx = rng.choice(th.numel(), size=10, replace=False)
    h = 1e-6
    scale = (2 * F).abs().max().item()
    for k in idx:
        tp, tm = th.clone(), th.clone()
        tp[k] += h
        tm[k] -= h
        fd = (exact_energy(desc, HAM, tp) - exact_energy(desc, HAM, tm)) / (2 * h)
        assert abs(2 * F[k].item() - fd) <= 1e-6 * scale + 1e-9, (int(k), 2 * F[k].item(), fd)


def test_sr_matrix_psd_and_small_step_descends():
    desc = ModelDesc.of(SHAPE)
    th = torch.tensor(di.draw_params(SHAPE, 31, "stress"))
    _, w, O, E = exact_sr_inputs(desc, HAM, th)
    Ebar, F, S = sr_moments(O, E, w)
    assert torch.allclose(S, S.T, atol=1e-14)
    assert torch.linalg.eigvalsh(S).min().item() >= -1e-12
    d = sr_update(O, E, w, shift=1e-3, eta=0.02)
    assert exact_energy(desc, HAM, th + d) < Ebar.item()


def test_sr_approaches_the_ground_state():
    desc = ModelDesc.of(SHAPE)
    th = torch.tensor(di.draw_params(SHAPE, 31, "stress"))
    e0 = float(np.linalg.eigvalsh(dense_h(HAM, SHAPE.N)).min())
    E_start = exact_energy(desc, HAM, th)
    hist = []
    for it in range(25):
        _, w, O, E = exact_sr_inputs(desc, HAM, th)
        shift = 1e-2 + (1e-4 - 1e-2) * it / 24  # the paper's linear diagonal-shift schedule
        th = th + sr_update(O, E, w, shift=shift, eta=0.05)
        hist.append(exact_energy(desc, HAM, th))
    assert hist[-1] < E_start
    assert hist[-1] - e0 <= 0.1 * (E_start - e0)
    assert hist[-1] >= e0 - 1e-9  # variational


def _complex_model():
    import dataclasses
    shape = dataclasses.replace(SHAPE, complex_out=1)
    th = torch.tensor(di.draw_params(shape, 31, "stress"))
    th[-2 * shape.d:] *= 5.0  # phases of order one
    return ModelDesc.of(shape), th


def test_complex_force_is_half_the_energy_gradient():
    """Complex psi, real parameters: 2 F = grad E with F = Re sum_b w_b conj(O_b - Obar)(E_b - E)."""
    desc, th = _complex_model()
    _, w, O, E = exact_sr_inputs(desc, HAM, th)
    assert O.is_complex() and E.imag.abs().max() > 1e-3
    Ebar, F, _ = sr_moments(O, E, w)
    assert abs(Ebar.imag) <= 1e-12 * abs(Ebar)  # <psi|H|psi> is real for a Hermitian H
    rng = np.random.Generator(np.random.PCG64(9))
    idx = rng.choice(th.numel(), size=10, replace=False)
    h = 1e-6
    scale = (2 * F).abs().max().item()
    for k in idx:
        tp, tm = th.clone(), th.clone()
        tp[k] += h
        tm[k] -= h
        fd = (exact_energy(desc, HAM, tp) - exact_energy(desc, HAM, tm)) / (2 * h)
        assert abs(2 * F[k].item() - fd) <= 1e-6 * scale + 1e-9, (int(k), 2 * F[k].item(), fd)


def test_complex_sr_matrix_psd_and_small_step_descends():
    desc, th = _complex_model()
    _, w, O, E = exact_sr_inputs(desc, HAM, th)
    Ebar, F, S = sr_moments(O, E, w)
    assert S.dtype == torch.float64 and F.dtype == torch.float64
    assert torch.allclose(S, S.T, atol=1e-14)
    assert torch.linalg.eigvalsh(S).min().item() >= -1e-12
    d = sr_update(O, E, w, shift=1e-3, eta=0.02)
    assert exact_energy(desc, HAM, th + d) < Ebar.real.item()
