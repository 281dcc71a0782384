"""Variational Monte Carlo with stochastic reconfiguration, FP64 on the CPU (test infrastructure
only).

Follows Sec. II (training by VMC and stochastic reconfiguration, Eq. (local-estimator)), Sec. VI
(natural-gradient descent: theta <- theta + eta * Delta-theta) and App. "Network parameters"
(standard SR, a diagonal shift). With samples s_b of weight w_b (sum_b w_b = 1: Monte Carlo
samples w_b = 1/B, or every configuration with w = |psi|^2 / Z for exact enumeration), the
log-derivatives O_bk = d log psi(s_b) / d theta_k and local energies E_b:
    E       = sum_b w_b E_b
    F_k     = sum_b w_b O_bk E_b - (sum_b w_b O_bk) E           (half the energy gradient)
    S_kl    = sum_b w_b O_bk O_bl - (sum_b w_b O_bk)(sum_b w_b O_bl)
    Delta   = -(S + shift * I)^-1 F,   theta <- theta + eta * Delta
(real parameters and a real, positive psi: no complex conjugates). A complex psi (complex read-out)
with real parameters has complex O and E_b; then F and S are the real parts of the same
moments with O conjugated on the left: F = Re sum_b w_b conj(O_b - Obar) (E_b - E),
S = Re sum_b w_b conj(O_b - Obar) (O_b - Obar)^T, and E is real up to sampling noise (its
imaginary part is reported as it comes). The solve here is a dense Cholesky factorisation; the
GPU solves the same system by conjugate gradients.
"""
from __future__ import annotations

import itertools

import torch

from .grad import grad_logpsi_batched
from .hamiltonian import connected, local_energy
from .model import DT, forward, plain_logratio


def sr_moments(O, E, w):
    """(E, F, S) of the definitions above."""
    O = torch.as_tensor(O)
    E = torch.as_tensor(E)
    w = torch.as_tensor(w, dtype=DT)
    if O.is_complex() or E.is_complex():
        O = O.to(torch.complex128)
        E = E.to(torch.complex128)
        Ebar = (w * E).sum()
        Oc = O - (w[:, None] * O).sum(0)
        F = (w[:, None] * Oc.conj() * (E - Ebar)[:, None]).sum(0).real
        S = (Oc.conj().T @ (w[:, None] * Oc)).real
        return Ebar, F, S
    O = O.to(DT)
    E = E.to(DT)
    Ebar = (w * E).sum()
    Obar = (w[:, None] * O).sum(0)
    Oc = O - Obar
    F = (w[:, None] * Oc * (E - Ebar)[:, None]).sum(0)
    S = Oc.T @ (w[:, None] * Oc)
    return Ebar, F, S


def sr_update(O, E, w, shift: float, eta: float):
    """eta * Delta = -eta (S + shift I)^-1 F by a dense Cholesky solve."""
    _, F, S = sr_moments(O, E, w)
    A = S + shift * torch.eye(S.shape[0], dtype=DT)
    Lc = torch.linalg.cholesky(A)
    return -eta * torch.cholesky_solve(F[:, None], Lc)[:, 0]


def all_configs(N: int) -> torch.Tensor:
    """Every +-1 configuration of N spins, [2^N, N] (int8)."""
    return torch.tensor(list(itertools.product((1, -1), repeat=N)), dtype=torch.int8)


def exact_energy(desc, ham, theta) -> float:
    """<psi|H|psi> / <psi|psi> by enumeration: sum_s |psi(s)|^2 E_loc(s) / sum_s |psi(s)|^2."""
    theta = torch.as_tensor(theta, dtype=DT)
    s = all_configs(desc.N * desc.token)
    sites, helem, n_conn, hdiag = connected(ham, s)
    lp, lr = plain_logratio(desc, theta, s, sites, n_conn)
    el = local_energy(hdiag, helem, n_conn, lr)
    p = torch.exp(2 * (lp.real - lp.real.max()))
    return float(((p * el).sum() / p.sum()).real)


def exact_weights(desc, theta, s) -> torch.Tensor:
    """|psi(s)|^2 / Z over the given (complete) set of configurations."""
    lp = forward(desc, torch.as_tensor(theta, dtype=DT), s)["logpsi"].real
    p = torch.exp(2 * (lp - lp.max()))
    return p / p.sum()


def exact_sr_inputs(desc, ham, theta):
    """(configurations, weights, O, E_loc) of exact enumeration."""
    theta = torch.as_tensor(theta, dtype=DT)
    s = all_configs(desc.N * desc.token)
    sites, helem, n_conn, hdiag = connected(ham, s)
    _, lr = plain_logratio(desc, theta, s, sites, n_conn)
    el = local_energy(hdiag, helem, n_conn, lr)
    w = exact_weights(desc, theta, s)
    O = grad_logpsi_batched(desc, theta, s)
    return s, w, O, el
