"""Pins of the oracle's token size (patching; Sec. V on the efficiency trade-off, and the token
sizes of the paper's experiments): N tokens of t spins each, token tau embedded as
sum_k E_k s_(t tau + k).

* equal embedding vectors (E_k = e, E_phi,k = f for every k) give the per-site network on the
  summed inputs x_tau = sum_k s_(t tau + k) (the forward takes real-valued inputs);
* E_k = E_phi,k = 0 for k >= 1 gives the per-site network on the spins s_(t tau): a wrong
  token-to-spin index map fails here;
* ABACUS equals full re-evaluation (Theorem 1 acts on tokens: a flip changes one token, a pair
  exchange one token or two neighbouring ones), one to four blocks, open and periodic;
* the |psi|^2-weighted mean of E_loc equals the Rayleigh quotient of the dense Hamiltonian of
  the N t spins (built independently from Pauli bit operations);
* log-derivatives equal central differences; the screened sampler equals exact
  Metropolis-Hastings.
"""
import dataclasses

import numpy as np
import pytest
import torch

import dn_inputs as di
import oracle as O
from oracle.grad import grad_logpsi_batched
from oracle.model import ModelDesc, forward
from oracle.sampler import exact_mh_sweep, screened_sweep, typewriter_sites
from test_oracle_hamiltonian import _all_confs, dense_h


def _pair(shape1, t, seed, equal=True):
    """Parameters of a token-t network and of the per-site network they reduce to."""
    shape_t = dataclasses.replace(shape1, token=t)
    d = shape1.d
    th1 = torch.tensor(di.draw_params(shape1, seed, "stress"))
    rest = th1[2 * d:]
    e, f = th1[:d], th1[d:2 * d]
    if equal:
        E = e.repeat(t)
        F = f.repeat(t)
    else:
        E = torch.cat([e, torch.zeros((t - 1) * d, dtype=torch.float64)])
        F = torch.cat([f, torch.zeros((t - 1) * d, dtype=torch.float64)])
    return shape_t, torch.cat([E, F, rest]), th1


@pytest.mark.parametrize("t", [2, 3])
@pytest.mark.parametrize("bc", ["open", "periodic"])
def test_equal_embeddings_give_summed_inputs(t, bc):
    shape1 = di.ModelShape(9, 2, 4, 3, bc=bc, act="silu")
    shape_t, tht, th1 = _pair(shape1, t, 5)
    sp = torch.tensor(di.uniform_spins(5, 9 * t, 3)).double()
    x = sp.reshape(5, 9, t).sum(-1)
    a = forward(ModelDesc.of(shape_t), tht, sp)["logpsi"]
    b = forward(ModelDesc.of(shape1), th1, x)["logpsi"]
    assert torch.allclose(a, b, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("t", [2, 3])
def test_first_position_only_gives_the_subchain(t):
    shape1 = di.ModelShape(10, 3, 3, 2, bc="open", act="tanh")
    shape_t, tht, th1 = _pair(shape1, t, 7, equal=False)
    sp = torch.tensor(di.uniform_spins(4, 10 * t, 8))
    a = forward(ModelDesc.of(shape_t), tht, sp)["logpsi"]
    b = forward(ModelDesc.of(shape1), th1, sp[:, ::t])["logpsi"]
    assert torch.allclose(a, b, rtol=1e-13, atol=1e-14)


CASES = [
    # (tokens, L, d, s, bc, act, ham kind, t)
    (8, 1, 3, 2, "open", "tanh", "lrtfim", 2),
    (7, 2, 4, 3, "open", "silu", "j1j2", 2),
    (8, 3, 3, 2, "periodic", "silu", "j1j2", 2),
    (6, 4, 3, 2, "periodic", "identity", "lrtfim", 2),
    (5, 2, 3, 2, "open", "silu", "j1j2", 3),
    (6, 2, 3, 2, "periodic", "tanh", "j1j2", 3),
]


@pytest.mark.parametrize("case", CASES)
def test_token_abacus_equals_full_reevaluation(case):
    N, L, d, s, bc, act_name, kind, t = case
    shape = di.ModelShape(N, L, d, s, bc=bc, act=act_name, token=t)
    desc = ModelDesc.of(shape)
    th = torch.tensor(di.draw_params(shape, 31, "stress"))
    sp = di.uniform_spins(3, N * t, 17)
    sites, helem, n_conn, hdiag = O.connected(di.HamSpec(kind, bc), sp)
    lp, lr = O.plain_logratio(desc, th, sp, sites, n_conn)
    la = O.abacus_logratio(desc, th, sp, sites, n_conn)
    assert lr.abs().max() > 0
    scale = max(lr.abs().max().item(), lp.abs().max().item())
    assert (la - lr).abs().max().item() <= 1e-12 * scale


@pytest.mark.parametrize("ham", [di.HamSpec("j1j2", "periodic", J1=1.0, J2=0.5),
                                 di.HamSpec("lrtfim", "open", J=1.0, alpha=3.0, h=1.0)])
def test_token_mean_local_energy_equals_rayleigh_quotient(ham):
    shape = di.ModelShape(4, 2, 3, 2, bc=ham.bc, act="silu", token=2)
    desc = ModelDesc.of(shape)
    th = torch.tensor(di.draw_params(shape, 12, "stress"))
    confs = _all_confs(8)
    res = O.eloc_plain(desc, ham, th, confs)
    lp = res["logpsi"].numpy()
    psi = np.exp(lp - lp.max())
    H = dense_h(ham, 8)
    rq = psi @ H @ psi / (psi @ psi)
    mean = np.sum(psi ** 2 * res["eloc"].numpy()) / np.sum(psi ** 2)
    assert abs(mean - rq) <= 1e-12 * max(1.0, abs(rq))


def test_token_gradient_matches_central_differences():
    shape = di.ModelShape(6, 2, 3, 2, bc="open", act="silu", token=2)
    desc = ModelDesc.of(shape)
    th = torch.tensor(di.draw_params(shape, 6005, "stress"))
    sp = torch.tensor(di.uniform_spins(2, 12, 3))
    G = grad_logpsi_batched(desc, th, sp)
    rng = np.random.Generator(np.random.PCG64(6005))
    idx = list(rng.choice(th.numel(), size=12, replace=False)) + [0, 3, 2 * 3 + 1, 2 * 3 * 2 - 1]
    eps = 1e-6
    for k in idx:  # the embedding entries of both positions among them
        tp, tm = th.clone(), th.clone()
        tp[k] += eps
        tm[k] -= eps
        fd = (forward(desc, tp, sp)["logpsi"] - forward(desc, tm, sp)["logpsi"]) / (2 * eps)
        scale = max(G[:, k].abs().max().item(), 1e-8)
        assert (fd - G[:, k]).abs().max().item() <= 1e-6 * scale + 1e-10


def test_token_screened_sampler_equals_exact_metropolis():
    shape = di.ModelShape(8, 2, 4, 3, act="silu", bc="open", token=2)
    desc = ModelDesc.of(shape)
    th = torch.tensor(di.draw_params(shape, 17, "stress"))
    th[-2 * shape.d:] *= 10.0
    chains = [torch.tensor(x).long() for x in di.uniform_spins(2, 16, 4)]
    refreshes = 0
    for sweep in range(4):
        parity = sweep % 2
        K = len(range(parity, 16, 2))
        rng = np.random.Generator(np.random.PCG64(950 + sweep))
        r, u = rng.random((2, K)), rng.random((2, K))
        for b in range(2):
            sites = typewriter_sites(16, 1, parity, r[b])
            ref = exact_mh_sweep(desc, th, chains[b], sites, u[b])
            got = screened_sweep(desc, th, chains[b], sites, u[b], 0.1, track=True)
            if got["unscreened_err"] <= 0.1:
                assert got["accepted"] == ref["accepted"]
            refreshes += got["refreshes"]
            chains[b] = got["spins"]
    assert refreshes > 0
