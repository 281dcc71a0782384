"""Pins of the oracle's Hamiltonians and local energy (Eq. (local-estimator); Sec. VI
long-range Ising chain; App. "Small system validation J1-J2", Eq. (j1j2_hamiltonian)).

The dense Hamiltonians here are built independently from Pauli bit operations (not
from the oracle's generator). Checks: the |psi|^2-weighted mean of E_loc equals
<psi|H|psi>/<psi|psi>; the generator's matrix is Hermitian and equals the dense one;
the Majumdar-Ghosh ground energy -3 N J1 / 8 at J2 = J1/2; trivial Ising limits;
the Kac factor as printed; the connected-element order on a hand-written example.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import dn_inputs as di
import oracle as O
from oracle.hamiltonian import kac
from oracle.model import ModelDesc

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _spin(x, i):
    return 1 - 2 * ((x >> i) & 1)          # bit 0 -> +1, bit 1 -> -1


def dense_h(ham, N):
    """H in the sz basis from sigma^z, sigma^x and S.S = (sz sz)/4 + (S+S- + S-S+)/2."""
    dim = 2 ** N
    H = np.zeros((dim, dim))
    if ham.kind == "lrtfim":
        if ham.paper_form:
            pre, hx = -ham.J / kac(N, ham.alpha), -ham.h     # sum over ordered pairs i != j
        else:
            pre, hx = ham.J, ham.h                          # sum over i < j
        for x in range(dim):
            e = 0.0
            for i in range(N):
                for j in range(N):
                    if i == j or (not ham.paper_form and j < i):
                        continue
                    r = abs(i - j)
                    if ham.bc == "periodic":
                        r = min(r, N - r)
                    e += pre * _spin(x, i) * _spin(x, j) / r ** ham.alpha
            H[x, x] += e
            for i in range(N):
                H[x ^ (1 << i), x] += hx
    else:
        for x in range(dim):
            for i in range(N):
                for dl, J in ((1, ham.J1), (2, ham.J2)):
                    j = i + dl
                    if j >= N:
                        if ham.bc != "periodic":
                            continue
                        j -= N
                    H[x, x] += J / 4 * _spin(x, i) * _spin(x, j)
                    if _spin(x, i) != _spin(x, j):
                        H[x ^ (1 << i) ^ (1 << j), x] += J / 2
    return H


def _all_confs(N):
    return np.array([[_spin(x, i) for i in range(N)] for x in range(2 ** N)], dtype=np.int8)


HAMS = [
    di.HamSpec("lrtfim", "open", J=1.0, alpha=3.0, h=1.0),
    di.HamSpec("lrtfim", "periodic", J=-1.3, alpha=2.0, h=0.7, paper_form=1),
    di.HamSpec("j1j2", "periodic", J1=1.0, J2=0.5),
    di.HamSpec("j1j2", "open", J1=0.8, J2=0.3),
]


@pytest.mark.parametrize("ham", HAMS)
def test_mean_local_energy_equals_rayleigh_quotient(ham):
    N = 8
    shape = di.ModelShape(N, 2, 3, 2, bc=ham.bc, act="silu")
    desc = ModelDesc.of(shape)
    th = torch.tensor(di.draw_params(shape, 12, "stress"))
    confs = _all_confs(N)
    res = O.eloc_plain(desc, ham, th, confs)
    lp = res["logpsi"].numpy()
    psi = np.exp(lp - lp.max())
    H = dense_h(ham, N)
    rq = psi @ H @ psi / (psi @ psi)
    mean = np.sum(psi ** 2 * res["eloc"].numpy()) / np.sum(psi ** 2)
    assert abs(mean - rq) <= 1e-12 * max(1.0, abs(rq))


@pytest.mark.parametrize("ham", HAMS)
def test_generator_matrix_is_hermitian_and_matches_dense(ham):
    N = 7 if ham.kind == "lrtfim" else 8
    confs = _all_confs(N)
    sites, helem, n_conn, hdiag = O.connected(ham, confs)
    Hg = np.zeros((2 ** N, 2 ** N))
    for x in range(2 ** N):
        Hg[x, x] = hdiag[x]
        for m in range(int(n_conn[x])):
            y = x
            for t in range(2):
                j = int(sites[x, m, t])
                if j >= 0:
                    y ^= 1 << j
            Hg[y, x] += helem[x, m].item()
    assert np.allclose(Hg, Hg.T, rtol=0, atol=1e-14)
    assert np.allclose(Hg, dense_h(ham, N), rtol=0, atol=1e-13)


@pytest.mark.parametrize("N", [8, 10])
def test_majumdar_ghosh_ground_energy(N):
    ham = di.HamSpec("j1j2", "periodic", J1=1.0, J2=0.5)
    confs = _all_confs(N)
    sites, helem, n_conn, hdiag = O.connected(ham, confs)
    Hg = np.diag(hdiag.numpy())
    for x in range(2 ** N):
        for m in range(int(n_conn[x])):
            Hg[x ^ (1 << int(sites[x, m, 0])) ^ (1 << int(sites[x, m, 1])), x] += helem[x, m].item()
    e0 = np.linalg.eigvalsh(Hg)[0]
    assert abs(e0 - (-3 * N * 1.0 / 8)) <= 1e-10


def test_ising_limits():
    N = 7
    confs = _all_confs(N)
    for ham, want in ((di.HamSpec("lrtfim", "open", J=1.0, alpha=2.0, h=0.0), None),
                      (di.HamSpec("lrtfim", "open", J=0.0, alpha=2.0, h=0.6), -N * 0.6)):
        sites, helem, n_conn, hdiag = O.connected(ham, confs)
        Hg = np.diag(hdiag.numpy())
        for x in range(2 ** N):
            for m in range(N):
                Hg[x ^ (1 << m), x] += helem[x, m].item()
        e0 = np.linalg.eigvalsh(Hg)[0]
        if want is None:
            want = hdiag.min().item()
        assert abs(e0 - want) <= 1e-12


def test_kac_factor_as_printed():
    # N_alpha(N) = 2 sum_{r=1}^{floor(N/2)} r^-alpha: N=4, alpha=1 -> 2 (1 + 1/2) = 3;
    # N=7, alpha=2 -> 2 (1 + 1/4 + 1/9)
    assert abs(kac(4, 1.0) - 3.0) < 1e-15
    assert abs(kac(7, 2.0) - 2 * (1 + 0.25 + 1 / 9)) < 1e-15


def test_connected_order_golden():
    with open(os.path.join(GOLD, "j1j2_order_n6.json")) as f:
        g = json.load(f)
    ham = di.HamSpec("j1j2", "periodic", J1=g["J1"], J2=g["J2"])
    sites, helem, n_conn, hdiag = O.connected(ham, np.array([g["spins"]], dtype=np.int8))
    n = int(n_conn[0])
    assert n == len(g["pairs"])
    assert sites[0, :n].tolist() == g["pairs"]
    assert np.allclose(helem[0, :n].numpy(), g["helem"])
    assert abs(hdiag[0].item() - g["hdiag"]) < 1e-15
