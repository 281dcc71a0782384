"""Pins of the oracle's forward pass (Sec. II, Eq. (wavefunc); Eq. (Dpractical); the
phi-stream CNN of App. "Details on the implementation of the DysonNet block").

* constant vertex (A_D = 0): Omega is linear in s with weights from dense matrices
  built here: A^T (1/N) diag(omega) [I + B1 + B2 B1 + ...] E, B_l = D_l G_l;
* identity nonlinearity: Omega is a polynomial of degree <= L+1 in s, so its Walsh
  coefficients above that degree vanish;
* one block, d = 1, w_c = 0, identity, periodic: the Jastrow form of App. "DysonNet can
  exactly represent power law decay" (Eq. (Jij_short)) with this model's residual,
  embedding and final-mixer factors;
* locality: the block-l vertex at site i depends only on spins within l*w_c of i;
* periodic networks are translation invariant.
"""
import itertools
import math

import numpy as np
import pytest
import torch

import dn_inputs as di
from oracle.model import ModelDesc, act, forward, mixers, unpack


def _model(shape, seed=3, scale="stress"):
    desc = ModelDesc.of(shape)
    th = torch.tensor(di.draw_params(shape, seed, scale))
    return desc, th


def _zero_block(desc, th, name):
    prm = unpack(desc, th)
    for lay in prm["layers"]:
        lay[name].zero_()
    return th


@pytest.mark.parametrize("L,bc,act_name", [(1, "open", "tanh"), (2, "open", "silu"), (3, "periodic", "silu")])
def test_constant_vertex_gives_linear_model(L, bc, act_name):
    shape = di.ModelShape(9, L, 3, 2, bc=bc, act=act_name)
    desc, th = _model(shape)
    th = _zero_block(desc, th.clone(), "A_D")
    prm = unpack(desc, th)
    T = mixers(desc, prm)
    N, d = desc.N, desc.d
    n = N * d
    # dense operators, index (i, c) -> i*d + c
    X = torch.eye(n, dtype=torch.float64)
    total = torch.eye(n, dtype=torch.float64)
    for l, lay in enumerate(prm["layers"]):
        G = torch.zeros(n, n, dtype=torch.float64)
        for c in range(d):
            G[c::d, c::d] = T[l][c]
        Dm = lay["U"] @ torch.diag(act(desc.act, lay["b"])) @ lay["V"]
        Dbig = torch.block_diag(*([Dm] * N))
        X = Dbig @ G @ X
        total = total + X
    omega = T[L].sum(dim=1)                     # [d, N] column sums of the final mixer
    Pw = torch.stack([(omega.T * prm["A"][:, k]).reshape(-1) / N for k in range(desc.d_out)])
    Emb = torch.zeros(n, N, dtype=torch.float64)
    for i in range(N):
        Emb[i * d:(i + 1) * d, i] = prm["E"]
    W = Pw @ total @ Emb                        # [d_out, N]
    s = torch.tensor(di.uniform_spins(6, N, 1)).double()
    Om = forward(desc, th, s)["Omega"]
    assert torch.allclose(Om, s @ W.T, rtol=0, atol=1e-13 * max(1.0, W.abs().max().item()))


def _walsh(values, N):
    """Walsh-Hadamard coefficients f_S = 2^-N sum_s f(s) prod_{i in S} s_i, indexed by bitmask."""
    f = values.copy()
    h = 1
    while h < len(f):
        for i in range(0, len(f), 2 * h):
            a, b = f[i:i + h].copy(), f[i + h:i + 2 * h].copy()
            f[i:i + h], f[i + h:i + 2 * h] = a + b, a - b
        h *= 2
    return f / len(f)


@pytest.mark.parametrize("L", [1, 2])
def test_identity_nonlinearity_gives_degree_L_plus_1(L):
    N = 8
    shape = di.ModelShape(N, L, 2, 2, act="identity", bc="open")
    desc, th = _model(shape, seed=9)
    confs = np.array([[1 - 2 * ((x >> i) & 1) for i in range(N)] for x in range(2 ** N)])
    Om = forward(desc, th, torch.tensor(confs))["Omega"].numpy()
    deg = np.array([bin(x).count("1") for x in range(2 ** N)])
    for k in range(desc.d_out):
        coef = _walsh(Om[:, k], N)
        assert np.max(np.abs(coef[deg > L + 1])) <= 1e-12 * np.max(np.abs(coef))
        assert np.max(np.abs(coef[deg == L + 1])) > 1e-8 * np.max(np.abs(coef))   # not vacuous


def test_jastrow_limit_closed_form():
    N = 7
    shape = di.ModelShape(N, 1, 1, 2, w_c=0, act="identity", bc="periodic")
    desc, th = _model(shape, seed=21)
    prm = unpack(desc, th)
    T = mixers(desc, prm)
    lay = prm["layers"][0]
    E, Ep = prm["E"][0], prm["E_phi"][0]
    W_D, w, K, k = lay["W_D"][0, 0], lay["w"][0], lay["K"][0, 0], lay["k"][0]
    A_D, b, U, V = lay["A_D"][0, 0], lay["b"][0], lay["U"][0, 0], lay["V"][0, 0]
    D1 = U * V * A_D * K * W_D * Ep                  # chi_i = D1' s_i + D0'; D_i = U V chi_i
    D0 = U * V * (A_D * (K * w + k) + b)
    g = T[0][0][:, 0]                                # g°_{(i-0) mod N}, i = 0..N-1
    gbar = g.sum()
    wbar = T[1][0].sum(dim=0)[0]                     # omega (constant on a ring)
    s = torch.tensor(di.uniform_spins(10, N, 4)).double()
    Om = forward(desc, th, s)["Omega"]
    for kk in range(2):
        pre = prm["A"][0, kk] * wbar * E / N
        hfield = pre * (1 + D0 * gbar)
        const = pre * D1 * N * g[0]
        want = const + hfield * s.sum(1)
        for i in range(N):
            for j in range(i + 1, N):
                Jij = pre * D1 * (g[(i - j) % N] + g[(j - i) % N])
                want = want + Jij * s[:, i] * s[:, j]
        assert torch.allclose(Om[:, kk], want, rtol=0, atol=1e-14)


@pytest.mark.parametrize("bc", ["open", "periodic"])
def test_vertex_locality(bc):
    N, L = 13, 3
    shape = di.ModelShape(N, L, 3, 2, bc=bc)
    desc, th = _model(shape)
    s = torch.tensor(di.uniform_spins(1, N, 2))
    f0 = forward(desc, th, s, cache=True)
    for j in (0, 5, N - 1):
        s1 = s.clone()
        s1[0, j] = -s1[0, j]
        f1 = forward(desc, th, s1, cache=True)
        for l in range(L):
            diff = (f1["chi"][l] - f0["chi"][l]).abs().amax(dim=-1)[0]
            for i in range(N):
                r = abs(i - j)
                if bc == "periodic":
                    r = min(r, N - r)
                if r > (l + 1) * desc.w_c:
                    assert diff[i] == 0.0
            assert diff.max() > 0


def test_periodic_translation_invariance():
    N = 12
    shape = di.ModelShape(N, 2, 4, 3, bc="periodic")
    desc, th = _model(shape)
    s = torch.tensor(di.uniform_spins(4, N, 8))
    lp = forward(desc, th, s)["logpsi"]
    for t in (1, 5, 11):
        lp2 = forward(desc, th, torch.roll(s, t, dims=1))["logpsi"]
        assert torch.allclose(lp, lp2, rtol=0, atol=1e-14)
