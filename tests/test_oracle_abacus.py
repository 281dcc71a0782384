"""Pins of the oracle's ABACUS update (Sec. III, Theorem 1; App. "Induction Proof of ABACUS").

Theorem 1 states that the recurrence reproduces the network output exactly for any
local update, so the oracle's ABACUS must equal its own full re-evaluation (the plain
definition) to roundoff, for single flips and pair exchanges, at edges and across the
periodic seam, at every depth, with and without the phi injection, at the small
baseline draw and at the stress draw. With a constant vertex the update has a closed
form: Omega is linear in s, so dOmega = -2 s_j w_j.
"""
import numpy as np
import pytest
import torch

import dn_inputs as di
import oracle as O
from oracle.model import ModelDesc, lcd, unpack, forward


def _err(a, b):
    return (a - b).abs().max().item() / max(b.abs().max().item(), 1e-300)


CASES = [
    # (N, L, d, s, bc, act, inject, ham kind)
    (10, 1, 3, 2, "open", "tanh", 0, "lrtfim"),
    (12, 2, 4, 3, "open", "silu", 0, "lrtfim"),
    (11, 3, 3, 2, "open", "silu", 0, "j1j2"),
    (12, 4, 3, 2, "periodic", "silu", 0, "j1j2"),
    (9, 2, 3, 2, "periodic", "tanh", 0, "lrtfim"),
    (10, 3, 3, 2, "periodic", "identity", 1, "j1j2"),
    (11, 4, 2, 2, "open", "silu", 1, "lrtfim"),
    (10, 2, 3, 2, "open", "tanh", 1, "j1j2"),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("scale", ["baseline", "stress"])
def test_abacus_equals_full_reevaluation(case, scale):
    N, L, d, s, bc, act_name, inj, kind = case
    shape = di.ModelShape(N, L, d, s, bc=bc, act=act_name, inject_phi=inj)
    desc = ModelDesc.of(shape)
    th = torch.tensor(di.draw_params(shape, 31, scale))
    ham = di.HamSpec(kind, bc)
    sp = di.uniform_spins(3, N, 17)
    sites, helem, n_conn, hdiag = O.connected(ham, sp)
    lp, lr = O.plain_logratio(desc, th, sp, sites, n_conn)
    la = O.abacus_logratio(desc, th, sp, sites, n_conn)
    assert lr.abs().max() > 0
    # The plain ratio is a difference of two full evaluations, so its rounding error scales
    # with |log psi|, not with the ratio (pair exchanges at the 0.1-scale draw give ratios
    # ~1e-20 against log psi ~1e-12). ABACUS forms dOmega directly. The bound is therefore
    # 1e-12 relative to the larger of the two magnitudes.
    scale = max(lr.abs().max().item(), lp.abs().max().item())
    assert (la - lr).abs().max().item() <= 1e-12 * scale


def test_abacus_wraparound_pairs():
    # the pairs that cross the periodic seam: (N-1, 0), (N-2, 0), (N-1, 1)
    N = 10
    shape = di.ModelShape(N, 3, 3, 2, bc="periodic", act="silu")
    desc = ModelDesc.of(shape)
    th = torch.tensor(di.draw_params(shape, 5, "stress"))
    sp = torch.tensor(di.uniform_spins(1, N, 3))
    sites = torch.tensor([[[N - 1, 0], [N - 2, 0], [N - 1, 1], [0, -1]]])
    n_conn = torch.tensor([4])
    _, lr = O.plain_logratio(desc, th, sp, sites, n_conn)
    la = O.abacus_logratio(desc, th, sp, sites, n_conn)
    assert _err(la, lr) <= 1e-12


def test_constant_vertex_closed_form():
    # A_D = 0 makes every vertex constant, so e^(l>=1) = 0 and Omega(s) = W s is linear:
    # dOmega for flipping j is -2 s_j W[:, j], with W read off from unit-vector evaluations.
    N = 11
    shape = di.ModelShape(N, 3, 3, 2, bc="open", act="silu")
    desc = ModelDesc.of(shape)
    th = torch.tensor(di.draw_params(shape, 41, "stress"))
    for lay in unpack(desc, th)["layers"]:
        lay["A_D"].zero_()
    eye = torch.eye(N, dtype=torch.float64)
    W = forward(desc, th, eye)["Omega"].T                    # [d_out, N], Omega(e_j)
    sp = torch.tensor(di.uniform_spins(2, N, 6))
    Om = forward(desc, th, sp)["Omega"]
    sites = torch.stack([torch.stack([torch.arange(N), -torch.ones(N, dtype=torch.int64)], 1)] * 2)
    n_conn = torch.tensor([N, N])
    la = O.abacus_logratio(desc, th, sp, sites, n_conn)
    want = torch.stack([torch.stack([lcd(Om[b], -2 * sp[b, j] * W[:, j]).sum() for j in range(N)])
                        for b in range(2)])
    assert _err(la, want) <= 1e-12


def test_output_links_are_jacobians():
    # T~^(m) = d Omega / d u^(m+1) at frozen vertices; checked by finite differences of a
    # frozen-vertex evaluation built from the dense background operators.
    from oracle.abacus import background_operators, output_links
    N = 8
    shape = di.ModelShape(N, 3, 2, 2, bc="open")
    desc = ModelDesc.of(shape)
    th = torch.tensor(di.draw_params(shape, 8, "stress"))
    s0 = torch.tensor(di.uniform_spins(1, N, 1))[0]
    ops = background_operators(desc, th, s0)
    Tt = output_links(desc, ops)
    n = N * desc.d
    rng = np.random.default_rng(2)
    for m in range(desc.L):
        dv = torch.tensor(rng.normal(size=n))
        # frozen-vertex propagation of a perturbation added to u^(m+1)
        du, acc = dv, torch.zeros(n, dtype=torch.float64)
        for l in range(m + 1, desc.L + 1):
            dh = ops["B"][l - 1] @ du
            acc = acc + dh
            du = dh
        assert torch.allclose(Tt[m] @ dv, ops["Pw"] @ acc, rtol=0, atol=1e-14)
