"""Pins of the oracle's block-diagonal vertex (Sec. V: D(sigma) block-diagonal in channel space,
a mixture-of-experts like structure): with d_block = b, D_j = U diag(chi_j) V maps each block of
b channels to itself.

* d_block = d is the dense vertex;
* the vertex matrices U diag(chi) V formed from the oracle's own parameters and gates vanish
  off the blocks, at every site and block, while chi itself is dense;
* the off-block entries of U and V in the parameter vector change nothing, and their gradients
  are zero;
* ABACUS equals full re-evaluation.
"""
import dataclasses

import torch

import dn_inputs as di
import oracle as O
from oracle.grad import grad_logpsi_batched
from oracle.model import ModelDesc, forward, unpack


def _shapes(b):
    dense = di.ModelShape(10, 2, 8, 3, bc="open", act="silu")
    return dense, dataclasses.replace(dense, d_block=b)


def test_full_block_is_dense():
    dense, blk = _shapes(8)
    th = torch.tensor(di.draw_params(dense, 3, "stress"))
    sp = di.uniform_spins(4, 10, 5)
    a = forward(ModelDesc.of(dense), th, sp)["logpsi"]
    b = forward(ModelDesc.of(blk), th, sp)["logpsi"]
    assert torch.equal(a, b)


def test_vertex_is_block_diagonal():
    _, blk = _shapes(4)
    desc = ModelDesc.of(blk)
    th = torch.tensor(di.draw_params(blk, 3, "stress"))
    out = forward(desc, th, di.uniform_spins(2, 10, 5), cache=True)
    prm = unpack(desc, th)
    c = torch.arange(8) // 4
    off = c[:, None] != c[None, :]
    for l, lay in enumerate(prm["layers"]):
        chi = out["chi"][l]                                   # [B, N, d]
        assert chi[..., 4:].abs().min() > 0                   # the gate itself is dense
        D = lay["U"][None, None] * chi[..., None, :] @ lay["V"][None, None]
        assert D[..., off].abs().max() == 0
        assert D[..., ~off].abs().max() > 1e-3


def _offblock_indices(shape):
    """Flat indices of the off-block entries of every block's U and V."""
    d, Wc, tk = shape.d, 2 * shape.w_c + 1, shape.token
    lay = 4 * d * d + 3 * d + Wc * d
    c = torch.arange(d) // shape.d_block
    off = (c[:, None] != c[None, :]).reshape(-1).nonzero()[:, 0]
    idx = []
    for l in range(shape.L):
        base = 2 * d * tk + l * lay
        offU = base + d * d + d + Wc * d + d + d * d + d
        idx += [offU + off, offU + d * d + off]
    return torch.cat(idx)


def test_offblock_entries_are_inert():
    _, blk = _shapes(4)
    desc = ModelDesc.of(blk)
    th = torch.tensor(di.draw_params(blk, 3, "stress"))
    idx = _offblock_indices(blk)
    th2 = th.clone()
    th2[idx] = torch.randn(idx.numel(), dtype=torch.float64)
    sp = di.uniform_spins(3, 10, 6)
    assert torch.equal(forward(desc, th, sp)["logpsi"], forward(desc, th2, sp)["logpsi"])
    G = grad_logpsi_batched(desc, th, sp)
    assert G[:, idx].abs().max() == 0
    assert G.abs().max() > 1e-3


def test_block_abacus_equals_full_reevaluation():
    for shape, kind in ((di.ModelShape(10, 3, 8, 3, bc="periodic", act="silu", d_block=4), "j1j2"),
                        (di.ModelShape(9, 2, 6, 2, bc="open", act="tanh", d_block=2), "lrtfim")):
        desc = ModelDesc.of(shape)
        th = torch.tensor(di.draw_params(shape, 31, "stress"))
        sp = di.uniform_spins(3, shape.N, 17)
        sites, helem, n_conn, hdiag = O.connected(di.HamSpec(kind, shape.bc), sp)
        lp, lr = O.plain_logratio(desc, th, sp, sites, n_conn)
        la = O.abacus_logratio(desc, th, sp, sites, n_conn)
        scale = max(lr.abs().max().item(), lp.abs().max().item())
        assert (la - lr).abs().max().item() <= 1e-12 * scale
