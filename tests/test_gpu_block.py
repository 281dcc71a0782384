"""GPU parity of the block-diagonal vertex (d_block > 0: U and V block-diagonal in channel
blocks; Sec. V) against the FP64 oracle, through the C ABI: log psi, log-ratios by ABACUS and by
full re-evaluation, E_loc, and the per-sample log-derivatives (whose off-block U and V entries
must be exactly zero). Tolerances as in the dense parity tests: 1e-10 in float64, 1e-4 in
float32 (normwise), the plain path's |Omega|^2 floor for its log-ratios.
"""
import sys

import pytest
import torch

import dn_inputs as di
import oracle as O
from oracle.grad import grad_logpsi_batched
from oracle.model import ModelDesc, forward
from test_oracle_block import _offblock_indices

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


def eps(x, ref):
    x, ref = torch.as_tensor(x).double().cpu(), torch.as_tensor(ref).double().cpu()
    return (x - ref).abs().max().item() / max(ref.abs().max().item(), 1e-300)


CASES = [
    (di.ModelShape(16, 2, 8, 4, act="silu", bc="open", d_block=4), di.HamSpec("lrtfim", "open"), "fp64", 3),
    (di.ModelShape(14, 3, 6, 3, act="tanh", bc="periodic", d_block=2), di.HamSpec("j1j2", "periodic"), "fp64", 3),
    (di.ModelShape(64, 3, 32, 16, bc="open", d_block=8), di.HamSpec("lrtfim", "open"), "fp32", 2),
    (di.ModelShape(40, 2, 32, 8, bc="periodic", d_block=8), di.HamSpec("j1j2", "periodic"), "fp32", 2),
]


@pytest.mark.parametrize("shape,ham,prec,B", CASES, ids=lambda x: str(x)[:48])
def test_block_logratio_eloc_and_grad_match_oracle(L, shape, ham, prec, B):
    th = torch.tensor(di.draw_params(shape, 23, "stress"))
    th[_offblock_indices(shape)] = 3.0  # present in the vector, unused by the model
    m = L.Model(shape, prec)
    m.set_params(th)
    desc = ModelDesc.of(shape)
    sp = di.uniform_spins(B, shape.N, 31)
    M_max = shape.N if ham.kind == "lrtfim" else 2 * shape.N
    ref = O.eloc_plain(desc, ham, th, sp, M_max)
    ref_ab = O.abacus_logratio(desc, th, sp, ref["sites"], ref["n_conn"])
    Om = forward(desc, th, sp)["Omega"]
    lr_scale = ref_ab.abs().max().item()
    if ham.kind == "j1j2":
        single = O.connected(di.HamSpec("lrtfim", shape.bc), sp)
        _, lr1 = O.plain_logratio(desc, th, sp, single[0], single[2])
        lr_scale = max(lr_scale, lr1.abs().max().item())
    spd = torch.tensor(sp, device="cuda")
    tol = 1e-10 if prec == "fp64" else 1e-4
    for path in ("abacus", "full"):
        lp, lr, el = (t.cpu() for t in m.eloc(ham, spd, M_max, path=path))
        floor = 0.0 if path == "abacus" else 1e3 * (2.2e-16 if prec == "fp64" else 6e-8) * max(
            1.0, Om.abs().max().item()) ** 2
        d_lr = (lr - ref_ab).abs().max().item()
        _say(f"block {shape.d}/{shape.d_block} L={shape.L} {prec} {path}: eps_logpsi {eps(lp, ref['logpsi']):.3e} "
             f"eps_eloc {eps(el, ref['eloc']):.3e} |d lr| {d_lr:.3e}")
        assert eps(lp, ref["logpsi"]) <= tol and eps(el, ref["eloc"]) <= tol
        assert d_lr <= tol * lr_scale + floor
    _, g, _ = m.grad_logpsi(spd)
    gref = grad_logpsi_batched(desc, th, sp)
    g = g.double().cpu()
    assert g[:, _offblock_indices(shape)].abs().max().item() == 0.0
    nrm = gref.norm(dim=1)
    e = ((g - gref).norm(dim=1) / nrm.clamp_min(1e-3 * nrm.max().item())).max().item()
    _say(f"  grad: eps_grad {e:.3e}")
    assert e <= (1e-10 if prec == "fp64" else 1e-4)
    m.close()


def test_block_size_must_divide_d(L):
    with pytest.raises(RuntimeError, match="d_block"):
        L.Model(di.ModelShape(16, 2, 8, 4, d_block=3), "fp64")
