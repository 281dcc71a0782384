"""The model variants together on the GPU against the FP64 oracle: token size 2, a complex
read-out and a block-diagonal vertex in one network (two and three blocks, open and periodic),
through the estimator (both paths), the allocation-free log psi, the log-derivatives and one SR
update. Tolerances as in the single-variant tests (float64: 1e-10; float32: 1e-4; phases
modulo 2 pi)."""
import math
import sys

import pytest
import torch

import dn_inputs as di
import oracle as O
from oracle.grad import grad_logpsi_batched
from oracle.model import ModelDesc, forward
from oracle.vmc import sr_update

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


def cdiff(x, ref):
    x, ref = torch.as_tensor(x).cpu(), torch.as_tensor(ref).cpu()
    return torch.complex(x.real - ref.real, torch.remainder(x.imag - ref.imag + math.pi, 2 * math.pi) - math.pi).abs()


@pytest.mark.parametrize("shape,ham,prec", [
    (di.ModelShape(9, 2, 8, 4, act="silu", bc="periodic", token=2, complex_out=1, d_block=4),
     di.HamSpec("j1j2", "periodic"), "fp64"),
    (di.ModelShape(10, 3, 8, 3, act="tanh", bc="open", token=2, complex_out=1, d_block=2),
     di.HamSpec("lrtfim", "open"), "fp64"),
    (di.ModelShape(40, 2, 32, 8, act="silu", bc="periodic", token=2, complex_out=1, d_block=8),
     di.HamSpec("j1j2", "periodic"), "fp32"),
], ids=lambda x: str(x)[:60])
def test_variants_together(L, shape, ham, prec):
    th = torch.tensor(di.draw_params(shape, 41, "stress"))
    th[-2 * shape.d:] *= 4.0  # phases of order one
    m = L.Model(shape, prec)
    m.set_params(th)
    desc = ModelDesc.of(shape)
    B, ns = 3, shape.n_spins
    sp = di.uniform_spins(B, ns, 43)
    M_max = ns if ham.kind == "lrtfim" else 2 * ns
    ref = O.eloc_plain(desc, ham, th, sp, M_max)
    ref_ab = O.abacus_logratio(desc, th, sp, ref["sites"], ref["n_conn"])
    Om = forward(desc, th, sp)["Omega"]
    lr_scale = ref_ab.abs().max().item()
    if ham.kind == "j1j2":
        single = O.connected(di.HamSpec("lrtfim", shape.bc), sp)
        _, lr1 = O.plain_logratio(desc, th, sp, single[0], single[2])
        lr_scale = max(lr_scale, lr1.abs().max().item())
    tol = 1e-10 if prec == "fp64" else 1e-4
    spd = torch.tensor(sp, device="cuda")
    for path in ("abacus", "full"):
        lp, lr, el = (t.cpu() for t in m.eloc(ham, spd, M_max, path=path))
        floor = 0.0 if path == "abacus" else 1e3 * (2.2e-16 if prec == "fp64" else 6e-8) * max(
            1.0, Om.abs().max().item()) ** 2
        e_lp = cdiff(lp, ref["logpsi"]).max().item() / ref["logpsi"].abs().max().item()
        e_el = (el - ref["eloc"]).abs().max().item() / ref["eloc"].abs().max().item()
        d_lr = cdiff(lr, ref_ab).max().item()
        _say(f"{shape.N}x{shape.token} L={shape.L} {prec} {path}: eps_logpsi {e_lp:.3e} eps_eloc {e_el:.3e} "
             f"|d lr| {d_lr:.3e} (scale {lr_scale:.3e})")
        assert e_lp <= tol and e_el <= tol and d_lr <= tol * lr_scale + floor
    lp_na = m.logpsi_noalloc(spd).cpu()
    assert torch.equal(lp_na, m.logpsi(spd).cpu())
    _, g, _ = m.grad_logpsi(spd)
    gref = grad_logpsi_batched(desc, th, sp)
    nrm = gref.abs().pow(2).sum(1).sqrt()
    e_g = ((g.to(torch.complex128).cpu() - gref).abs().pow(2).sum(1).sqrt()
           / nrm.clamp_min(1e-3 * nrm.max().item())).max().item()
    _say(f"  eps_grad {e_g:.3e}")
    assert e_g <= tol
    _, _, el = m.eloc(ham, spd, M_max)
    delta, energy, _ = m.sr_update(g, el, None, shift=1e-2, eta=0.1, max_iter=1000, tol=1e-13)
    ref_delta = sr_update(gref, ref["eloc"], torch.full((B,), 1.0 / B, dtype=torch.float64), 1e-2, 0.1)
    e_d = (delta.cpu() - ref_delta).norm().item() / ref_delta.norm().item()
    _say(f"  sr: rel err of delta {e_d:.3e}")
    assert e_d <= (1e-8 if prec == "fp64" else 1e-4)
    m.close()
