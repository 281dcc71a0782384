"""GPU parity of the BF16-mixed precision mode against the FP64 oracle.

In this mode both channel-mixing products of every block (forward, adjoint and the ABACUS
deep propagation) run on the bf16 matrix cores with float accumulation; fields, the
phi stream, the Toeplitz mixer, the slice recompute and the log-ratio read-out stay in
float / float64. Error bounds follow from the bf16 unit roundoff u = 2^-8 (round to
nearest even, 8 significant bits): each mixing product rounds its two operands, so each
block changes Omega (and the propagated dOmega) by about 2u relative, and L blocks by
about 2Lu. With a factor 2 of margin:
  * ABACUS log-ratios:   |lr - lr*| <= 4 L u * lr_scale (lr_scale as in the float tests:
                          max|lr*|, or for pair exchanges the larger single-flip ratios);
  * plain log-ratios:    the difference of two evaluations, |Omega|^2 scale (as in float);
  * log psi:             |d log psi| <= 4 L u * max|Omega| * max(1, max|Omega|);
  * E_loc:               |dE| <= max_b sum_m |h_bm| psi(s'_m)/psi(s_b) * (bound on |d lr|).
The measured errors are printed next to the bounds.
"""
import sys

import pytest
import torch

import dn_inputs as di
import oracle as O
from oracle.model import ModelDesc, forward

pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -8


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2603_11189_amd import _lib
    _lib.lib()
    return _lib


CASES = [
    # the J1-J2 chain of the BF16 workload (N=128, four blocks, d=64, periodic, balanced spins)
    (di.ModelShape(128, 4, 64, 32, bc="periodic"), di.HamSpec("j1j2", "periodic"), 6, "balanced"),
    (di.ModelShape(96, 3, 32, 16, bc="open"), di.HamSpec("lrtfim", "open", alpha=2.0, h=0.5), 6, "uniform"),
    (di.ModelShape(70, 2, 48, 8, act="tanh", bc="open"), di.HamSpec("j1j2", "open"), 5, "uniform"),
]


@pytest.mark.parametrize("shape,ham,B,spins", CASES, ids=lambda x: str(x)[:40])
@pytest.mark.parametrize("scale", ["baseline", "stress"])
def test_bf16_logratio_and_eloc(L, shape, ham, B, spins, scale):
    _say("bf16", shape, ham.kind, scale)
    th = torch.tensor(di.draw_params(shape, 41, scale))
    m = L.Model(shape, "bf16")
    m.set_params(th)
    desc = ModelDesc.of(shape)
    f = di.uniform_spins if spins == "uniform" else di.balanced_spins
    sp = f(B, shape.N, 43)
    M_max = shape.N if ham.kind == "lrtfim" else 2 * shape.N
    ref = O.eloc_plain(desc, ham, th, sp, M_max)
    Om = forward(desc, th, sp)["Omega"]
    om = Om.abs().max().item()
    lr_scale = ref["logratio"].abs().max().item()
    if ham.kind == "j1j2":
        single = O.connected(di.HamSpec("lrtfim", shape.bc), sp)
        _, lr1 = O.plain_logratio(desc, th, sp, single[0], single[2])
        lr_scale = max(lr_scale, lr1.abs().max().item())
    b = 4 * shape.L * U_BF16
    spd = torch.tensor(sp, device="cuda")
    mask = torch.arange(M_max)[None, :] < ref["n_conn"][:, None]
    weight = (ref["helem"].abs() * torch.exp(ref["logratio"]) * mask).sum(-1).max().item()
    for path in ("abacus", "full"):
        lp, lr, el = (t.cpu() for t in m.eloc(ham, spd, M_max, path=path))
        d_lr = (lr - ref["logratio"]).abs().max().item()
        d_lp = (lp - ref["logpsi"]).abs().max().item()
        d_el = (el - ref["eloc"]).abs().max().item()
        lr_bound = b * (lr_scale if path == "abacus" else max(lr_scale, om * om))
        lp_bound = b * om * max(1.0, om)
        el_bound = weight * lr_bound
        _say(f"  {path}: |d lr| {d_lr:.3e} (bound {lr_bound:.3e})  |d logpsi| {d_lp:.3e} "
             f"(bound {lp_bound:.3e})  |d E| {d_el:.3e} (bound {el_bound:.3e})  "
             f"eps_eloc {d_el / ref['eloc'].abs().max().item():.3e}")
        assert d_lr <= lr_bound and d_lp <= lp_bound and d_el <= el_bound
    m.close()


def test_bf16_needs_wide_channels(L):
    with pytest.raises(L.DysonNetError) as ei:
        L.Model(di.ModelShape(32, 2, 16, 8), "bf16")
    assert ei.value.status == L.DN_EUNSUPPORTED


def test_bf16_gradients_run_in_float(L):
    """The per-sample log-derivatives of a BF16-mixed model come from the float forward and
    backward, bit for bit those of the same model in float."""
    shape = di.ModelShape(64, 2, 32, 16, bc="open")
    th = torch.tensor(di.draw_params(shape, 5, "stress"))
    sp = torch.tensor(di.uniform_spins(8, 64, 6), device="cuda")
    out = []
    for prec in ("bf16", "fp32"):
        m = L.Model(shape, prec)
        m.set_params(th)
        out.append(m.grad_logpsi(sp))
        m.close()
    assert torch.equal(out[0][1], out[1][1]) and torch.equal(out[0][0], out[1][0])
