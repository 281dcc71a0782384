"""GPU parity of ABACUS with the phi stream injected into the h stream (the practical block of
Fig. 1c: the mixer of block l reads h^(l-1) + phi^(l); the residual sum holds no phi) against
the FP64 oracle, through the C ABI.

With injection the input change of block l + 1 is dh^(l) + dphi^(l+1), a vector on the slice
S_(l+1). The GPU therefore takes the full-chain propagation at every depth from two blocks up.
One block has no tiled block: the per-flip finish takes its whole input change
e^(0) + dphi^(1).

Log-ratios are compared with the oracle's ABACUS in float64 mode (it is pinned to full
re-evaluation with and without injection) and with the oracle's plain ratio in float32 mode;
the GPU's full path is compared with the same. E_loc and log psi are compared with the oracle's
plain estimator. Measures and tolerances are those of the per-site parity tests: normwise
eps(x) = max|x - x*| / max|x*|; 1e-10 in float64 mode, 1e-4 in float32 mode; the full path's
log-ratios with their |Omega|^2 rounding floor; pair ratios relative to the single-flip ratios
of the same samples.

Cases: one to four blocks, open and periodic, single flips and pair exchanges (across the
seam), token size 2, a complex read-out, the screened sampler's decisions exactly, a ragged
batch with injected instances.
"""
import sys

import numpy as np
import pytest
import torch

import dn_inputs as di
import oracle as O
from oracle.grad import grad_logpsi_batched
from oracle.model import ModelDesc, forward
from oracle.sampler import screened_sweep, typewriter_sites

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
    x, ref = torch.as_tensor(x), torch.as_tensor(ref)
    if x.is_complex() or ref.is_complex():
        x, ref = torch.view_as_real(x.to(torch.complex128).cpu()), torch.view_as_real(ref.to(torch.complex128).cpu())
    x, ref = x.double().cpu(), ref.double().cpu()
    return (x - ref).abs().max().item() / max(ref.abs().max().item(), 1e-300)


CASES = [
    # shape, ham, prec, B
    (di.ModelShape(16, 1, 8, 4, act="tanh", bc="open", inject_phi=1), di.HamSpec("lrtfim", "open"), "fp64", 4),
    (di.ModelShape(17, 1, 6, 3, act="silu", bc="periodic", inject_phi=1), di.HamSpec("j1j2", "periodic"), "fp64", 3),
    (di.ModelShape(9, 1, 6, 3, act="silu", bc="periodic", inject_phi=1, token=2), di.HamSpec("j1j2", "periodic"),
     "fp64", 3),
    (di.ModelShape(70, 1, 32, 16, bc="periodic", inject_phi=1), di.HamSpec("j1j2", "periodic"), "fp32", 3),
    # wider CNN windows: S_1 of a pair cluster nine sites wide at w_c = 3, S_2 eleven at w_c = 2
    (di.ModelShape(19, 1, 6, 3, act="silu", bc="open", w_c=3, inject_phi=1), di.HamSpec("j1j2", "open"), "fp64", 3),
    (di.ModelShape(21, 2, 6, 3, act="tanh", bc="periodic", w_c=2, inject_phi=1), di.HamSpec("j1j2", "periodic"),
     "fp64", 3),
    (di.ModelShape(16, 2, 8, 4, act="tanh", bc="open", inject_phi=1), di.HamSpec("lrtfim", "open"), "fp64", 4),
    (di.ModelShape(18, 2, 6, 3, act="silu", bc="periodic", inject_phi=1), di.HamSpec("j1j2", "periodic"), "fp64", 3),
    (di.ModelShape(20, 3, 8, 4, act="silu", bc="open", inject_phi=1), di.HamSpec("j1j2", "open"), "fp64", 3),
    (di.ModelShape(22, 4, 6, 3, act="tanh", bc="periodic", inject_phi=1), di.HamSpec("lrtfim", "periodic"), "fp64", 3),
    (di.ModelShape(19, 3, 5, 3, act="identity", bc="periodic", inject_phi=1), di.HamSpec("j1j2", "periodic"), "fp64", 3),
    (di.ModelShape(10, 2, 6, 3, act="silu", bc="periodic", inject_phi=1, token=2), di.HamSpec("j1j2", "periodic"),
     "fp64", 3),
    (di.ModelShape(11, 3, 6, 3, act="tanh", bc="open", inject_phi=1, token=2), di.HamSpec("lrtfim", "open"), "fp64", 3),
    (di.ModelShape(18, 3, 6, 3, act="silu", bc="periodic", inject_phi=1, complex_out=1), di.HamSpec("j1j2", "periodic"),
     "fp64", 3),
    (di.ModelShape(64, 2, 32, 16, bc="open", inject_phi=1), di.HamSpec("lrtfim", "open"), "fp32", 4),
    (di.ModelShape(70, 3, 20, 8, bc="periodic", inject_phi=1), di.HamSpec("j1j2", "periodic"), "fp32", 3),
    (di.ModelShape(130, 4, 64, 16, bc="open", inject_phi=1), di.HamSpec("j1j2", "open"), "fp32", 2),
]


@pytest.mark.parametrize("shape,ham,prec,B", CASES, ids=lambda x: str(x)[:56])
@pytest.mark.parametrize("scale", ["baseline", "stress"])
def test_inject_logratio_and_eloc_match_oracle(L, shape, ham, prec, B, scale):
    _say("inject", shape, ham.kind, prec, scale)
    th = torch.tensor(di.draw_params(shape, 29, scale))
    m = L.Model(shape, prec)
    m.set_params(th)
    desc = ModelDesc.of(shape)
    ns = shape.n_spins
    sp = di.uniform_spins(B, ns, 37)
    M_max = ns if ham.kind == "lrtfim" else 2 * ns
    ref = O.eloc_plain(desc, ham, th, sp, M_max)
    # float64: the oracle's ABACUS, free of the plain ratio's |log psi| rounding; float32: the
    # plain ratio (the definition), whose rounding lies far below the float32 tolerance
    ref_ab = O.abacus_logratio(desc, th, sp, ref["sites"], ref["n_conn"]) if prec == "fp64" else ref["logratio"]
    Om = forward(desc, th, sp)["Omega"]
    mag = lambda x: (torch.view_as_real(x) if x.is_complex() else x).abs().max().item()  # noqa: E731
    lr_scale = mag(ref_ab)
    if ham.kind == "j1j2":  # pair exchanges: measured against the single-flip ratios of the samples
        single = O.connected(di.HamSpec("lrtfim", shape.bc), sp)
        _, lr1 = O.plain_logratio(desc, th, sp, single[0], single[2])
        lr_scale = max(lr_scale, mag(lr1))
    spd = torch.tensor(sp, device="cuda")
    tol = 1e-10 if prec == "fp64" else 1e-4
    for path in ("abacus", "full"):
        lp, lr, el = (t.cpu() for t in m.eloc(ham, spd, M_max, path=path))
        e_lp, e_el = eps(lp, ref["logpsi"]), eps(el, ref["eloc"])
        d_lr = mag(lr - ref_ab)
        floor = 0.0
        if path == "full":
            u = 2.2e-16 if prec == "fp64" else 6e-8
            floor = 1e3 * u * max(1.0, Om.abs().max().item()) ** 2
        _say(f"  {path}: eps_logpsi {e_lp:.3e} eps_eloc {e_el:.3e} |d lr| {d_lr:.3e} (scale {lr_scale:.3e})")
        assert e_lp <= tol and e_el <= tol
        assert d_lr <= tol * lr_scale + floor
    m.close()


def test_inject_sweep_matches_oracle(L):
    shape = di.ModelShape(14, 3, 4, 3, act="silu", bc="periodic", inject_phi=1)
    desc = ModelDesc.of(shape)
    th = torch.tensor(di.draw_params(shape, 17, "stress"))
    th[-2 * shape.d:] *= 10.0
    m = L.Model(shape, "fp64")
    m.set_params(th)
    B, ns = 3, shape.n_spins
    spins = torch.tensor(di.uniform_spins(B, ns, 4), device="cuda")
    host = [spins[b].cpu().long() for b in range(B)]
    refreshes = 0
    for sweep in range(4):
        parity = sweep % 2
        K = len(range(parity, ns, 2))
        rng = np.random.Generator(np.random.PCG64(970 + sweep))
        r, u = rng.random((B, K)), rng.random((B, K))
        acc, ref = m.screened_sweep(spins, 1, parity, torch.tensor(r, device="cuda"), torch.tensor(u, device="cuda"),
                                    0.1)
        acc, ref = acc.cpu(), ref.cpu()
        for b in range(B):
            sites = typewriter_sites(ns, 1, parity, r[b])
            want = screened_sweep(desc, th, host[b], sites, u[b], 0.1)
            assert acc[b].tolist() == [int(x) for x in want["accepted"]], (sweep, b)
            assert int(ref[b]) == want["refreshes"], (sweep, b)
            host[b] = want["spins"]
            refreshes += want["refreshes"]
        assert torch.equal(spins.cpu().long(), torch.stack(host)), sweep
    assert refreshes > 0
    m.close()


def test_inject_ragged_matches_oracle(L):
    cases = [
        (di.ModelShape(20, 2, 16, 8, bc="periodic", inject_phi=1), di.HamSpec("j1j2", "periodic"), 4, "fp64"),
        (di.ModelShape(19, 1, 8, 4, act="tanh", bc="open", inject_phi=1), di.HamSpec("lrtfim", "open"), 5, "fp64"),
        (di.ModelShape(35, 3, 32, 16, bc="open", inject_phi=1), di.HamSpec("lrtfim", "open"), 3, "fp32"),
    ]
    models, thetas, spins, lps, els = [], [], [], [], []
    for i, (shape, ham, B, prec) in enumerate(cases):
        th = torch.tensor(di.draw_params(shape, 7800 + i, "stress"))
        m = L.Model(shape, prec)
        m.set_params(th)
        models.append(m)
        thetas.append(th)
        spins.append(torch.tensor(di.uniform_spins(B, shape.n_spins, 7900 + i), device="cuda"))
        lps.append(torch.full((B,), float("nan"), dtype=torch.float64, device="cuda"))
        els.append(torch.full((B,), float("nan"), dtype=torch.float64, device="cuda"))
    # the first graph-mode call runs eagerly and records; the next two replay the recording
    # (with the background phi copies as memcpy nodes) on new spins in the same tensors, with
    # other GPU work in between
    for call in range(3):
        if call:
            for i, (shape, ham, B, prec) in enumerate(cases):
                spins[i].copy_(torch.tensor(di.uniform_spins(B, shape.n_spins, 7950 + 10 * call + i), device="cuda"))
                lps[i].fill_(float("nan"))
                els[i].fill_(float("nan"))
            junk = torch.randn(1 << 20, device="cuda")
            (junk * 2).sum().item()
        L.ragged_eloc(models, [c[1] for c in cases], spins, lps, els, n_streams=2, mode="graph")
        torch.cuda.synchronize()
        for i, (shape, ham, B, prec) in enumerate(cases):
            M_max = shape.n_spins if ham.kind == "lrtfim" else 2 * shape.n_spins
            ref = O.eloc_plain(ModelDesc.of(shape), ham, thetas[i], spins[i].cpu().numpy(), M_max)
            tol = 1e-10 if prec == "fp64" else 1e-4
            e_el, e_lp = eps(els[i], ref["eloc"]), eps(lps[i], ref["logpsi"])
            _say(f"  ragged call {call} inst {i}: eps_eloc {e_el:.3e} eps_logpsi {e_lp:.3e}")
            assert e_el <= tol and e_lp <= tol, (call, i)
    for m in models:
        m.close()


GRAD_CASES = [
    (di.ModelShape(12, 1, 4, 2, act="tanh", bc="open", inject_phi=1), "fp64"),
    (di.ModelShape(14, 2, 6, 3, act="silu", bc="periodic", inject_phi=1), "fp64"),
    (di.ModelShape(16, 3, 8, 4, act="identity", bc="open", w_c=2, inject_phi=1), "fp64"),
    (di.ModelShape(15, 4, 6, 3, act="silu", bc="periodic", inject_phi=1), "fp64"),
    (di.ModelShape(9, 3, 6, 3, act="tanh", bc="periodic", inject_phi=1, token=2), "fp64"),
    (di.ModelShape(14, 2, 6, 3, act="silu", bc="open", inject_phi=1, complex_out=1), "fp64"),
    (di.ModelShape(40, 3, 20, 6, act="silu", bc="open", inject_phi=1), "fp32"),
]


@pytest.mark.parametrize("shape,prec", GRAD_CASES, ids=lambda x: str(x)[:56])
@pytest.mark.parametrize("scale", ["baseline", "stress"])
def test_inject_grad_matches_oracle(L, shape, prec, scale):
    """Log-derivatives with phi injected (the backward adds the mixer input's gradient to the
    phi stream's) against the oracle's autodiff; measure and bounds of the per-site gradient
    tests: eps_grad = max_b ||g_b - g*_b|| / max(||g*_b||, 1e-3 max_b' ||g*_b'||), 1e-10 in
    float64 mode, 1e-4 in float32 mode."""
    _say("inject grad", shape, prec, scale)
    th = torch.tensor(di.draw_params(shape, 6105, scale))
    m = L.Model(shape, prec)
    m.set_params(th)
    sp = di.uniform_spins(5, shape.n_spins, 7)
    lp, g, _ = m.grad_logpsi(torch.tensor(sp, device="cuda"))
    ref = grad_logpsi_batched(ModelDesc.of(shape), th, sp)
    g = g.cpu()
    if ref.is_complex():  # real and imaginary parts side by side
        g, ref = torch.cat([g.real, g.imag], 1), torch.cat([ref.real, ref.imag], 1)
    g, ref = g.double(), ref.double()
    nrm = ref.norm(dim=1)
    e = ((g - ref).norm(dim=1) / nrm.clamp_min(max(1e-3 * nrm.max().item(), 1e-300))).max().item()
    _say(f"  eps_grad {e:.3e}")
    assert e <= (1e-10 if prec == "fp64" else 1e-4)
    m.close()
