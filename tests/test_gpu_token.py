"""GPU parity of token size > 1 (patching: N tokens of `token` spins, token tau embedded as
sum_k E_k s_(token tau + k)) against the FP64 oracle, through the C ABI.

Measures and tolerances are those of the per-site parity tests (normwise eps(x) =
max|x - x*| / max|x*|; 1e-10 in float64 mode, 1e-4 in float32 mode; the plain path's log-ratios
with their |Omega|^2 rounding floor; pair ratios relative to the single-flip ratios of the same
samples). Cases: one to four blocks (the fused one/two-block kernel with its per-position links,
the deep chain), open and periodic, single flips and pair exchanges inside one token and across
two, token sizes 2 and 3; gradients against the oracle's autodiff; the screened sampler's
decisions exactly; a ragged batch with a token instance; the paper's benchmark shape (1000 spins
in 500 tokens of two, two blocks, d = 2, s = 12) at full size on sampled outputs.
"""
import dataclasses
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
    x, ref = torch.as_tensor(x).double().cpu(), torch.as_tensor(ref).double().cpu()
    return (x - ref).abs().max().item() / max(ref.abs().max().item(), 1e-300)


CASES = [
    # shape (N in tokens), ham, prec, B
    (di.ModelShape(8, 1, 8, 4, act="tanh", bc="open", token=2), di.HamSpec("lrtfim", "open"), "fp64", 4),
    (di.ModelShape(10, 2, 8, 4, act="silu", bc="open", token=2), di.HamSpec("lrtfim", "open", alpha=2.0, h=0.5),
     "fp64", 3),
    (di.ModelShape(9, 2, 6, 3, act="silu", bc="periodic", token=2), di.HamSpec("j1j2", "periodic"), "fp64", 3),
    (di.ModelShape(11, 3, 6, 3, act="tanh", bc="open", token=2), di.HamSpec("j1j2", "open"), "fp64", 3),
    (di.ModelShape(10, 4, 8, 4, act="silu", bc="periodic", token=3), di.HamSpec("j1j2", "periodic"), "fp64", 2),
    (di.ModelShape(7, 2, 5, 3, act="tanh", bc="open", token=3), di.HamSpec("j1j2", "open"), "fp64", 3),
    (di.ModelShape(64, 2, 32, 16, bc="open", token=2), di.HamSpec("lrtfim", "open"), "fp32", 3),
    (di.ModelShape(70, 3, 20, 8, bc="periodic", token=2), di.HamSpec("j1j2", "periodic"), "fp32", 2),
]


@pytest.mark.parametrize("shape,ham,prec,B", CASES, ids=lambda x: str(x)[:48])
def test_token_logratio_and_eloc_match_oracle(L, shape, ham, prec, B):
    _say("token", shape, ham.kind, prec)
    th = torch.tensor(di.draw_params(shape, 23, "stress"))
    m = L.Model(shape, prec)
    m.set_params(th)
    desc = ModelDesc.of(shape)
    ns = shape.n_spins
    sp = di.uniform_spins(B, ns, 31)
    M_max = ns if ham.kind == "lrtfim" else 2 * ns
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
        e_lp, e_el = eps(lp, ref["logpsi"]), eps(el, ref["eloc"])
        d_lr = (lr - ref_ab).abs().max().item()
        floor = 0.0
        if path == "full":
            u = 2.2e-16 if prec == "fp64" else 6e-8
            floor = 1e3 * u * max(1.0, Om.abs().max().item()) ** 2
        _say(f"  {path}: eps_logpsi {e_lp:.3e} eps_eloc {e_el:.3e} |d lr| {d_lr:.3e} (scale {lr_scale:.3e})")
        assert e_lp <= tol and e_el <= tol
        assert d_lr <= tol * lr_scale + floor
    m.close()


GRAD_CASES = [
    (di.ModelShape(8, 1, 4, 2, act="tanh", bc="open", token=2), "fp64"),
    (di.ModelShape(9, 2, 6, 3, act="silu", bc="periodic", token=2), "fp64"),
    (di.ModelShape(6, 3, 5, 3, act="identity", bc="open", token=3), "fp64"),
    (di.ModelShape(40, 2, 20, 6, act="silu", bc="periodic", token=2), "fp32"),
]


@pytest.mark.parametrize("shape,prec", GRAD_CASES, ids=lambda x: str(x)[:48])
def test_token_grad_matches_oracle(L, shape, prec):
    th = torch.tensor(di.draw_params(shape, 6005, "stress"))
    m = L.Model(shape, prec)
    m.set_params(th)
    sp = di.uniform_spins(4, shape.n_spins, 7)
    _, g, _ = m.grad_logpsi(torch.tensor(sp, device="cuda"))
    ref = grad_logpsi_batched(ModelDesc.of(shape), th, sp)
    g = g.double().cpu()
    nrm = ref.norm(dim=1)
    e = ((g - ref).norm(dim=1) / nrm.clamp_min(1e-3 * nrm.max().item())).max().item()
    _say(f"token grad N={shape.N}x{shape.token} L={shape.L} {prec}: eps_grad {e:.3e}")
    assert e <= (1e-10 if prec == "fp64" else 1e-4)
    m.close()


def test_token_sweep_matches_oracle(L):
    shape = di.ModelShape(8, 2, 4, 3, act="silu", bc="open", token=2)
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
        rng = np.random.Generator(np.random.PCG64(960 + sweep))
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


def test_token_ragged_matches_oracle(L):
    cases = [
        (di.ModelShape(20, 2, 16, 8, bc="periodic", token=2), di.HamSpec("j1j2", "periodic"), 4, "fp64"),
        (di.ModelShape(19, 1, 8, 4, act="tanh", bc="open"), di.HamSpec("lrtfim", "open"), 5, "fp64"),
        (di.ModelShape(35, 3, 32, 16, bc="open", token=2), di.HamSpec("lrtfim", "open"), 3, "fp32"),
    ]
    models, thetas, spins, lps, els = [], [], [], [], []
    for i, (shape, ham, B, prec) in enumerate(cases):
        th = torch.tensor(di.draw_params(shape, 7600 + i, "stress"))
        m = L.Model(shape, prec)
        m.set_params(th)
        models.append(m)
        thetas.append(th)
        spins.append(torch.tensor(di.uniform_spins(B, shape.n_spins, 7700 + i), device="cuda"))
        lps.append(torch.full((B,), float("nan"), dtype=torch.float64, device="cuda"))
        els.append(torch.full((B,), float("nan"), dtype=torch.float64, device="cuda"))
    L.ragged_eloc(models, [c[1] for c in cases], spins, lps, els, n_streams=2, mode="graph")
    torch.cuda.synchronize()
    for i, (shape, ham, B, prec) in enumerate(cases):
        M_max = shape.n_spins if ham.kind == "lrtfim" else 2 * shape.n_spins
        ref = O.eloc_plain(ModelDesc.of(shape), ham, thetas[i], spins[i].cpu().numpy(), M_max)
        tol = 1e-10 if prec == "fp64" else 1e-4
        e_el, e_lp = eps(els[i], ref["eloc"]), eps(lps[i], ref["logpsi"])
        _say(f"  ragged inst {i} token={shape.token}: eps_eloc {e_el:.3e} eps_logpsi {e_lp:.3e}")
        assert e_el <= tol and e_lp <= tol
    for m in models:
        m.close()


def test_paper_benchmark_shape_sampled(L):
    """1000 spins in 500 tokens of two, two blocks, d = 2, s = 12, periodic, the paper-form
    long-range Ising chain (J = -5, alpha = 6, h = 1), float32, 64 samples: two samples recomputed
    by the oracle element by element, and ABACUS against full re-evaluation for all."""
    shape = di.ModelShape(500, 2, 2, 12, bc="periodic", act="silu", token=2)
    ham = di.HamSpec("lrtfim", "periodic", J=-5.0, alpha=6.0, h=1.0, paper_form=1)
    th = torch.tensor(di.draw_params(shape, 2010, "stress"))
    m = L.Model(shape, "fp32")
    m.set_params(th)
    B, ns = 64, shape.n_spins
    sp = di.uniform_spins(B, ns, 1010)
    spd = torch.tensor(sp, device="cuda")
    lpa, lra, ela = m.eloc(ham, spd, ns, path="abacus")
    lpf, lrf, elf = m.eloc(ham, spd, ns, path="full")
    torch.cuda.synchronize()
    desc = ModelDesc.of(shape)
    pick = [0, B - 1]
    ref = O.eloc_plain(desc, ham, th, sp[pick], ns)
    Om = forward(desc, th, sp[pick])["Omega"]
    lr_scale = ref["logratio"].abs().max().item()
    floor = 1e3 * 6e-8 * max(1.0, Om.abs().max().item()) ** 2
    d_af = (lra.cpu() - lrf.cpu()).abs().max().item()
    d_lr = (lra.cpu()[pick] - ref["logratio"]).abs().max().item()
    _say(f"paper shape: |d lr| abacus-full {d_af:.3e}, abacus-oracle {d_lr:.3e} (scale {lr_scale:.3e}), "
         f"eps_eloc {eps(ela.cpu()[pick], ref['eloc']):.3e}")
    assert d_af <= 1e-4 * lr_scale + floor and eps(ela, elf) <= 1e-4
    assert d_lr <= 1e-4 * lr_scale
    assert eps(ela.cpu()[pick], ref["eloc"]) <= 1e-4 and eps(lpa.cpu()[pick], ref["logpsi"]) <= 1e-4
    m.close()
