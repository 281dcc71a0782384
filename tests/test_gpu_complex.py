"""GPU parity of the complex read-out (complex_out = 1: a complex output matrix A, one complex
unit Omega_0 + i Omega_1, complex log psi; Sec. II) against the FP64 oracle, through the C ABI.

Phases are compared modulo 2 pi: for complex values x, x* the measure is
ceps(x, x*) = max |Re(x - x*) + i wrap(Im(x - x*))| / max |x*| (wrap to [-pi, pi]). E_loc is an
ordinary complex number (no wrap). Tolerances follow the real parity tests: 1e-10 in float64
mode, 1e-4 in float32 mode, with the plain path's |Omega|^2 rounding floor for its log-ratios.
The read-out is scaled so that the phases are of order one. The sampler test compares decisions,
refresh counts and final configurations exactly (taken in float64 on both sides).
Log-derivatives O = d Re log psi + i d Im log psi are held to the oracle's autodiff with the
gradient measure of the real tests (normwise per sample, floored at 1e-3 of the batch's largest
norm): 1e-10 in float64, 1e-4 in float32; the torch.autograd wrapper to the oracle's autodiff of
the same real loss; the SR update to the oracle's dense solve of the conjugated moments (1e-8 in
float64, 1e-4 with float32 log-derivatives).
"""
import dataclasses
import math
import sys

import numpy as np
import pytest
import torch

import dn_inputs as di
import oracle as O
from oracle.grad import grad_logpsi_batched
from oracle.model import ModelDesc, forward
from oracle.sampler import exact_mh_sweep, screened_sweep, typewriter_sites
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


def _wrap(y):
    return torch.remainder(y + math.pi, 2 * math.pi) - math.pi


def cdiff(x, ref):
    x, ref = torch.as_tensor(x).cpu(), torch.as_tensor(ref).cpu()
    return torch.complex(x.real - ref.real, _wrap(x.imag - ref.imag)).abs()


def ceps(x, ref):
    return cdiff(x, ref).max().item() / max(torch.as_tensor(ref).abs().max().item(), 1e-300)


def eps(x, ref):
    x, ref = torch.as_tensor(x).cpu(), torch.as_tensor(ref).cpu()
    return (x - ref).abs().max().item() / max(ref.abs().max().item(), 1e-300)


def _cshape(shape):
    return dataclasses.replace(shape, complex_out=1)


def _params(shape, seed, scale="stress", a_scale=5.0):
    th = torch.tensor(di.draw_params(shape, seed, scale))
    th[-2 * shape.d:] *= a_scale  # phases of order one
    return th


CASES = [
    # shape, ham, prec, B: one block (fused kernel), two blocks (fused, pivot-0 link), deep chains
    (di.ModelShape(16, 1, 8, 4, act="tanh", bc="open"), di.HamSpec("lrtfim", "open"), "fp64", 4),
    (di.ModelShape(20, 2, 8, 4, act="silu", bc="open"), di.HamSpec("lrtfim", "open", alpha=2.0, h=0.5), "fp64", 3),
    (di.ModelShape(22, 3, 6, 3, act="tanh", bc="open"), di.HamSpec("j1j2", "open"), "fp64", 3),
    (di.ModelShape(20, 4, 8, 4, act="silu", bc="periodic"), di.HamSpec("j1j2", "periodic"), "fp64", 3),
    (di.ModelShape(64, 2, 32, 16, bc="open"), di.HamSpec("lrtfim", "open"), "fp32", 3),
    (di.ModelShape(40, 2, 64, 32, bc="periodic"), di.HamSpec("j1j2", "periodic"), "fp32", 2),
    (di.ModelShape(70, 3, 20, 8, bc="periodic"), di.HamSpec("j1j2", "periodic"), "fp32", 2),
]


@pytest.mark.parametrize("shape,ham,prec,B", CASES, ids=lambda x: str(x)[:40])
def test_complex_logratio_and_eloc_match_oracle(L, shape, ham, prec, B):
    shape = _cshape(shape)
    _say("complex", shape, ham.kind, prec)
    th = _params(shape, 23)
    m = L.Model(shape, prec)
    m.set_params(th)
    desc = ModelDesc.of(shape)
    sp = di.uniform_spins(B, shape.N, 31)
    M_max = shape.N if ham.kind == "lrtfim" else 2 * shape.N
    ref = O.eloc_plain(desc, ham, th, sp, M_max)
    ref_ab = O.abacus_logratio(desc, th, sp, ref["sites"], ref["n_conn"])
    Om = forward(desc, th, sp)["Omega"]
    lr_scale = ref_ab.abs().max().item()
    if ham.kind == "j1j2":  # pair ratios: relative to the single-flip ratios of the same samples
        single = O.connected(di.HamSpec("lrtfim", shape.bc), sp)
        _, lr1 = O.plain_logratio(desc, th, sp, single[0], single[2])
        lr_scale = max(lr_scale, lr1.abs().max().item())
    assert ref_ab.imag.abs().max() > 1e-2 and ref["logpsi"].imag.abs().max() > 1e-2
    spd = torch.tensor(sp, device="cuda")
    tol = 1e-10 if prec == "fp64" else 1e-4
    for path in ("abacus", "full"):
        lp, lr, el = (t.cpu() for t in m.eloc(ham, spd, M_max, path=path))
        assert lp.dtype == torch.complex128 and lr.dtype == torch.complex128 and el.dtype == torch.complex128
        e_lp, e_el = ceps(lp, ref["logpsi"]), eps(el, ref["eloc"])
        d_lr = cdiff(lr, ref_ab).max().item()
        floor = 0.0
        if path == "full":
            u = 2.2e-16 if prec == "fp64" else 6e-8
            floor = 1e3 * u * max(1.0, Om.abs().max().item()) ** 2
        _say(f"  {path}: eps_logpsi {e_lp:.3e} eps_eloc {e_el:.3e} |d lr| {d_lr:.3e} (scale {lr_scale:.3e})")
        assert e_lp <= tol and e_el <= tol
        assert d_lr <= tol * lr_scale + floor
        # entries beyond n_conn are zero
        for b in range(B):
            assert torch.all(lr[b, int(ref["n_conn"][b]):] == 0)
    lp2 = m.logpsi(spd).cpu()
    assert ceps(lp2, ref["logpsi"]) <= tol
    lp3 = m.logpsi_noalloc(spd).cpu()
    assert torch.equal(lp3, lp2)
    m.close()


def test_complex_local_energy_entry_point(L):
    shape = _cshape(di.ModelShape(18, 2, 8, 4, bc="open"))
    ham = di.HamSpec("lrtfim", "open")
    th = _params(shape, 5)
    sp = di.uniform_spins(4, 18, 9)
    ref = O.eloc_plain(ModelDesc.of(shape), ham, th, sp, 18)
    hd = ref["hdiag"].cuda()
    he = ref["helem"].cuda()
    nc = ref["n_conn"].to(torch.int32).cuda()
    el = L.local_energy(hd, he, nc, ref["logratio"].cuda()).cpu()
    assert el.dtype == torch.complex128
    assert eps(el, ref["eloc"]) <= 1e-13


@pytest.mark.parametrize("shape,spacing,eps_s", [
    (di.ModelShape(16, 2, 4, 3, act="silu", bc="open"), 1, 0.1),
    (di.ModelShape(15, 3, 3, 2, act="tanh", bc="periodic"), 2, 0.05),
], ids=lambda x: str(x)[:40])
def test_complex_sweep_matches_oracle(L, shape, spacing, eps_s):
    shape = _cshape(shape)
    desc = ModelDesc.of(shape)
    th = _params(shape, 17, a_scale=10.0)
    m = L.Model(shape, "fp64")
    m.set_params(th)
    B = 3
    spins = torch.tensor(di.uniform_spins(B, shape.N, 4), device="cuda")
    host = [spins[b].cpu().long() for b in range(B)]
    total_ref = 0
    for sweep in range(4):
        parity = sweep % 2
        K = len(range(parity, (shape.N + spacing - 1) // spacing, 2))
        rng = np.random.Generator(np.random.PCG64(800 + sweep))
        r, u = rng.random((B, K)), rng.random((B, K))
        acc, ref = m.screened_sweep(spins, spacing, parity, torch.tensor(r, device="cuda"),
                                    torch.tensor(u, device="cuda"), eps_s)
        acc, ref = acc.cpu(), ref.cpu()
        for b in range(B):
            sites = typewriter_sites(shape.N, spacing, parity, r[b])
            want = screened_sweep(desc, th, host[b], sites, u[b], eps_s, track=True)
            assert acc[b].tolist() == [int(x) for x in want["accepted"]], (sweep, b)
            assert int(ref[b]) == want["refreshes"], (sweep, b)
            if want["unscreened_err"] <= eps_s:
                assert exact_mh_sweep(desc, th, host[b], sites, u[b])["accepted"] == want["accepted"]
            host[b] = want["spins"]
            total_ref += want["refreshes"]
        assert torch.equal(spins.cpu().long(), torch.stack(host)), sweep
    _say(f"complex sampler N={shape.N} L={shape.L}: refreshes {total_ref}")
    m.close()


def test_complex_ragged_matches_oracle(L):
    """A complex and a real instance in one graph-mode submission."""
    cases = [
        (_cshape(di.ModelShape(40, 2, 16, 8, bc="periodic")), di.HamSpec("j1j2", "periodic"), 4, "fp64"),
        (di.ModelShape(19, 1, 8, 4, act="tanh", bc="open"), di.HamSpec("lrtfim", "open"), 5, "fp64"),
        (_cshape(di.ModelShape(70, 3, 32, 16, bc="open")), di.HamSpec("lrtfim", "open"), 3, "fp32"),
    ]
    models, thetas, spins, lps, els = [], [], [], [], []
    for i, (shape, ham, B, prec) in enumerate(cases):
        th = _params(shape, 7300 + i)
        m = L.Model(shape, prec)
        m.set_params(th)
        models.append(m)
        thetas.append(th)
        spins.append(torch.tensor(di.uniform_spins(B, shape.N, 7400 + i), device="cuda"))
        lps.append(torch.full((B,), float("nan"), dtype=m.out_dtype, device="cuda"))
        els.append(torch.full((B,), float("nan"), dtype=m.out_dtype, device="cuda"))
    for call in range(2):
        if call:
            for i, (shape, ham, B, prec) in enumerate(cases):
                spins[i].copy_(torch.tensor(di.uniform_spins(B, shape.N, 7500 + i)))
        L.ragged_eloc(models, [c[1] for c in cases], spins, lps, els, n_streams=2, mode="graph")
        torch.cuda.synchronize()
        for i, (shape, ham, B, prec) in enumerate(cases):
            M_max = shape.N if ham.kind == "lrtfim" else 2 * shape.N
            ref = O.eloc_plain(ModelDesc.of(shape), ham, thetas[i], spins[i].cpu().numpy(), M_max)
            tol = 1e-10 if prec == "fp64" else 1e-4
            e_el = eps(els[i], ref["eloc"])
            e_lp = ceps(lps[i], ref["logpsi"]) if shape.complex_out else eps(lps[i], ref["logpsi"])
            _say(f"  ragged call {call} inst {i} complex={shape.complex_out}: eps_eloc {e_el:.3e} eps_logpsi {e_lp:.3e}")
            assert e_el <= tol and e_lp <= tol
    for m in models:
        m.close()


def test_complex_full_size_sampled(L):
    """The N=256, four-block, d=64 network with a complex read-out, float32, 256 samples: two
    samples recomputed by the oracle, element by element (ABACUS) and against full
    re-evaluation for the whole batch."""
    w = di.WORKLOADS["tfim_n256_l4_d64"]
    shape, ham = _cshape(w.model), w.ham
    B = 256
    th = _params(shape, w.param_seed, a_scale=3.0)
    m = L.Model(shape, "fp32")
    m.set_params(th)
    sp = w.spin_batch(B)
    spd = torch.tensor(sp, device="cuda")
    lpa, lra, ela = m.eloc(ham, spd, shape.N, path="abacus")
    lpf, lrf, elf = m.eloc(ham, spd, shape.N, path="full")
    torch.cuda.synchronize()
    desc = ModelDesc.of(shape)
    pick = [0, B - 1]
    ref = O.eloc_plain(desc, ham, th, sp[pick], shape.N)
    Om = forward(desc, th, sp[pick])["Omega"]
    lr_scale = ref["logratio"].abs().max().item()
    floor = 1e3 * 6e-8 * max(1.0, Om.abs().max().item()) ** 2
    d_af = cdiff(lra, lrf).max().item()
    _say(f"complex full size: |d lr| abacus vs full {d_af:.3e} (scale {lr_scale:.3e}, floor {floor:.1e})")
    assert d_af <= 1e-4 * lr_scale + floor and eps(ela, elf) <= 1e-4
    d_lr = cdiff(lra.cpu()[pick], ref["logratio"]).max().item()
    _say(f"  abacus vs oracle: |d lr| {d_lr:.3e} eps_eloc {eps(ela.cpu()[pick], ref['eloc']):.3e} "
         f"eps_logpsi {ceps(lpa.cpu()[pick], ref['logpsi']):.3e}")
    assert d_lr <= 1e-4 * lr_scale
    assert eps(ela.cpu()[pick], ref["eloc"]) <= 1e-4 and ceps(lpa.cpu()[pick], ref["logpsi"]) <= 1e-4
    m.close()


def eps_grad(g, ref):
    g, ref = g.to(torch.complex128).cpu(), ref.to(torch.complex128).cpu()
    nrm = ref.abs().pow(2).sum(1).sqrt()
    err = (g - ref).abs().pow(2).sum(1).sqrt()
    return (err / nrm.clamp_min(max(1e-3 * nrm.max().item(), 1e-300))).max().item()


GRAD_CASES = [
    (di.ModelShape(12, 1, 4, 2, act="tanh", bc="open"), "fp64"),
    (di.ModelShape(14, 2, 6, 3, act="silu", bc="periodic"), "fp64"),
    (di.ModelShape(16, 3, 8, 4, act="identity", bc="open", w_c=2), "fp64"),
    (di.ModelShape(40, 2, 20, 6, act="silu", bc="periodic"), "fp32"),
]


@pytest.mark.parametrize("shape,prec", GRAD_CASES, ids=lambda x: str(x)[:44])
def test_complex_grad_matches_oracle(L, shape, prec):
    shape = _cshape(shape)
    th = _params(shape, 6005)
    m = L.Model(shape, prec)
    m.set_params(th)
    sp = di.uniform_spins(5, shape.N, 7)
    lp, g, _ = m.grad_logpsi(torch.tensor(sp, device="cuda"))
    assert g.is_complex() and lp.dtype == torch.complex128
    ref = grad_logpsi_batched(ModelDesc.of(shape), th, sp)
    lp_ref = forward(ModelDesc.of(shape), th, sp)["logpsi"]
    e, e_lp = eps_grad(g, ref), ceps(lp, lp_ref)
    _say(f"complex grad {shape.N} L={shape.L} {prec}: eps_grad {e:.3e} eps_logpsi {e_lp:.3e}")
    assert ref.imag.abs().max() > 1e-3
    assert e <= (1e-10 if prec == "fp64" else 1e-4)
    assert e_lp <= (1e-10 if prec == "fp64" else 1e-4)
    m.close()


def test_complex_weighted_sum_and_autograd(L):
    from paper_2603_11189_amd.autograd import logpsi as lp_fn
    shape = _cshape(di.ModelShape(16, 2, 8, 4, act="silu", bc="open"))
    th = _params(shape, 3)
    m = L.Model(shape, "fp64")
    m.set_params(th)
    sp = di.uniform_spins(6, 16, 2)
    spd = torch.tensor(sp, device="cuda")
    w = torch.linspace(-1.0, 2.0, 6, dtype=torch.float64, device="cuda")
    _, g, ws = m.grad_logpsi(spd, weights=w)
    assert torch.allclose(ws, (w[:, None] * g).sum(0), rtol=1e-12, atol=1e-14)
    # a real loss of the complex log psi: the library's backward against the oracle's autodiff
    a = torch.linspace(0.5, -1.0, 6, dtype=torch.float64)
    c = torch.linspace(-0.3, 1.2, 6, dtype=torch.float64)
    p = th.clone().cuda().requires_grad_(True)
    out = lp_fn(m, p, spd)
    (a.cuda() * out.real + c.cuda() * out.imag).sum().backward()
    q = th.clone().requires_grad_(True)
    ref = forward(ModelDesc.of(shape), q, sp)["logpsi"]
    (a * ref.real + c * ref.imag).sum().backward()
    err = (p.grad.cpu() - q.grad).abs().max().item() / q.grad.abs().max().item()
    _say(f"complex autograd: rel err {err:.3e}")
    assert err <= 1e-10
    m.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_complex_sr_update_matches_dense_solve(L, prec):
    shape = _cshape(di.ModelShape(12, 2, 4, 2, bc="open"))
    ham = di.HamSpec("lrtfim", "open", J=-1.0, alpha=2.0, h=-0.8)
    desc = ModelDesc.of(shape)
    th = _params(shape, 51)
    m = L.Model(shape, prec)
    m.set_params(th)
    B = 48
    sp = di.uniform_spins(B, shape.N, 52)
    spd = torch.tensor(sp, device="cuda")
    _, g, _ = m.grad_logpsi(spd)
    _, _, el = m.eloc(ham, spd, shape.N)
    shift, eta = 1e-2, 0.1
    delta, energy, iters = m.sr_update(g, el, None, shift=shift, eta=eta, max_iter=1000, tol=1e-13)
    ref_O = grad_logpsi_batched(desc, th, sp)
    ref = O.eloc_plain(desc, ham, th, sp, shape.N)
    w_ref = torch.full((B,), 1.0 / B, dtype=torch.float64)
    ref_delta = sr_update(ref_O, ref["eloc"], w_ref, shift, eta)
    e = (delta.cpu() - ref_delta).norm().item() / ref_delta.norm().item()
    E_ref = (w_ref * ref["eloc"]).sum()
    e_E = abs(complex(energy.item()) - complex(E_ref.item()))
    _say(f"complex sr {prec}: CG iterations {iters}, rel err of delta {e:.3e}, |d E| {e_E:.3e}, "
         f"Im E {E_ref.imag.item():.3e}")
    assert e <= (1e-8 if prec == "fp64" else 1e-4)
    assert e_E <= (1e-12 if prec == "fp64" else 1e-6) * max(1.0, abs(E_ref.item()))
    m.close()
