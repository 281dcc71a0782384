"""GPU parity of the ragged batch (dn_ragged_eloc): instances of different shapes, depths,
widths, precisions and Hamiltonians in one submission, against the FP64 oracle instance by
instance. Graph mode is checked on its first (eager, recording) call and on replays after the
spins were refilled in place, which changes every instance's generator output (and, for the
J1-J2 chain, its number of connected elements). Tolerances are those of the single-model
parity tests: 1e-10 in float64 mode, 1e-4 in float32 mode (normwise, eps(x) =
max|x - x*| / max|x*|).
"""
import sys

import numpy as np
import pytest
import torch

import dn_inputs as di
import oracle as O
from oracle.model import ModelDesc

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


# (shape, Hamiltonian, B, precision, spin recipe): ragged tails (N not a multiple of 64),
# one to four blocks, every padded width, both chains and boundary conditions.
SMALL = [
    (di.ModelShape(19, 1, 8, 4, act="tanh", bc="open"), di.HamSpec("lrtfim", "open"), 6, "fp64", "uniform"),
    (di.ModelShape(40, 2, 16, 8, bc="periodic"), di.HamSpec("j1j2", "periodic"), 5, "fp64", "balanced"),
    (di.ModelShape(70, 3, 32, 16, bc="open"), di.HamSpec("lrtfim", "open", alpha=2.0, h=0.5), 4, "fp32",
     "uniform"),
    (di.ModelShape(130, 4, 64, 32, bc="open"), di.HamSpec("j1j2", "open"), 3, "fp32", "uniform"),
    (di.ModelShape(33, 2, 20, 6, act="identity", bc="periodic"),
     di.HamSpec("lrtfim", "periodic", J=-5.0, alpha=6.0, h=1.0, paper_form=1), 7, "fp32", "uniform"),
]


def _spins(recipe, B, N, seed):
    f = di.uniform_spins if recipe == "uniform" else di.balanced_spins
    return f(B, N, seed)


def _m_max(shape, ham):
    return shape.N if ham.kind == "lrtfim" else 2 * shape.N


def _setup(L, cases, seed0):
    models, thetas, spins, lps, els = [], [], [], [], []
    for i, (shape, ham, B, prec, recipe) in enumerate(cases):
        th = torch.tensor(di.draw_params(shape, seed0 + i, "stress"))
        m = L.Model(shape, prec)
        m.set_params(th)
        models.append(m)
        thetas.append(th)
        spins.append(torch.tensor(_spins(recipe, B, shape.N, seed0 + 50 + i), device="cuda"))
        lps.append(torch.full((B,), float("nan"), dtype=torch.float64, device="cuda"))
        els.append(torch.full((B,), float("nan"), dtype=torch.float64, device="cuda"))
    return models, thetas, spins, lps, els


def _check(cases, thetas, spins, lps, els, tag):
    torch.cuda.synchronize()
    for i, (shape, ham, B, prec, _) in enumerate(cases):
        sp = spins[i].cpu().numpy()
        ref = O.eloc_plain(ModelDesc.of(shape), ham, thetas[i], sp, _m_max(shape, ham))
        tol = 1e-10 if prec == "fp64" else 1e-4
        e_el, e_lp = eps(els[i], ref["eloc"]), eps(lps[i], ref["logpsi"])
        _say(f"  {tag} inst {i} N={shape.N} L={shape.L} d={shape.d} {ham.kind} {prec}: "
             f"eps_eloc {e_el:.3e} eps_logpsi {e_lp:.3e}")
        assert e_el <= tol and e_lp <= tol, (tag, i, e_el, e_lp)


@pytest.mark.parametrize("mode,n_streams", [("eager", 1), ("eager", 3), ("graph", 1), ("graph", 4)])
def test_ragged_small_matches_oracle(L, mode, n_streams):
    _say("ragged small", mode, n_streams)
    models, thetas, spins, lps, els = _setup(L, SMALL, 7100)
    hams = [c[1] for c in SMALL]
    L.ragged_eloc(models, hams, spins, lps, els, n_streams=n_streams, mode=mode)
    _check(SMALL, thetas, spins, lps, els, f"{mode} call 1")
    # new spins in the same tensors: a graph-mode call now replays the recording
    for rep in range(2):
        for i, (shape, ham, B, prec, recipe) in enumerate(SMALL):
            spins[i].copy_(torch.tensor(_spins(recipe, B, shape.N, 9000 + 10 * rep + i)))
            els[i].fill_(float("nan"))
            lps[i].fill_(float("nan"))
        L.ragged_eloc(models, hams, spins, lps, els, n_streams=n_streams, mode=mode)
        _check(SMALL, thetas, spins, lps, els, f"{mode} call {rep + 2}")
    for m in models:
        m.close()


def test_ragged_replay_after_param_update(L):
    """Parameters change in place: the recorded graph reads the new tables."""
    cases = SMALL[2:4]
    models, thetas, spins, lps, els = _setup(L, cases, 7300)
    hams = [c[1] for c in cases]
    L.ragged_eloc(models, hams, spins, lps, els, mode="graph")
    for i, (shape, *_rest) in enumerate(cases):
        thetas[i] = torch.tensor(di.draw_params(shape, 7400 + i, "stress"))
        models[i].set_params(thetas[i])
    L.ragged_eloc(models, hams, spins, lps, els, mode="graph")
    _check(cases, thetas, spins, lps, els, "after set_params")
    for m in models:
        m.close()


def test_ragged_argument_errors(L):
    shape = di.ModelShape(40, 2, 16, 8)
    m = L.Model(shape, "fp32")
    sp = torch.tensor(di.uniform_spins(4, 40, 1), device="cuda")
    el = torch.empty(4, dtype=torch.float64, device="cuda")
    ham = di.HamSpec("lrtfim", "open")
    with pytest.raises(L.DysonNetError) as ei:       # parameters not set
        L.ragged_eloc([m], [ham], [sp], None, [el])
    assert ei.value.status == L.DN_ESTATE
    m.set_params(torch.tensor(di.draw_params(shape, 1, "baseline")))
    with pytest.raises(L.DysonNetError) as ei:       # one model twice
        L.ragged_eloc([m, m], [ham, ham], [sp, sp], None, [el, el])
    assert ei.value.status == L.DN_EINVAL
    with pytest.raises(L.DysonNetError) as ei:       # J1-J2 on a chain too short
        small = L.Model(di.ModelShape(4, 1, 8, 4), "fp32")
        small.set_params(torch.tensor(di.draw_params(di.ModelShape(4, 1, 8, 4), 1, "baseline")))
        L.ragged_eloc([small], [di.HamSpec("j1j2", "open")],
                      [torch.ones((2, 4), dtype=torch.int8, device="cuda")], None, [el[:2]])
    assert ei.value.status == L.DN_EINVAL
    # empty instances are skipped
    L.ragged_eloc([m], [ham], [sp[:0]], None, [el[:0]])
    m.close()


def test_ragged_full_size_sampled(L):
    """The 32-instance ragged batch (N ~ U{32..512}, L ~ U{2,3,4}, B ~ U{256..2048}, d=64,
    s=32, float32) in the benchmark's launch configuration (graph mode, 4 streams): every
    instance's E_loc and log psi checked against the oracle on one sample, and on a second
    replay with the instance's spins rolled by one sample."""
    ws = di.ragged_instances()
    models, thetas, spins, lps, els = [], [], [], [], []
    for w in ws:
        th = torch.tensor(w.params("stress"))
        m = L.Model(w.model, "fp32")
        m.set_params(th)
        models.append(m)
        thetas.append(th)
        spins.append(torch.tensor(w.spin_batch(), device="cuda"))
        lps.append(torch.empty(w.B, dtype=torch.float64, device="cuda"))
        els.append(torch.empty(w.B, dtype=torch.float64, device="cuda"))
    hams = [w.ham for w in ws]
    _say("ragged full size: 32 instances, total B", sum(w.B for w in ws))
    for call in range(2):
        if call == 1:
            for s in spins:
                s.copy_(torch.roll(s, 1, dims=0))
        L.ragged_eloc(models, hams, spins, lps, els, n_streams=4, mode="graph")
        torch.cuda.synchronize()
        for i, w in enumerate(ws):
            b = (37 * i + 11 * call) % w.B
            sp = spins[i][b:b + 1].cpu().numpy()
            ref = O.eloc_plain(ModelDesc.of(w.model), w.ham, thetas[i], sp, w.model.N)
            # one sample's E_loc can sit near zero: measure against the size of its terms
            terms = ref["hdiag"][0].abs() + (ref["helem"][0].abs() * torch.exp(ref["logratio"][0])).sum()
            e_el = abs(els[i][b].item() - ref["eloc"][0].item()) / terms.item()
            e_lp = abs(lps[i][b].item() - ref["logpsi"][0].item()) / max(abs(ref["logpsi"][0].item()), 1e-3)
            _say(f"  call {call} inst {i} N={w.model.N} L={w.model.L} b={b}: eps_eloc {e_el:.3e} "
                 f"eps_logpsi {e_lp:.3e}")
            assert e_el <= 1e-4 and e_lp <= 1e-4
            assert bool(torch.isfinite(els[i]).all())
    for m in models:
        m.close()


def test_autotune_keeps_results(L):
    """The autotuner only changes launch shapes: results stay at the oracle's values."""
    shape = di.ModelShape(70, 3, 32, 16, bc="open")
    ham = di.HamSpec("lrtfim", "open", alpha=2.0, h=0.5)
    th = torch.tensor(di.draw_params(shape, 77, "stress"))
    m = L.Model(shape, "fp32")
    m.set_params(th)
    nt, bud = m.autotune(ham, B_probe=64)
    _say("autotune:", nt, bud >> 20, "MiB")
    assert nt in (1, 2, 3, 4) and bud in (256 << 20, 1 << 30, 3 << 30)
    sp = di.uniform_spins(5, shape.N, 78)
    ref = O.eloc_plain(ModelDesc.of(shape), ham, th, sp, shape.N)
    lp, lr, el = m.eloc(ham, torch.tensor(sp, device="cuda"), shape.N, path="abacus")
    assert eps(el.cpu(), ref["eloc"]) <= 1e-4 and eps(lp.cpu(), ref["logpsi"]) <= 1e-4
    m.close()


def test_ragged_rerecords_after_workspace_growth(L):
    """A model used elsewhere between submissions may have to grow (move) its workspace; the
    next ragged call must then record a new graph instead of replaying one that points at the
    old buffers."""
    cases = SMALL[2:4]
    models, thetas, spins, lps, els = _setup(L, cases, 7500)
    hams = [c[1] for c in cases]
    L.ragged_eloc(models, hams, spins, lps, els, mode="graph")
    L.ragged_eloc(models, hams, spins, lps, els, mode="graph")   # a replay
    # a much larger batch on the first model grows its flip and cache buffers
    shape, ham = cases[0][0], cases[0][1]
    big = torch.tensor(di.uniform_spins(512, shape.N, 7600), device="cuda")
    models[0].eloc(ham, big, shape.N, path="abacus")
    for i, (shape, ham, B, prec, recipe) in enumerate(cases):
        spins[i].copy_(torch.tensor(_spins(recipe, B, shape.N, 7700 + i)))
    L.ragged_eloc(models, hams, spins, lps, els, mode="graph")
    _check(cases, thetas, spins, lps, els, "after workspace growth")
    for m in models:
        m.close()
