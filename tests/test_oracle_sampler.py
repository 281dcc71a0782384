"""Pins of the oracle's screened typewriter sampler (Sec. IV, Algorithm 2; App. "Screened
Metropolis sampler is exact"; App. "Practical implementation of the screened typewriter sampler").

* typewriter schedule: one proposal in every other block of width `spacing`, inside its block;
* the screened rule reproduces exact Metropolis-Hastings decision for decision (same draws u)
  whenever eps bounds |min(1, R~) - min(1, R)| for every decision taken without a refresh (the
  appendix's theorem), on networks of one to three blocks, open and periodic, with a sharpened
  read-out (acceptance well inside (0, 1)) and tightly packed proposals;
* the screen is not vacuous: without it (eps = 0) the bare independent-scattering chain takes a
  decision exact Metropolis-Hastings does not, on the same networks and draws;
* eps = 1 refreshes at every proposal, so every ratio is exact;
* with eps = 0 the chain is the bare independent-scattering chain written out here by brute force:
  updates from full evaluations of single flips of the starting configuration, ratios
  prod_units cosh^2(Omega + dOmega) / cosh^2(Omega) with Omega accumulating the accepted updates.
"""
import math

import numpy as np
import pytest
import torch

import dn_inputs as di
from oracle.model import ModelDesc, forward
from oracle.sampler import exact_mh_sweep, screened_sweep, typewriter_sites, update_eps_buffer


def _draws(shape, K, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random(K), rng.random(K)


def _peaked(shape, seed, scale=10.0):
    th = torch.tensor(di.draw_params(shape, seed, "stress"))
    th[-2 * shape.d:] *= scale  # the read-out A
    return th


@pytest.mark.parametrize("N,spacing,parity", [(16, 3, 0), (16, 3, 1), (17, 4, 1), (10, 10, 0), (12, 1, 0)])
def test_typewriter_sites_one_per_visited_block(N, spacing, parity):
    nblk = (N + spacing - 1) // spacing
    blocks = list(range(parity, nblk, 2))
    r, _ = _draws(None, len(blocks), 5)
    r[0] = 0.9999999999  # the last site of a block
    sites = typewriter_sites(N, spacing, parity, r)
    assert len(sites) == len(blocks)
    for j, b in zip(sites, blocks):
        assert b * spacing <= j < min((b + 1) * spacing, N)
    assert sites == sorted(sites)


CASES = [
    (di.ModelShape(14, 1, 4, 3, act="tanh", bc="open"), 1, 0.02),
    (di.ModelShape(16, 2, 4, 3, act="silu", bc="open"), 1, 0.1),
    (di.ModelShape(15, 2, 3, 2, act="silu", bc="periodic"), 2, 0.1),
    (di.ModelShape(14, 3, 3, 2, act="tanh", bc="open"), 2, 0.05),
]


def _chain(shape, spacing, eps, sweeps=4, B=3):
    """B chains (the GPU sampler test's setup), several half-sweeps of alternating parity."""
    desc = ModelDesc.of(shape)
    th = _peaked(shape, 17)
    chains = [torch.tensor(x).long() for x in di.uniform_spins(B, shape.N, 4)]
    out = []
    for sweep in range(sweeps):
        parity = sweep % 2
        K = len(range(parity, (shape.N + spacing - 1) // spacing, 2))
        rng = np.random.Generator(np.random.PCG64(700 + sweep))
        r, u = rng.random((B, K)), rng.random((B, K))
        for b in range(B):
            sites = typewriter_sites(shape.N, spacing, parity, r[b])
            ref = exact_mh_sweep(desc, th, chains[b], sites, u[b])
            got = screened_sweep(desc, th, chains[b], sites, u[b], eps, track=True)
            out.append((ref, got))
            chains[b] = ref["spins"]
    return out


@pytest.mark.parametrize("shape,spacing,eps", CASES, ids=lambda x: str(x)[:40])
def test_screened_equals_exact_metropolis(shape, spacing, eps):
    refreshes = 0
    for ref, got in _chain(shape, spacing, eps):
        assert got["unscreened_err"] <= eps  # the theorem's precondition on this trajectory ...
        assert got["accepted"] == ref["accepted"]  # ... so every decision is the exact one
        assert torch.equal(got["spins"], ref["spins"])
        refreshes += got["refreshes"]
    assert refreshes > 0


def test_screen_is_not_vacuous():
    differs = 0
    for shape, spacing, _ in CASES:
        for ref, got in _chain(shape, spacing, 0.0):
            differs += sum(a != b for a, b in zip(got["accepted"], ref["accepted"]))
    assert differs > 0


def test_unit_tolerance_refreshes_every_proposal():
    shape = di.ModelShape(12, 2, 4, 3, bc="open")
    desc = ModelDesc.of(shape)
    th = _peaked(shape, 3)
    s = torch.tensor(di.uniform_spins(1, 12, 2)[0])
    r, u = _draws(shape, 3, 9)
    sites = typewriter_sites(12, 2, 0, r)
    got = screened_sweep(desc, th, s, sites, u, eps=1.0)
    ref = exact_mh_sweep(desc, th, s, sites, u)
    assert got["refreshes"] == len(sites)
    assert got["accepted"] == ref["accepted"]


def test_zero_tolerance_is_the_independent_scattering_chain():
    shape = di.ModelShape(13, 2, 3, 2, bc="open")
    desc = ModelDesc.of(shape)
    th = _peaked(shape, 8)
    s0 = torch.tensor(di.uniform_spins(1, 13, 6)[0])
    r, u = _draws(shape, 6, 12)
    sites = typewriter_sites(13, 1, 1, r)
    got = screened_sweep(desc, th, s0, sites, u, eps=0.0)
    assert got["refreshes"] == 0
    Om0 = forward(desc, th, s0[None])["Omega"][0]
    Om = Om0.clone()
    s = s0.clone()
    for k, j in enumerate(sites):
        sp = s0.clone()
        sp[j] = -sp[j]
        dO = forward(desc, th, sp[None])["Omega"][0] - Om0
        R = float(torch.prod(torch.cosh(Om + dO) ** 2 / torch.cosh(Om) ** 2))
        a = float(u[k]) < min(1.0, R)
        assert a == got["accepted"][k]
        if a:
            s[j] = -s[j]
            Om = Om + dO
    assert torch.equal(s, got["spins"])


# ---- the practical tolerance schedule eps(n) (App. "Practical implementation of the screened
# typewriter sampler"): a buffer indexed by the flips accepted since the background


def test_constant_buffer_equals_fixed_tolerance():
    shape, spacing, eps = CASES[1]
    desc = ModelDesc.of(shape)
    th = _peaked(shape, 17)
    s0 = torch.tensor(di.uniform_spins(1, shape.N, 4)[0]).long()
    rng = np.random.Generator(np.random.PCG64(71))
    K = len(range(0, shape.N, 2))
    r, u = rng.random(K), rng.random(K)
    sites = typewriter_sites(shape.N, spacing, 0, r)
    a = screened_sweep(desc, th, s0, sites, u, eps)
    b = screened_sweep(desc, th, s0, sites, u, 0.0, eps_buf=[eps] * 5)
    assert a["accepted"] == b["accepted"] and torch.equal(a["spins"], b["spins"])
    assert a["refreshes"] == b["refreshes"] and a["events"] == b["events"]


def test_buffer_update_rule_worked_example():
    # entries start at the default 0.2 (not yet set); gamma = 1.5; n beyond the buffer uses its
    # last entry
    buf, is_set = [0.2] * 3, [False] * 3
    update_eps_buffer(buf, is_set, [(1, 0.03)], 1.5)
    assert buf == [0.2, 0.03, 0.2] and is_set == [False, True, False]   # first visit: e~ itself
    update_eps_buffer(buf, is_set, [(1, 0.05), (1, 0.01)], 1.5)
    assert math.isclose(buf[1], 0.075)                                    # max(0.03, 1.5 * 0.05)
    update_eps_buffer(buf, is_set, [(7, 0.004), (2, 0.001)], 1.5)
    assert buf[2] == 0.004 and is_set[2]       # n = 7 -> entry 2 (first visit), then max(0.004, 0.0015)
    update_eps_buffer(buf, is_set, [(0, 0.0)], 1.5)
    assert buf[0] == 0.0 and is_set[0]


def _adaptive_run(shape, spacing, sweeps, B, gamma, default, seed):
    desc = ModelDesc.of(shape)
    th = _peaked(shape, 17)
    chains = [torch.tensor(x).long() for x in di.uniform_spins(B, shape.N, 4)]
    buf, is_set = [default] * 6, [False] * 6
    refreshes, out = [], []
    for sweep in range(sweeps):
        parity = sweep % 2
        K = len(range(parity, (shape.N + spacing - 1) // spacing, 2))
        rng = np.random.Generator(np.random.PCG64(seed + sweep))
        r, u = rng.random((B, K)), rng.random((B, K))
        events, nref = [], 0
        for b in range(B):
            sites = typewriter_sites(shape.N, spacing, parity, r[b])
            got = screened_sweep(desc, th, chains[b], sites, u[b], 0.0, track=True, eps_buf=list(buf))
            ref = exact_mh_sweep(desc, th, chains[b], sites, u[b])
            out.append((ref, got))
            events += got["events"]
            nref += got["refreshes"]
            chains[b] = got["spins"]
        update_eps_buffer(buf, is_set, events, gamma)
        refreshes.append(nref)
    return out, refreshes, buf, is_set


def test_adaptive_schedule_calibrates_and_stays_exact():
    shape = di.ModelShape(16, 2, 4, 3, act="silu", bc="open")
    out, refreshes, buf, is_set = _adaptive_run(shape, 1, 6, 3, 1.5, 0.2, 930)
    for ref, got in out:
        for n, e in got["events"]:
            if n == 0:  # no accepted flip since the background: the approximate ratio is exact
                assert e <= 1e-12
        if got["unscreened_excess"] <= 0.0:  # every unscreened decision's error within its tolerance
            assert got["accepted"] == ref["accepted"]
    assert any(is_set) and max(b for b, s_ in zip(buf, is_set) if s_) < 0.2
    # the conservative default freezes at every ambiguous draw within 0.2; calibrated entries
    # freeze far less often
    assert refreshes[-1] < refreshes[0]
