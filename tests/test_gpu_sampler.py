"""GPU screened typewriter sampler (dn_screened_sweep, through the C ABI) against the FP64 oracle's
sampler (Sec. IV, Algorithm 2; App. "Screened Metropolis sampler is exact").

Float64 networks with a sharpened read-out (acceptance well inside (0, 1)) and tightly packed
proposals (spacing 1 and 2), so that the independent-scattering ratios are visibly approximate and
the screen does work. Several chains, several half-sweeps of alternating parity, draws from seeded
generators. The accept/reject decisions are integers taken in float64 on both sides: the GPU's
decisions, refresh counts and final configurations must equal the oracle sampler's exactly, and,
whenever the oracle reports that eps bounded the error of every decision taken without a refresh,
they must equal exact Metropolis-Hastings for the same draws.
"""
import sys

import numpy as np
import pytest
import torch

import dn_inputs as di
from oracle.model import ModelDesc
from oracle.sampler import exact_mh_sweep, screened_sweep, typewriter_sites, update_eps_buffer

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


def _peaked(shape, seed, scale=10.0):
    th = torch.tensor(di.draw_params(shape, seed, "stress"))
    th[-2 * shape.d:] *= scale  # the read-out A
    return th


CASES = [
    # shape, spacing, eps (the last case's eps does not bound the error: decisions then follow
    # the screened chain, which the oracle reproduces all the same)
    (di.ModelShape(14, 1, 4, 3, act="tanh", bc="open"), 1, 0.02),
    (di.ModelShape(16, 2, 4, 3, act="silu", bc="open"), 1, 0.1),
    (di.ModelShape(15, 2, 3, 2, act="silu", bc="periodic"), 2, 0.1),
    (di.ModelShape(14, 3, 3, 2, act="tanh", bc="open"), 2, 0.05),
    (di.ModelShape(16, 2, 4, 3, act="silu", bc="open"), 1, 0.02),
]


@pytest.mark.parametrize("shape,spacing,eps", CASES, ids=lambda x: str(x)[:40])
def test_sweep_matches_oracle(L, shape, spacing, eps):
    desc = ModelDesc.of(shape)
    th = _peaked(shape, 17)
    m = L.Model(shape, "fp64")
    m.set_params(th)
    B = 3
    spins = torch.tensor(di.uniform_spins(B, shape.N, 4), device="cuda")
    host = [spins[b].cpu().long() for b in range(B)]
    total_ref, total_acc, exact_ok = 0, 0, True
    for sweep in range(4):
        parity = sweep % 2
        nblk = (shape.N + spacing - 1) // spacing
        K = len(range(parity, nblk, 2))
        rng = np.random.Generator(np.random.PCG64(700 + sweep))
        r = rng.random((B, K))
        u = rng.random((B, K))
        acc, ref = m.screened_sweep(spins, spacing, parity, torch.tensor(r, device="cuda"),
                                    torch.tensor(u, device="cuda"), eps)
        acc, ref = acc.cpu(), ref.cpu()
        for b in range(B):
            sites = typewriter_sites(shape.N, spacing, parity, r[b])
            want = screened_sweep(desc, th, host[b], sites, u[b], eps, track=True)
            assert acc[b].tolist() == [int(x) for x in want["accepted"]], (sweep, b)
            assert int(ref[b]) == want["refreshes"], (sweep, b)
            if want["unscreened_err"] <= eps:
                mh = exact_mh_sweep(desc, th, host[b], sites, u[b])
                assert mh["accepted"] == want["accepted"]
            else:
                exact_ok = False
            host[b] = want["spins"]
            total_ref += want["refreshes"]
            total_acc += sum(want["accepted"])
        assert torch.equal(spins.cpu().long(), torch.stack(host)), sweep
    _say(f"sampler N={shape.N} L={shape.L} spacing {spacing} eps {eps}: accepted {total_acc}, refreshes "
         f"{total_ref}, eps bounded every unscreened decision: {exact_ok}")
    m.close()


def test_sweep_argument_errors(L):
    shape = di.ModelShape(12, 1, 4, 2)
    m = L.Model(shape, "fp64")
    m.set_params(torch.tensor(di.draw_params(shape, 1, "stress")))
    sp = torch.tensor(di.uniform_spins(2, 12, 1), device="cuda")
    r = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    for spacing, parity, eps in ((0, 0, 0.1), (2, 2, 0.1), (2, 0, -1.0)):
        with pytest.raises(L.DysonNetError) as ei:
            m.screened_sweep(sp, spacing, parity, r, r, eps) if spacing > 0 and parity < 2 else \
                L._check(L.lib().dn_screened_sweep(m.handle, L._ptr(sp), 2, spacing, parity, L._ptr(r), L._ptr(r),
                                                   eps, L._ptr(r), L._ptr(r), None))
        assert ei.value.status == L.DN_EINVAL
    m.close()


@pytest.mark.parametrize("shape,spacing,prec", [
    (di.ModelShape(16, 2, 4, 3, act="silu", bc="open"), 1, "fp64"),
    (di.ModelShape(15, 2, 3, 2, act="silu", bc="periodic"), 2, "fp64"),
    (di.ModelShape(14, 3, 3, 2, act="tanh", bc="open"), 1, "fp64"),
], ids=lambda x: str(x)[:40])
def test_adaptive_sweep_matches_oracle(L, shape, spacing, prec):
    """The tolerance buffer eps(n) (App. "Practical implementation of the screened typewriter
    sampler"): decisions, refresh counts and configurations equal the oracle's after every
    half-sweep, and so does the buffer (its flags exactly, its values to 1e-12 absolute: the
    errors are differences of float64 acceptance probabilities formed on both sides)."""
    desc = ModelDesc.of(shape)
    th = _peaked(shape, 17)
    m = L.Model(shape, prec)
    m.set_params(th)
    B, n_eps, gamma, default = 4, 5, 1.5, 0.2
    spins = torch.tensor(di.uniform_spins(B, shape.N, 4), device="cuda")
    host = [spins[b].cpu().long() for b in range(B)]
    buf = torch.full((n_eps,), default, dtype=torch.float64, device="cuda")
    flag = torch.zeros(n_eps, dtype=torch.int32, device="cuda")
    hbuf, hset = [default] * n_eps, [False] * n_eps
    refr = []
    for sweep in range(6):
        parity = sweep % 2
        K = len(range(parity, (shape.N + spacing - 1) // spacing, 2))
        rng = np.random.Generator(np.random.PCG64(930 + sweep))
        r, u = rng.random((B, K)), rng.random((B, K))
        acc, ref = m.screened_sweep_adaptive(spins, spacing, parity, torch.tensor(r, device="cuda"),
                                             torch.tensor(u, device="cuda"), buf, flag, gamma)
        acc, ref = acc.cpu(), ref.cpu()
        events, total = [], 0
        for b in range(B):
            sites = typewriter_sites(shape.N, spacing, parity, r[b])
            want = screened_sweep(desc, th, host[b], sites, u[b], 0.0, eps_buf=list(hbuf))
            assert acc[b].tolist() == [int(x) for x in want["accepted"]], (sweep, b)
            assert int(ref[b]) == want["refreshes"], (sweep, b)
            host[b] = want["spins"]
            events += want["events"]
            total += want["refreshes"]
        update_eps_buffer(hbuf, hset, events, gamma)
        assert torch.equal(spins.cpu().long(), torch.stack(host)), sweep
        assert flag.cpu().tolist() == [int(x) for x in hset], sweep
        assert (buf.cpu() - torch.tensor(hbuf, dtype=torch.float64)).abs().max().item() <= 1e-12, sweep
        refr.append(total)
    _say(f"adaptive sampler N={shape.N} L={shape.L}: refreshes per half-sweep {refr}, "
         f"buffer {[round(x, 4) for x in hbuf]}")
    assert any(hset)
    m.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_two_block_sweep_few_proposals_matches_oracle(L, prec):
    """A two-block network with few proposals per chain propagates them through block 1 over the
    whole chain (no pivot-0 link): that path in float32 (three-term split products) and
    BF16-mixed (hi + lo products) mode, decisions and refreshes against the float64 oracle. The
    draws are fixed; a decision could only differ where u lies within the mode's rounding of the
    ratio, which these draws do not meet."""
    shape = di.ModelShape(40, 2, 32, 8, act="silu", bc="periodic")
    desc = ModelDesc.of(shape)
    th = _peaked(shape, 23)
    m = L.Model(shape, prec)
    m.set_params(th)
    B, spacing, eps = 4, 4, 0.05
    spins = torch.tensor(di.uniform_spins(B, shape.N, 9), device="cuda")
    host = [spins[b].cpu().long() for b in range(B)]
    total_acc = 0
    for sweep in range(4):
        parity = sweep % 2
        nblk = (shape.N + spacing - 1) // spacing
        K = len(range(parity, nblk, 2))
        rng = np.random.Generator(np.random.PCG64(780 + sweep))
        r, u = rng.random((B, K)), rng.random((B, K))
        acc, ref = m.screened_sweep(spins, spacing, parity, torch.tensor(r, device="cuda"),
                                    torch.tensor(u, device="cuda"), eps)
        acc, ref = acc.cpu(), ref.cpu()
        for b in range(B):
            sites = typewriter_sites(shape.N, spacing, parity, r[b])
            want = screened_sweep(desc, th, host[b], sites, u[b], eps)
            assert acc[b].tolist() == [int(x) for x in want["accepted"]], (sweep, b)
            assert int(ref[b]) == want["refreshes"], (sweep, b)
            host[b] = want["spins"]
            total_acc += sum(want["accepted"])
        assert torch.equal(spins.cpu().long(), torch.stack(host)), sweep
    _say(f"two-block sweep {prec}: accepted {total_acc}")
    assert total_acc > 0
    m.close()
