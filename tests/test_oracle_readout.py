"""Pins of the oracle's read-out non-linearity and of the stress parameter draw.

* ``logcosh`` (f = log cosh, Sec. II Eq. (wavefunc)) equals log(cosh x) computed in 60-digit
  decimal arithmetic, on both sides of the |x| = 1 branch point and far into the range where
  cosh overflows a double: a wrong constant in either branch (say a missing ln 2) fails here
  directly, not only through ABACUS == plain;
* ``lcd(a, d) = log cosh(a + d) - log cosh(a)`` (the log-ratio of one read-out unit, formed
  without cancellation) equals the same difference taken in 60-digit arithmetic;
* the stress draw is not vacuous: every block's share of the read-out,
  rho_l = ||sum_i omega_i h^(l)_i|| / ||sum_i omega_i h^(0)_i||, lies in [1e-2, 1e2] for every
  benchmark workload. For zero-magnetisation configurations of a periodic chain omega is
  constant and the embedding's share omega E sum_i s_i vanishes identically; there the
  shares are taken relative to block 1 (and the vanishing is asserted).
"""
import decimal
import math

import pytest
import torch

import dn_inputs as di
from oracle.model import ModelDesc, forward, lcd, logcosh

decimal.getcontext().prec = 60
D = decimal.Decimal


def _logcosh_dec(x: float) -> decimal.Decimal:
    xd = D(repr(x))
    return (((xd.exp() + (-xd).exp()) / 2).ln())


XS = [0.0, 1e-300, 1e-12, 3e-8, 1e-3, 0.1, 0.5, 0.9, 0.999999, 1.0, 1.000001, 1.1, 2.0, 5.0,
      18.0, 19.5, 30.0, 100.0, 709.0, 711.0, 800.0, 5000.0]


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_logcosh_matches_high_precision(sign):
    xs = [sign * x for x in XS]
    got = logcosh(torch.tensor(xs, dtype=torch.float64))
    for x, g in zip(xs, got.tolist()):
        ref = float(_logcosh_dec(x))
        # a few units in the last place of the result
        assert abs(g - ref) <= 4 * 2.2e-16 * abs(ref) + 1e-320, (x, g, ref)


def test_logcosh_is_even_and_branch_continuous():
    x = torch.tensor([1.0 - 1e-15, 1.0, 1.0 + 2.2e-16, 1.0 + 1e-15], dtype=torch.float64)
    v = logcosh(x)
    assert torch.equal(v, logcosh(-x))
    assert (v[1:] - v[:-1]).abs().max().item() <= 1e-14


def test_lcd_matches_high_precision():
    g = torch.Generator().manual_seed(7)
    a = torch.cat([torch.randn(200, generator=g, dtype=torch.float64) * 3,
                   torch.tensor([0.0, 0.0, 0.7, -0.7, 20.0, -20.0, 1.0, -1.0], dtype=torch.float64)])
    dl = torch.cat([torch.randn(200, generator=g, dtype=torch.float64) * torch.logspace(-9, 1, 200, dtype=torch.float64),
                    torch.tensor([1e-7, -1.0, 1.0, -1.0000001, 0.999999, 3.0, -1e-5, 1e-5], dtype=torch.float64)])
    got = lcd(a, dl)
    for ai, di_, gi in zip(a.tolist(), dl.tolist(), got.tolist()):
        # the inputs are the doubles a and d; a + d itself is exact in the decimal reference
        ref = (((D(repr(ai)) + D(repr(di_))).exp() + (-(D(repr(ai)) + D(repr(di_)))).exp()) / 2).ln() - _logcosh_dec(ai)
        ref = float(ref)
        # relative to the change (the quantity lcd is built to keep), with a floor for results
        # that cancel below the inputs' own rounding
        assert abs(gi - ref) <= 1e-13 * abs(ref) + 4e-16 * abs(di_) * (1 + abs(math.tanh(ai))), (ai, di_, gi, ref)


@pytest.mark.parametrize("name", list(di.WORKLOADS))
def test_stress_draw_every_block_carries_signal(name):
    w = di.WORKLOADS[name]
    desc = ModelDesc.of(w.model)
    fw = forward(desc, torch.tensor(w.params("stress")), w.spin_batch(8), cache=True)
    om = fw["omega"]
    share = [torch.einsum("bic,ci->bc", h, om).norm().item() for h in fw["h"]]
    if w.spins == "balanced" and w.model.bc == "periodic":
        assert share[0] <= 1e-12 * share[1]
        ref = share[1]
    else:
        ref = share[0]
    rho = [s / ref for s in share[1:]]
    assert all(1e-2 <= r <= 1e2 for r in rho), rho
    # and the baseline draw is the near-linear regime the stress draw exists to avoid
    fwb = forward(desc, torch.tensor(w.params("baseline")), w.spin_batch(8), cache=True)
    shb = [torch.einsum("bic,ci->bc", h, fwb["omega"]).norm().item() for h in fwb["h"]]
    if not (w.spins == "balanced" and w.model.bc == "periodic"):
        assert shb[-1] / shb[0] < 1e-2
