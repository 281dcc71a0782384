"""Pins of the oracle's complex read-out: a complex output matrix A makes log psi complex
(Sec. II, Eq. (wavefunc) and the remark below it on complex wavefunctions). The two real
read-out columns form one complex unit Omega = Omega_0 + i Omega_1, log psi = log cosh(Omega).

* ``logcosh_c`` and ``lcd_c`` equal log cosh z and log(cosh(a + d) / cosh a) taken in 50-digit
  complex arithmetic (mpmath), phases compared modulo 2 pi, on both sides of every branch and
  next to a zero of cosh;
* exp(log psi) equals numpy's complex cosh of the network's own Omega;
* Im A = 0 gives the real network with A[:, 1] = 0 (zero phase); Im A -> -Im A conjugates psi;
* ABACUS equals full re-evaluation for the complex network (Theorem 1 is about Omega, so the
  complex read-out changes nothing upstream), at every depth, open and periodic, flips and pairs;
* the |psi|^2-weighted mean of the complex E_loc equals psi^H H psi / psi^H psi with H the dense
  matrix built independently from Pauli bit operations, and its imaginary part vanishes;
* the screened sampler's decisions equal exact Metropolis-Hastings on |psi|^2;
* the complex log-derivatives equal central differences of Re and Im log psi.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import torch

import dn_inputs as di
import oracle as O
from oracle.grad import grad_logpsi_batched
from oracle.model import ModelDesc, forward, lcd_c, logcosh_c
from oracle.sampler import exact_mh_sweep, screened_sweep, typewriter_sites
from test_oracle_hamiltonian import _all_confs, dense_h

mp.mp.dps = 50


def _wrap(y):
    return y - 2 * math.pi * round(y / (2 * math.pi))


def _cplx(shape, seed=31, scale="stress"):
    return dataclass_replace(shape, complex_out=1), torch.tensor(di.draw_params(shape, seed, scale))


def dataclass_replace(shape, **kw):
    import dataclasses
    return dataclasses.replace(shape, **kw)


XS = [0.0, 1e-9, -0.3, 0.7, -1.0, 2.5, -5.0, 30.0, -400.0]
YS = [0.0, 1e-7, 0.2, -1.3, 1.5707, -1.5708, 3.0, -3.1, 7.5, 100.0]


def test_logcosh_c_matches_high_precision():
    z = torch.tensor([complex(x, y) for x in XS for y in YS], dtype=torch.complex128)
    got = logcosh_c(z)
    for zi, gi in zip(z.tolist(), got.tolist()):
        ref = mp.log(mp.cosh(mp.mpc(zi.real, zi.imag)))
        re, im = float(mp.re(ref)), float(mp.im(ref))
        # the inputs are doubles; sin/cos of |y| up to 100 carry ~|y| eps of absolute error
        assert abs(gi.real - re) <= 1e-13 * abs(re) + 4e-16 * (1 + abs(zi.imag)), (zi, gi, re)
        assert abs(_wrap(gi.imag - im)) <= 1e-13 * abs(im) + 4e-16 * (1 + abs(zi.imag)), (zi, gi, im)


def test_logcosh_c_next_to_a_zero_of_cosh():
    # cosh(x + i pi/2) = i sinh x: |cosh| ~ |x| next to the zero at i pi/2
    for x in [1e-6, -3e-4, 0.01]:
        z = torch.tensor([complex(x, math.pi / 2)], dtype=torch.complex128)
        g = logcosh_c(z)[0].item()
        ref = mp.log(mp.cosh(mp.mpc(x, math.pi / 2)))
        assert abs(g.real - float(mp.re(ref))) <= 1e-13 * abs(float(mp.re(ref)))
        assert abs(_wrap(g.imag - float(mp.im(ref)))) <= 1e-12


def test_real_axis_reduces_to_logcosh():
    x = torch.tensor(XS, dtype=torch.float64)
    g = logcosh_c(torch.complex(x, torch.zeros_like(x)))
    assert torch.equal(g.imag, torch.zeros_like(x))
    assert torch.allclose(g.real, O.model.logcosh(x), rtol=1e-15, atol=0)


def test_lcd_c_matches_high_precision():
    g = torch.Generator().manual_seed(11)
    n = 300
    a = torch.complex(torch.randn(n, generator=g, dtype=torch.float64) * 3,
                      torch.randn(n, generator=g, dtype=torch.float64) * 2)
    mag = torch.logspace(-9, 0.7, n, dtype=torch.float64)
    ang = torch.rand(n, generator=g, dtype=torch.float64) * 2 * math.pi
    dl = torch.polar(mag, ang)
    extra_a = torch.tensor([0.3 + 1.0j, -2 + 0.1j, 0.5 + 1.5j, 20 - 3j], dtype=torch.complex128)
    extra_d = torch.tensor([1.0 + 0j, 0.6 + 0.8j, 0.0 + 0.07j, -1e-6 + 2e-6j], dtype=torch.complex128)
    a = torch.cat([a, extra_a])
    dl = torch.cat([dl, extra_d])
    got = lcd_c(a, dl)
    for ai, di_, gi in zip(a.tolist(), dl.tolist(), got.tolist()):
        A = mp.mpc(ai.real, ai.imag)
        ref = mp.log(mp.cosh(A + mp.mpc(di_.real, di_.imag)) / mp.cosh(A))
        re, im = float(mp.re(ref)), float(mp.im(ref))
        # relative to the change, with a floor for results below the inputs' own rounding
        th = abs(complex(mp.tanh(A)))
        fl = 4e-16 * abs(di_) * (1 + th) + 1e-15 * abs(ai) * abs(di_)
        assert abs(gi.real - re) <= 1e-12 * abs(ref) + fl, (ai, di_, gi, re)
        assert abs(_wrap(gi.imag - im)) <= 1e-12 * abs(ref) + fl, (ai, di_, gi, im)


def test_exp_logpsi_is_cosh_of_omega():
    shape, th = _cplx(di.ModelShape(12, 2, 4, 3, bc="open"))
    desc = ModelDesc.of(shape)
    sp = di.uniform_spins(6, 12, 4)
    out = forward(desc, th, sp)
    Om = out["Omega"].numpy()
    ref = np.cosh(Om[:, 0] + 1j * Om[:, 1])
    got = np.exp(out["logpsi"].numpy())
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.abs(out["logpsi"].imag.numpy()).max() > 1e-3  # a phase is there


def test_real_a_gives_the_real_network_and_sign_flip_conjugates():
    shape = di.ModelShape(11, 3, 3, 2, bc="periodic", act="tanh")
    th = torch.tensor(di.draw_params(shape, 5, "stress"))
    d = shape.d
    th_r = th.clone()
    th_r[-2 * d + 1::2] = 0.0                                  # Im A = 0 (and A[:, 1] = 0)
    sp = di.uniform_spins(5, 11, 6)
    real = forward(ModelDesc.of(shape), th_r, sp)["logpsi"]
    cplx = forward(ModelDesc.of(dataclass_replace(shape, complex_out=1)), th_r, sp)["logpsi"]
    assert torch.equal(cplx.imag, torch.zeros_like(real))
    assert torch.allclose(cplx.real, real, rtol=1e-14, atol=1e-15)
    th_c = th.clone()
    th_c[-2 * d + 1::2] *= -1.0
    desc = ModelDesc.of(dataclass_replace(shape, complex_out=1))
    a = forward(desc, th, sp)["logpsi"]
    b = forward(desc, th_c, sp)["logpsi"]
    assert torch.allclose(a.real, b.real, rtol=1e-14, atol=1e-15)
    assert max(abs(_wrap(x + y)) for x, y in zip(a.imag.tolist(), b.imag.tolist())) <= 1e-13


CASES = [
    (10, 1, 3, 2, "open", "tanh", "lrtfim"),
    (12, 2, 4, 3, "open", "silu", "j1j2"),
    (11, 3, 3, 2, "periodic", "silu", "j1j2"),
    (10, 4, 3, 2, "periodic", "identity", "lrtfim"),
]


@pytest.mark.parametrize("case", CASES)
def test_complex_abacus_equals_full_reevaluation(case):
    N, L, d, s, bc, act_name, kind = case
    shape, th = _cplx(di.ModelShape(N, L, d, s, bc=bc, act=act_name))
    desc = ModelDesc.of(shape)
    sp = di.uniform_spins(3, N, 17)
    sites, helem, n_conn, hdiag = O.connected(di.HamSpec(kind, bc), sp)
    lp, lr = O.plain_logratio(desc, th, sp, sites, n_conn)
    la = O.abacus_logratio(desc, th, sp, sites, n_conn)
    assert lr.dtype == torch.complex128 and la.dtype == torch.complex128
    scale = max(lr.abs().max().item(), lp.abs().max().item())
    assert (la.real - lr.real).abs().max().item() <= 1e-12 * scale
    dph = torch.remainder(la.imag - lr.imag + math.pi, 2 * math.pi) - math.pi
    assert dph.abs().max().item() <= 1e-12 * scale
    assert lr.imag.abs().max() > 1e-3


@pytest.mark.parametrize("ham", [di.HamSpec("j1j2", "periodic", J1=1.0, J2=0.5),
                                 di.HamSpec("lrtfim", "open", J=1.0, alpha=3.0, h=1.0)])
def test_complex_mean_local_energy_equals_rayleigh_quotient(ham):
    N = 8
    shape, th = _cplx(di.ModelShape(N, 2, 3, 2, bc=ham.bc, act="silu"), seed=12)
    th[-2 * shape.d:] *= 8.0  # phases of order one
    desc = ModelDesc.of(shape)
    confs = _all_confs(N)
    res = O.eloc_plain(desc, ham, th, confs)
    lp = res["logpsi"].numpy()
    psi = np.exp(lp - lp.real.max())
    H = dense_h(ham, N)
    rq = np.vdot(psi, H @ psi) / np.vdot(psi, psi)
    p = np.abs(psi) ** 2
    mean = np.sum(p * res["eloc"].numpy()) / np.sum(p)
    assert abs(rq.imag) <= 1e-13 * abs(rq)
    assert abs(mean - rq.real) <= 1e-12 * max(1.0, abs(rq))
    assert np.abs(res["eloc"].numpy().imag).max() > 1e-3  # E_loc itself is complex


def test_complex_screened_sampler_equals_exact_metropolis():
    shape = di.ModelShape(16, 2, 4, 3, act="silu", bc="open", complex_out=1)
    desc = ModelDesc.of(shape)
    th = torch.tensor(di.draw_params(shape, 17, "stress"))
    th[-2 * shape.d:] *= 10.0
    chains = [torch.tensor(x).long() for x in di.uniform_spins(2, 16, 4)]
    refreshes = 0
    for sweep in range(4):
        parity = sweep % 2
        K = len(range(parity, (16 + 1 - 1) // 1, 2))
        rng = np.random.Generator(np.random.PCG64(900 + sweep))
        r, u = rng.random((2, K)), rng.random((2, K))
        for b in range(2):
            sites = typewriter_sites(16, 1, parity, r[b])
            ref = exact_mh_sweep(desc, th, chains[b], sites, u[b])
            got = screened_sweep(desc, th, chains[b], sites, u[b], 0.1, track=True)
            assert got["unscreened_err"] <= 0.1
            assert got["accepted"] == ref["accepted"]
            assert torch.equal(got["spins"], ref["spins"])
            refreshes += got["refreshes"]
            chains[b] = ref["spins"]
    assert refreshes > 0


def test_complex_gradient_matches_central_differences():
    shape, th = _cplx(di.ModelShape(10, 2, 3, 2, bc="periodic", act="silu"), seed=6005)
    desc = ModelDesc.of(shape)
    sp = torch.tensor(di.uniform_spins(2, 10, 3))
    G = grad_logpsi_batched(desc, th, sp)
    assert G.dtype == torch.complex128
    rng = np.random.Generator(np.random.PCG64(6005))
    idx = rng.choice(th.numel(), size=16, replace=False)
    eps = 1e-6
    for k in idx:
        tp, tm = th.clone(), th.clone()
        tp[k] += eps
        tm[k] -= eps
        a, b = forward(desc, tp, sp)["logpsi"], forward(desc, tm, sp)["logpsi"]
        fd_re = (a.real - b.real) / (2 * eps)
        fd_im = torch.remainder(a.imag - b.imag + math.pi, 2 * math.pi) - math.pi
        fd_im = fd_im / (2 * eps)
        scale = max(G[:, k].abs().max().item(), 1e-8)
        assert (fd_re - G[:, k].real).abs().max().item() <= 1e-6 * scale + 1e-10
        assert (fd_im - G[:, k].imag).abs().max().item() <= 1e-6 * scale + 1e-10
