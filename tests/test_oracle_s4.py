"""Pins of the oracle's S4 Green's-function taps (kernel generation).

Each test checks the taps produced by matrix powers against an independent route the
paper gives: the resolvent at the N-th roots of unity (Sec. V, Eq. (resolvent)), the
Woodbury/Cauchy form of the DPLR resolvent (App. "Details on the implementation of the
DysonNet block", Eq. (greenWoodbury), with its low-rank term re-derived), the state
recurrence itself (Sec. V, Eq. (ssm_discretized) as the causal scan), an FFT
convolution, the s = 1 closed form, and the exact low-rank structure of SSM kernels
(App. "Exact algorithm ... arbitrary network depth", Proposition on HODLR kernels).
"""
import math

import numpy as np
import pytest
import torch

import dn_inputs as di
from oracle.model import ModelDesc, s4_discretize, s4_taps, toeplitz_matrices, unpack


def _setup(N, s, d=3, bc="open", seed=11, scale="stress"):
    shape = di.ModelShape(N, 1, d, s, bc=bc)
    desc = ModelDesc.of(shape)
    th = torch.tensor(di.draw_params(shape, seed, scale))
    prm = unpack(desc, th)
    return desc, prm


def _resolvent(Ad, Bd, C, z):
    s = Ad.shape[-1]
    x = np.linalg.solve(np.eye(s) - z * Ad, Bd)
    return C @ x


@pytest.mark.parametrize("N,s", [(8, 2), (12, 3), (16, 4)])
def test_periodic_taps_match_resolvent(N, s):
    # DFT_k of the aliased real kernel equals the resolvent combination at z_k = e^{2 pi i k/N}:
    # 1/2 [R+(z) + conj R+(zb) + R-(zb) + conj R-(z) - C-B - conj(C-B)], R(z) = C (I - z A_d)^-1 B_d.
    desc, prm = _setup(N, s, bc="periodic")
    for p4 in prm["s4"]:
        taps = s4_taps(desc, p4).numpy()
        circ = taps[:, N - 1:]                      # offsets 0..N-1 = g°_p
        Ad, Bd, Cp, Cm, *_ = [t.numpy() for t in s4_discretize(desc, p4)]
        for c in range(desc.d):
            for k in range(N):
                z = np.exp(2j * math.pi * k / N)
                zb = np.conj(z)
                dft = np.sum(circ[c] * z ** np.arange(N))
                Rp, Rpb = _resolvent(Ad[c], Bd[c], Cp[c], z), _resolvent(Ad[c], Bd[c], Cp[c], zb)
                Rm, Rmb = _resolvent(Ad[c], Bd[c], Cm[c], z), _resolvent(Ad[c], Bd[c], Cm[c], zb)
                cb = Cm[c] @ Bd[c]
                want = 0.5 * (Rp + np.conj(Rpb) + Rmb + np.conj(Rm) - cb - np.conj(cb))
                assert abs(dft - want) <= 1e-12 * max(1.0, abs(want))


@pytest.mark.parametrize("N,s", [(10, 2), (16, 3)])
def test_bilinear_resolvent_matches_cauchy_woodbury(N, s):
    # C (I - z A_d)^-1 B_d = c(z) C (g(z) I - Delta Abar)^-1 Bbar, c = 2 Delta/(1+z), g = 2(1-z)/(1+z),
    # and for Abar = Lambda + p q^T (Sherman-Morrison on the diagonal Cauchy sums):
    # C (gI - Delta Abar)^-1 Bbar = G0(Bbar,C) + Delta G0(p,C) G0(Bbar,q) / (1 - Delta G0(p,q)),
    # G0(u,v) = sum_i v_i u_i / (g - Delta Lambda_i).   (z = -1 excluded: c and g are singular there.)
    desc, prm = _setup(N, s)
    for p4 in prm["s4"]:
        Ad, Bd, Cp, Cm, delta, Abar, Bbar = [t.numpy() for t in s4_discretize(desc, p4)]
        lam = -np.exp(p4["lam_re"].numpy()) + 1j * p4["lam_im"].numpy()
        p = p4["p_re"].numpy() + 1j * p4["p_im"].numpy()
        q = p4["q_re"].numpy() + 1j * p4["q_im"].numpy()
        for c in range(desc.d):
            for k in range(N):
                z = np.exp(2j * math.pi * k / N)
                if abs(1 + z) < 1e-9:
                    continue
                cz, gz, D = 2 * delta[c] / (1 + z), 2 * (1 - z) / (1 + z), delta[c]
                G0 = lambda u, v: np.sum(v * u / (gz - D * lam[c]))  # noqa: E731
                for C in (Cp[c], Cm[c]):
                    wood = G0(Bbar[c], C) + D * G0(p[c], C) * G0(Bbar[c], q[c]) / (1 - D * G0(p[c], q[c]))
                    want = cz * wood
                    got = _resolvent(Ad[c], Bd[c], C, z)
                    assert abs(got - want) <= 1e-11 * max(1.0, abs(want))


def _scan_apply(Ad, Bd, Cp, Cm, u, periodic):
    """Bidirectional state recurrence x_i = A x_{i-1} + B u_i read out by C+ (r >= 0) and C- (r >= 1)."""
    N, s = len(u), Ad.shape[0]
    fwd = np.zeros((N, s), complex)
    bwd = np.zeros((N, s), complex)
    x = np.zeros(s, complex)
    if periodic:
        Q = np.linalg.inv(np.eye(s) - np.linalg.matrix_power(Ad, N))
        acc = sum(np.linalg.matrix_power(Ad, N - 1 - j) @ Bd * u[j] for j in range(N))
        x = Q @ acc                                   # steady state x_{N-1}
    for i in range(N):
        x = Ad @ x + Bd * u[i]
        fwd[i] = x
    zz = np.zeros(s, complex)
    if periodic:
        acc = sum(np.linalg.matrix_power(Ad, r) @ Bd * u[(r - 1) % N] for r in range(1, N + 1))
        zz = Q @ acc                                  # steady state z_{N-1}
        bwd[N - 1] = zz
        for i in range(N - 2, -1, -1):
            zz = Ad @ (zz + Bd * u[i + 1])
            bwd[i] = zz
    else:
        for i in range(N - 2, -1, -1):
            zz = Ad @ (zz + Bd * u[i + 1])
            bwd[i] = zz
    return (fwd @ Cp).real + (bwd @ Cm).real


@pytest.mark.parametrize("bc", ["open", "periodic"])
def test_toeplitz_equals_recurrence_scan_and_fft(bc):
    N, s = 14, 3
    desc, prm = _setup(N, s, bc=bc)
    rng = np.random.default_rng(5)
    for p4 in prm["s4"]:
        taps = s4_taps(desc, p4)
        T = toeplitz_matrices(desc, taps).numpy()
        Ad, Bd, Cp, Cm, *_ = [t.numpy() for t in s4_discretize(desc, p4)]
        for c in range(desc.d):
            u = rng.normal(size=N)
            direct = T[c] @ u
            scan = _scan_apply(Ad[c], Bd[c], Cp[c], Cm[c], u, bc == "periodic")
            assert np.max(np.abs(direct - scan)) <= 1e-12 * max(1.0, np.max(np.abs(direct)))
            tc = taps[c].numpy()
            if bc == "open":   # linear convolution with taps at offsets -(N-1)..N-1 via zero-padded FFT
                n = 4 * N
                full = np.fft.irfft(np.fft.rfft(tc, n) * np.fft.rfft(u, n), n)
                fft = full[N - 1:2 * N - 1]
            else:              # circular convolution with g°_p
                fft = np.fft.irfft(np.fft.rfft(tc[N - 1:]) * np.fft.rfft(u), N)
            assert np.max(np.abs(direct - fft)) <= 1e-12 * max(1.0, np.max(np.abs(direct)))


def test_single_state_closed_form():
    # s = 1: Abar = lambda + p q; A_d = (1 + D/2 Abar)/(1 - D/2 Abar); B_d = D Bbar/(1 - D/2 Abar);
    # g_r = Re(C+ B_d A_d^r), g_-r = Re(C- B_d A_d^r).
    N = 9
    desc, prm = _setup(N, 1, d=4)
    for p4 in prm["s4"]:
        taps = s4_taps(desc, p4).numpy()
        lam = -np.exp(p4["lam_re"].numpy()[:, 0]) + 1j * p4["lam_im"].numpy()[:, 0]
        pq = (p4["p_re"].numpy()[:, 0] + 1j * p4["p_im"].numpy()[:, 0]) * \
             (p4["q_re"].numpy()[:, 0] + 1j * p4["q_im"].numpy()[:, 0])
        Bb = p4["B_re"].numpy()[:, 0] + 1j * p4["B_im"].numpy()[:, 0]
        Cp = p4["Cp_re"].numpy()[:, 0] + 1j * p4["Cp_im"].numpy()[:, 0]
        Cm = p4["Cm_re"].numpy()[:, 0] + 1j * p4["Cm_im"].numpy()[:, 0]
        D = np.exp(np.log(1e-2) + np.log(10) * np.arange(4) / 3 + p4["dt"].numpy())
        ab = lam + pq
        ad = (1 + D / 2 * ab) / (1 - D / 2 * ab)
        bd = D * Bb / (1 - D / 2 * ab)
        for r in range(N):
            assert np.allclose(taps[:, N - 1 + r], (Cp * bd * ad ** r).real, rtol=0, atol=1e-14)
            if r:
                assert np.allclose(taps[:, N - 1 - r], (Cm * bd * ad ** r).real, rtol=0, atol=1e-14)


def test_offdiagonal_blocks_have_rank_at_most_2s():
    # Each direction of a real SSM kernel is Re(sum of s exponentials): the strictly
    # lower block of its Toeplitz matrix has rank <= 2s (s complex modes + conjugates).
    N, s = 32, 2
    desc, prm = _setup(N, s, d=2)
    for p4 in prm["s4"]:
        taps = s4_taps(desc, p4)
        T = toeplitz_matrices(desc, taps).numpy()
        for c in range(desc.d):
            blk = T[c][N // 2:, :N // 2]             # rows below, columns left: causal offsets only
            sv = np.linalg.svd(blk, compute_uv=False)
            assert np.sum(sv > 1e-10 * sv[0]) <= 2 * s
            blk2 = T[c][:N // 2, N // 2:]            # anti-causal offsets only
            sv2 = np.linalg.svd(blk2, compute_uv=False)
            assert np.sum(sv2 > 1e-10 * sv2[0]) <= 2 * s


def test_discretised_state_matrix_is_stable_at_both_draws():
    for scale in ("baseline", "stress"):
        shape = di.WORKLOADS["tfim_n256_l4_d64"].model
        desc = ModelDesc.of(shape)
        th = torch.tensor(di.draw_params(shape, 1005, scale))
        prm = unpack(desc, th)
        for p4 in prm["s4"]:
            Ad = s4_discretize(desc, p4)[0]
            assert torch.linalg.eigvals(Ad).abs().max().item() < 1.0
