"""Connected elements, diagonal energies and the local energy, FP64 (test infrastructure only).

Hamiltonians of the paper's benchmarks:
  * long-range transverse-field Ising chain (Sec. VI, benchmarking Hamiltonian), in the
    paper's Kac-normalised form, -(J/N_alpha) sum_{i != j} sz sz / r^alpha - h sum sx, with
    N_alpha = 2 sum_{r=1}^{floor(N/2)} r^-alpha, or in the plain form
    sum_{i<j} J sz sz / dist^alpha + h sum sx (paper_form = 0);
  * J1-J2 Heisenberg chain (App. "Small system validation J1-J2",
    Eq. (j1j2_hamiltonian)) with S = sigma/2, so each bond contributes (J/4) s_i s_j on
    the diagonal and J/2 between configurations that differ by exchanging an
    antiparallel pair.
Local energy: Eq. (local-estimator), E_loc(s) = sum_s' <s|H|s'> psi(s')/psi(s).

Connected-element order (it fixes the layout of logratio[B, M]): Ising, element m flips
site m; J1-J2, for i = 0..N-1 and then delta = 1, 2, the bond (i, i+delta) is emitted when
its spins are antiparallel (bonds that leave an open chain are skipped).
"""
from __future__ import annotations

import math

import torch

from .model import DT, plain_logratio


def _dist(ham, N: int, i: int, j: int) -> int:
    r = abs(i - j)
    if ham.bc == "periodic":
        r = min(r, N - r)
    return r


def kac(N: int, alpha: float) -> float:
    """Kac factor N_alpha(N) = 2 sum_{r=1}^{floor(N/2)} r^-alpha (Sec. VI)."""
    return 2.0 * sum(r ** (-alpha) for r in range(1, N // 2 + 1))


def ising_couplings(ham, N: int):
    """(c_zz per unordered pair, c_x): the diagonal pair weight and the sx matrix element."""
    if ham.paper_form:
        return -2.0 * ham.J / kac(N, ham.alpha), -ham.h
    return ham.J, ham.h


def connected(ham, spins, M_max: int | None = None):
    """Generator of the connected configurations of each sample.

    Returns sites [B, M_max, 2] (second entry -1 for a single flip; unused rows -1),
    helem [B, M_max] (0 beyond n_conn), n_conn [B], hdiag [B]. Pure Python loops:
    this is the readable definition, used at small B.
    """
    s = torch.as_tensor(spins).to(torch.int64)
    B, N = s.shape
    if M_max is None:
        M_max = N if ham.kind == "lrtfim" else 2 * N
    sites = torch.full((B, M_max, 2), -1, dtype=torch.int64)
    helem = torch.zeros((B, M_max), dtype=DT)
    n_conn = torch.zeros(B, dtype=torch.int64)
    hdiag = torch.zeros(B, dtype=DT)
    if ham.kind == "lrtfim":
        czz, cx = ising_couplings(ham, N)
        for b in range(B):
            e = 0.0
            for i in range(N):
                for j in range(i + 1, N):
                    e += czz * float(s[b, i] * s[b, j]) / _dist(ham, N, i, j) ** ham.alpha
            hdiag[b] = e
            assert M_max >= N
            for m in range(N):
                sites[b, m, 0] = m
                helem[b, m] = cx
            n_conn[b] = N
    elif ham.kind == "j1j2":
        assert N >= 5, "J1-J2 needs N >= 5 so that no bond repeats"
        Jd = {1: ham.J1, 2: ham.J2}
        for b in range(B):
            e, m = 0.0, 0
            for i in range(N):
                for dl in (1, 2):
                    j = i + dl
                    if j >= N:
                        if ham.bc != "periodic":
                            continue
                        j -= N
                    e += Jd[dl] / 4.0 * float(s[b, i] * s[b, j])
                    if s[b, i] != s[b, j]:
                        assert m < M_max, "M_max too small"
                        sites[b, m, 0], sites[b, m, 1] = i, j
                        helem[b, m] = Jd[dl] / 2.0
                        m += 1
            hdiag[b] = e
            n_conn[b] = m
    else:
        raise ValueError(ham.kind)
    return sites, helem, n_conn, hdiag


def local_energy(hdiag, helem, n_conn, logratio):
    """E_loc = hdiag + sum_{m < n_conn} helem_m exp(logratio_m) (Eq. (local-estimator))."""
    M = helem.shape[1]
    mask = torch.arange(M)[None, :] < torch.as_tensor(n_conn)[:, None]
    t = helem * torch.exp(logratio)
    terms = torch.where(mask, t, torch.zeros_like(t))
    return hdiag + terms.sum(-1)


def eloc_plain(desc, ham, theta, spins, M_max: int | None = None):
    """Local energy with log-ratios from full re-evaluation. Returns a dict of all parts."""
    sites, helem, n_conn, hdiag = connected(ham, spins, M_max)
    lp, lr = plain_logratio(desc, theta, spins, sites, n_conn)
    return {"logpsi": lp, "logratio": lr, "eloc": local_energy(hdiag, helem, n_conn, lr),
            "sites": sites, "helem": helem, "n_conn": n_conn, "hdiag": hdiag}
