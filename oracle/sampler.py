"""Screened typewriter Metropolis sampler, FP64 on the CPU (test infrastructure only).

Follows Sec. IV ("Screened typewriter sampler", Algorithm 2), App. "Screened Metropolis
sampler is exact" and App. "Practical implementation of the screened typewriter sampler":

* typewriter schedule: the chain is cut into blocks of width `spacing`; one half-sweep visits
  every other block (parity 0: blocks 0, 2, 4, ...; parity 1: blocks 1, 3, ...) and proposes one
  single-site flip per visited block, at a site drawn uniformly inside the block (the uniform
  draws r_k in [0, 1) are inputs, so the choice is floor(r_k * width));
* the proposals' updates Delta-Omega_k are formed by ABACUS against one background (the
  configuration at the start of the half-sweep, or at the last refresh), and the acceptance
  ratio of proposal k treats the flips accepted so far as independent scatterers (independent
  scattering approximation): R~ = |f(Omega + dOmega_k) / f(Omega)|^2 with Omega the background
  output plus the dOmega of every flip accepted since;
* screened acceptance with tolerance eps: with P = min(1, R~), a draw u with |u - P| <= eps is
  ambiguous: the background is rebuilt at the current configuration, the remaining proposals'
  updates are recomputed (the first of them is then exact), and the test is repeated; otherwise
  accept iff u < P. When eps bounds |R~ - R| for the exact ratio R, every decision equals the
  exact Metropolis-Hastings decision for the same u.
The reference chain is plain Metropolis-Hastings: R = |psi(s')|^2 / |psi(s)|^2 from two full
evaluations, accept iff u < min(1, R). f = prod_k cosh (log psi = sum_k log cosh Omega_k), so
R~ = exp(2 sum_k lcd(Omega_k, dOmega_k)) (for a complex-output network the real part of the
complex log-ratio of its units: |psi|^2 decides).

The practical tolerance schedule of the same appendix: a buffer eps(n) indexed by the number n
of flips accepted since the current background (the last entry serves every larger n), read
when a proposal is screened. At each refresh the frozen proposal's approximate and exact
acceptance probabilities give the empirical error e~ = |min(1, R~) - min(1, R)|, recorded with
the n at which the chain froze. The buffer entries start at a conservative default; an entry
still at its default is overwritten with e~, any other becomes max(eps(n), gamma e~) with
gamma > 1. Here the buffer is one per sampler (shared by its chains) and held fixed during a
half-sweep; the half-sweep's events are applied afterwards, chain by chain in chain order and
in order of occurrence within a chain (``update_eps_buffer``).
"""
from __future__ import annotations

import math
from typing import Dict, List

import torch

from .abacus import abacus_logratio
from .model import DT, forward, ratio


def typewriter_sites(N: int, spacing: int, parity: int, r) -> List[int]:
    """One proposal per visited block b = parity, parity + 2, ...: site b*spacing +
    floor(r_k * width_b), width_b = min(spacing, N - b*spacing); r_k the k-th visited block's draw."""
    sites = []
    nblk = (N + spacing - 1) // spacing
    for k, b in enumerate(range(parity, nblk, 2)):
        lo = b * spacing
        width = min(spacing, N - lo)
        sites.append(lo + min(int(math.floor(float(r[k]) * width)), width - 1))
    return sites


def _logpsi(desc, theta, s) -> float:
    return forward(desc, theta, torch.as_tensor(s)[None])["logpsi"][0].real.item()


def exact_mh_sweep(desc, theta, spins, sites: List[int], u) -> Dict:
    """Plain Metropolis-Hastings over the listed single-site proposals."""
    theta = torch.as_tensor(theta, dtype=DT)
    s = torch.as_tensor(spins).to(torch.int64).clone()
    lp = _logpsi(desc, theta, s)
    acc = []
    for k, j in enumerate(sites):
        sp = s.clone()
        sp[j] = -sp[j]
        lp1 = _logpsi(desc, theta, sp)
        R = math.exp(2.0 * (lp1 - lp))
        a = float(u[k]) < min(1.0, R)
        acc.append(a)
        if a:
            s, lp = sp, lp1
    return {"spins": s, "accepted": acc}


def _updates(desc, theta, s, sites: List[int]):
    """(Omega of s, [dOmega of flipping each site against the background s]) by ABACUS."""
    B = torch.as_tensor(s)[None]
    M = len(sites)
    st = torch.full((1, M, 2), -1, dtype=torch.int64)
    for m, j in enumerate(sites):
        st[0, m, 0] = j
    _, parts = abacus_logratio(desc, theta, B, st, torch.tensor([M]), return_parts=True)
    Om = forward(desc, theta, B)["Omega"][0]
    return Om, [p["dOmega"] for p in parts]


def screened_sweep(desc, theta, spins, sites: List[int], u, eps: float, track: bool = False,
                   eps_buf=None) -> Dict:
    """Algorithm 2 on one chain: returns the final spins, the decisions, the number of refreshes,
    the largest |R~ - R| seen at a refresh (R exact at the refreshed background), the refresh
    events [(n, e~)] (n flips accepted since the background when the chain froze, e~ the
    empirical error of its acceptance probability) and, with track, the largest
    |min(1, R~) - min(1, R)| over the decisions taken without a refresh (R from two full
    evaluations) and the largest excess of that difference over the tolerance the decision used:
    a decision taken without a refresh has |u - min(1, R~)| > eps, so it is the exact one
    whenever the difference is <= eps. The tolerance is eps, or eps_buf[min(n, len - 1)] when a
    buffer is given."""
    theta = torch.as_tensor(theta, dtype=DT)
    s = torch.as_tensor(spins).to(torch.int64).clone()
    Om, dOm = _updates(desc, theta, s, sites)
    base = 0                      # index of the first proposal the current updates cover
    n = 0                         # flips accepted since the current background
    acc, refreshes, isa_err, unscreened, excess, events = [], 0, 0.0, 0.0, -math.inf, []
    for k, j in enumerate(sites):
        Rt = math.exp(2.0 * ratio(desc, Om, dOm[k - base]).real.item())
        P = min(1.0, Rt)
        tol = eps if eps_buf is None else float(eps_buf[min(n, len(eps_buf) - 1)])
        if abs(float(u[k]) - P) <= tol:
            # ambiguous: rebuild the background at the current configuration
            refreshes += 1
            Om, dOm = _updates(desc, theta, s, sites[k:])
            base = k
            R = math.exp(2.0 * ratio(desc, Om, dOm[0]).real.item())
            isa_err = max(isa_err, abs(Rt - R))
            events.append((n, abs(P - min(1.0, R))))
            P = min(1.0, R)
            n = 0
        elif track:
            sp = s.clone()
            sp[j] = -sp[j]
            R = math.exp(2.0 * (_logpsi(desc, theta, sp) - _logpsi(desc, theta, s)))
            unscreened = max(unscreened, abs(P - min(1.0, R)))
            excess = max(excess, abs(P - min(1.0, R)) - tol)
        a = float(u[k]) < P
        acc.append(a)
        if a:
            s[j] = -s[j]
            Om = Om + dOm[k - base]
            n += 1
    return {"spins": s, "accepted": acc, "refreshes": refreshes, "isa_err": isa_err,
            "unscreened_err": unscreened, "unscreened_excess": excess, "events": events}


def update_eps_buffer(buf: List[float], is_set: List[bool], events, gamma: float) -> None:
    """Apply refresh events [(n, e~)] in order: the entry min(n, len - 1) takes e~ if it still
    holds its default, else max(entry, gamma e~)."""
    for n, e in events:
        i = min(n, len(buf) - 1)
        if not is_set[i]:
            buf[i] = e
            is_set[i] = True
        else:
            buf[i] = max(buf[i], gamma * e)
