"""ABACUS local update with link tensors built from their definitions (test infrastructure only).

Follows Sec. III (Eqs. (fullprod), (Tl), (Lmn), (recur_step), (recur_out), Theorem 1)
and the pivot-class induction of App. "Induction Proof of ABACUS". Background operators
are materialised as dense (N*d) x (N*d) matrices, so this is for small N*d only; it is
the brute-force check of the method, not a fast path.

Readings of the paper:
  * the printed recurrence and read-out omit the words whose only scattering is the
    input change E*Delta-sigma itself ("pivot 0"); the induction's base case contains
    it. Here it is included: e^(0) = E (s' - s) on the cluster, with links from it to
    every later layer and to the output;
  * the printed read-out adds P_M h~^(L) on top of T^(L); T^(L) already is the
    read-out of the last layer, so it is counted once;
  * the quantity returned is Delta-Omega (the change of the pre-nonlinearity output),
    turned into log psi(s')/psi(s) = sum_k [logcosh(Omega_k + dOmega_k) - logcosh(Omega_k)];
  * h~0^(l) is the unscattered field entering the layer-l vertex, i.e. the slice of
    v0^(l) = G^(l) u0^(l);
  * slices are exact supports S_l = {i : dist(i, C) <= l*w_c} of the vertex change
    (ring distance for periodic chains, clipped for open ones), which covers clusters
    of more than one site.
With the phi stream injected into the h stream, the perturbation entering layer l+1
is z^(l) = e^(l) + Delta-phi^(l+1) (support S_{l+1}).
"""
from __future__ import annotations

from typing import List

import torch

from .model import CT, DT, forward, ratio, unpack, mixers


def _slice(desc, cluster: List[int], radius: int) -> List[int]:
    N = desc.N
    out = []
    for i in range(N):
        best = N
        for j in cluster:
            r = abs(i - j)
            if desc.bc == "periodic":
                r = min(r, N - r)
            best = min(best, r)
        if best <= radius:
            out.append(i)
    return out


def _idx(sites: List[int], d: int) -> torch.Tensor:
    return torch.tensor([i * d + c for i in sites for c in range(d)], dtype=torch.int64)


def background_operators(desc, theta, s0):
    """Dense background operators of one sample s0 (frozen vertices D0 = D(s0))."""
    theta = torch.as_tensor(theta, dtype=DT)
    prm = unpack(desc, theta)
    T = mixers(desc, prm)
    fw = forward(desc, theta, torch.as_tensor(s0)[None], cache=True, T=T)
    N, d, L = desc.N, desc.d, desc.L
    n = N * d
    G, Bm = [], []
    for l in range(L):
        Gl = torch.zeros(n, n, dtype=DT)
        for c in range(d):
            Gl[c::d, c::d] = T[l][c]
        lay = prm["layers"][l]
        D0 = torch.zeros(n, n, dtype=DT)
        chi = fw["chi"][l][0]
        for i in range(N):
            D0[i * d:(i + 1) * d, i * d:(i + 1) * d] = lay["U"] @ torch.diag(chi[i]) @ lay["V"]
        G.append(Gl)
        Bm.append(D0 @ Gl)
    Pw = torch.zeros(desc.d_out, n, dtype=DT)
    for k in range(desc.d_out):
        Pw[k] = (fw["omega"].T * prm["A"][:, k]).reshape(-1) / N
    return {"fw": fw, "prm": prm, "T": T, "G": G, "B": Bm, "Pw": Pw}


def chain(ops, a: int, b: int) -> torch.Tensor:
    """X_{a..b} = B^(b) ... B^(a) with 1-based block indices (identity if a > b)."""
    n = ops["Pw"].shape[1]
    X = torch.eye(n, dtype=DT)
    for l in range(a, b + 1):
        X = ops["B"][l - 1] @ X
    return X


def output_links(desc, ops) -> List[torch.Tensor]:
    """T~^(m) = A^T P_omega sum_{l=m+1..L} X_{m+1..l}: read-out of a perturbation entering u^(m+1).

    Without injection the paper's T^(m) (Eq. (Tl)) is A^T P_omega + T~^(m) for m < L and
    A^T P_omega for m = L.
    """
    L = desc.L
    out = []
    for m in range(L):
        acc = torch.zeros_like(ops["Pw"])
        for l in range(m + 1, L + 1):
            acc = acc + ops["Pw"] @ chain(ops, m + 1, l)
        out.append(acc)
    return out


def abacus_logratio(desc, theta, spins, sites, n_conn, return_parts: bool = False):
    """log psi(s')/psi(s) for every listed cluster update by the ABACUS recurrence.

    For each sample: materialise background operators; for each cluster C (the tokens of the
    flipped spins):
      e^(0) = E (s' - s) on C (each flipped spin through the embedding of its token position);
      for l = 1..L:  x^(l) = P_S v0^(l) + sum_{m<l} P_{S_l} G^(l) X_{m+1..l-1} z^(m)
                     e^(l) = Delta-D^(l) x^(l) on S_l,  Delta-D_i = U diag(chi'_i - chi0_i) V
      dOmega = A^T P_omega sum_l e^(l) + sum_m T~^(m) z^(m)
    where z^(m) = e^(m) (+ Delta-phi^(m+1) when phi is injected). The updated vertices
    chi' and phi' are taken from the phi stream of s', and their changes are asserted
    to vanish outside the slices.
    """
    theta = torch.as_tensor(theta, dtype=DT)
    s = torch.as_tensor(spins).to(torch.int64)
    B, N = s.shape[0], desc.N   # N tokens (N * token spins)
    M = sites.shape[1]
    d, L, wc = desc.d, desc.L, desc.w_c
    out = torch.zeros(B, M, dtype=CT if desc.complex_out else DT)
    parts = []
    for b in range(B):
        ops = background_operators(desc, theta, s[b])
        fw0, prm = ops["fw"], ops["prm"]
        Ttil = output_links(desc, ops)
        Om0 = fw0["Omega"][0]
        Y = {}
        for l in range(1, L + 1):
            for m in range(0, l):
                Y[(l, m)] = ops["G"][l - 1] @ chain(ops, m + 1, l - 1)
        for mi in range(int(n_conn[b])):
            flips = [int(x) for x in sites[b, mi] if int(x) >= 0]   # spin indices
            C = sorted({j // desc.token for j in flips})            # the cluster, in tokens
            sp = s[b].clone()
            for j in flips:
                sp[j] = -sp[j]
            fw1 = forward(desc, theta, sp[None], cache=True, T=ops["T"])
            S = [_slice(desc, C, l * wc) for l in range(L + 1)]
            dchi = [fw1["chi"][l][0] - fw0["chi"][l][0] for l in range(L)]
            dphi = [fw1["phi"][l][0] - fw0["phi"][l][0] for l in range(L + 1)]
            for l in range(1, L + 1):
                outside = [i for i in range(N) if i not in S[l]]
                if outside:
                    assert dchi[l - 1][outside].abs().max() <= 1e-13, "vertex change leaks"
                    assert dphi[l][outside].abs().max() <= 1e-13, "phi change leaks"
            e = [torch.zeros(N, d, dtype=DT) for _ in range(L + 1)]
            for j in flips:
                e[0][j // desc.token] += prm["E"][j % desc.token] * float(sp[j] - s[b, j])
            z, zs = [], []
            for l in range(1, L + 1):
                z.append(e[l - 1] + (dphi[l] if desc.inject_phi else 0.0))
                zs.append(S[l] if desc.inject_phi else S[l - 1])
                rows = _idx(S[l], d)
                x = fw0["v"][l - 1][0].reshape(-1)[rows]
                for m in range(l):
                    cols = _idx(zs[m], d)
                    x = x + Y[(l, m)][rows][:, cols] @ z[m].reshape(-1)[cols]
                x = x.reshape(len(S[l]), d)
                lay = prm["layers"][l - 1]
                for t, i in enumerate(S[l]):
                    e[l][i] = lay["U"] @ (dchi[l - 1][i] * (lay["V"] @ x[t]))
            dOm = sum(ops["Pw"] @ e[l].reshape(-1) for l in range(L + 1))
            for m in range(L):
                dOm = dOm + Ttil[m] @ z[m].reshape(-1)
            out[b, mi] = ratio(desc, Om0, dOm)
            if return_parts:
                parts.append({"b": b, "m": mi, "dOmega": dOm, "slices": S})
    if return_parts:
        return out, parts
    return out
