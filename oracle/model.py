"""DysonNet forward pass and plain log-ratios, FP64 on the CPU (test infrastructure only).

Follows the paper's definition of the network (Sec. II, Definition of the block and
Eq. (wavefunc)), its S4 realisation of the Green's function (Sec. V, Eqs.
(ssm_discretized)-(resolvent); App. "Details on the implementation of the DysonNet
block", Eq. (discretization)) and its practical vertex (Eq. (Dpractical) and the
CNN phi-stream of the same appendix). The plain log-ratio is the definition of the
quantity ABACUS accelerates: log psi(s') - log psi(s) from two full evaluations
(Eq. (local-estimator)).

Layout: activations are [batch, site, channel]; matrices are [out, in].

Readings of the paper used here (where it is silent, ambiguous or garbled):
  * products of blocks apply block 1 first (Eq. (COBALT_recurrence));
  * the residual sum runs over h^(0) = E s and every block output (Eq. (wavefunc), M=0..L);
  * phi^(0) = E_phi s; block l computes phi^(l) and gates with chi^(l) = g(A_D phi^(l) + b),
    so block l's vertex sees spins within l*w_c;
  * the bidirectional SSM is the causal bilinear-discretised recurrence read out by C+
    for offsets r >= 0 and by C- for r >= 1 (the printed "lattice Laplace" form is
    not used); taps are Re(C^T A_d^r B_d) with no conjugation;
  * periodic networks use the aliased kernel (resolvent at the N-th roots of unity);
  * Lambda = -exp(raw) + i*raw', A-bar = diag(Lambda) + p q^T, step
    Delta_c = exp(ln 0.01 + ln 10 * c/(d-1) + raw);
  * f = log cosh on each of d_out read-out units, log psi = sum_k logcosh(Omega_k);
  * complex_out = 1 makes A complex (Sec. II, below Eq. (wavefunc): a complex A gives a
    complex wavefunction): the d_out real columns pair up as A[:, 2j] + i A[:, 2j+1], so
    there are d_out/2 complex units and log psi = sum_j logcosh(Omega_2j + i Omega_2j+1)
    is complex; its imaginary part (the phase) is reported in (-pi, pi];
  * inject_phi adds phi^(l) to the h stream before the mixer (Fig. 1c); the residual
    sum holds only the h stream;
  * token size t (patching, Sec. V on the efficiency trade-off): the network runs on N tokens,
    token tau holding the spins t tau .. t tau + t - 1, embedded as h^(0)_tau = sum_k E_k s_(t tau + k)
    and phi^(0)_tau = sum_k E_phi,k s_(t tau + k) (one embedding vector per position k inside a
    token; t = 1 is the per-site embedding);
  * block-diagonal vertex (Sec. V, the mixture-of-experts remark): with d_block = b > 0 the
    vertex D = U diag(chi) V acts within channel blocks of b: U and V are block-diagonal, their
    off-block entries of the parameter vector are not used (zero), chi and the phi stream are
    unchanged.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List

import torch

DT = torch.float64
CT = torch.complex128


@dataclass(frozen=True)
class ModelDesc:
    N: int
    L: int
    d: int
    s: int
    d_out: int = 2
    w_c: int = 1
    bc: str = "open"
    act: str = "silu"
    inject_phi: int = 0
    complex_out: int = 0
    token: int = 1
    d_block: int = 0

    @staticmethod
    def of(shape) -> "ModelDesc":
        return ModelDesc(shape.N, shape.L, shape.d, shape.s, shape.d_out, shape.w_c,
                         shape.bc, shape.act, shape.inject_phi, getattr(shape, "complex_out", 0),
                         getattr(shape, "token", 1), getattr(shape, "d_block", 0))


def act(name: str, x: torch.Tensor) -> torch.Tensor:
    """The local nonlinearity g (SiLU in the paper's block appendix; tanh/identity as options)."""
    if name == "silu":
        return x * torch.sigmoid(x)
    if name == "tanh":
        return torch.tanh(x)
    if name == "identity":
        return x
    raise ValueError(name)


def block_mask(desc: ModelDesc):
    """1 on the channel blocks of the vertex (d_block > 0), else None."""
    if not desc.d_block:
        return None
    c = torch.arange(desc.d) // desc.d_block
    return (c[:, None] == c[None, :]).to(DT)


def unpack(desc: ModelDesc, theta: torch.Tensor) -> Dict:
    """Split the flat FP64 parameter vector into named tensors (canonical order)."""
    d, s, Wc, L = desc.d, desc.s, 2 * desc.w_c + 1, desc.L
    pos = [0]

    def take(*shape):
        n = 1
        for x in shape:
            n *= x
        t = theta[pos[0]:pos[0] + n].reshape(*shape)
        pos[0] += n
        return t

    prm = {"E": take(desc.token, d), "E_phi": take(desc.token, d), "layers": [], "s4": []}
    blk = block_mask(desc)
    for _ in range(L):
        lay = {"W_D": take(d, d), "w": take(d), "K": take(Wc, d), "k": take(d),
               "A_D": take(d, d), "b": take(d), "U": take(d, d), "V": take(d, d)}
        if blk is not None:
            lay["U"] = lay["U"] * blk
            lay["V"] = lay["V"] * blk
        prm["layers"].append(lay)
    for _ in range(L + 1):
        rows = [take(12 * s + 1) for _ in range(d)]
        blk = torch.stack(rows)  # [d, 12s+1]
        names = ["lam_re", "lam_im", "p_re", "p_im", "q_re", "q_im", "B_re", "B_im",
                 "Cp_re", "Cp_im", "Cm_re", "Cm_im"]
        ent = {nm: blk[:, i * s:(i + 1) * s] for i, nm in enumerate(names)}
        ent["dt"] = blk[:, 12 * s]
        prm["s4"].append(ent)
    prm["A"] = take(d, desc.d_out)
    assert pos[0] == theta.numel(), (pos[0], theta.numel())
    return prm


def s4_discretize(desc: ModelDesc, p4: Dict):
    """Bilinear discretisation of the DPLR state matrix, per channel.

    App. "Details on the implementation of the DysonNet block", Eq. (discretization):
    A = (I - Delta/2 Abar)^-1 (I + Delta/2 Abar), B = (I - Delta/2 Abar)^-1 Delta Bbar,
    with Abar = Lambda + p q^T (Sec. V, S4 Ansatz). Returns (A_d [d,s,s], B_d [d,s],
    C+ [d,s], C- [d,s], Delta [d], Abar [d,s,s], Bbar [d,s]) in complex128.
    """
    d, s = desc.d, desc.s
    lam = torch.complex(-torch.exp(p4["lam_re"]), p4["lam_im"])
    p = torch.complex(p4["p_re"], p4["p_im"])
    q = torch.complex(p4["q_re"], p4["q_im"])
    Bbar = torch.complex(p4["B_re"], p4["B_im"])
    Cp = torch.complex(p4["Cp_re"], p4["Cp_im"])
    Cm = torch.complex(p4["Cm_re"], p4["Cm_im"])
    Abar = torch.diag_embed(lam) + p[:, :, None] * q[:, None, :]
    c = torch.arange(d, dtype=DT)
    delta = torch.exp(math.log(1e-2) + math.log(10.0) * c / max(d - 1, 1) + p4["dt"])
    eye = torch.eye(s, dtype=CT).expand(d, s, s)
    half = (delta / 2).to(CT)[:, None, None]
    Mm = eye - half * Abar
    Ad = torch.linalg.solve(Mm, eye + half * Abar)
    Bd = torch.linalg.solve(Mm, (delta.to(CT)[:, None] * Bbar)[..., None])[..., 0]
    return Ad, Bd, Cp, Cm, delta, Abar, Bbar


def _powers(Ad: torch.Tensor, x0: torch.Tensor, n: int) -> torch.Tensor:
    """[x0, A x0, A^2 x0, ..., A^(n-1) x0] along a new axis 1 (plain repeated products)."""
    out = [x0]
    x = x0
    for _ in range(n - 1):
        x = (Ad @ x[..., None])[..., 0]
        out.append(x)
    return torch.stack(out, dim=1)  # [d, n, s]


def s4_taps(desc: ModelDesc, p4: Dict, check_stable: bool = True) -> torch.Tensor:
    """Real Green's-function taps of one mixer, [d, 2N-1] indexed by offset r + N - 1.

    Open chain (zero padding): g_r = Re(C+^T A_d^r B_d) for r >= 0 and
    g_{-r} = Re(C-^T A_d^r B_d) for r >= 1 (Sec. V bidirectional SSM; Eq. (resolvent)
    is the transform of this impulse response). Periodic chain: the aliased kernel
    g°_p = Re(C+^T A_d^p Q B_d) + Re(C-^T A_d^(N-p) Q B_d), Q = (I - A_d^N)^-1, stored at
    offsets r in [-(N-1), N-1] as g°_{r mod N}.
    """
    N = desc.N
    Ad, Bd, Cp, Cm, *_ = s4_discretize(desc, p4)
    if check_stable:
        rho = torch.linalg.eigvals(Ad.detach()).abs().max().item()
        assert rho < 1.0, f"unstable discretised state matrix (spectral radius {rho})"
    if desc.bc == "open":
        X = _powers(Ad, Bd, N)                          # [d, N, s]
        kp = (X * Cp[:, None, :]).sum(-1).real          # [d, N]
        km = (X * Cm[:, None, :]).sum(-1).real
        neg = torch.flip(km[:, 1:], dims=[1])           # offsets -(N-1)..-1
        return torch.cat([neg, kp], dim=1)              # [d, 2N-1]
    s = desc.s
    AN = torch.linalg.matrix_power(Ad, N)
    eye = torch.eye(s, dtype=CT).expand_as(AN)
    y = torch.linalg.solve(eye - AN, Bd[..., None])[..., 0]
    Y = _powers(Ad, y, N + 1)                           # A^p Q B, p = 0..N
    cp = (Y[:, :N] * Cp[:, None, :]).sum(-1).real       # p = 0..N-1
    cm = (torch.flip(Y[:, 1:], dims=[1]) * Cm[:, None, :]).sum(-1).real  # A^(N-p), p=0..N-1
    circ = cp + cm                                      # [d, N], g°_p
    r = torch.arange(-(N - 1), N)
    return circ[:, r % N]


def toeplitz_matrices(desc: ModelDesc, taps: torch.Tensor) -> torch.Tensor:
    """Dense per-channel mixer matrices T[c, i, i'] = g_c(i - i') (definition of G, Sec. II)."""
    N = desc.N
    i = torch.arange(N)
    idx = (i[:, None] - i[None, :]) + N - 1
    return taps[:, idx]                                 # [d, N, N]


def logcosh(x: torch.Tensor) -> torch.Tensor:
    """log cosh x, accurate in relative terms everywhere.

    |x| <= 1: log1p(2 sinh^2(x/2)) (cosh x = 1 + 2 sinh^2(x/2), no cancellation near 0);
    |x| > 1:  |x| + log1p(exp(-2|x|)) - ln 2 (no overflow).
    """
    ax = x.abs()
    small = ax <= 1.0
    xs = torch.where(small, x, torch.zeros_like(x))
    near = torch.log1p(2 * torch.sinh(xs / 2) ** 2)
    far = ax + torch.log1p(torch.exp(-2 * ax)) - math.log(2.0)
    return torch.where(small, near, far)


def lcd(a: torch.Tensor, delta: torch.Tensor) -> torch.Tensor:
    """log cosh(a + delta) - log cosh(a) without cancellation.

    Uses cosh(a+delta)/cosh(a) = 1 + 2 sinh^2(delta/2) + tanh(a) sinh(delta) for
    |delta| <= 1 and the plain difference otherwise.
    """
    small = delta.abs() <= 1.0
    ds = torch.where(small, delta, torch.zeros_like(delta))
    inner = 2 * torch.sinh(ds / 2) ** 2 + torch.tanh(a) * torch.sinh(ds)
    return torch.where(small, torch.log1p(inner), logcosh(a + delta) - logcosh(a))


def wrap_phase(y: torch.Tensor) -> torch.Tensor:
    """The representative of y modulo 2 pi in [-pi, pi]."""
    return y - (2 * math.pi) * torch.round(y / (2 * math.pi))


def _ctanh(z: torch.Tensor) -> torch.Tensor:
    """tanh(x + iy) = (sinh 2x + i sin 2y) / (cosh 2x + cos 2y); +-1 once |x| > 20."""
    x, y = z.real, z.imag
    big = x.abs() > 20.0
    xs = torch.where(big, torch.zeros_like(x), x)
    den = torch.cosh(2 * xs) + torch.cos(2 * y)
    re = torch.where(big, torch.sign(x), torch.sinh(2 * xs) / den)
    im = torch.where(big, torch.zeros_like(y), torch.sin(2 * y) / den)
    return torch.complex(re, im)


def logcosh_c(z: torch.Tensor) -> torch.Tensor:
    """log cosh(x + iy) for complex z, phase in (-pi, pi].

    cosh(x + iy) = cosh x cos y + i sinh x sin y, so |cosh z|^2 / cosh^2 x equals both
    1 - (sin y / cosh x)^2 and tanh^2 x + (cos y / cosh x)^2. log|cosh z| = logcosh(x) + 1/2 log
    of that ratio, taken as log1p of the first form while (sin y / cosh x)^2 <= 1/2 and as the
    log of the second (a sum of squares, no cancellation near the zeros of cosh) beyond;
    arg cosh z = atan2(tanh x sin y, cos y).
    """
    x, y = z.real, z.imag
    ch = torch.cosh(x)
    q = torch.sin(y) / ch
    c = torch.cos(y) / ch
    th = torch.tanh(x)
    near_zero = q * q > 0.5
    ratio = torch.where(near_zero, torch.log(th * th + c * c), torch.log1p(-q * q))
    re = logcosh(x) + 0.5 * ratio
    im = torch.atan2(th * torch.sin(y), torch.cos(y))
    return torch.complex(re, im)


def lcd_c(a: torch.Tensor, delta: torch.Tensor) -> torch.Tensor:
    """log cosh(a + delta) - log cosh(a) for complex a, delta, phase in [-pi, pi].

    For |delta| <= 1: cosh(a + delta)/cosh(a) = 1 + w, w = 2 sinh^2(delta/2) + tanh(a) sinh(delta),
    and log(1 + w) = 1/2 log|1 + w|^2 + i atan2(Im w, 1 + Re w); otherwise the difference of
    logcosh_c with the phase wrapped.
    """
    small = delta.abs() <= 1.0
    ds = torch.where(small, delta, torch.zeros_like(delta))
    w = 2 * torch.sinh(ds / 2) ** 2 + _ctanh(a) * torch.sinh(ds)
    # |1 + w|^2 = 1 + u, u = 2 Re w + |w|^2: log1p(u) while |u| <= 1/2, else the log of the sum
    # of squares (1 + Re w)^2 + (Im w)^2 (no cancellation when 1 + w is near zero)
    u = 2 * w.real + w.real ** 2 + w.imag ** 2
    mod = torch.where(u.abs() <= 0.5, torch.log1p(u), torch.log((1 + w.real) ** 2 + w.imag ** 2))
    near = torch.complex(0.5 * mod, torch.atan2(w.imag, 1 + w.real))
    far = logcosh_c(a + delta) - logcosh_c(a)
    far = torch.complex(far.real, wrap_phase(far.imag))
    return torch.where(small, near, far)


def _units(desc: ModelDesc, Om: torch.Tensor) -> torch.Tensor:
    """The complex read-out units Omega_2j + i Omega_2j+1 of a complex-output network."""
    return torch.complex(Om[..., 0::2], Om[..., 1::2])


def readout(desc: ModelDesc, Omega: torch.Tensor) -> torch.Tensor:
    """log psi from the read-out pre-activations Omega [..., d_out]."""
    if desc.complex_out:
        lp = logcosh_c(_units(desc, Omega)).sum(-1)
        return torch.complex(lp.real, wrap_phase(lp.imag))
    return logcosh(Omega).sum(-1)


def ratio(desc: ModelDesc, Om0: torch.Tensor, dOm: torch.Tensor) -> torch.Tensor:
    """log psi(s')/psi(s) from Omega(s) and dOmega = Omega(s') - Omega(s)."""
    if desc.complex_out:
        lr = lcd_c(_units(desc, Om0), _units(desc, dOm)).sum(-1)
        return torch.complex(lr.real, wrap_phase(lr.imag))
    return lcd(Om0, dOm).sum(-1)


def _shift(desc: ModelDesc, a: torch.Tensor, r: int) -> torch.Tensor:
    """out[:, i] = a[:, i + r] with zero padding (open) or wrap-around (periodic)."""
    if r == 0:
        return a
    if desc.bc == "periodic":
        return torch.roll(a, shifts=-r, dims=1)
    out = torch.zeros_like(a)
    N = a.shape[1]
    if r > 0:
        out[:, :N - r] = a[:, r:]
    else:
        out[:, -r:] = a[:, :N + r]
    return out


def mixers(desc: ModelDesc, prm: Dict, check_stable: bool = True) -> List[torch.Tensor]:
    """Dense Toeplitz/circulant matrices of the L block mixers and the final mixer G^f."""
    return [toeplitz_matrices(desc, s4_taps(desc, p4, check_stable)) for p4 in prm["s4"]]


def forward(desc: ModelDesc, theta: torch.Tensor, spins, cache: bool = False, T=None):
    """Evaluate the network on a batch of configurations (Sec. II, Eq. (wavefunc)).

    phi^(0) = E_phi s, h^(0) = E s (per token: sum_k E_k s_(t tau + k)); for each block l:
      a = W_D phi + w,  phi <- g(sum_r K_r * a_{i+r} + k)          (phi-stream CNN)
      chi = g(A_D phi + b)                                          (Eq. (Dpractical))
      v = G^(l) u with u = h (+ phi if inject_phi)                   (Green's-function mixer)
      h <- U (chi * (V v))                                          (vertex D = U diag(chi) V)
    R = sum_{l=0..L} h^(l);  Omega = A^T (1/N) sum_i omega_i * R_i with omega the column
    sums of the final mixer (mean pooling after G^f);  log psi = sum_k logcosh(Omega_k).
    Returns a dict with "logpsi" [B], "Omega" [B, d_out] and, if cache, the per-block
    intermediates.
    """
    prm = unpack(desc, theta)
    if T is None:
        T = mixers(desc, prm)
    s = torch.as_tensor(spins).to(DT)
    if s.dim() == 1:
        s = s[None]
    N = desc.N
    g = lambda x: act(desc.act, x)  # noqa: E731
    st = s.reshape(s.shape[0], N, desc.token)         # [B, token index, position in the token]
    phi = st @ prm["E_phi"]
    h = st @ prm["E"]
    R = h
    out = {"h": [h], "phi": [phi], "a": [], "chi": [], "v": [], "u": []}
    for l, lay in enumerate(prm["layers"]):
        a = phi @ lay["W_D"].T + lay["w"]
        conv = sum(lay["K"][r + desc.w_c] * _shift(desc, a, r)
                   for r in range(-desc.w_c, desc.w_c + 1))
        phi = g(conv + lay["k"])
        chi = g(phi @ lay["A_D"].T + lay["b"])
        u = h + phi if desc.inject_phi else h
        v = torch.einsum("cij,bjc->bic", T[l], u)
        h = (chi * (v @ lay["V"].T)) @ lay["U"].T
        R = R + h
        if cache:
            out["a"].append(a)
            out["phi"].append(phi)
            out["chi"].append(chi)
            out["v"].append(v)
            out["u"].append(u)
            out["h"].append(h)
    omega = T[desc.L].sum(dim=1)                          # [d, N]: sum_j g^f_c(j - i)
    Omega = torch.einsum("bic,ci,ck->bk", R, omega, prm["A"]) / N
    out["Omega"] = Omega
    out["logpsi"] = readout(desc, Omega)
    out["omega"] = omega
    out["T"] = T
    out["prm"] = prm
    return out


def logpsi(desc: ModelDesc, theta, spins) -> torch.Tensor:
    return forward(desc, torch.as_tensor(theta, dtype=DT), spins)["logpsi"]


def flip_configs(spins: torch.Tensor, sites: torch.Tensor, n_conn: torch.Tensor):
    """Connected configurations s'_m of each sample: s with the listed site(s) flipped.

    sites [B, M, 2] holds one or two site indices per element (second = -1 for a
    single flip). Returns s' [B, M, N] (entries m >= n_conn[b] are copies of s).
    """
    s = torch.as_tensor(spins).to(torch.int64)
    B, N = s.shape
    M = sites.shape[1]
    sp = s[:, None, :].repeat(1, M, 1)
    for b in range(B):
        for m in range(int(n_conn[b])):
            for t in range(2):
                j = int(sites[b, m, t])
                if j >= 0:
                    sp[b, m, j] = -sp[b, m, j]
    return sp


def plain_logratio(desc: ModelDesc, theta, spins, sites, n_conn, chunk: int = 512):
    """log psi(s'_m) - log psi(s) for every connected configuration, by full re-evaluation.

    This is the definition used in Eq. (local-estimator): each ratio comes from two
    complete forward passes. Returns (logpsi [B], logratio [B, M]) with zeros for
    m >= n_conn[b].
    """
    theta = torch.as_tensor(theta, dtype=DT)
    s = torch.as_tensor(spins).to(torch.int64)
    B, N = s.shape
    M = sites.shape[1]
    prm = unpack(desc, theta)
    T = mixers(desc, prm)
    base = forward(desc, theta, s, T=T)["logpsi"]
    sp = flip_configs(s, sites, n_conn).reshape(B * M, N)
    vals = []
    for c0 in range(0, B * M, chunk):
        vals.append(forward(desc, theta, sp[c0:c0 + chunk], T=T)["logpsi"])
    lp = torch.cat(vals).reshape(B, M)
    lr = lp - base[:, None]
    if desc.complex_out:
        lr = torch.complex(lr.real, wrap_phase(lr.imag))
    mask = torch.arange(M)[None, :] < torch.as_tensor(n_conn)[:, None]
    return base, torch.where(mask, lr, torch.zeros_like(lr))
