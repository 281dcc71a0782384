"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random numbers and names workloads. It holds none of the
method's arithmetic: parameters are returned as one flat float64 vector in the
canonical order (documented in ``param_blocks``), spins as int8 arrays of +-1.
Both the oracle and the HIP library unpack the flat vector with their own code.

Random source: NumPy ``Generator(PCG64(seed))``; every draw is in the order listed.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Tuple

import numpy as np

ACTS = ("silu", "tanh", "identity")
BCS = ("open", "periodic")


@dataclasses.dataclass(frozen=True)
class ModelShape:
    """Hyper-parameters of one DysonNet (names follow the paper's notation)."""

    N: int            # chain length in tokens (network sites); the chain holds N * token spins
    L: int            # number of DysonNet blocks
    d: int            # embedding (channel) dimension
    s: int            # S4 state size per channel
    d_out: int = 2    # log-cosh read-out units
    w_c: int = 1      # half-width of the phi-stream CNN (kernel 2*w_c+1)
    bc: str = "open"  # network boundary condition: "open" (zero padding) or "periodic"
    act: str = "silu"  # local nonlinearity g: "silu" | "tanh" | "identity"
    inject_phi: int = 0  # 1: add phi^(l) to the h stream before the mixer (Fig. 1c form)
    complex_out: int = 0  # 1: complex read-out matrix A (column pairs as real and imaginary parts)
    token: int = 1    # spins per token (patching): token tau embeds spins token*tau .. token*tau + token - 1
    d_block: int = 0  # > 0: the vertex acts within channel blocks of this size (U, V block-diagonal)

    def __post_init__(self):
        assert self.act in ACTS and self.bc in BCS
        assert self.N >= 1 and self.L >= 1 and self.d >= 1 and self.s >= 1 and self.token >= 1

    @property
    def n_spins(self) -> int:
        return self.N * self.token


@dataclasses.dataclass(frozen=True)
class HamSpec:
    """Hamiltonian of the local estimator.

    kind "lrtfim": long-range transverse-field Ising chain. paper_form=0 is
        H = sum_{i<j} J/dist^alpha sz_i sz_j + h sum_i sx_i, paper_form=1 is
        H = -(J/N_alpha) sum_{i!=j} sz sz/dist^alpha - h sum sx with the Kac factor.
        dist is |i-j| for bc "open", min(|i-j|, N-|i-j|) for "periodic".
    kind "j1j2": J1 sum S_i.S_{i+1} + J2 sum S_i.S_{i+2} with S = sigma/2.
    """

    kind: str = "lrtfim"
    bc: str = "open"
    J: float = 1.0
    alpha: float = 3.0
    h: float = 1.0
    paper_form: int = 0
    J1: float = 1.0
    J2: float = 0.5


def param_blocks(m: ModelShape) -> List[Tuple[str, int, float]]:
    """(name, length, stress-draw std) for every block of the flat parameter vector.

    Order: E[token, d], E_phi[token, d] (one embedding vector per position inside a token);
      per block l=1..L: W_D[d,d], w[d], K[2w_c+1,d], k[d], A_D[d,d], b[d], U[d,d], V[d,d];
      per mixer (blocks 1..L, then the final mixer f), per channel c:
        Lambda_re-raw[s], Lambda_im[s], p_re[s], p_im[s], q_re[s], q_im[s],
        B_re[s], B_im[s], C+_re[s], C+_im[s], C-_re[s], C-_im[s], log-step offset[1];
      A[d, d_out].
    Matrices are row-major with the output index first.
    """
    d, s, Wc = m.d, m.s, 2 * m.w_c + 1
    rd = 1.0 / math.sqrt(d)
    te = 1.0 / math.sqrt(m.token)  # a token sums `token` embedded spins
    out = [("E", m.token * d, te), ("E_phi", m.token * d, te)]
    for l in range(m.L):
        out += [
            (f"W_D{l}", d * d, rd), (f"w{l}", d, 0.5), (f"K{l}", Wc * d, 1.0 / math.sqrt(Wc)),
            (f"k{l}", d, 0.5), (f"A_D{l}", d * d, rd), (f"b{l}", d, 0.5),
            (f"U{l}", d * d, rd), (f"V{l}", d * d, rd),
        ]
    for mix in range(m.L + 1):
        for c in range(d):
            for nm, std in (("lam_re", 0.1), ("lam_im", 0.1), ("p_re", 0.1), ("p_im", 0.1),
                            ("q_re", 0.1), ("q_im", 0.1), ("B_re", 1.0), ("B_im", 1.0),
                            ("Cp_re", 1 / math.sqrt(s)), ("Cp_im", 1 / math.sqrt(s)),
                            ("Cm_re", 1 / math.sqrt(s)), ("Cm_im", 1 / math.sqrt(s))):
                out.append((f"s4_{mix}_{c}_{nm}", s, std))
            out.append((f"s4_{mix}_{c}_dt", 1, 0.1))
    out.append(("A", d * m.d_out, rd))
    return out


def param_count(m: ModelShape) -> int:
    return sum(n for _, n, _ in param_blocks(m))


def draw_params(m: ModelShape, seed: int, scale: str = "baseline") -> np.ndarray:
    """Flat float64 parameter vector.

    scale "baseline": every raw entry ~ N(0, 0.1^2).
    scale "stress": per-block std from ``param_blocks`` (order-one signal in every layer).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if scale == "baseline":
        return rng.normal(0.0, 0.1, size=param_count(m)).astype(np.float64)
    if scale != "stress":
        raise ValueError(scale)
    parts = [rng.normal(0.0, std, size=n) for _, n, std in param_blocks(m)]
    return np.concatenate(parts).astype(np.float64)


def uniform_spins(B: int, N: int, seed: int) -> np.ndarray:
    """B x N iid uniform +-1 spins (int8)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (2 * rng.integers(0, 2, size=(B, N)) - 1).astype(np.int8)


def balanced_spins(B: int, N: int, seed: int) -> np.ndarray:
    """B rows, each a uniform random permutation of N/2 (+1) and N/2 (-1) (zero magnetisation)."""
    assert N % 2 == 0
    rng = np.random.Generator(np.random.PCG64(seed))
    base = np.array([1] * (N // 2) + [-1] * (N // 2), dtype=np.int8)
    return np.stack([rng.permutation(base) for _ in range(B)]).astype(np.int8)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    model: ModelShape
    ham: HamSpec
    B: int
    param_seed: int
    spin_seed: int
    spins: str = "uniform"   # or "balanced"
    prec: str = "fp32"       # fp64 | fp32 | bf16

    def params(self, scale: str = "baseline") -> np.ndarray:
        seed = self.param_seed if scale == "baseline" else self.param_seed + 100
        return draw_params(self.model, seed, scale)

    def spin_batch(self, B: int | None = None) -> np.ndarray:
        B = self.B if B is None else B
        f = uniform_spins if self.spins == "uniform" else balanced_spins
        return f(self.B, self.model.N, self.spin_seed)[:B]


# The five workloads of the benchmark statement, as concrete seeded recipes.
WORKLOADS: Dict[str, Workload] = {
    # tiny: N=16, one block, d=8, s=4, tanh, open, FP64, 64 samples
    "tfim_n16_l1_d8": Workload(
        "tfim_n16_l1_d8", ModelShape(16, 1, 8, 4, act="tanh", bc="open"),
        HamSpec("lrtfim", "open", J=1.0, alpha=3.0, h=1.0), 64, 1001, 2001, prec="fp64"),
    # N=64, two blocks, d=32, s=16, FP32, 4096 samples
    "tfim_n64_l2_d32": Workload(
        "tfim_n64_l2_d32", ModelShape(64, 2, 32, 16, act="silu", bc="open"),
        HamSpec("lrtfim", "open", J=1.0, alpha=3.0, h=1.0), 4096, 1002, 2002),
    # J1-J2 chain N=128, periodic, zero-magnetisation sector, four blocks, d=64, s=32
    "j1j2_n128_l4_d64": Workload(
        "j1j2_n128_l4_d64", ModelShape(128, 4, 64, 32, act="silu", bc="periodic"),
        HamSpec("j1j2", "periodic", J1=1.0, J2=0.5), 8192, 1003, 2003, spins="balanced", prec="bf16"),
    # headline: N=256, four blocks, d=64, s=32, FP32, 2048 samples, alpha=2, h=0.5
    "tfim_n256_l4_d64": Workload(
        "tfim_n256_l4_d64", ModelShape(256, 4, 64, 32, act="silu", bc="open"),
        HamSpec("lrtfim", "open", J=1.0, alpha=2.0, h=0.5), 2048, 1005, 2005),
    # same shape at two blocks (the paper's depth)
    "tfim_n256_l2_d64": Workload(
        "tfim_n256_l2_d64", ModelShape(256, 2, 64, 32, act="silu", bc="open"),
        HamSpec("lrtfim", "open", J=1.0, alpha=2.0, h=0.5), 2048, 1006, 2006),
}


def ragged_small_instances(n_inst: int = 64, base_seed: int = 3500):
    """Many small instances, where per-call host work matters: N ~ U{16..128}, L ~ U{1,2},
    d ~ {16, 32} (state size d / 2), B ~ U{32..256}."""
    out = []
    for i in range(n_inst):
        rng = np.random.Generator(np.random.PCG64(base_seed + i))
        N = int(rng.integers(16, 129))
        L = int(rng.integers(1, 3))
        d = int(rng.choice([16, 32]))
        B = int(rng.integers(32, 257))
        out.append(Workload(f"ragged_small_{i}", ModelShape(N, L, d, d // 2, act="silu", bc="open"),
                            HamSpec("lrtfim", "open", J=1.0, alpha=3.0, h=1.0), B,
                            6000 + i, 7000 + i))
    return out


def ragged_instances(n_inst: int = 32, base_seed: int = 3000):
    """The ragged batch: instance i draws N ~ U{32..512}, L ~ U{2,3,4}, B ~ U{256..2048}."""
    out = []
    for i in range(n_inst):
        rng = np.random.Generator(np.random.PCG64(base_seed + i))
        N = int(rng.integers(32, 513))
        L = int(rng.integers(2, 5))
        B = int(rng.integers(256, 2049))
        out.append(Workload(f"ragged_{i}", ModelShape(N, L, 64, 32, act="silu", bc="open"),
                            HamSpec("lrtfim", "open", J=1.0, alpha=3.0, h=1.0), B,
                            5000 + i, 4000 + i))
    return out
