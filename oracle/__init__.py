"""FP64 CPU oracle of the DysonNet local estimator (test infrastructure only).

This package is a plain, slow, obviously correct reference of what the GPU path
computes. It is used only by ``tests/``, by ``__graft_entry__.smoke()`` and by the
``cpu_baseline`` leg of ``bench.py``; the product path never imports it.

It shares no code with the HIP library: it reads the flat parameter vector with its
own unpacking, computes the S4 Green's-function taps by matrix powers in complex128,
evaluates the network by direct Toeplitz sums, forms log-ratios by full
re-evaluation (the plain definition) and, separately, by the ABACUS recurrence with
links materialised from their definitions. All arithmetic is float64 (complex128 for
the state-space part) using plain PyTorch CPU tensors.

Modules
  model        parameter unpacking, S4 kernel generation, forward pass, plain log-ratio
  abacus       ABACUS local update with dense link tensors (small N)
  hamiltonian  connected elements, diagonal energies, local energy
  grad         per-sample d log psi / d theta by reverse-mode autodiff of ``model``

Every function cites the passage of the paper it follows. Readings of passages that
are silent, ambiguous or garbled are stated where they are used.
Nothing here is "parity unpinned": each part is pinned by a test in
``tests/test_oracle_*.py`` against closed forms, invariants or brute force.
"""
from .model import (ModelDesc, unpack, s4_discretize, s4_taps, toeplitz_matrices,
                    forward, logpsi, plain_logratio, lcd, logcosh, flip_configs)
from .hamiltonian import connected, local_energy, eloc_plain
from .abacus import abacus_logratio

__all__ = [
    "ModelDesc", "unpack", "s4_discretize", "s4_taps", "toeplitz_matrices", "forward",
    "logpsi", "plain_logratio", "lcd", "logcosh", "flip_configs", "connected",
    "local_energy", "eloc_plain", "abacus_logratio",
]
