"""MI355X-native DysonNet local estimator (HIP kernels for gfx950 behind a C ABI).

The product path is ``libdysonnet.so`` (built from ``csrc/`` by ``build.py``); this package
only binds it. Importing the package does not load the library; the first call does, and
raises if it has not been built.
"""
from ._lib import (DysonNetError, Model, connected, local_energy, param_count, lib, EXPORTS,  # noqa: F401
                   LIB_PATH)
