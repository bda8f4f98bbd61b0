"""libaddns: algebraic non-overlapping domain-decomposition preconditioned
(F)GMRES for Oseen saddle-point systems on AMD MI355X (gfx950).

The compute path is the HIP library ``libaddns.so`` built from ``csrc/``;
``addns`` is its thin ctypes binding.  Importing the binding does not load
the library; the first call does, and fails loudly if it is missing.
"""
from . import addns  # noqa: F401
