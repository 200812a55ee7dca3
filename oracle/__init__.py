"""Oracle for the Store-zechin permanent -- TEST INFRASTRUCTURE, not product.

Plain, slow, obviously correct CPU implementations written from the paper
(Su & Zheng, "The Multiphoton Boson Sampling Machine Doesn't Beat Early
Classical Computers for Five-boson Sampling"):

* :mod:`oracle.exact`  -- exact arithmetic in Python: eq. (1) by brute force,
  Store-zechin (section 4) with op counting per Tables 1-3, Ryser eq. (4),
  the section 5.2 machine-time model, primes, bound and Garner CRT;
* :mod:`oracle.native` -- the same Store-zechin stored sub-permanents in C
  (``perm_oracle.c``): fp64 FMA chain for complex128, exact 128-bit
  accumulation mod p for integers, per(|A|); memo (paper's order) and
  layers (OpenMP) evaluation;
* repeated columns (bunched bosons): one stored minor per count vector
  instead of one per subset -- exact (:func:`exact.per_multi_exact`), fp64
  chain and residues in C (:func:`native.per_multi_c128`,
  :func:`native.per_multi_int`).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import anything from here.  The oracle shares no code with
the HIP library and never imports it.
"""
from . import exact, native  # noqa: F401

__all__ = ["exact", "native"]
