"""Seeded synthetic inputs shared by the tests, the bench and the oracle's callers.

This module holds no arithmetic of the permanent method: it only draws
matrices.  Every generator takes an explicit seed and uses NumPy's PCG64, so
the same bytes come out on every machine.

Workloads (the paper's problem is the permanent of an n x n matrix, eq. (1);
boson-sampling amplitudes are permanents of n x n submatrices of an
interferometer unitary, section 2):

* :func:`uniform_int`     -- iid integers in [lo, hi] (small exact case);
* :func:`bernoulli01`     -- iid 0/1 entries with P(1) = p (#P-complete class
                             named in section 2);
* :func:`complex_gaussian`-- iid complex Gaussians, real and imaginary parts
                             N(0, 1/2);
* :func:`dyadic_complex`  -- complex entries whose parts are multiples of
                             2^-bits (exact rational references exist);
* :func:`haar_unitary`    -- Haar-random unitary via QR with the phase fix of
                             Mezzadri (2007); stands in for the photonic
                             interferometer, whose matrix is not available;
* :func:`submatrix_batch` -- packed row-major n x n submatrices of a unitary on
                             random distinct rows/columns, n uniform in a range;
* :func:`poisson_trace`   -- arrival times and sizes of a serving trace;
* :func:`bunched_pattern` -- output counts of n photons landing in `modes`
                             detectors uniformly at random (collisions
                             allowed), zero counts dropped;
* :func:`bunched_output`  -- the n x m matrix of a bunched output: rows = the
                             n input modes, columns = the m occupied output
                             modes of a Haar unitary, with their counts.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Tuple

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_int(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """n x n int64 matrix with iid entries uniform on {lo, ..., hi}."""
    return _rng(seed).integers(lo, hi + 1, size=(n, n), dtype=np.int64)


def bernoulli01(n: int, seed: int, p: float = 0.5) -> np.ndarray:
    """n x n int64 matrix of iid Bernoulli(p) entries."""
    return (_rng(seed).random((n, n)) < p).astype(np.int64)


def complex_gaussian(n: int, seed: int) -> np.ndarray:
    """n x n complex128 matrix, real and imaginary parts iid N(0, 1/2)."""
    g = _rng(seed).standard_normal((2, n, n))
    return ((g[0] + 1j * g[1]) / np.sqrt(2.0)).astype(np.complex128)


def dyadic_complex(n: int, seed: int, bits: int = 30, scale: float = 1.0) -> np.ndarray:
    """complex_gaussian rounded so both parts are integer multiples of 2^-bits."""
    z = complex_gaussian(n, seed) * scale
    q = float(2 ** bits)
    return (np.round(z.real * q) / q + 1j * (np.round(z.imag * q) / q)).astype(np.complex128)


def haar_unitary(m: int, seed: int) -> np.ndarray:
    """m x m Haar-random unitary: QR of a complex Gaussian, R's diagonal phases
    moved into Q (Mezzadri, Notices AMS 54 (2007))."""
    g = _rng(seed).standard_normal((2, m, m))
    z = (g[0] + 1j * g[1]) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    ph = d / np.abs(d)
    return (q * ph[None, :]).astype(np.complex128)


@dataclass
class Batch:
    ns: np.ndarray        # int32[count], matrix orders
    offsets: np.ndarray   # int64[count], element offset of each matrix in ``mats``
    mats: np.ndarray      # complex128[sum n^2], row-major matrices back to back

    @property
    def count(self) -> int:
        return int(self.ns.shape[0])

    def matrix(self, i: int) -> np.ndarray:
        n = int(self.ns[i])
        o = int(self.offsets[i])
        return self.mats[o:o + n * n].reshape(n, n)


def submatrix_batch(U: np.ndarray, count: int, n_lo: int, n_hi: int, seed: int) -> Batch:
    """``count`` submatrices of U on random distinct rows and columns, with
    orders uniform on {n_lo, ..., n_hi}, packed row-major back to back."""
    rng = _rng(seed)
    m = U.shape[0]
    ns = rng.integers(n_lo, n_hi + 1, size=count).astype(np.int32)
    offsets = np.zeros(count, dtype=np.int64)
    if count:
        offsets[1:] = np.cumsum(ns.astype(np.int64) ** 2)[:-1]
    total = int((ns.astype(np.int64) ** 2).sum())
    mats = np.empty(total, dtype=np.complex128)
    # Draw rows/cols per matrix: argsort of uniform keys is a random
    # permutation; take its first n entries (distinct indices).
    for lo_n in range(n_lo, n_hi + 1):
        idx = np.nonzero(ns == lo_n)[0]
        if idx.size == 0:
            continue
        k = idx.size
        rows = np.argsort(rng.random((k, m)), axis=1)[:, :lo_n]
        cols = np.argsort(rng.random((k, m)), axis=1)[:, :lo_n]
        sub = U[rows[:, :, None], cols[:, None, :]]  # (k, n, n)
        flat = sub.reshape(k, lo_n * lo_n)
        pos = offsets[idx][:, None] + np.arange(lo_n * lo_n)[None, :]
        mats[pos] = flat
    return Batch(ns=ns, offsets=offsets, mats=mats)


@dataclass
class Trace:
    t_arrive: np.ndarray  # float64[count] seconds from the start
    ns: np.ndarray        # int32[count]
    mats: list            # list of complex128 (n, n) arrays


def poisson_trace(U: np.ndarray, count: int, rate_per_s: float, seed: int,
                  small=(5, 12), large=(20, 28), p_small: float = 0.8) -> Trace:
    """Poisson arrivals (exponential gaps of mean 1/rate) of submatrix
    permanents; with probability ``p_small`` the order is uniform on ``small``,
    else uniform on ``large``."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps) - gaps[0]
    is_small = rng.random(count) < p_small
    ns = np.where(is_small, rng.integers(small[0], small[1] + 1, size=count),
                  rng.integers(large[0], large[1] + 1, size=count)).astype(np.int32)
    m = U.shape[0]
    mats = []
    for n in ns:
        rows = rng.permutation(m)[:n]
        cols = rng.permutation(m)[:n]
        mats.append(np.ascontiguousarray(U[np.ix_(rows, cols)]))
    return Trace(t_arrive=t, ns=ns, mats=mats)


def split_parts(z: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Real and imaginary parts as float64 arrays (a convenience for tests)."""
    return np.ascontiguousarray(z.real), np.ascontiguousarray(z.imag)


def bunched_pattern(n: int, modes: int, seed: int) -> np.ndarray:
    """Counts (int32, all >= 1, summing to n) of the occupied modes when n
    photons land in `modes` detectors independently and uniformly."""
    hits = _rng(seed).integers(0, modes, size=n)
    c = np.bincount(hits, minlength=modes)
    return c[c > 0].astype(np.int32)


def bunched_output(n: int, mult, seed: int, modes: int = 0) -> np.ndarray:
    """n x m complex128 block of a Haar unitary on `modes` >= max(n, m) modes
    (default 2 * max(n, m)): rows = input modes 0..n-1, columns = m random
    distinct output modes, one per entry of `mult` (the counts are carried
    separately).  The output amplitude of the bunched pattern is the permanent
    of this block with column j repeated mult[j] times, over the square root
    of prod mult[j]!."""
    m = len(mult)
    M = modes or 2 * max(n, m)
    U = haar_unitary(M, seed)
    cols = _rng(seed + 1).choice(M, size=m, replace=False)
    return np.ascontiguousarray(U[:n][:, cols])
