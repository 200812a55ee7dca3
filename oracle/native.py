"""ctypes front end of the C oracle (``oracle/perm_oracle.c``) -- test infrastructure.

Only tests/, ``__graft_entry__.smoke()`` and bench.py's CPU-baseline leg may
use this module.  :func:`build` compiles the C file with gcc into
``oracle/_build/libpermoracle.so``; the functions here load it on first use
(building it if it is missing).

The C code evaluates the Store-zechin stored sub-permanents (section 4 of the
paper) on dense bitmask-indexed tables; see the header of perm_oracle.c for
the per-entry arithmetic (fp64 FMA chain for complex, exact 128-bit
accumulation then ``%`` for residues).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import List, Optional, Sequence

import numpy as np

from . import exact

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "perm_oracle.c")
_BUILD_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD_DIR, "libpermoracle.so")
_lock = threading.Lock()
_lib: Optional[ctypes.CDLL] = None

MODE_MEMO = 0
MODE_LAYERS = 1


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, OpenMP, no FP contraction)."""
    os.makedirs(_BUILD_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load() -> ctypes.CDLL:
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build(force=False)
            lib = ctypes.CDLL(_LIB_PATH)
            dp = ctypes.POINTER(ctypes.c_double)
            up = ctypes.POINTER(ctypes.c_uint64)
            lib.oracle_per_c128.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_int, dp]
            lib.oracle_per_c128.restype = ctypes.c_int
            lib.oracle_per_abs.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp]
            lib.oracle_per_abs.restype = ctypes.c_int
            lib.oracle_per_modp.argtypes = [ctypes.c_int, up, ctypes.c_uint64, ctypes.c_int,
                                            ctypes.c_int, up]
            lib.oracle_per_modp.restype = ctypes.c_int
            lib.oracle_ryser_bound.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
            lib.oracle_ryser_bound.restype = ctypes.c_int
            ip = ctypes.POINTER(ctypes.c_int32)
            lib.oracle_multi_c128.argtypes = [ctypes.c_int, ctypes.c_int, ip, dp, ctypes.c_int, dp]
            lib.oracle_multi_c128.restype = ctypes.c_int
            lib.oracle_multi_modp.argtypes = [ctypes.c_int, ctypes.c_int, ip, up, ctypes.c_uint64, ctypes.c_int, up]
            lib.oracle_multi_modp.restype = ctypes.c_int
            lib.oracle_ryser_modp.argtypes = [ctypes.c_int, up, ctypes.c_uint64, ctypes.c_int, up]
            lib.oracle_ryser_modp.restype = ctypes.c_int
            lib.oracle_mulmod_pm61.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
            lib.oracle_mulmod_pm61.restype = ctypes.c_uint64
            lib.oracle_per_gauss_modp.argtypes = [ctypes.c_int, up, up, ctypes.c_uint64, ctypes.c_int, up]
            lib.oracle_per_gauss_modp.restype = ctypes.c_int
            lib.oracle_per_c128_many.argtypes = [ctypes.c_int64, ip, ctypes.POINTER(ctypes.c_int64), dp,
                                                 ctypes.c_int, dp]
            lib.oracle_per_c128_many.restype = ctypes.c_int
            lib.oracle_max_threads.argtypes = []
            lib.oracle_max_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _check(rc: int, what: str):
    if rc == -2:
        raise MemoryError(f"{what}: out of host memory")
    if rc != 0:
        raise ValueError(f"{what}: bad arguments (rc={rc})")


def _as_c128(A) -> np.ndarray:
    A = np.ascontiguousarray(np.asarray(A, dtype=np.complex128))
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("square matrix expected")
    return A


def per_c128(A, mode: int = MODE_LAYERS, nthreads: int = 0) -> complex:
    """fp64 Store-zechin permanent of a complex matrix (canonical FMA chain)."""
    A = _as_c128(A)
    n = A.shape[0]
    out = np.zeros(2, dtype=np.float64)
    flat = A.view(np.float64)
    rc = _load().oracle_per_c128(n, flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 mode, nthreads, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    _check(rc, "oracle_per_c128")
    return complex(out[0], out[1])


def per_c128_bits(A, mode: int = MODE_LAYERS, nthreads: int = 0) -> np.ndarray:
    """Same as :func:`per_c128` but returns the two doubles as uint64 bit patterns."""
    z = per_c128(A, mode, nthreads)
    return np.array([z.real, z.imag], dtype=np.float64).view(np.uint64)


def per_abs(A, nthreads: int = 0) -> float:
    """fp64 per(|A|), the scale of the complex tolerance |d| <= tol * per(|A|)."""
    A = _as_c128(A)
    n = A.shape[0]
    out = np.zeros(1, dtype=np.float64)
    flat = A.view(np.float64)
    rc = _load().oracle_per_abs(n, flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                nthreads, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    _check(rc, "oracle_per_abs")
    return float(out[0])


def ryser_bound(A, mm: int, depth: int, nthreads: int = 0) -> float:
    """Rigorous bound on the rounding error of an fp64 evaluation of Ryser's
    eq. (4) with ranges of at most 2^mm one-column-change subsets, FMA complex
    products, and every product passing through at most `depth` additions
    (derivation in perm_oracle.c).  n <= 24."""
    A = _as_c128(A)
    n = A.shape[0]
    out = np.zeros(1, dtype=np.float64)
    flat = A.view(np.float64)
    rc = _load().oracle_ryser_bound(n, flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(mm), int(depth),
                                    nthreads, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    _check(rc, "oracle_ryser_bound")
    return float(out[0])


def per_modp(R, p: int, mode: int = MODE_LAYERS, nthreads: int = 0) -> int:
    """Store-zechin permanent mod p of a matrix of residues in [0, p), p < 2^61."""
    R = np.ascontiguousarray(np.asarray(R, dtype=np.uint64))
    if R.ndim != 2 or R.shape[0] != R.shape[1]:
        raise ValueError("square matrix expected")
    n = R.shape[0]
    out = np.zeros(1, dtype=np.uint64)
    up = ctypes.POINTER(ctypes.c_uint64)
    rc = _load().oracle_per_modp(n, R.ctypes.data_as(up), ctypes.c_uint64(p), mode, nthreads,
                                 out.ctypes.data_as(up))
    _check(rc, "oracle_per_modp")
    return int(out[0])


def per_int(A, mode: int = MODE_LAYERS, nthreads: int = 0, redundant: int = 1) -> int:
    """Exact integer permanent: C residues per prime, Garner in Python."""
    def per_mod(res: List[List[int]], p: int) -> int:
        return per_modp(np.array(res, dtype=np.uint64).reshape(len(res), len(res)), p,
                        mode=mode, nthreads=nthreads)
    return exact.per_int_multimodular(A, per_mod, redundant=redundant)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


# ------------------------------------------------------------ repeated columns
def _mult_arg(mult, m: int) -> np.ndarray:
    t = np.ascontiguousarray(np.asarray(mult, dtype=np.int32))
    if t.ndim != 1 or t.shape[0] != m:
        raise ValueError("one multiplicity per column")
    return t


def per_multi_c128(A, mult, nthreads: int = 0) -> complex:
    """fp64 permanent of the matrix with column j of the n x m matrix A
    repeated mult[j] times: one stored minor per count vector, the complex
    chain of :func:`per_c128`, then times prod mult[j]! (see perm_oracle.c)."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.complex128))
    if A.ndim != 2:
        raise ValueError("matrix expected")
    n, m = A.shape
    t = _mult_arg(mult, m)
    out = np.zeros(2, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = _load().oracle_multi_c128(n, m, t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   A.view(np.float64).ctypes.data_as(dp), nthreads, out.ctypes.data_as(dp))
    _check(rc, "oracle_multi_c128")
    return complex(out[0], out[1])


def multi_modp(R, mult, p: int, nthreads: int = 0) -> int:
    """G(mult) mod p for an n x m matrix of residues in [0, p) (unscaled)."""
    R = np.ascontiguousarray(np.asarray(R, dtype=np.uint64))
    if R.ndim != 2:
        raise ValueError("matrix expected")
    n, m = R.shape
    t = _mult_arg(mult, m)
    out = np.zeros(1, dtype=np.uint64)
    up = ctypes.POINTER(ctypes.c_uint64)
    rc = _load().oracle_multi_modp(n, m, t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), R.ctypes.data_as(up),
                                   ctypes.c_uint64(p), nthreads, out.ctypes.data_as(up))
    _check(rc, "oracle_multi_modp")
    return int(out[0])


def per_multi_int(A, mult, nthreads: int = 0, redundant: int = 1) -> int:
    """Exact integer permanent with repeated columns: C residues of G per
    prime, Garner and the factorial scale in Python."""
    m = np.asarray(A).shape[1]

    def g_mod(res: List[List[int]], p: int) -> int:
        return multi_modp(np.array(res, dtype=np.uint64).reshape(len(res), m), mult, p, nthreads=nthreads)
    return exact.per_multi_int_multimodular(A, mult, g_mod, redundant=redundant)


# ------------------------------------------------ eq. (4) mod p, O(n) memory
def ryser_modp(R, p: int, nthreads: int = 0) -> int:
    """per(R) mod p by Ryser's eq. (4) over all 2^n column subsets in
    Gray-code order (perm_oracle.c); R holds residues in [0, p) and
    p = 2^61 - c with c < 2^16.  O(n) memory, so n may exceed the tables'
    limit (up to 40; the time is 2^n * n^2 / threads)."""
    R = np.ascontiguousarray(np.asarray(R, dtype=np.uint64))
    if R.ndim != 2 or R.shape[0] != R.shape[1]:
        raise ValueError("square matrix expected")
    out = np.zeros(1, dtype=np.uint64)
    up = ctypes.POINTER(ctypes.c_uint64)
    rc = _load().oracle_ryser_modp(R.shape[0], R.ctypes.data_as(up), ctypes.c_uint64(p), nthreads,
                                   out.ctypes.data_as(up))
    _check(rc, "oracle_ryser_modp")
    return int(out[0])


def mulmod_pm61(x: int, y: int, p: int) -> int:
    """The modular product the eq. (4) oracle uses (for its own pin)."""
    return int(_load().oracle_mulmod_pm61(ctypes.c_uint64(x), ctypes.c_uint64(y), ctypes.c_uint64(p)))


def per_int_ryser(A, nthreads: int = 0, redundant: int = 1) -> int:
    """Exact integer permanent by eq. (4) mod primes 2^61 - c and Garner,
    with the redundant-prime check (any order up to 40)."""
    def per_mod(res: List[List[int]], p: int) -> int:
        return ryser_modp(np.array(res, dtype=np.uint64).reshape(len(res), len(res)), p, nthreads=nthreads)
    return exact.per_int_multimodular(A, per_mod, redundant=redundant)


# ------------------------------------------- Gaussian integers, exact values
def per_gauss_modp(X, Y, p: int, nthreads: int = 0):
    """(Re, Im) of per(X + iY) mod p for integer matrices given as residues
    in [0, p) (stored sub-permanents over Z[i] mod p, perm_oracle.c)."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.uint64))
    Y = np.ascontiguousarray(np.asarray(Y, dtype=np.uint64))
    if X.ndim != 2 or X.shape[0] != X.shape[1] or X.shape != Y.shape:
        raise ValueError("two square matrices of one shape expected")
    out = np.zeros(2, dtype=np.uint64)
    up = ctypes.POINTER(ctypes.c_uint64)
    rc = _load().oracle_per_gauss_modp(X.shape[0], X.ctypes.data_as(up), Y.ctypes.data_as(up),
                                       ctypes.c_uint64(p), nthreads, out.ctypes.data_as(up))
    _check(rc, "oracle_per_gauss_modp")
    return int(out[0]), int(out[1])


def per_gauss_int(X, Y, nthreads: int = 0, redundant: int = 1):
    """Exact per(X + iY) for integer matrices X, Y, as a pair of Python ints.

    Both parts are bounded by prod_i sum_j (|x_ij| + |y_ij|) >= prod_i sum_j
    |g_ij| >= |per|; primes are chosen for that bound, each part is
    recombined by Garner and checked on the redundant prime(s)."""
    Xi = [[int(v) for v in row] for row in np.asarray(X)]
    Yi = [[int(v) for v in row] for row in np.asarray(Y)]
    n = len(Xi)
    B = 1
    for i in range(n):
        B *= sum(abs(Xi[i][j]) + abs(Yi[i][j]) for j in range(n))
    ps = exact.primes_for_bound(B, redundant=redundant)
    used = ps[: len(ps) - redundant]
    res = []
    for p in ps:
        xr = np.array([[v % p for v in row] for row in Xi], dtype=np.uint64).reshape(n, n)
        yr = np.array([[v % p for v in row] for row in Yi], dtype=np.uint64).reshape(n, n)
        res.append(per_gauss_modp(xr, yr, p, nthreads=nthreads))
    re = exact.garner([r[0] for r in res[: len(used)]], used)
    im = exact.garner([r[1] for r in res[: len(used)]], used)
    for (a, b), p in zip(res[len(used):], ps[len(used):]):
        if re % p != a or im % p != b:
            raise ArithmeticError("redundant prime disagrees with recombined value")
    return re, im


def per_dyadic_exact(A, bits: int, nthreads: int = 0):
    """Exact per(A) of a complex matrix whose parts are integer multiples of
    2^-bits: per(A) = 2^(-n bits) per(2^bits A), the latter over Z[i].
    Returns (Re, Im) as fractions.Fraction."""
    from fractions import Fraction
    A = _as_c128(A)
    n = A.shape[0]
    q = float(2 ** bits)
    X = A.real * q
    Y = A.imag * q
    if not (np.all(X == np.round(X)) and np.all(Y == np.round(Y))):
        raise ValueError("entries are not multiples of 2^-bits")
    re, im = per_gauss_int(X.astype(np.int64), Y.astype(np.int64), nthreads=nthreads)
    s = Fraction(1, 2 ** (n * bits))
    return re * s, im * s


# ----------------------------------------------- many small complex matrices
def per_c128_many(ns, offsets, mats, nthreads: int = 0) -> np.ndarray:
    """per_c128 (paper's memo order) of every matrix of a packed batch:
    matrix i has order ns[i] <= 20 and starts at complex element offsets[i]
    of mats.  Returns complex128[count]."""
    ns = np.ascontiguousarray(np.asarray(ns, dtype=np.int32))
    offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    mats = np.ascontiguousarray(np.asarray(mats, dtype=np.complex128))
    count = int(ns.shape[0])
    out = np.zeros(count, dtype=np.complex128)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = _load().oracle_per_c128_many(count, ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      mats.view(np.float64).ctypes.data_as(dp), nthreads,
                                      out.view(np.float64).ctypes.data_as(dp))
    _check(rc, "oracle_per_c128_many")
    return out
