"""Pins of the oracle functions that reach beyond the fp64 tables: eq. (4)
mod p in O(n) memory (orders 31..34), stored minors over the Gaussian
integers mod p (exact values of dyadic complex matrices, hence the true
fp64 error of the chain), the many-matrix driver, and per(|A|).  CPU only.

Each pin is something other than the function itself: brute force over the
symmetric group (eq. (1), section 3.1), closed forms, exact integer
arithmetic, or the independent stored-minor recurrence of section 4."""
import math
import random
import statistics
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact
from oracle.exact import GaussQ
from paper_1802_02779_amd import inputs

from test_oracle_native import chain_error_bound

PRIMES = exact.primes_61(6)


def derangements(m):
    d = [1, 0]
    for k in range(2, m + 1):
        d.append((k - 1) * (d[-1] + d[-2]))
    return d[m]


# ------------------------------------------------------- the modular product
def test_mulmod_matches_integer_arithmetic(oracle_lib):
    rng = random.Random(5)
    for p in PRIMES:
        edge = [0, 1, 2, p - 1, p - 2, (p - 1) // 2, 1 << 60, p - (1 << 32)]
        cases = [(x, y) for x in edge for y in edge]
        cases += [(rng.randrange(p), rng.randrange(p)) for _ in range(2000)]
        for x, y in cases:
            assert oracle_lib.mulmod_pm61(x, y, p) == x * y % p, (p, x, y)


# ------------------------------------------------------------- eq. (4) mod p
@pytest.mark.parametrize("n", range(0, 8))
def test_ryser_modp_vs_definition(oracle_lib, n):
    """Random residues anywhere in [0, p) (large ones exercise the
    reduction): eq. (4) mod p equals eq. (1) evaluated in exact integers."""
    rng = random.Random(100 + n)
    for p in PRIMES[:3]:
        R = [[rng.randrange(p) for _ in range(n)] for _ in range(n)]
        ref = exact.per_definition(R) % p if n else 1
        got = oracle_lib.ryser_modp(np.array(R, dtype=np.uint64).reshape(n, n), p)
        assert got == ref, (n, p)


@pytest.mark.parametrize("n", [8, 11, 14, 17])
def test_ryser_modp_vs_stored_minors(oracle_lib, n):
    """Two independent methods (eq. (4) against the stored minors of
    section 4), same residues."""
    rng = np.random.default_rng(n)
    p = PRIMES[n % 3]
    R = rng.integers(0, p, size=(n, n), dtype=np.uint64)
    assert oracle_lib.ryser_modp(R, p, nthreads=4) == oracle_lib.per_modp(R, p, nthreads=4)


@pytest.mark.parametrize("n", [1, 9, 18, 21])
def test_ryser_int_closed_forms(oracle_lib, n):
    J = np.ones((n, n), dtype=np.int64)
    I = np.eye(n, dtype=np.int64)
    assert oracle_lib.per_int_ryser(J) == math.factorial(n)
    assert oracle_lib.per_int_ryser(I) == 1
    assert oracle_lib.per_int_ryser(J - I) == derangements(n)
    assert oracle_lib.per_int_ryser(-2 * J) == math.factorial(n) * (-2) ** n


@pytest.mark.parametrize("n", [2, 6, 12, 15])
def test_ryser_int_vs_stored_minors(oracle_lib, n):
    A = inputs.uniform_int(n, -1000, 1000, seed=n)
    assert oracle_lib.per_int_ryser(A) == oracle_lib.per_int(A)
    B = inputs.bernoulli01(n, seed=n)
    assert oracle_lib.per_int_ryser(B) == oracle_lib.per_int(B)


def test_ryser_modp_rejects_bad_arguments(oracle_lib):
    p = PRIMES[0]
    with pytest.raises(ValueError):
        oracle_lib.ryser_modp(np.full((3, 3), p, dtype=np.uint64), p)   # residue not below p
    with pytest.raises(ValueError):
        oracle_lib.ryser_modp(np.zeros((3, 3), dtype=np.uint64), 1000003)  # not of the form 2^61 - c
    with pytest.raises(ValueError):
        oracle_lib.ryser_modp(np.zeros((41, 41), dtype=np.uint64), p)


# ------------------------------------------------- Gaussian integers mod p
def _gauss_matrix(n, seed, lo=-9, hi=9):
    rng = np.random.default_rng(seed)
    X = rng.integers(lo, hi + 1, size=(n, n), dtype=np.int64)
    Y = rng.integers(lo, hi + 1, size=(n, n), dtype=np.int64)
    return X, Y


@pytest.mark.parametrize("n", range(0, 8))
def test_gauss_vs_definition(oracle_lib, n):
    X, Y = _gauss_matrix(n, 300 + n, -(10 ** 6), 10 ** 6)
    ref = exact.per_definition([[GaussQ(int(X[i, j]), int(Y[i, j])) for j in range(n)] for i in range(n)]) \
        if n else GaussQ(1, 0)
    re, im = oracle_lib.per_gauss_int(X, Y)
    assert (Fraction(re), Fraction(im)) == (ref.re, ref.im), n


@pytest.mark.parametrize("n", [6, 13, 18])
def test_gauss_rank_one_closed_form(oracle_lib, n):
    """per(u v^T) = n! prod u_i prod v_j over Z[i]."""
    rng = np.random.default_rng(n)
    u = [complex(int(a), int(b)) for a, b in rng.integers(-7, 8, size=(n, 2))]
    v = [complex(int(a), int(b)) for a, b in rng.integers(-7, 8, size=(n, 2))]
    uq = [GaussQ(int(z.real), int(z.imag)) for z in u]
    vq = [GaussQ(int(z.real), int(z.imag)) for z in v]
    X = np.array([[int((uq[i] * vq[j]).re) for j in range(n)] for i in range(n)], dtype=np.int64)
    Y = np.array([[int((uq[i] * vq[j]).im) for j in range(n)] for i in range(n)], dtype=np.int64)
    ref = GaussQ(math.factorial(n), 0)
    for z in uq + vq:
        ref = ref * z
    assert oracle_lib.per_gauss_int(X, Y) == (int(ref.re), int(ref.im))


@pytest.mark.parametrize("n", [5, 9])
def test_gauss_vs_fp64_chain_where_exact(oracle_lib, n):
    """Entries in {-1, 0, 1} + i{-1, 0, 1}: every stored value is a Gaussian
    integer below 2^53 in modulus, so the fp64 chain is exact and must equal
    the Z[i] value."""
    X, Y = _gauss_matrix(n, 400 + n, -1, 1)
    z = oracle_lib.per_c128(X + 1j * Y)
    assert (z.real, z.imag) == tuple(float(v) for v in oracle_lib.per_gauss_int(X, Y))


def test_gauss_multiplication_convention(oracle_lib):
    """A planted swap of the product's parts would break this 2x2 case:
    per([[a, b], [c, d]]) = a d + b c with (1+2i)(3+4i) + (2-i)(i) = -4 + 12i."""
    X = np.array([[1, 2], [0, 3]], dtype=np.int64)
    Y = np.array([[2, -1], [1, 4]], dtype=np.int64)
    # a = 1+2i, b = 2-i, c = i, d = 3+4i: (1+2i)(3+4i) = -5+10i, (2-i)(i) = 1+2i
    assert oracle_lib.per_gauss_int(X, Y) == (-4, 12)


# --------------------- the true fp64 error of the chain on dyadic matrices
@pytest.mark.parametrize("n", [16, 18, 20])
def test_chain_error_on_dyadic_within_bound(oracle_lib, n):
    """Dyadic complex Gaussian matrices (parts multiples of 2^-30): the exact
    permanent over Z[i], and the fp64 chain within the derived bound
    e_n * per(|A|)."""
    A = inputs.dyadic_complex(n, seed=n, bits=30)
    re, im = oracle_lib.per_dyadic_exact(A, 30, nthreads=4)
    z = oracle_lib.per_c128(A, nthreads=4)
    err = math.hypot(float(Fraction(z.real) - re), float(Fraction(z.imag) - im))
    bound = chain_error_bound(n) * oracle_lib.per_abs(A, nthreads=4) * (1 + 1e-12)
    assert err <= bound, (n, err, bound)


def test_chain_error_statistical_gate(oracle_lib):
    """Over 16 seeded dyadic 20x20 Gaussian matrices the median relative error
    of the fp64 chain against the exact value is at most 1e-12 (the stated
    tolerance 1e-10 * per(|A|) is vacuous at this size)."""
    rel = []
    for seed in range(16):
        A = inputs.dyadic_complex(20, seed=5000 + seed, bits=30)
        re, im = oracle_lib.per_dyadic_exact(A, 30, nthreads=4)
        z = oracle_lib.per_c128(A, nthreads=4)
        err = math.hypot(float(Fraction(z.real) - re), float(Fraction(z.imag) - im))
        rel.append(err / math.hypot(float(re), float(im)))
    assert statistics.median(rel) <= 1e-12, rel


# ------------------------------------------------------------------ per(|A|)
@pytest.mark.parametrize("n", [3, 7, 12])
def test_per_abs_rank_one(oracle_lib, n):
    """per(|u v^T|) = n! prod |u_i| prod |v_j| for complex u, v: fixes the
    modulus as the Euclidean one (|re| + |im|, or max, would miss it)."""
    rng = np.random.default_rng(n)
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    A = np.outer(u, v)
    ref = math.factorial(n) * float(np.prod(np.abs(u)) * np.prod(np.abs(v)))
    got = oracle_lib.per_abs(A)
    assert abs(got - ref) <= 1e-13 * n * ref, (got, ref)


def test_per_abs_of_purely_imaginary_and_rotated(oracle_lib):
    """Multiplying every entry by a unit phase leaves per(|A|) unchanged."""
    A = inputs.complex_gaussian(9, seed=3)
    base = oracle_lib.per_abs(A)
    for ph in (1j, np.exp(0.7j), -1):
        assert abs(oracle_lib.per_abs(A * ph) - base) <= 1e-13 * base


# ------------------------------------------------------ many small matrices
def test_many_matches_single(oracle_lib):
    U = inputs.haar_unitary(64, seed=3)
    b = inputs.submatrix_batch(U, 400, 0, 12, seed=9)
    got = oracle_lib.per_c128_many(b.ns, b.offsets, b.mats, nthreads=4)
    for i in range(b.count):
        z = oracle_lib.per_c128(b.matrix(i), mode=oracle_lib.MODE_MEMO)
        assert np.array([z]).view(np.uint64).tolist() == np.array([got[i]]).view(np.uint64).tolist(), i
