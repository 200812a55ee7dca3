"""Pins of the C oracle (oracle/perm_oracle.c): exact values, closed forms,
invariances and a derived fp64 error bound.  CPU only."""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact
from oracle.exact import GaussQ
from paper_1802_02779_amd import inputs

U64 = 2.0 ** -53


def chain_error_bound(n):
    """Relative bound e_n with |computed - per(A)| <= e_n * per(|A|) for the
    fp64 FMA chain (each stored value of order k sums 2k rounded FMAs per
    part; Cauchy-Schwarz puts both parts under sqrt(2)*gamma_{2k}; the error of
    the k predecessors propagates with weight per(|A|) of the minor):
        e_1 = 0,  e_k = e_{k-1} + sqrt(2) * gamma_{2k} * (1 + e_{k-1}),
        gamma_m = m u / (1 - m u),  u = 2^-53."""
    e = 0.0
    for k in range(2, n + 1):
        g = 2 * k * U64 / (1 - 2 * k * U64)
        e = e + math.sqrt(2.0) * g * (1 + e)
    return e


def exact_complex(A):
    """Exact per(A) of a complex128 matrix: Ryser eq. (4) in exact rationals
    for n <= 11, else the exact Store-zechin evaluation (pinned separately
    against eq. (1) and eq. (4))."""
    M = exact.as_exact_matrix(A)
    return exact.per_ryser(M) if len(M) <= 11 else exact.per_store_zechin(M)


def close_within(z, ref_exact, bound_abs):
    d = GaussQ.from_complex(z) - ref_exact
    err = math.hypot(float(d.re), float(d.im))
    return err <= bound_abs, err


# -------------------------------------------- evaluation orders agree bitwise
@pytest.mark.parametrize("n", [2, 3, 5, 8, 11, 14, 16])
def test_memo_and_layers_bitwise_complex(oracle_lib, n):
    A = inputs.complex_gaussian(n, seed=n)
    a = oracle_lib.per_c128_bits(A, mode=oracle_lib.MODE_MEMO)
    b = oracle_lib.per_c128_bits(A, mode=oracle_lib.MODE_LAYERS, nthreads=4)
    assert (a == b).all()


@pytest.mark.parametrize("n", [2, 4, 9, 13, 16])
def test_memo_and_layers_equal_modp(oracle_lib, n):
    p = exact.primes_61(1)[0]
    R = np.array(exact.residues_of(inputs.uniform_int(n, -99, 99, seed=n), p), dtype=np.uint64)
    assert oracle_lib.per_modp(R, p, mode=oracle_lib.MODE_MEMO) == \
        oracle_lib.per_modp(R, p, mode=oracle_lib.MODE_LAYERS, nthreads=3)


# -------------------------------------------------- complex vs exact values
@pytest.mark.parametrize("n", range(1, 8))
def test_complex_vs_definition(oracle_lib, n):
    for seed in range(3):
        A = inputs.complex_gaussian(n, seed=1000 * n + seed)
        ref = exact.per_definition(A)
        z = oracle_lib.per_c128(A)
        ok, err = close_within(z, ref, chain_error_bound(n) * oracle_lib.per_abs(A) * (1 + 1e-12))
        assert ok, (n, seed, err)


@pytest.mark.parametrize("n", [9, 11, 14])
def test_complex_dyadic_vs_exact(oracle_lib, n):
    A = inputs.dyadic_complex(n, seed=n, bits=20)
    ref = exact_complex(A)
    z = oracle_lib.per_c128(A)
    bound = chain_error_bound(n) * oracle_lib.per_abs(A) * (1 + 1e-12)
    ok, err = close_within(z, ref, bound)
    assert ok, (err, bound)
    # the tolerance stated for complex results is far wider than the chain's
    assert bound < 1e-10 * oracle_lib.per_abs(A)


def test_error_bound_small_against_tolerance():
    assert chain_error_bound(30) < 2e-13


# ------------------------------------------------------- integer pins (C)
@pytest.mark.parametrize("n", range(0, 8))
def test_int_vs_definition_huge_entries(oracle_lib, n):
    rng = np.random.default_rng(n)
    A = rng.integers(-(2 ** 63), 2 ** 63 - 1, size=(n, n), dtype=np.int64, endpoint=True)
    assert oracle_lib.per_int(A) == exact.per_definition(A)
    assert oracle_lib.per_int(A, mode=oracle_lib.MODE_MEMO) == exact.per_definition(A)


@pytest.mark.parametrize("n", [1, 5, 10, 16, 20])
def test_int_closed_forms(oracle_lib, n):
    def D(m):
        d = [1, 0]
        for k in range(2, m + 1):
            d.append((k - 1) * (d[-1] + d[-2]))
        return d[m]
    J = np.ones((n, n), dtype=np.int64)
    I = np.eye(n, dtype=np.int64)
    assert oracle_lib.per_int(J) == math.factorial(n)
    assert oracle_lib.per_int(I) == 1
    assert oracle_lib.per_int(J - I) == D(n)
    assert oracle_lib.per_int(3 * J) == math.factorial(n) * 3 ** n
    Z = inputs.uniform_int(n, -5, 5, seed=n)
    Z[n // 2, :] = 0
    assert oracle_lib.per_int(Z) == 0
    T = np.triu(inputs.uniform_int(n, -3, 3, seed=n + 50))
    assert oracle_lib.per_int(T) == math.prod(int(x) for x in np.diag(T))


def test_int_block_diagonal(oracle_lib):
    A = inputs.uniform_int(5, -9, 9, seed=1)
    B = inputs.uniform_int(6, -9, 9, seed=2)
    M = np.zeros((11, 11), dtype=np.int64)
    M[:5, :5] = A
    M[5:, 5:] = B
    assert oracle_lib.per_int(M) == exact.per_definition(A) * exact.per_store_zechin(B)


def test_int_invariances(oracle_lib):
    n = 14
    A = inputs.uniform_int(n, -50, 50, seed=3)
    p = oracle_lib.per_int(A)
    rng = np.random.default_rng(0)
    assert oracle_lib.per_int(A[rng.permutation(n)]) == p
    assert oracle_lib.per_int(A[:, rng.permutation(n)]) == p
    assert oracle_lib.per_int(np.ascontiguousarray(A.T)) == p
    B = A.copy()
    B[4] *= -7
    assert oracle_lib.per_int(B) == -7 * p


# ------------------------------------------------- complex closed forms
@pytest.mark.parametrize("n", [4, 10, 18])
def test_complex_rank_one(oracle_lib, n):
    rng = np.random.default_rng(n)
    u = np.exp(1j * rng.uniform(0, 2 * np.pi, n)) * rng.uniform(0.5, 1.5, n)
    v = np.exp(1j * rng.uniform(0, 2 * np.pi, n)) * rng.uniform(0.5, 1.5, n)
    A = np.outer(u, v)
    z = oracle_lib.per_c128(A)
    ref = math.factorial(n) * np.prod(u) * np.prod(v)
    # per(|A|) = |ref| here; the entries themselves carry rounding (|da| <= u|a|)
    tol = (chain_error_bound(n) + 4 * n * U64) * oracle_lib.per_abs(A)
    assert abs(z - ref) <= tol


def test_complex_power_of_two_scaling_bitwise(oracle_lib):
    n = 12
    A = inputs.complex_gaussian(n, seed=77)
    z = oracle_lib.per_c128(A)
    B = A.copy()
    B[5] *= 8.0
    C = A.copy()
    C[:, 2] *= 0.25
    assert oracle_lib.per_c128(B) == z * 8.0
    assert oracle_lib.per_c128(C) == z * 0.25


def test_complex_invariances_within_bound(oracle_lib):
    n = 13
    A = inputs.complex_gaussian(n, seed=5)
    z = oracle_lib.per_c128(A)
    tol = 2 * chain_error_bound(n) * oracle_lib.per_abs(A)
    rng = np.random.default_rng(1)
    for B in (A[rng.permutation(n)], A[:, rng.permutation(n)], np.ascontiguousarray(A.T)):
        assert abs(oracle_lib.per_c128(B) - z) <= tol


def test_complex_zero_row_is_exact_zero(oracle_lib):
    A = inputs.complex_gaussian(9, seed=3)
    A[0] = 0
    assert oracle_lib.per_c128(A) == 0


def test_per_abs(oracle_lib):
    A = inputs.complex_gaussian(10, seed=4)
    assert oracle_lib.per_abs(A) >= abs(oracle_lib.per_c128(A))
    R = np.abs(inputs.complex_gaussian(10, seed=8))
    assert abs(oracle_lib.per_abs(R) - oracle_lib.per_c128(R).real) <= 1e-13 * oracle_lib.per_abs(R)
    assert oracle_lib.per_c128(R).imag == 0


@pytest.mark.parametrize("n", [5, 9, 12])
def test_per_abs_complex_rank_one(oracle_lib, n):
    """per(|u v^T|) = n! prod_i |u_i| prod_j |v_j| for complex u, v: entrywise
    moduli of a complex rank-one matrix (a modulus other than the Euclidean
    one, such as |re| + |im|, fails this)."""
    rng = np.random.default_rng(100 + n)
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    A = np.outer(u, v)
    want = math.factorial(n) * float(np.prod(np.abs(u))) * float(np.prod(np.abs(v)))
    assert abs(oracle_lib.per_abs(A) - want) <= 1e-12 * want
    # a unit phase on every entry leaves every modulus, hence per(|A|), as it was
    P = np.exp(2j * np.pi * rng.random((n, n)))
    assert abs(oracle_lib.per_abs(A * P) - want) <= 1e-12 * want


def test_bad_arguments_rejected(oracle_lib):
    with pytest.raises(ValueError):
        oracle_lib.per_c128(np.zeros((31, 31), dtype=np.complex128))
    with pytest.raises(ValueError):
        oracle_lib.per_modp(np.full((3, 3), 7, dtype=np.uint64), 5)


# ------------------------------------------------------------ Ryser bound
def _gray_ryser_fp64(A, mm):
    """Plain fp64 evaluation of eq. (4) with the structure the bound covers:
    ranges of 2^mm Gray-code subsets, each starting from directly formed row
    sums and changing one column per subset; sequential summation."""
    n = A.shape[0]
    acc = 0j
    for x0 in range(0, 1 << n, 1 << mm):
        S = x0 ^ (x0 >> 1)
        r = [0j] * n
        for j in range(n):
            if (S >> j) & 1:
                for i in range(n):
                    r[i] = r[i] + complex(A[i, j])
        sg = -1.0 if bin(S).count("1") & 1 else 1.0
        for t in range(1 << mm):
            if t:
                j = (t & -t).bit_length() - 1
                S ^= 1 << j
                s = 1.0 if (S >> j) & 1 else -1.0
                for i in range(n):
                    r[i] = r[i] + s * complex(A[i, j])
                sg = -sg
            p = r[0]
            for v in r[1:]:
                p = p * v
            acc = acc + sg * p
    return acc * (-1) ** n


def _exact_complex(A):
    n = A.shape[0]
    Q = [[GaussQ(Fraction(float(A[i, j].real)), Fraction(float(A[i, j].imag))) for j in range(n)]
         for i in range(n)]
    v = exact.per_store_zechin(Q)
    return complex(float(v.re), float(v.im))


@pytest.mark.parametrize("n,kind", [(5, "gauss"), (6, "gauss"), (7, "gauss"), (6, "huge_column"),
                                    (7, "scaled_rows")])
def test_ryser_bound_covers_an_fp64_evaluation(oracle_lib, n, kind):
    """eq. (4) in fp64 against the exact permanent: the derived bound holds
    for both a one-range (maximal drift) and a direct (2^0) evaluation, on
    Gaussian and on badly scaled inputs where cancellation is extreme."""
    rng = np.random.default_rng(40 + n)
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2)
    if kind == "huge_column":
        A[:, 0] *= 1e8
    elif kind == "scaled_rows":
        A *= (10.0 ** np.arange(n))[:, None]
    ref = _exact_complex(A)
    for mm in (0, n):
        got = _gray_ryser_fp64(A, mm)
        bound = oracle_lib.ryser_bound(A, mm, (1 << n) + 1)
        assert abs(got - ref) <= bound, (n, kind, mm, abs(got - ref), bound)


def test_ryser_bound_grows_with_drift_and_depth(oracle_lib):
    A = inputs.complex_gaussian(8, seed=5)
    b = [oracle_lib.ryser_bound(A, mm, 64) for mm in (0, 4, 8)]
    assert b[0] < b[1] < b[2]
    assert oracle_lib.ryser_bound(A, 2, 16) < oracle_lib.ryser_bound(A, 2, 4096)


def test_ryser_bound_scales_with_the_matrix(oracle_lib):
    """Every term of the bound is homogeneous of degree n in A."""
    A = inputs.complex_gaussian(7, seed=6)
    b1 = oracle_lib.ryser_bound(A, 3, 200)
    b2 = oracle_lib.ryser_bound(2.0 * A, 3, 200)
    assert b2 == pytest.approx(b1 * 2.0 ** 7, rel=1e-12)
