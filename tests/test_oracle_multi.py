"""Pins of the repeated-column oracle (count-vector tables): the exact
Python DP, the C fp64 chain and the C residues.  CPU only.

What pins it to something other than itself:
  * brute force over S_n (eq. 1) of the explicitly expanded n x n matrix;
  * the subset oracle (already pinned against eq. 1, eq. 4 and Tables 1-3)
    on the expanded matrix -- exact for integers, bitwise for complex when
    every multiplicity is 1 (then the two tables hold the same chains);
  * closed forms: one column repeated n times, the all-ones matrix,
    rank-one matrices;
  * exact invariances (row permutations; column permutations carrying their
    multiplicities)."""
import itertools
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
    e = 0.0
    for k in range(2, n + 1):
        g = 2 * k * U64 / (1 - 2 * k * U64)
        e = e + math.sqrt(2.0) * g * (1 + e)
    return e


def random_mult(rng, n, m):
    """m positive counts summing to n."""
    cuts = sorted(rng.sample(range(1, n), m - 1)) if m > 1 else []
    b = [0] + cuts + [n]
    return [b[i + 1] - b[i] for i in range(m)]


def bits(z):
    return np.array([z.real, z.imag], dtype=np.float64).view(np.uint64).tolist()


# ------------------------------------------------------------- exact DP
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_exact_equals_brute_force_of_expanded_int(n):
    rng = random.Random(1000 + n)
    for rep in range(4):
        m = rng.randint(1, n)
        t = random_mult(rng, n, m)
        A = np.array([[rng.randint(-9, 9) for _ in range(m)] for _ in range(n)], dtype=np.int64)
        assert exact.per_multi_exact(A, t) == exact.per_definition(exact.expand_columns(A, t)), (n, t)


@pytest.mark.parametrize("n", [2, 4, 6])
def test_exact_equals_brute_force_of_expanded_complex(n):
    rng = random.Random(2000 + n)
    m = max(1, n // 2)
    t = random_mult(rng, n, m)
    A = inputs.dyadic_complex(n, seed=n, bits=12)[:, :m]
    assert exact.per_multi_exact(A, t) == exact.per_definition(exact.expand_columns(A, t))


@pytest.mark.parametrize("n", [2, 5, 8])
def test_exact_all_ones_is_store_zechin(n):
    A = inputs.uniform_int(n, -5, 5, seed=n)
    assert exact.per_multi_exact(A, [1] * n) == exact.per_store_zechin(exact.as_exact_matrix(A))


def test_exact_closed_forms():
    # one column repeated n times: n! * prod_i a_i
    col = np.array([[3], [-2], [5], [7], [1]], dtype=np.int64)
    assert exact.per_multi_exact(col, [5]) == math.factorial(5) * 3 * -2 * 5 * 7 * 1
    # all-ones matrix: n! whatever the multiplicities
    for t in ([2, 3, 1], [6], [1, 1, 4], [2, 2, 2]):
        n = sum(t)
        assert exact.per_multi_exact(np.ones((n, len(t)), dtype=np.int64), t) == math.factorial(n)
    # rank one u v^T: n! prod u_i prod v_j^t_j
    u = [2, -1, 3, 1, 2, -2]
    v = [1, 3, -2]
    t = [3, 1, 2]
    A = np.array([[ui * vj for vj in v] for ui in u], dtype=np.int64)
    ref = math.factorial(6) * math.prod(u) * math.prod(vj ** tj for vj, tj in zip(v, t))
    assert exact.per_multi_exact(A, t) == ref


def test_exact_rejects_bad_multiplicities():
    A = np.ones((3, 2), dtype=np.int64)
    with pytest.raises(ValueError):
        exact.per_multi_exact(A, [1, 1])
    with pytest.raises(ValueError):
        exact.per_multi_exact(A, [3, 0])
    assert exact.per_multi_exact(np.zeros((0, 0), dtype=np.int64), []) == 1


def test_count_vectors_colex_order():
    t = [2, 1, 2]
    layer = exact.count_vectors(t, 2)
    # all vectors of sum 2, ordered by the last column first
    assert layer == [(2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1), (0, 0, 2)]
    assert sum(len(exact.count_vectors(t, k)) for k in range(6)) == 3 * 2 * 3


# ----------------------------------------------------------- C, complex
@pytest.mark.parametrize("n", [1, 2, 5, 9, 13, 16])
def test_native_all_ones_bitwise_equals_subset_oracle(oracle_lib, n):
    A = inputs.complex_gaussian(n, seed=300 + n)
    assert bits(oracle_lib.per_multi_c128(A, [1] * n)) == bits(oracle_lib.per_c128(A))


@pytest.mark.parametrize("n", [3, 6, 9, 12])
def test_native_exact_on_small_gaussian_integers(oracle_lib, n):
    """Parts in {-1, 0, 1}: every intermediate and the factorial scale are
    integers below 2^53, so fp64 must give the exact value bit for bit."""
    rng = np.random.default_rng(400 + n)
    r = random.Random(400 + n)
    for rep in range(3):
        m = r.randint(1, n)
        t = random_mult(r, n, m)
        A = (rng.integers(-1, 2, size=(n, m)) + 1j * rng.integers(-1, 2, size=(n, m))).astype(np.complex128)
        q = exact.per_multi_exact(A, t)
        ref = complex(float(q.re), float(q.im))
        assert bits(oracle_lib.per_multi_c128(A, t)) == bits(ref), (n, t)


@pytest.mark.parametrize("n", [4, 8, 12])
def test_native_gaussian_within_chain_bound(oracle_lib, n):
    r = random.Random(500 + n)
    for rep in range(3):
        m = r.randint(1, n)
        t = random_mult(r, n, m)
        A = inputs.dyadic_complex(n, seed=500 + 7 * n + rep, bits=20)[:, :m]
        got = oracle_lib.per_multi_c128(A, t)
        q = exact.per_multi_exact(A, t)
        # |a| <= |re| + |im|: an exact upper bound of per(|A|) of the expansion
        absA = np.abs(A.real) + np.abs(A.imag)
        scale = float(exact.per_multi_exact(absA, t))
        tol = (chain_error_bound(n) + 4 * U64) * scale
        d = GaussQ.from_complex(got) - q
        assert math.hypot(float(d.re), float(d.im)) <= tol, (n, t)


@pytest.mark.parametrize("n", [10, 14, 18])
def test_native_complex_close_to_subset_oracle_of_expansion(oracle_lib, n):
    """Two different fp64 chains of the same permanent: both within the
    chain bound of the exact value, so within twice it of each other."""
    r = random.Random(600 + n)
    m = n // 2
    t = random_mult(r, n, m)
    A = inputs.bunched_output(n, t, seed=n)
    a = oracle_lib.per_multi_c128(A, t)
    E = exact.expand_columns(A, t)
    b = oracle_lib.per_c128(E)
    tol = 2 * (chain_error_bound(n) + 4 * U64) * oracle_lib.per_abs(E) * (1 + 1e-9)
    assert abs(a - b) <= tol, (n, t, abs(a - b), tol)


def test_native_edge_cases(oracle_lib):
    assert oracle_lib.per_multi_c128(np.zeros((0, 0), dtype=np.complex128), []) == 1
    a = np.array([[2.5 - 1.25j]])
    assert bits(oracle_lib.per_multi_c128(a, [1])) == bits(2.5 - 1.25j)
    col = np.array([[1 + 1j], [2 - 1j], [0.5j]])
    # 3! * (1+i)(2-i)(0.5i), every step exact
    assert oracle_lib.per_multi_c128(col, [3]) == 6 * (1 + 1j) * (2 - 1j) * 0.5j
    with pytest.raises(ValueError):
        oracle_lib.per_multi_c128(np.ones((3, 2), dtype=np.complex128), [1, 1])
    with pytest.raises(ValueError):
        oracle_lib.per_multi_c128(np.ones((3, 2), dtype=np.complex128), [3, 0])


# ----------------------------------------------------------- C, mod p
@pytest.mark.parametrize("n", [2, 5, 8])
def test_native_modp_equals_exact_g(oracle_lib, n):
    r = random.Random(700 + n)
    p = exact.primes_61(2)[1]
    for rep in range(3):
        m = r.randint(1, n)
        t = random_mult(r, n, m)
        A = np.array([[r.randint(-50, 50) for _ in range(m)] for _ in range(n)], dtype=np.int64)
        g = exact.per_multi_exact(A, t) // math.prod(math.factorial(x) for x in t)
        R = np.array([[int(v) % p for v in row] for row in A], dtype=np.uint64)
        assert oracle_lib.multi_modp(R, t, p) == g % p


@pytest.mark.parametrize("n", [6, 12, 16, 18])
def test_native_int_equals_subset_oracle_of_expansion(oracle_lib, n):
    """Exact integers: the count-vector table against the subset table of the
    explicitly expanded matrix (independent algorithms, equal values)."""
    r = random.Random(800 + n)
    for rep in range(2):
        m = r.randint(2, n - 1)
        t = random_mult(r, n, m)
        A = np.array([[r.randint(-3, 3) for _ in range(m)] for _ in range(n)], dtype=np.int64)
        assert oracle_lib.per_multi_int(A, t) == oracle_lib.per_int(exact.expand_columns(A, t)), (n, t)


def test_native_int_extreme_entries(oracle_lib):
    rng = np.random.default_rng(81)
    for n, t in ((3, [2, 1]), (5, [1, 3, 1]), (6, [6])):
        A = rng.integers(-(2 ** 63), 2 ** 63 - 1, size=(n, len(t)), dtype=np.int64, endpoint=True)
        A[0, 0] = -(2 ** 63)
        assert oracle_lib.per_multi_int(A, t) == exact.per_multi_exact(A, t)


def test_native_int_invariances(oracle_lib):
    r = random.Random(900)
    n, t = 14, [3, 1, 4, 2, 1, 3]
    A = np.array([[r.randint(-4, 4) for _ in range(len(t))] for _ in range(n)], dtype=np.int64)
    v = oracle_lib.per_multi_int(A, t)
    rows = list(range(n))
    r.shuffle(rows)
    assert oracle_lib.per_multi_int(A[rows], t) == v
    cols = list(range(len(t)))
    r.shuffle(cols)
    assert oracle_lib.per_multi_int(A[:, cols], [t[c] for c in cols]) == v
    # scaling row 0 by 3 scales the permanent by 3
    B = A.copy()
    B[0] *= 3
    assert oracle_lib.per_multi_int(B, t) == 3 * v
