"""Exact-arithmetic oracle for the permanent (test infrastructure only).

Nothing in the product path may import this module.  It is imported by
``tests/``, by ``__graft_entry__.smoke()`` and by the CPU-baseline leg of
``bench.py``, and by nothing else.

Every function works in exact arithmetic: Python ``int`` for integer
matrices, :class:`GaussQ` (pairs of ``fractions.Fraction``) for complex
matrices whose parts are given as floats (every finite double is an exact
dyadic rational, so ``Fraction(float)`` loses nothing).

Paper passages followed (Su & Zheng, "The Multiphoton Boson Sampling Machine
Doesn't Beat Early Classical Computers for Five-boson Sampling"):

* eq. (1), section 3.1 -- the definition of per(A), used by
  :func:`per_definition` (brute force over the symmetric group);
* properties 1-4, section 3.1 -- used by the tests, not here;
* section 3.2 -- the naive operation counts, :func:`naive_op_counts`;
* eqs. (2)-(4), section 3.3 -- Ryser's inclusion-exclusion form, used by
  :func:`per_ryser` (eq. 4) and :func:`ryser_op_counts`;
* section 4 (and 4.1-4.3, Tables 1-3) -- Store-zechin: develop along the last
  row, recursively, storing every sub-permanent the first time it is met and
  reusing it afterwards; :func:`per_store_zechin` follows it step by step and
  can count multiplications/additions per top-level term exactly as Tables
  1-3 lay them out;
* section 5.2 -- the ENIAC/TRADIC operation-rate model, :func:`machine_time_ms`.

Parity pins for this module live in ``tests/test_oracle_exact.py``.
"""
from __future__ import annotations

import itertools
import math
from collections import Counter
from fractions import Fraction
from typing import Callable, Dict, List, Optional, Sequence, Tuple


# --------------------------------------------------------------------------
# exact complex numbers
# --------------------------------------------------------------------------
class GaussQ:
    """Exact complex rational x + i*y (x, y Fractions)."""

    __slots__ = ("re", "im")

    def __init__(self, re=0, im=0):
        self.re = Fraction(re)
        self.im = Fraction(im)

    @staticmethod
    def from_complex(z: complex) -> "GaussQ":
        return GaussQ(Fraction(float(z.real)), Fraction(float(z.imag)))

    def __add__(self, o):
        o = _gq(o)
        return GaussQ(self.re + o.re, self.im + o.im)

    __radd__ = __add__

    def __sub__(self, o):
        o = _gq(o)
        return GaussQ(self.re - o.re, self.im - o.im)

    def __rsub__(self, o):
        return _gq(o) - self

    def __neg__(self):
        return GaussQ(-self.re, -self.im)

    def __mul__(self, o):
        o = _gq(o)
        return GaussQ(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    __rmul__ = __mul__

    def __eq__(self, o):
        o = _gq(o)
        return self.re == o.re and self.im == o.im

    def __hash__(self):
        return hash((self.re, self.im))

    def __abs__(self):
        return math.hypot(float(self.re), float(self.im))

    def to_complex(self) -> complex:
        return complex(float(self.re), float(self.im))

    def __repr__(self):
        return f"GaussQ({self.re}, {self.im})"


def _gq(x) -> GaussQ:
    if isinstance(x, GaussQ):
        return x
    if isinstance(x, complex):
        return GaussQ.from_complex(x)
    return GaussQ(x, 0)


def as_exact_matrix(A) -> List[List]:
    """Convert a square matrix (nested lists or numpy array) to exact entries.

    Integer dtypes become Python ints, float dtypes Fractions, complex dtypes
    GaussQ.  No rounding happens anywhere.
    """
    try:
        import numpy as np  # local import: numpy is only needed for arrays
    except ImportError:  # pragma: no cover
        np = None
    if np is not None and isinstance(A, np.ndarray):
        if A.ndim != 2 or A.shape[0] != A.shape[1]:
            raise ValueError("square matrix expected")
        if np.issubdtype(A.dtype, np.integer) or A.dtype == np.bool_:
            return [[int(v) for v in row] for row in A]
        if np.issubdtype(A.dtype, np.complexfloating):
            return [[GaussQ.from_complex(complex(v)) for v in row] for row in A]
        if np.issubdtype(A.dtype, np.floating):
            return [[Fraction(float(v)) for v in row] for row in A]
        raise TypeError(f"unsupported dtype {A.dtype}")
    rows = [list(r) for r in A]
    n = len(rows)
    if any(len(r) != n for r in rows):
        raise ValueError("square matrix expected")
    out = []
    for r in rows:
        out.append([_gq(v) if isinstance(v, complex) else v for v in r])
    return out


def _zero_like(A):
    for row in A:
        for v in row:
            return v * 0
    return 0


# --------------------------------------------------------------------------
# eq. (1): the definition, brute force over S_n
# --------------------------------------------------------------------------
def per_definition(A):
    """per(A) = sum over permutations sigma of prod_i a[i, sigma(i)]  (eq. 1).

    Exponential in n! -- meant for n <= 8.
    """
    M = as_exact_matrix(A)
    n = len(M)
    if n == 0:
        return 1
    total = _zero_like(M)
    for sigma in itertools.permutations(range(n)):
        prod = M[0][sigma[0]]
        for i in range(1, n):
            prod = prod * M[i][sigma[i]]
        total = total + prod
    return total


# --------------------------------------------------------------------------
# section 4: Store-zechin, developed along the last row with stored minors
# --------------------------------------------------------------------------
class OpCounter:
    """Counts x and + the way Tables 1-3 attribute them.

    Each top-level term j of the development along the last row (the j-th
    summand a[n, j] * per(A_{n; j})) is charged with the one multiplication
    by a[n, j] plus every multiplication and addition spent on sub-permanents
    that were first evaluated while that term was being expanded.  The
    additions that join the n top-level terms are charged to the "sigma" row.
    """

    def __init__(self, n: int):
        self.n = n
        self.term_mul = [0] * n
        self.term_add = [0] * n
        self.sigma_add = 0
        self.current = -1
        self.minors_computed = 0

    def totals(self) -> Tuple[int, int]:
        return sum(self.term_mul), sum(self.term_add) + self.sigma_add


def per_store_zechin(A, ops: Optional[OpCounter] = None, memo: Optional[dict] = None):
    """Store-zechin (section 4): permanent developed along the last row.

    per(rows 1..k, columns S) = sum over j in S, in ascending order, of
        a[k, j] * per(rows 1..k-1, columns S minus {j})
    (property 4 of section 3.1 applied to the last remaining row), recursively
    down to sub-permanents of order 2, whose value is the 2x2 expansion
    a[2, x] * a[1, y] + a[2, y] * a[1, x].  Every sub-permanent is stored the
    first time it is evaluated and looked up on every later use, so each
    repeated minor is computed once (sections 4.2 and 4.3).

    A minor is keyed by its remaining column set S (a frozenset of 0-based
    column indices); its rows are always the first |S| rows.  Exact
    arithmetic.  ``memo`` may be passed in to inspect the stored minors.
    """
    M = as_exact_matrix(A)
    n = len(M)
    if n == 0:
        return 1
    if n == 1:
        return M[0][0]
    if memo is None:
        memo = {}

    def minor(S: Tuple[int, ...]):
        # S: ascending tuple of remaining columns; rows 0..len(S)-1 remain.
        k = len(S)
        if k == 1:
            return M[0][S[0]]
        if S in memo:
            return memo[S]
        if k == 2:
            x, y = S
            val = M[1][x] * M[0][y] + M[1][y] * M[0][x]
            if ops is not None:
                ops.term_mul[ops.current] += 2
                ops.term_add[ops.current] += 1
        else:
            val = None
            for idx, j in enumerate(S):
                sub = minor(S[:idx] + S[idx + 1:])
                term = M[k - 1][j] * sub
                val = term if val is None else val + term
            if ops is not None:
                ops.term_mul[ops.current] += k
                ops.term_add[ops.current] += k - 1
        if ops is not None:
            ops.minors_computed += 1
        memo[S] = val
        return val

    full = tuple(range(n))
    if n == 2:
        # The order-2 base case is the whole matrix.
        if ops is not None:
            ops.current = 0
        return minor(full)
    total = None
    for j in range(n):
        if ops is not None:
            ops.current = j
        sub = minor(full[:j] + full[j + 1:])
        term = M[n - 1][j] * sub
        if ops is not None:
            ops.term_mul[j] += 1
        total = term if total is None else total + term
    if ops is not None:
        ops.sigma_add += n - 1
    return total


def store_zechin_op_table(n: int) -> OpCounter:
    """Op counts of Store-zechin for an n x n matrix, laid out as in Tables 1-3.

    The counts do not depend on the values, so a matrix of ones is used.
    """
    if n < 3:
        raise ValueError("the paper's tables start at n = 3")
    ops = OpCounter(n)
    per_store_zechin([[1] * n for _ in range(n)], ops=ops)
    return ops


def expansion_multiplicities(n: int) -> Dict[int, Counter]:
    """Occurrences of each minor in the *un-stored* expansion tree.

    Expanding along the last row without storing anything, the minor with the
    last L rows removed and column set C removed is reached once per ordering
    of the removed columns.  Returns {L: Counter(removed-column-set ->
    occurrences)} for L = 1..n-2 (down to order-2 minors).  Sections 4.2 and
    4.3 state these counts for n = 4 and n = 5.
    """
    out: Dict[int, Counter] = {}

    def walk(removed: Tuple[int, ...]):
        L = len(removed)
        if L >= 1:
            out.setdefault(L, Counter())[frozenset(removed)] += 1
        if n - L <= 2:
            return
        for j in range(n):
            if j not in removed:
                walk(removed + (j,))

    walk(())
    return out


# --------------------------------------------------------------------------
# section 3.3: Ryser, eq. (4)
# --------------------------------------------------------------------------
def per_ryser(A):
    """per(A) = (-1)^n * sum_{S subset of columns} (-1)^{|S|} prod_i sum_{j in S} a_ij.

    Eq. (4), evaluated in exact arithmetic; every subset is visited, the empty
    one included (its product is 0 for n >= 1).
    """
    M = as_exact_matrix(A)
    n = len(M)
    if n == 0:
        return 1
    zero = _zero_like(M)
    total = zero
    for mask in range(1 << n):
        cols = [j for j in range(n) if mask >> j & 1]
        prod = None
        for i in range(n):
            s = zero
            for j in cols:
                s = s + M[i][j]
            prod = s if prod is None else prod * s
        sign = -1 if (n - len(cols)) % 2 else 1
        total = total + prod * sign
    return total


def naive_op_counts(n: int) -> Tuple[int, int]:
    """Section 3.2: n!(n-1) multiplications and n!-1 additions."""
    f = math.factorial(n)
    return f * (n - 1), f - 1


def ryser_op_counts(n: int, refs_count: bool = False) -> Tuple[int, int]:
    """Section 3.3: (2^n-1)(n-1) multiplications; (2^n-n)(n+1)-2 additions.

    With ``refs_count`` the addition count is the one the paper attributes to
    its references [1][2], (2^n-2)(n+1).
    """
    mul = (2 ** n - 1) * (n - 1)
    add = (2 ** n - 2) * (n + 1) if refs_count else (2 ** n - n) * (n + 1) - 2
    return mul, add


# --------------------------------------------------------------------------
# section 5.2: operation-rate model of ENIAC and TRADIC
# --------------------------------------------------------------------------
MACHINES = {
    # additions per second, multiplications per second
    "ENIAC": (5000.0, 357.0),
    "TRADIC": (62500.0, 3333.0),
}


def machine_time_ms(mults: int, adds: int, machine: str) -> float:
    """Running time in ms: each operation takes 1/rate seconds (section 5.2)."""
    add_rate, mul_rate = MACHINES[machine]
    return 1000.0 * (mults / mul_rate + adds / add_rate)


# --------------------------------------------------------------------------
# exact integers beyond 64 bits: bound, primes, Chinese remaindering
# --------------------------------------------------------------------------
_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime_u64(x: int) -> bool:
    """Deterministic Miller-Rabin for x < 3.3e24 (the first 12 primes as bases)."""
    if x < 2:
        return False
    for p in _MR_BASES:
        if x % p == 0:
            return x == p
    d, s = x - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        y = pow(a, d, x)
        if y in (1, x - 1):
            continue
        for _ in range(s - 1):
            y = y * y % x
            if y == x - 1:
                break
        else:
            return False
    return True


def primes_61(count: int) -> List[int]:
    """The ``count`` largest primes below 2^61, in descending order."""
    out = []
    x = (1 << 61) - 1
    while len(out) < count:
        if is_prime_u64(x):
            out.append(x)
        x -= 2
    return out


def perm_bound(A) -> int:
    """|per(A)| <= min(prod_i sum_j |a_ij|, n! * max|a_ij|^n), exact ints."""
    M = as_exact_matrix(A)
    n = len(M)
    if n == 0:
        return 1
    rows = 1
    mx = 0
    for r in M:
        s = 0
        for v in r:
            s += abs(int(v))
            mx = max(mx, abs(int(v)))
        rows *= s
    return min(rows, math.factorial(n) * mx ** n)


def primes_for_bound(B: int, redundant: int = 1) -> List[int]:
    """Smallest prefix of :func:`primes_61` whose product exceeds 2B, plus
    ``redundant`` further primes used only to check the recombined value."""
    ps = primes_61(80)
    prod, r = 1, 0
    while prod <= 2 * B:
        prod *= ps[r]
        r += 1
    r = max(r, 1)
    return ps[: r + redundant]


def garner(residues: Sequence[int], primes: Sequence[int]) -> int:
    """Chinese remaindering in mixed radix (Garner), lifted to (-P/2, P/2]."""
    if len(residues) != len(primes):
        raise ValueError("one residue per prime")
    digits: List[int] = []
    for i, (r, p) in enumerate(zip(residues, primes)):
        # value of the digits so far, mod p
        acc, scale = 0, 1
        for d, q in zip(digits, primes[:i]):
            acc = (acc + d * scale) % p
            scale = scale * q % p
        digits.append((r - acc) * pow(scale, -1, p) % p)
    value, scale = 0, 1
    for d, q in zip(digits, primes):
        value += d * scale
        scale *= q
    if value > scale // 2:
        value -= scale
    return value


def residues_of(A, p: int) -> List[List[int]]:
    """Entries reduced into [0, p) (Python's % already lands there)."""
    M = as_exact_matrix(A)
    return [[int(v) % p for v in r] for r in M]


def per_int_multimodular(A, per_mod: Callable[[List[List[int]], int], int],
                         redundant: int = 1) -> int:
    """Exact integer permanent from residues: choose primes by the bound,
    evaluate per(A) mod each prime with ``per_mod``, recombine with Garner on
    all but the redundant primes, then require the redundant ones to agree."""
    B = perm_bound(A)
    ps = primes_for_bound(B, redundant=redundant)
    used = ps[: len(ps) - redundant]
    res = [per_mod(residues_of(A, p), p) for p in ps]
    v = garner(res[: len(used)], used)
    for r, p in zip(res[len(used):], ps[len(used):]):
        if v % p != r:
            raise ArithmeticError("redundant prime disagrees with recombined value")
    return v


# --------------------------------------------------------------------------
# repeated columns (bunched bosons): stored minors over count vectors
# --------------------------------------------------------------------------
def _exact_rect(A) -> List[List]:
    """Exact entries of an n x m matrix (the conversions of as_exact_matrix)."""
    try:
        import numpy as np
    except ImportError:  # pragma: no cover
        np = None
    if np is not None and isinstance(A, np.ndarray):
        if A.ndim != 2:
            raise ValueError("matrix expected")
        if np.issubdtype(A.dtype, np.integer) or A.dtype == np.bool_:
            return [[int(v) for v in row] for row in A]
        if np.issubdtype(A.dtype, np.complexfloating):
            return [[GaussQ.from_complex(complex(v)) for v in row] for row in A]
        if np.issubdtype(A.dtype, np.floating):
            return [[Fraction(float(v)) for v in row] for row in A]
        raise TypeError(f"unsupported dtype {A.dtype}")
    return [[_gq(v) if isinstance(v, complex) else v for v in r] for r in A]


def expand_columns(A, mult: Sequence[int]):
    """The n x n matrix whose columns are column j of the n x m matrix A
    repeated mult[j] times, in order (a numpy array when A is one)."""
    mult = [int(t) for t in mult]
    try:
        import numpy as np
        if isinstance(A, np.ndarray):
            return np.repeat(A, mult, axis=1)
    except ImportError:  # pragma: no cover
        pass
    return [[v for v, t in zip(r, mult) for _ in range(t)] for r in A]


def count_vectors(mult: Sequence[int], k: int) -> List[Tuple[int, ...]]:
    """Every c with 0 <= c_j <= mult[j] and sum(c) = k, ordered by
    (c_{m-1}, ..., c_0) lexicographically (colex: the last column is the most
    significant).  This is the order in which a layer of the table is laid out."""
    out = [c for c in itertools.product(*[range(t + 1) for t in reversed(mult)]) if sum(c) == k]
    return [tuple(reversed(c)) for c in out]


def per_multi_exact(A, mult: Sequence[int]):
    """per(expand_columns(A, mult)) with one stored minor per count vector.

    Columns j and the copies of it are identical, so every column subset
    with c_j copies of each column has the same minor (section 4's stored
    sub-permanents; the repeating terms of Tables 1-3 become one entry):
        G(c) = sum_{j: c_j > 0} a[|c|-1][j] * G(c - e_j),  G(0) = 1,
    G counts each assignment of rows to distinct columns once, and each
    assignment stands for prod_j mult[j]! bijections onto the copies, so
    per = G(mult) * prod_j mult[j]!.  Exact ints / GaussQ."""
    M = _exact_rect(A)
    mult = tuple(int(t) for t in mult)
    n, m = len(M), len(mult)
    if any(t < 1 for t in mult) or sum(mult) != n or any(len(r) != m for r in M):
        raise ValueError("mult must be positive, one per column, summing to the row count")
    if n == 0:
        return 1
    G = {tuple([0] * m): 1}
    for k in range(1, n + 1):
        H = {}
        for c in count_vectors(mult, k):
            acc = None
            for j in range(m):
                if c[j] == 0:
                    continue
                prev = c[:j] + (c[j] - 1,) + c[j + 1:]
                term = M[k - 1][j] * G[prev]
                acc = term if acc is None else acc + term
            H[c] = acc
        G = H
    scale = 1
    for t in mult:
        scale *= math.factorial(t)
    return G[mult] * scale


def per_multi_int_multimodular(A, mult: Sequence[int], g_mod: Callable[[List[List[int]], int], int],
                               redundant: int = 1) -> int:
    """Exact integer permanent with repeated columns from residues of G:
    primes by the bound of the expanded matrix (G divides per, so the bound
    covers G), G mod p from ``g_mod``, Garner, the redundant primes checked,
    then times prod_j mult[j]!."""
    M = _exact_rect(A)
    B = perm_bound(expand_columns(M, mult))
    ps = primes_for_bound(B, redundant=redundant)
    used = ps[: len(ps) - redundant]
    res = [g_mod([[int(v) % p for v in r] for r in M], p) for p in ps]
    g = garner(res[: len(used)], used)
    for r, p in zip(res[len(used):], ps[len(used):]):
        if g % p != r:
            raise ArithmeticError("redundant prime disagrees with recombined value")
    for t in mult:
        g *= math.factorial(int(t))
    return g
