"""Orders 31..34, beyond the oracle's 2^n tables: integer 0/1 results are
exact against values the oracle computed by eq. (4) mod p in O(n) memory
(stored in tests/golden/large_configs.json) and against closed forms at
every order; two independent GPU algorithms -- the Store-zechin layer sweep
and Ryser's eq. (4) -- agree bit for bit for integers, and within the
measured 1e-6 gate (as at n = 26, 28) for complex Gaussian inputs.
Workspaces here reach 112 GB; the cache is emptied after each test."""
import json
import math
import os

import numpy as np
import pytest

from paper_1802_02779_amd import inputs

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def chain_error_bound(n):
    e = 0.0
    for k in range(2, n + 1):
        g = 2 * k * U64 / (1 - 2 * k * U64)
        e = e + math.sqrt(2.0) * g * (1 + e)
    return e


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1802_02779_amd import perm
    perm.lib()
    yield perm
    torch.cuda.empty_cache()


@pytest.fixture(autouse=True)
def _release():
    yield
    import torch
    torch.cuda.empty_cache()


def bits(z):
    return np.asarray([z], dtype=np.complex128).view(np.uint64).tolist()


@pytest.mark.parametrize("n", [31, 32, 34])
def test_int_bernoulli_sweep_equals_ryser(P, n):
    B = inputs.bernoulli01(n, seed=n)
    print(f"[gpu] int 0/1 n={n} store-zechin", flush=True)
    sz = P.perm_solve(B)
    print(f"[gpu] int 0/1 n={n} ryser", flush=True)
    ry = P.perm_ryser(B)
    assert sz == ry, (n, sz, ry)
    assert sz > 0


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large_configs.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("n", [31, 32, 33, 34])
def test_int_bernoulli_vs_stored_oracle(P, golden, n):
    """Bernoulli(1/2) 0/1 matrices (seed 0): exact against the oracle's
    eq. (4) mod p values."""
    print(f"[gpu] int 0/1 n={n} vs stored oracle value", flush=True)
    assert P.perm_solve(inputs.bernoulli01(n, seed=0)) == int(golden[f"int_n{n}_bern_s0"]["value"])


@pytest.mark.parametrize("n", [31, 32, 33, 34])
def test_int_closed_forms(P, n):
    J = np.ones((n, n), dtype=np.int64)
    I = np.eye(n, dtype=np.int64)
    d = [1, 0]
    for k in range(2, n + 1):
        d.append((k - 1) * (d[-1] + d[-2]))
    print(f"[gpu] closed forms n={n}", flush=True)
    assert P.perm_solve(J) == math.factorial(n)
    assert P.perm_solve(J - I) == d[n]
    assert P.perm_ryser(J) == math.factorial(n)
    assert P.perm_solve(I) == 1


@pytest.mark.parametrize("n", [31, 34])
def test_complex_deterministic_and_agrees_with_ryser(P, n):
    import torch
    A = inputs.complex_gaussian(n, seed=n)
    d_a = torch.from_numpy(A).cuda()
    d_r = torch.zeros(3, dtype=torch.complex128, device="cuda")
    ws = P.device_buffer(P.perm_workspace_bytes(P.PERM_COMPLEX128, n))
    print(f"[gpu] complex n={n} store-zechin x2", flush=True)
    P.perm_solve_async(n, d_a, n, d_r[0:1], ws)
    P.perm_solve_async(n, d_a, n, d_r[1:2], ws)
    del ws
    wr = P.device_buffer(P.perm_ryser_workspace_bytes(P.PERM_COMPLEX128, n))
    print(f"[gpu] complex n={n} ryser", flush=True)
    P.perm_ryser_async(n, d_a, n, d_r[2:3], wr)
    r = d_r.cpu().numpy()
    assert bits(r[0]) == bits(r[1])
    rel = abs(r[2] - r[0]) / abs(r[0])
    print(f"[gpu] complex n={n} relative difference Ryser / Store-zechin {rel:.3e}", flush=True)
    assert rel < 1e-6


def test_complex_rank_one_n34(P):
    n = 34
    rng = np.random.default_rng(34)
    u = np.exp(1j * rng.uniform(0, 2 * np.pi, n)) * rng.uniform(0.8, 1.2, n)
    v = np.exp(1j * rng.uniform(0, 2 * np.pi, n)) * rng.uniform(0.8, 1.2, n)
    A = np.outer(u, v)
    print("[gpu] rank one n=34", flush=True)
    z = P.perm_solve(A)
    ref = math.factorial(n) * np.prod(u) * np.prod(v)
    # per(|A|) = |ref| for a rank-one matrix; the chain bound plus the
    # rounding of the reference itself (2n products)
    assert abs(z - ref) <= (chain_error_bound(n) + 4 * n * U64) * abs(ref)


@pytest.mark.parametrize("n", [31, 32, 33, 34])
def test_complex_exact_on_sparse_integer_matrices(P, n):
    """0/1 matrices with at most three ones per row (the diagonal, the
    superdiagonal and, from the third row on, one random column): every
    stored value is an integer bounded by the product of the row sums,
    4 * 3^32 < 2^53, so the complex sweep's fp64 chain is exact and must give
    the integer permanent bit for bit -- an exact pin of the complex path's
    tables and indexing at orders beyond the oracle's tables."""
    rng = np.random.default_rng(100 + n)
    A = np.eye(n, dtype=np.int64)
    A[np.arange(n - 1), np.arange(1, n)] = 1
    A[np.arange(2, n), rng.integers(0, n, size=n - 2)] = 1
    assert math.prod(int(r) for r in A.sum(axis=1)) < 2 ** 53
    print(f"[gpu] sparse 0/1 n={n}: integer and complex sweeps", flush=True)
    want = P.perm_solve(A)
    assert want == P.perm_ryser(A)
    assert 0 < want < 2 ** 53
    z = P.perm_solve(A.astype(np.complex128))
    assert z == complex(float(want), 0.0), (z, want)
