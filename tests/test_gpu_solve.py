"""GPU parity of perm_solve / perm_solve_async against the oracle.

Complex results are compared bit for bit with the oracle's fp64 FMA chain
(both evaluate every stored sub-permanent with the same chain, so any
difference is a bug) and, as the stated gate, within 1e-10 * per(|A|).
Integer results are exact.  Full-size workloads compare against values the
oracle wrote into tests/golden/large_configs.json.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import exact, native
from paper_1802_02779_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large_configs.json")
TOL = 1e-10


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1802_02779_amd import perm
    perm.lib()
    return perm


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def c_bits(z):
    return tuple(int(x) for x in np.array([z.real, z.imag], dtype=np.float64).view(np.uint64))


def check_complex(P, A, label=""):
    print(f"[gpu] complex n={A.shape[0]} {label}", flush=True)
    z = P.perm_solve(A)
    ref = native.per_c128(A)
    assert c_bits(z) == c_bits(ref), (label, z, ref)
    assert abs(z - ref) <= TOL * native.per_abs(A)
    return z


# ----------------------------------------------------------- complex128
@pytest.mark.parametrize("n", list(range(2, 23)))
def test_complex_gaussian_bitwise(P, n):
    seeds = range(3) if n <= 16 else range(1)
    for s in seeds:
        check_complex(P, inputs.complex_gaussian(n, seed=100 * n + s), f"seed={s}")


@pytest.mark.parametrize("n", [3, 5, 8])
def test_complex_vs_exact_definition(P, n):
    A = inputs.complex_gaussian(n, seed=n)
    ref = exact.per_definition(A)
    z = P.perm_solve(A)
    d = abs(z - ref.to_complex())
    assert d <= 1e-14 * native.per_abs(A) + 1e-300


def test_complex_dyadic_exact_value(P):
    # parts are multiples of 2^-20: the exact permanent is a known rational
    A = inputs.dyadic_complex(10, seed=3, bits=20)
    ref = exact.per_ryser(exact.as_exact_matrix(A)).to_complex()
    z = P.perm_solve(A)
    assert abs(z - ref) <= 1e-13 * native.per_abs(A)


def test_complex_haar_submatrices(P):
    U = inputs.haar_unitary(64, seed=7)
    rng = np.random.default_rng(7)
    for n in (5, 9, 14, 19):
        r = rng.permutation(64)[:n]
        c = rng.permutation(64)[:n]
        check_complex(P, np.ascontiguousarray(U[np.ix_(r, c)]), "haar")


def test_complex_lda_and_async(P):
    import torch
    n = 17
    big = inputs.complex_gaussian(24, seed=9)
    A = np.ascontiguousarray(big[:n, :n])
    z = check_complex(P, A, "packed")
    # host call with lda > n through the raw ABI
    import ctypes
    L = P.lib()
    ws = P.device_buffer(P.perm_workspace_bytes(P.PERM_COMPLEX128, n))
    out = P.perm_c128_t()
    big = np.ascontiguousarray(big)
    rc = L.perm_solve(1, n, big.ctypes.data, 24, ctypes.byref(out), ws.data_ptr(), ws.numel(),
                      torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    assert c_bits(complex(out.re, out.im)) == c_bits(z)
    # device input with lda = 24, device output
    d_big = torch.from_numpy(big).cuda()
    d_res = torch.zeros(1, dtype=torch.complex128, device="cuda")
    P.perm_solve_async(n, d_big, 24, d_res, ws)
    torch.cuda.synchronize()
    assert c_bits(complex(d_res.cpu().numpy()[0])) == c_bits(z)


def test_complex_trivial_orders_async(P):
    import torch
    ws = P.device_buffer(256)
    res = torch.zeros(1, dtype=torch.complex128, device="cuda")
    P.perm_solve_async(0, None, 1, res, ws)
    torch.cuda.synchronize()
    assert complex(res.cpu().numpy()[0]) == 1
    a = torch.tensor([[3.0 - 2.0j]], dtype=torch.complex128, device="cuda")
    P.perm_solve_async(1, a, 1, res, ws)
    torch.cuda.synchronize()
    assert complex(res.cpu().numpy()[0]) == 3.0 - 2.0j
    assert P.perm_solve(np.array([[1 + 1j, 2], [3, 4j]])) == (1 + 1j) * 4j + 2 * 3


def test_workspace_too_small(P):
    n = 12
    ws = P.device_buffer(P.perm_workspace_bytes(P.PERM_COMPLEX128, n) - 1)
    with pytest.raises(P.PermError) as e:
        P.perm_solve(inputs.complex_gaussian(n, seed=1), workspace=ws)
    assert e.value.code == P.PERM_ENOMEM


def test_complex_invariances(P):
    n = 20
    A = inputs.complex_gaussian(n, seed=21)
    z = P.perm_solve(A)
    pa = native.per_abs(A)
    rng = np.random.default_rng(3)
    for B in (A[rng.permutation(n)], A[:, rng.permutation(n)], np.ascontiguousarray(A.T)):
        assert abs(P.perm_solve(np.ascontiguousarray(B)) - z) <= 1e-12 * pa
    # power-of-two scaling of one row or column is exact: bitwise
    B = A.copy()
    B[7] *= 4.0
    C = A.copy()
    C[:, 11] *= 0.5
    assert c_bits(P.perm_solve(B)) == c_bits(z * 4.0)
    assert c_bits(P.perm_solve(C)) == c_bits(z * 0.5)
    D = A.copy()
    D[13] = 0
    assert P.perm_solve(D) == 0


def test_complex_rank_one_large(P):
    n = 28
    rng = np.random.default_rng(28)
    u = np.exp(1j * rng.uniform(0, 2 * np.pi, n)) * rng.uniform(0.8, 1.2, n)
    v = np.exp(1j * rng.uniform(0, 2 * np.pi, n)) * rng.uniform(0.8, 1.2, n)
    A = np.outer(u, v)
    z = P.perm_solve(A)
    ref = math.factorial(n) * np.prod(u) * np.prod(v)
    assert abs(z - ref) <= 1e-12 * abs(ref)


def test_determinism_and_tuning_variants(P):
    n = 20
    A = inputs.complex_gaussian(n, seed=5)
    ref = c_bits(native.per_c128(A))
    saved = P.perm_tuning_get()
    try:
        for t in range(3, 16):
            for remap, thin in ((0, -1), (1, 0), (3, 5000), (16, 64), (64, 16)):
                tu = P.perm_tuning_t.from_buffer_copy(saved)
                tu.layer_t[n] = t
                tu.layer_xcd_remap[n] = remap
                tu.layer_flags[n] = remap & 1
                tu.layer_thin[n] = thin
                P.perm_tuning_set(tu)
                assert c_bits(P.perm_solve(A)) == ref, (t, remap, thin)
    finally:
        P.perm_tuning_set(saved)
    for _ in range(5):
        assert c_bits(P.perm_solve(A)) == ref


# --------------------------------------------------------- full sizes
FULL_COMPLEX = [("c128_n23_s0", 23, 0), ("c128_n24_s0", 24, 0), ("c128_n25_s0", 25, 0),
                ("c128_n26_s0", 26, 0), ("c128_n26_s1", 26, 1), ("c128_n27_s0", 27, 0),
                ("c128_n28_s0", 28, 0), ("c128_n29_s0", 29, 0), ("c128_n30_s0", 30, 0)]


@pytest.mark.parametrize("key,n,seed", FULL_COMPLEX)
def test_full_size_complex(P, golden, key, n, seed):
    g = golden[key]
    A = inputs.complex_gaussian(n, seed=seed)
    print(f"[gpu] full size {key}", flush=True)
    z = P.perm_solve(A)
    assert c_bits(z) == (int(g["re_bits"], 16), int(g["im_bits"], 16)), (z, g["value"])
    assert abs(z - complex(*g["value"])) <= TOL * g["per_abs"]


# ------------------------------------------------------------- int64
@pytest.mark.parametrize("n", list(range(2, 15)) + [16, 18, 20])
def test_int_random(P, n):
    print(f"[gpu] int n={n}", flush=True)
    A = inputs.uniform_int(n, -99, 99, seed=n)
    assert P.perm_solve(A) == native.per_int(A)


@pytest.mark.parametrize("n", [2, 5, 8, 11])
def test_int_huge_entries(P, n):
    rng = np.random.default_rng(1000 + n)
    A = rng.integers(-(2 ** 63), 2 ** 63 - 1, size=(n, n), dtype=np.int64, endpoint=True)
    ref = exact.per_definition(A) if n <= 8 else native.per_int(A)
    assert P.perm_solve(A) == ref


def test_int_config_n10(P, golden):
    for s in range(16):
        A = inputs.uniform_int(10, 0, 9, seed=s)
        assert P.perm_solve(A) == int(golden[f"int_n10_u09_s{s}"]["value"])


@pytest.mark.parametrize("n", [25, 27, 29, 30])
def test_int_full_size_bernoulli(P, golden, n):
    print(f"[gpu] int n={n} Bernoulli", flush=True)
    A = inputs.bernoulli01(n, seed=0)
    assert P.perm_solve(A) == int(golden[f"int_n{n}_bern_s0"]["value"])


def test_complex_dyadic_n20_true_error(P):
    """Dyadic complex Gaussian matrices of order 20 (parts multiples of
    2^-30), whose exact permanents the oracle computes over the Gaussian
    integers: the GPU result is bitwise the oracle's fp64 chain, lies within
    the derived chain bound of the exact value, and over 16 seeds the median
    relative error is at most 1e-12."""
    from fractions import Fraction
    import statistics
    from test_oracle_native import chain_error_bound
    rel = []
    for seed in range(16):
        A = inputs.dyadic_complex(20, seed=7000 + seed, bits=30)
        print(f"[gpu] dyadic n=20 seed={seed}", flush=True)
        z = P.perm_solve(A)
        assert c_bits(z) == c_bits(native.per_c128(A)), seed
        re, im = native.per_dyadic_exact(A, 30)
        err = math.hypot(float(Fraction(z.real) - re), float(Fraction(z.imag) - im))
        assert err <= chain_error_bound(20) * native.per_abs(A) * (1 + 1e-12), seed
        rel.append(err / math.hypot(float(re), float(im)))
    assert statistics.median(rel) <= 1e-12, rel


def test_int_plain_prefix_row_sum_branch(P):
    """Rows with two nonzero entries (a_ii = v_i, a_i,i+1 = 1, a_n-1,0 = 1):
    per = prod v_i + 1, and the layer bound min(R_{k-1}, k M_{k-1}) takes
    the row sum R = v + 1 in every row but the first.  With v_0 = 2^30,
    v_1..v_4 = 2^10 and v_i = 1 after them the bound allows plain 64-bit
    layers up to k = 4 (the stored value F({0..3}) is 2^60) and the largest
    stored value of layer 5 is 2^70; the value needs two primes and the
    redundant one, one sweep.  A row index off by one in the row-sum branch
    would take rows 1..k (factors 2^10 and then 2) and run every layer in
    plain arithmetic, which overflows."""
    n = 24
    v = [2 ** 30] + [2 ** 10] * 4 + [1] * (n - 5)
    A = np.zeros((n, n), dtype=np.int64)
    for i in range(n):
        A[i, i] = v[i]
        A[i, (i + 1) % n] = 1
    want = math.prod(v) + 1
    # plain layers by the rule, computed here: product of the per-row factors
    B, K = 1, 0
    for k in range(1, n + 1):
        R, M = int(np.abs(A[k - 1]).sum()), int(np.abs(A[k - 1]).max())
        B *= min(R, k * M)
        if B > 2 ** 63 - 1:
            break
        K = k
    assert K == 4
    P.perm_profile_enable(True)
    try:
        P.perm_profile_read()
        got = P.perm_solve(A)
        prof = P.perm_profile_read()
    finally:
        P.perm_profile_enable(False)
    assert got == want == native.per_int(A)
    assert prof.int_plain_layers == K - 1  # layers 2..K


def test_int_plain_layers_computed_once_for_many_primes(P):
    """A 0/1 matrix of order 33 needs four primes, more than one sweep
    carries: the plain layers (2..21 here) run once and serve every prime."""
    n = 33
    A = inputs.bernoulli01(n, seed=5)
    P.perm_profile_enable(True)
    try:
        P.perm_profile_read()
        got = P.perm_solve(A)
        prof = P.perm_profile_read()
    finally:
        P.perm_profile_enable(False)
    assert got == P.perm_ryser(A)
    B, K = 1, 0
    for k in range(1, n + 1):
        row = np.abs(A[k - 1])
        B *= min(int(row.sum()), k * int(row.max()))
        if B > 2 ** 63 - 1:
            break
        K = k
    assert prof.int_plain_layers == K - 1, (prof.int_plain_layers, K)


def test_int_closed_forms_n30(P):
    n = 30
    J = np.ones((n, n), dtype=np.int64)
    I = np.eye(n, dtype=np.int64)
    d = [1, 0]
    for k in range(2, n + 1):
        d.append((k - 1) * (d[-1] + d[-2]))
    print("[gpu] int n=30 closed forms", flush=True)
    assert P.perm_solve(J) == math.factorial(n) == 265252859812191058636308480000000
    assert P.perm_solve(J - I) == d[n] == 97581073836835777732377428235481
    assert P.perm_solve(I) == 1
    assert P.perm_solve(-J) == math.factorial(n)  # (-1)^30 * 30!
    T = np.triu(inputs.uniform_int(n, 1, 3, seed=4))
    assert P.perm_solve(T) == math.prod(int(x) for x in np.diag(T))


def test_int_invariances_and_small_workspace(P):
    n = 18
    A = inputs.uniform_int(n, -30, 30, seed=8)
    ref = native.per_int(A)
    rng = np.random.default_rng(2)
    assert P.perm_solve(np.ascontiguousarray(A[rng.permutation(n)])) == ref
    assert P.perm_solve(np.ascontiguousarray(A[:, rng.permutation(n)])) == ref
    assert P.perm_solve(np.ascontiguousarray(A.T)) == ref
    B = A.copy()
    B[3] *= -5
    assert P.perm_solve(B) == -5 * ref
    # a workspace that holds one prime's tables only: more sweeps, same value
    from math import comb
    one = P.perm_workspace_bytes(P.PERM_INT64, n) - 2 * 2 * 8 * max(comb(n, k) for k in range(n + 1)) + 1024
    assert P.perm_solve(A, workspace=P.device_buffer(one)) == ref


@pytest.mark.parametrize("n,c", [(16, 1), (20, 1), (22, 1), (24, 3), (24, 7), (21, 2)])
def test_int_plain_prefix_switch(P, n, c):
    """c * J with row signs: every stored value of layer k is +-k! c^k, equal
    to the bound that decides how many layers run in plain 64-bit arithmetic
    before the residues take over (all layers for 1 * J_16 and 1 * J_20, up to
    k = 20 for 1 * J_22, k = 14 for 3 * J, k = 12 for 7 * J, k = 16 for 2 * J), so a layer
    taken past the bound would overflow and show."""
    sign = np.where(np.arange(n) % 3 == 1, -1, 1).astype(np.int64)
    A = c * np.ones((n, n), dtype=np.int64) * sign[:, None]
    want = math.factorial(n) * c ** n * int(np.prod(sign))
    print(f"[gpu] int plain prefix n={n} c={c}", flush=True)
    assert P.perm_solve(A) == want
    B = inputs.uniform_int(n, -c, c, seed=n + c)
    assert P.perm_solve(B) == native.per_int(B)


@pytest.mark.parametrize("n", [20, 24])
def test_int_plain_layer_width_variants(P, n):
    """Bit 1 of layer_flags widens the low window of the plain 64-bit layers
    only: every width gives the same exact value."""
    A01 = inputs.bernoulli01(n, seed=3)
    A9 = inputs.uniform_int(n, 0, 9, seed=3)
    want = (native.per_int(A01), native.per_int(A9))
    saved = P.perm_tuning_get()
    try:
        for t in range(max(1, n - 22), 15):
            for flags in (0, 2, 3):
                tu = P.perm_tuning_t.from_buffer_copy(saved)
                tu.layer_t[n] = t
                tu.layer_flags[n] = flags
                P.perm_tuning_set(tu)
                assert (P.perm_solve(A01), P.perm_solve(A9)) == want, (n, t, flags)
    finally:
        P.perm_tuning_set(saved)


def test_cache_aware_tile_order(P, golden):
    """Bit 2 of layer_flags (tiles that share high windows dealt to one XCD
    together) changes only which workgroup computes which tile: complex
    results stay bitwise equal to the oracle's chain, integer results exact,
    for every low-window width, XCD run length and thin-tile threshold tried
    and at the full sizes under the shipped tuning table."""
    import os
    saved = P.perm_tuning_get()
    try:
        for n in (16, 20, 22):
            A = inputs.complex_gaussian(n, seed=40 + n)
            ref = c_bits(native.per_c128(A))
            for t in sorted({max(2, n - 18), n - 12, 8, 10, 12}):
                for remap, thin in ((0, 0), (1, -1), (64, 16), (256, 0)):
                    tu = P.perm_tuning_t.from_buffer_copy(saved)
                    tu.layer_t[n] = t
                    tu.layer_xcd_remap[n] = remap
                    tu.layer_thin[n] = thin
                    tu.layer_flags[n] = 4
                    P.perm_tuning_set(tu)
                    print(f"[gpu] tile order n={n} t={t} remap={remap} thin={thin}", flush=True)
                    assert c_bits(P.perm_solve(A)) == ref, (n, t, remap, thin)
        A = inputs.uniform_int(22, 0, 9, seed=8)
        want = native.per_int(A)
        for flags in (4, 6):
            tu = P.perm_tuning_t.from_buffer_copy(saved)
            tu.layer_flags[22] = flags
            P.perm_tuning_set(tu)
            assert P.perm_solve(A) == want, flags
        path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "paper_1802_02779_amd", "tuning", "gfx950.json")
        if P.perm_tuning_load(path) != 0:
            pytest.skip("the shipped tuning table is for another GPU key")
        tu = P.perm_tuning_get()
        for n in range(23, 31):
            tu.layer_flags[n] |= 4
        P.perm_tuning_set(tu)
        for key, n, seed in FULL_COMPLEX:
            g = golden[key]
            print(f"[gpu] tile order full size {key}", flush=True)
            z = P.perm_solve(inputs.complex_gaussian(n, seed=seed))
            assert c_bits(z) == (int(g["re_bits"], 16), int(g["im_bits"], 16)), key
        for n in (25, 27, 29, 30):
            print(f"[gpu] tile order int n={n}", flush=True)
            assert P.perm_solve(inputs.bernoulli01(n, seed=0)) == int(golden[f"int_n{n}_bern_s0"]["value"])
    finally:
        P.perm_tuning_set(saved)


def test_full_sizes_under_shipped_tuning(P, golden):
    """The timed workloads in the configuration bench.py times: the shipped
    tuning table loaded, device-resident complex solves (n = 26, 28) and the
    n = 30 0/1 exact solve, against the stored oracle values."""
    import os
    import torch
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_1802_02779_amd", "tuning", "gfx950.json")
    saved = P.perm_tuning_get()
    try:
        if P.perm_tuning_load(path) != 0:
            pytest.skip("the shipped tuning table is for another GPU key")
        for key, n, _ in FULL_COMPLEX:
            g = golden[key]
            A = inputs.complex_gaussian(n, seed=int(key.rsplit("_s", 1)[1]))
            d_a = torch.from_numpy(A).cuda()
            d_r = torch.zeros(1, dtype=torch.complex128, device="cuda")
            ws = P.device_buffer(P.perm_workspace_bytes(P.PERM_COMPLEX128, n))
            print(f"[gpu] shipped tuning {key}", flush=True)
            for _ in range(2):
                P.perm_solve_async(n, d_a, n, d_r, ws)
            z = complex(d_r.cpu().numpy()[0])
            assert c_bits(z) == (int(g["re_bits"], 16), int(g["im_bits"], 16)), key
            del ws
        for n in (25, 27, 29, 30):
            print(f"[gpu] shipped tuning int n={n}", flush=True)
            assert P.perm_solve(inputs.bernoulli01(n, seed=0)) == int(golden[f"int_n{n}_bern_s0"]["value"])
    finally:
        P.perm_tuning_set(saved)
        torch.cuda.empty_cache()


def test_concurrent_solves_on_separate_streams(P, golden):
    """perm_solve_async is re-entrant with distinct workspaces and streams:
    four host threads queue different matrices (n = 20..26) on their own
    streams at the same time; every result equals the same matrix solved
    alone, bit for bit."""
    import threading
    import torch
    ns = [20, 23, 24, 26]
    mats = [inputs.complex_gaussian(n, seed=500 + n) for n in ns]
    alone = [c_bits(P.perm_solve(A)) for A in mats]
    streams = [torch.cuda.Stream() for _ in ns]
    d_a = [torch.from_numpy(A).cuda() for A in mats]
    d_r = [torch.zeros(1, dtype=torch.complex128, device="cuda") for _ in ns]
    ws = [P.device_buffer(P.perm_workspace_bytes(P.PERM_COMPLEX128, n)) for n in ns]
    torch.cuda.synchronize()
    errors = []

    def work(i):
        try:
            for _ in range(3):
                P.perm_solve_async(ns[i], d_a[i], ns[i], d_r[i], ws[i], stream=streams[i])
            streams[i].synchronize()
        except Exception as e:  # noqa: BLE001 -- reported below
            errors.append(e)

    print("[gpu] four concurrent solves", flush=True)
    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(ns))]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    for i in range(len(ns)):
        assert c_bits(complex(d_r[i].cpu().numpy()[0])) == alone[i], ns[i]
