"""GPU parity of the repeated-column path (perm_solve_multi[_async]) against
the count-vector oracle: complex128 bit for bit (same chain, same scale),
int64 exact.  Shapes span one tile to many tiles and chunks, ragged layer
ends, a single column repeated 64 times, and the stored full-size bunched
workloads (40 photons in 20 detectors: a largest layer of 3.9e7 count
vectors)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import exact, native
from paper_1802_02779_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1802_02779_amd import perm
    perm.lib()
    return perm


def bits(z):
    return np.asarray([z], dtype=np.complex128).view(np.uint64).tolist()


SHAPES = [[2], [1, 2], [2, 1, 1], [3, 3], [1] * 12 + [3], [3] + [1] * 12, [2] * 10, [6, 6, 6], [1, 7, 1, 7, 1],
          [4, 1, 3, 2, 1, 2, 3, 1, 2], [64], [32, 32], [2] * 12 + [1] * 6]


@pytest.mark.parametrize("mult", SHAPES, ids=[str(i) for i in range(len(SHAPES))])
def test_c128_bitwise_equals_oracle(P, mult):
    n = sum(mult)
    A = inputs.complex_gaussian(n, seed=n + len(mult))[:, :len(mult)]
    print(f"[gpu] multi c128 mult={mult}", flush=True)
    got = P.perm_solve_multi(A, mult)
    ref = native.per_multi_c128(A, mult)
    assert bits(got) == bits(ref), (mult, got, ref)


@pytest.mark.parametrize("n,M", [(8, 4), (12, 6), (16, 8), (20, 10), (24, 12), (26, 10), (30, 15)])
def test_c128_bunched_patterns(P, n, M):
    for seed in range(2):
        t = inputs.bunched_pattern(n, M, seed)
        A = inputs.bunched_output(n, t, seed)
        print(f"[gpu] multi c128 bunched n={n} M={M} seed={seed} mult={t.tolist()}", flush=True)
        assert bits(P.perm_solve_multi(A, t)) == bits(native.per_multi_c128(A, t)), (n, M, seed)


@pytest.mark.parametrize("n", [2, 9, 16, 20])
def test_all_ones_is_perm_solve(P, n):
    A = inputs.complex_gaussian(n, seed=50 + n)
    assert bits(P.perm_solve_multi(A, [1] * n)) == bits(P.perm_solve(A))


def test_c128_async_lda_deterministic(P):
    import torch
    t = [3, 1, 2, 4, 1, 2, 3]
    n, m, lda = sum(t), len(t), 11
    A = inputs.bunched_output(n, t, seed=5)
    big = np.zeros((n, lda), dtype=np.complex128)
    big[:, :m] = A
    d_a = torch.from_numpy(big).cuda()
    d_r = torch.zeros(2, dtype=torch.complex128, device="cuda")
    ws = P.device_buffer(P.perm_multi_workspace_bytes(P.PERM_COMPLEX128, t))
    P.perm_solve_multi_async(n, t, d_a, lda, d_r[0:1], ws)
    P.perm_solve_multi_async(n, t, d_a, lda, d_r[1:2], ws)
    r = d_r.cpu().numpy()
    assert bits(r[0]) == bits(r[1])
    assert bits(r[0]) == bits(native.per_multi_c128(A, t))
    small = P.device_buffer(64)
    with pytest.raises(P.PermError) as e:
        P.perm_solve_multi(A, t, workspace=small)
    assert e.value.code == -3  # PERM_ENOMEM


def test_c128_small_gaussian_integers_exact(P):
    rng = np.random.default_rng(77)
    for t in ([3, 2, 1], [2, 2, 2, 2], [5, 1, 4]):
        n, m = sum(t), len(t)
        A = (rng.integers(-1, 2, size=(n, m)) + 1j * rng.integers(-1, 2, size=(n, m))).astype(np.complex128)
        q = exact.per_multi_exact(A, t)
        assert P.perm_solve_multi(A, t) == complex(float(q.re), float(q.im)), t


@pytest.mark.parametrize("key,n,M", [("multi_c128_n36_M18_s0", 36, 18), ("multi_c128_n40_M20_s0", 40, 20)])
def test_c128_full_size_stored(P, golden_dir, key, n, M):
    cfg = json.load(open(os.path.join(golden_dir, "large_configs.json")))[key]
    t = inputs.bunched_pattern(n, M, 0)
    assert t.tolist() == cfg["mult"]
    A = inputs.bunched_output(n, t, 0)
    print(f"[gpu] multi c128 {key}", flush=True)
    got = P.perm_solve_multi(A, t)
    assert bits(got) == [int(cfg["re_bits"], 16), int(cfg["im_bits"], 16)]


# ------------------------------------------------------------------ int64
@pytest.mark.parametrize("mult", [[2, 1], [3, 3], [2] * 8, [4, 1, 3, 2, 1, 2, 3], [1] * 9 + [4], [20], [5, 5, 5, 5]])
def test_int_exact_vs_oracle(P, mult):
    rng = np.random.default_rng(sum(mult) * 7 + len(mult))
    n, m = sum(mult), len(mult)
    A = rng.integers(-9, 10, size=(n, m), dtype=np.int64)
    print(f"[gpu] multi int mult={mult}", flush=True)
    assert P.perm_solve_multi(A, mult) == native.per_multi_int(A, mult), mult


def test_int_extreme_entries(P):
    rng = np.random.default_rng(83)
    for t in ([2, 1], [1, 3, 1], [6]):
        n = sum(t)
        A = rng.integers(-(2 ** 63), 2 ** 63 - 1, size=(n, len(t)), dtype=np.int64, endpoint=True)
        A[0, 0] = -(2 ** 63)
        assert P.perm_solve_multi(A, t) == exact.per_multi_exact(A, t), t


def test_int_closed_forms(P):
    t = inputs.bunched_pattern(40, 20, 0)
    n = 40
    assert P.perm_solve_multi(np.ones((n, len(t)), dtype=np.int64), t) == math.factorial(n)
    col = np.arange(1, 41, dtype=np.int64).reshape(40, 1) % 5 + 1
    assert P.perm_solve_multi(col, [40]) == math.factorial(40) * math.prod(int(v) for v in col[:, 0])


def test_int_full_size_stored(P, golden_dir):
    cfg = json.load(open(os.path.join(golden_dir, "large_configs.json")))["multi_int_n36_M18_bern_s0"]
    t = inputs.bunched_pattern(36, 18, 0)
    B = inputs.bernoulli01(36, seed=0)[:, :len(t)]
    print("[gpu] multi int n=36", flush=True)
    assert str(P.perm_solve_multi(B, t)) == cfg["value"]


# ------------------------------------------------------- maximum sizes
U64 = 2.0 ** -53
BIG = [2] * 20 + [1] * 2  # n = 42, largest layer 1.48e9 count vectors (47 GB of layer pair)


def chain_error_bound(n):
    e = 0.0
    for k in range(2, n + 1):
        g = 2 * k * U64 / (1 - 2 * k * U64)
        e = e + math.sqrt(2.0) * g * (1 + e)
    return e


def test_c128_rank_one_largest_layers(P):
    """Rank one u v^T: per = n! prod u_i prod v_j^mult[j]; per(|A|) = |per|,
    so the chain bound applies relative to |per| (plus the rounding of the
    scale and of the reference itself)."""
    import torch
    n, m = sum(BIG), len(BIG)
    rng = np.random.default_rng(42)
    u = np.exp(1j * rng.uniform(0, 2 * np.pi, n)) * rng.uniform(0.8, 1.2, n)
    v = np.exp(1j * rng.uniform(0, 2 * np.pi, m)) * rng.uniform(0.8, 1.2, m)
    A = np.outer(u, v)
    print(f"[gpu] multi c128 rank one n={n} m={m}", flush=True)
    z = P.perm_solve_multi(A, BIG)
    torch.cuda.empty_cache()
    ref = math.factorial(n) * np.prod(u) * np.prod(v ** np.array(BIG))
    assert abs(z - ref) <= (chain_error_bound(n) + (4 * n + 8) * U64) * abs(ref)


def test_int_all_ones_largest_layers(P):
    import torch
    n, m = sum(BIG), len(BIG)
    print(f"[gpu] multi int all-ones n={n} m={m}", flush=True)
    assert P.perm_solve_multi(np.ones((n, m), dtype=np.int64), BIG) == math.factorial(n)
    torch.cuda.empty_cache()


def test_plan_cache_eviction_on_device(P):
    """More distinct shapes than the plan cache holds, twice over: plans are
    dropped (after a device synchronization) and rebuilt; every result stays
    bitwise equal to the oracle."""
    shapes = [[2] * k + [1, 3] for k in range(1, 11)] + [[3] * k + [2] for k in range(1, 9)]  # 18 > 16
    for rep in range(2):
        for t in shapes:
            n = sum(t)
            A = inputs.complex_gaussian(n, seed=n)[:, :len(t)]
            assert bits(P.perm_solve_multi(A, t)) == bits(native.per_multi_c128(A, t)), (rep, t)


# ----------------------------------------------------- rows and columns
@pytest.mark.parametrize("rm,cm", [([2, 1, 3], [1, 1, 1, 1, 1, 1]), ([1] * 6, [3, 3]), ([2, 2], [2, 1, 1]),
                                   ([4, 1, 1], [2, 2, 2])])
def test_bunched_rows_and_columns(P, rm, cm):
    """Repeated rows and columns: exact integers equal eq. (1) on the fully
    expanded matrix; complex equals the oracle's chain in the orientation the
    rule picks, bit for bit."""
    rng = np.random.default_rng(sum(rm) * 10 + len(rm))
    A = rng.integers(-4, 5, size=(len(rm), len(cm)), dtype=np.int64)
    full = np.repeat(np.repeat(A, rm, axis=0), cm, axis=1)
    assert P.perm_solve_bunched(A, rm, cm) == exact.per_definition(full)
    Z = inputs.complex_gaussian(max(len(rm), len(cm)), seed=7)[:len(rm), :len(cm)]
    got = P.perm_solve_bunched(Z, rm, cm)
    if P.bunched_orientation(rm, cm):
        ref = native.per_multi_c128(np.repeat(Z.T, cm, axis=0), rm)
    else:
        ref = native.per_multi_c128(np.repeat(Z, rm, axis=0), cm)
    assert bits(got) == bits(ref)


@pytest.mark.parametrize("c,t", [(3, [2] * 12), (1, [3] * 8 + [1] * 4), (2, [1] * 6 + [4] * 4)])
def test_int_plain_prefix_switch(P, c, t):
    """c * (an n x m block of ones) with row signs: count vectors whose used
    columns appear once reach the bound that decides how many layers run in
    plain 64-bit arithmetic before the residues take over; the value is
    n! c^n times the signs, and a random block matches the oracle."""
    n, m = sum(t), len(t)
    sign = np.where(np.arange(n) % 4 == 2, -1, 1).astype(np.int64)
    A = c * np.ones((n, m), dtype=np.int64) * sign[:, None]
    print(f"[gpu] multi int plain prefix c={c} mult={t}", flush=True)
    assert P.perm_solve_multi(A, t) == math.factorial(n) * c ** n * int(np.prod(sign))
    rng = np.random.default_rng(n * 7 + c)
    B = rng.integers(-c, c + 1, size=(n, m), dtype=np.int64)
    assert P.perm_solve_multi(B, t) == native.per_multi_int(B, t)
