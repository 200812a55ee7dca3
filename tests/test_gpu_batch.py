"""GPU parity of perm_solve_batch (persistent on-chip kernel, graph replay)."""
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


def c_bits_arr(z):
    z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128))
    return z.view(np.uint64).reshape(-1, 2)


def run_batch(P, batch, flags=0, ws=None, results=None):
    import torch
    d_mats = torch.from_numpy(batch.mats).cuda()
    if results is None:
        results = torch.zeros(batch.count, dtype=torch.complex128, device="cuda")
    if ws is None:
        ws = P.device_buffer(P.perm_batch_workspace_bytes(P.PERM_COMPLEX128, batch.ns))
    P.perm_solve_batch(P.PERM_COMPLEX128, batch.ns, batch.offsets, d_mats, results, ws,
                       flags=flags | P.PERM_BATCH_SYNC)
    return results.cpu().numpy(), d_mats, results, ws


def oracle_bits(batch):
    out = np.empty(batch.count, dtype=np.complex128)
    for i in range(batch.count):
        out[i] = native.per_c128(batch.matrix(i), mode=native.MODE_MEMO)
    return c_bits_arr(out)


def test_batch_mixed_orders_bitwise(P):
    U = inputs.haar_unitary(64, seed=11)
    b = inputs.submatrix_batch(U, 3000, 0, 12, seed=1)
    print("[gpu] batch 3000 mixed n=0..12", flush=True)
    got, *_ = run_batch(P, b)
    assert (c_bits_arr(got) == oracle_bits(b)).all()


def test_batch_equals_single_solve(P):
    U = inputs.haar_unitary(64, seed=12)
    b = inputs.submatrix_batch(U, 200, 3, 12, seed=2)
    got, *_ = run_batch(P, b)
    for i in range(0, 200, 7):
        assert (c_bits_arr([P.perm_solve(b.matrix(i))]) == c_bits_arr([got[i]])).all()


def test_batch_single_order_each(P):
    U = inputs.haar_unitary(64, seed=13)
    for n in range(0, 13):
        b = inputs.submatrix_batch(U, 97, n, n, seed=n)
        got, *_ = run_batch(P, b)
        assert (c_bits_arr(got) == oracle_bits(b)).all(), n


def test_batch_graph_replays(P):
    import torch
    U = inputs.haar_unitary(64, seed=14)
    b = inputs.submatrix_batch(U, 5000, 3, 12, seed=3)
    ref = oracle_bits(b)
    got, d_mats, results, ws = run_batch(P, b, flags=P.PERM_BATCH_GRAPH)
    assert (c_bits_arr(got) == ref).all()
    for rep in range(4):
        results.zero_()  # eager work between replays
        torch.cuda.synchronize()
        P.perm_solve_batch(P.PERM_COMPLEX128, b.ns, b.offsets, d_mats, results, ws,
                           flags=P.PERM_BATCH_GRAPH | P.PERM_BATCH_REUSE | P.PERM_BATCH_SYNC)
        assert (c_bits_arr(results.cpu().numpy()) == ref).all(), rep


def test_batch_group_variants(P):
    U = inputs.haar_unitary(64, seed=15)
    b = inputs.submatrix_batch(U, 600, 3, 12, seed=4)
    ref = oracle_bits(b)
    saved = P.perm_tuning_get()
    try:
        for g in (16, 32, 64, 128, 256, 512):
            t = P.perm_tuning_t.from_buffer_copy(saved)
            for n in range(13):
                t.batch_group[n] = g
            P.perm_tuning_set(t)
            got, *_ = run_batch(P, b)
            assert (c_bits_arr(got) == ref).all(), g
    finally:
        P.perm_tuning_set(saved)


def test_batch_empty(P):
    import torch
    ws = P.device_buffer(256)
    res = torch.zeros(1, dtype=torch.complex128, device="cuda")
    P.perm_solve_batch(P.PERM_COMPLEX128, np.zeros(0, np.int32), np.zeros(0, np.int64),
                       res, res, ws, flags=P.PERM_BATCH_SYNC)


def test_batch_int64(P):
    rng = np.random.default_rng(21)
    ns = rng.integers(0, 13, size=300).astype(np.int32)
    offsets = np.zeros(300, dtype=np.int64)
    offsets[1:] = np.cumsum(ns.astype(np.int64) ** 2)[:-1]
    mats = np.empty(int((ns.astype(np.int64) ** 2).sum()), dtype=np.int64)
    for i, n in enumerate(ns):
        lo, hi = (-(2 ** 63), 2 ** 63 - 1) if i % 5 == 0 else (-50, 50)
        mats[offsets[i]:offsets[i] + n * n] = rng.integers(lo, hi, size=n * n, dtype=np.int64, endpoint=True)
    ws = P.device_buffer(P.perm_batch_workspace_bytes(P.PERM_INT64, ns))
    print("[gpu] int batch 300", flush=True)
    got = P.perm_solve_batch(P.PERM_INT64, ns, offsets, mats, None, ws)
    for i, n in enumerate(ns):
        A = mats[offsets[i]:offsets[i] + n * n].reshape(n, n)
        ref = exact.per_definition(A) if n <= 6 else native.per_int(A)
        assert got[i] == ref, (i, n)


def test_batch_full_size_sampled(P):
    """The timed workload at full size (2^20 submatrices of order 3..12 of the
    seeded 64x64 Haar unitary, one graph launch, then a replay): 1500 sampled
    outputs, plus the first and last of every order, bitwise equal to the
    oracle's; the replay bitwise equal to the first launch."""
    import torch
    count = 1 << 20
    U = inputs.haar_unitary(64, seed=2018)
    b = inputs.submatrix_batch(U, count, 3, 12, seed=1)
    print("[gpu] batch 2^20 full size", flush=True)
    got, d_mats, results, ws = run_batch(P, b, flags=P.PERM_BATCH_GRAPH)
    rng = np.random.default_rng(7)
    idx = set(rng.choice(count, size=1500, replace=False).tolist())
    for n in range(3, 13):
        where = np.flatnonzero(b.ns == n)
        idx.update([int(where[0]), int(where[-1])])
    idx = sorted(idx)
    ref = c_bits_arr([native.per_c128(b.matrix(i), mode=native.MODE_MEMO) for i in idx])
    assert (c_bits_arr(got[idx]) == ref).all()
    results.zero_()
    torch.cuda.synchronize()
    P.perm_solve_batch(P.PERM_COMPLEX128, b.ns, b.offsets, d_mats, results, ws,
                       flags=P.PERM_BATCH_GRAPH | P.PERM_BATCH_REUSE | P.PERM_BATCH_SYNC)
    assert (c_bits_arr(results.cpu().numpy()) == c_bits_arr(got)).all()
    del d_mats, results, ws
    torch.cuda.empty_cache()


def test_batch_full_size_every_output_digest(P):
    """Every one of the 2^20 outputs of the timed workload against the
    oracle: results start as NaN (a skipped matrix would stay NaN), the
    graph launch fills them, and the SHA-256 of all results (little-endian
    complex128, batch order) must equal the digest the oracle's results gave
    (tests/golden/make_large_configs.py); per-order digests name the order
    on a mismatch.  A replay after eager work gives the same digest."""
    import hashlib
    import json
    import os
    import torch
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large_configs.json")) as f:
        g = json.load(f)["batch_2p20_s2018_s1"]
    count = 1 << 20
    U = inputs.haar_unitary(64, seed=2018)
    b = inputs.submatrix_batch(U, count, 3, 12, seed=1)
    assert g["count"] == count
    results = torch.full((count,), float("nan"), dtype=torch.complex128, device="cuda")
    print("[gpu] batch 2^20 digest", flush=True)
    got, d_mats, results, ws = run_batch(P, b, flags=P.PERM_BATCH_GRAPH, results=results)

    def check(arr):
        assert not np.isnan(arr.view(np.float64)).any()
        if hashlib.sha256(np.ascontiguousarray(arr).astype("<c16").tobytes()).hexdigest() != g["sha256"]:
            bad = [n for n in range(3, 13)
                   if hashlib.sha256(np.ascontiguousarray(arr[b.ns == n]).astype("<c16").tobytes()).hexdigest()
                   != g["sha256_by_order"][str(n)]]
            raise AssertionError(f"batch results differ from the oracle's for orders {bad}")

    check(got)
    results.fill_(float("nan"))
    torch.cuda.synchronize()
    P.perm_solve_batch(P.PERM_COMPLEX128, b.ns, b.offsets, d_mats, results, ws,
                       flags=P.PERM_BATCH_GRAPH | P.PERM_BATCH_REUSE | P.PERM_BATCH_SYNC)
    check(results.cpu().numpy())
    del d_mats, results, ws
    torch.cuda.empty_cache()
