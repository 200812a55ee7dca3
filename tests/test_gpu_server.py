"""GPU tests of the continuous-batching server (perm_server_*)."""
import time

import numpy as np
import pytest

from oracle import native
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
    return tuple(np.array([z.real, z.imag], dtype=np.float64).view(np.uint64).tolist())


def wait_all(P, srv, tickets, timeout=60.0):
    out = {}
    t0 = time.time()
    pending = set(tickets)
    while pending:
        for t in list(pending):
            r = P.perm_server_poll(srv, t)
            if r is not None:
                out[t] = r
                pending.discard(t)
        assert time.time() - t0 < timeout, f"{len(pending)} requests still pending"
        time.sleep(0.0005)
    return out


def test_results_alone_equal_results_in_mix(P):
    U = inputs.haar_unitary(64, seed=31)
    rng = np.random.default_rng(31)
    ns = list(rng.integers(5, 13, size=60)) + list(rng.integers(18, 25, size=8))
    rng.shuffle(ns)
    mats = []
    for n in ns:
        r, c = rng.permutation(64)[:n], rng.permutation(64)[:n]
        mats.append(np.ascontiguousarray(U[np.ix_(r, c)]))
    pool = P.device_buffer(2 << 30)
    srv = P.perm_server_create(pool, max_large_slots=2, queue_capacity=1000, small_n_max=12, max_small_batch=16)
    try:
        print("[gpu] server mix of 68 requests", flush=True)
        tickets = [P.perm_server_submit(srv, A) for A in mats]
        res = wait_all(P, srv, tickets)
    finally:
        P.perm_server_destroy(srv)
    for t, A in zip(tickets, mats):
        z, st = res[t]
        assert st.status == 0 and st.n == A.shape[0]
        assert st.t_submit <= st.t_admit <= st.t_done
        assert bits(z) == bits(P.perm_solve(A)) == bits(native.per_c128(A))


def test_backpressure_and_footprint_errors(P):
    pool = P.device_buffer(256 << 20)
    A26 = inputs.complex_gaussian(22, seed=1)
    srv = P.perm_server_create(pool, budget_bytes=200 << 20, max_large_slots=1, queue_capacity=3,
                               small_n_max=12, max_small_batch=64)
    try:
        # 16 * 2^24 = 256 MiB > 200 MiB budget
        with pytest.raises(P.PermError) as e:
            P.perm_server_submit(srv, inputs.complex_gaussian(24, seed=0))
        assert e.value.code == P.PERM_ENOMEM
        with pytest.raises(P.PermError) as e:
            P.perm_server_submit(srv, np.zeros((P.PERM_N_MAX + 1, P.PERM_N_MAX + 1), dtype=np.complex128))
        assert e.value.code == P.PERM_ERANGE
        codes, tickets = [], []
        for _ in range(20):
            try:
                tickets.append(P.perm_server_submit(srv, A26))
            except P.PermError as err:
                codes.append(err.code)
        assert codes and all(c == P.PERM_EAGAIN for c in codes)
        res = wait_all(P, srv, tickets)
        ref = bits(P.perm_solve(A26))
        assert all(bits(z) == ref for z, _ in res.values())
        with pytest.raises(P.PermError) as e:
            P.perm_server_poll(srv, tickets[0])  # already consumed
        assert e.value.code == P.PERM_ENOTFOUND
        with pytest.raises(P.PermError) as e:
            P.perm_server_poll(srv, 10 ** 9)
        assert e.value.code == P.PERM_ENOTFOUND
    finally:
        P.perm_server_destroy(srv)


def test_budget_admits_one_large_at_a_time(P):
    n = 22
    pool = P.device_buffer(1 << 30)
    charge = 16 << n
    srv = P.perm_server_create(pool, budget_bytes=int(1.5 * charge), max_large_slots=4, queue_capacity=64,
                               small_n_max=12, max_small_batch=64)
    mats = [inputs.complex_gaussian(n, seed=s) for s in range(6)]
    try:
        tickets = [P.perm_server_submit(srv, A) for A in mats]
        res = wait_all(P, srv, tickets)
    finally:
        P.perm_server_destroy(srv)
    spans = sorted((res[t][1].t_start, res[t][1].t_done) for t in tickets)
    for (s0, d0), (s1, d1) in zip(spans, spans[1:]):
        assert s1 >= d0, "two requests ran together although the budget holds one"
    for t, A in zip(tickets, mats):
        assert bits(res[t][0]) == bits(native.per_c128(A))


def test_destroy_with_pending_requests(P):
    pool = P.device_buffer(512 << 20)
    srv = P.perm_server_create(pool, max_large_slots=1, queue_capacity=100, small_n_max=12, max_small_batch=8)
    for s in range(20):
        P.perm_server_submit(srv, inputs.complex_gaussian(24, seed=s))
    t0 = time.time()
    P.perm_server_destroy(srv)
    assert time.time() - t0 < 30


def test_large_orders_overlap_and_match_stored_values(P):
    """Six large requests (n = 25..28) admitted together into a 16 GiB pool
    (carve-outs reach past 4 GiB), mixed with small ones: each result is
    bitwise the stored oracle value (or, for the seeds without one, the same
    matrix solved alone), and requests really are in flight together."""
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large_configs.json")) as f:
        golden = json.load(f)
    reqs = [(28, 0), (28, 1), (28, 2), (27, 0), (26, 1), (25, 0)]
    mats = [inputs.complex_gaussian(n, seed=s) for n, s in reqs]
    refs = []
    for (n, s), A in zip(reqs, mats):
        g = golden.get(f"c128_n{n}_s{s}")
        refs.append((int(g["re_bits"], 16), int(g["im_bits"], 16)) if g else bits(P.perm_solve(A)))
    U = inputs.haar_unitary(64, seed=41)
    rng = np.random.default_rng(41)
    small = []
    for n in rng.integers(5, 13, size=24):
        r, c = rng.permutation(64)[:n], rng.permutation(64)[:n]
        small.append(np.ascontiguousarray(U[np.ix_(r, c)]))
    pool = P.device_buffer(16 << 30)
    srv = P.perm_server_create(pool, max_large_slots=6, queue_capacity=100, small_n_max=12, max_small_batch=8)
    try:
        print("[gpu] server: 6 large (n=25..28) + 24 small", flush=True)
        tl = [P.perm_server_submit(srv, A) for A in mats]
        ts = [P.perm_server_submit(srv, A) for A in small]
        res = wait_all(P, srv, tl + ts, timeout=120.0)
    finally:
        P.perm_server_destroy(srv)
        del pool
    for t, (n, s), ref in zip(tl, reqs, refs):
        z, st = res[t]
        assert st.status == 0 and st.n == n
        assert bits(z) == ref, (n, s)
    for t, A in zip(ts, small):
        assert bits(res[t][0]) == bits(native.per_c128(A))
    spans = [(res[t][1].t_start, res[t][1].t_done) for t in tl]
    overlapping = sum(1 for i in range(len(spans)) for j in range(i + 1, len(spans))
                      if spans[i][0] < spans[j][1] and spans[j][0] < spans[i][1])
    assert overlapping >= 1, spans
