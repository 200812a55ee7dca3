"""The cache-aware tile order of the layer sweep (host side, CPU only).

Every layer launch with bit 2 of layer_flags reads its tiles from this list,
so each tiled k' group must list every high part T (an m-subset of the
n - t high columns) exactly once, padded to a multiple of 8 slots so that
each of the 8 XCDs gets the same number of workgroups.  A missing or doubled
tile would leave stored values unwritten or race, which the GPU parity tests
catch only at the orders they run; this checks every layer of several orders.
"""
import os
from itertools import combinations
from math import comb

import numpy as np
import pytest

NO_TILE = 0xFFFFFFFF


@pytest.fixture(scope="module")
def perm():
    from paper_1802_02779_amd import perm as p
    if not os.path.exists(p.LIB_PATH):
        from paper_1802_02779_amd import build
        build.build()
    p.lib()
    return p


def tiled_groups(n, t, k, thin=128):
    nh = n - t
    return [(kp, k - kp) for kp in range(max(0, k - nh), min(k, t) + 1) if comb(t, kp) >= thin]


def popcount(a):
    return np.array([bin(int(x)).count("1") for x in a])


@pytest.mark.parametrize("n,t", [(16, 8), (20, 10), (24, 12), (26, 12), (28, 12)])
@pytest.mark.parametrize("value_bytes", [16, 8, 24])
def test_every_group_lists_each_high_part_once(perm, n, t, value_bytes):
    nh = n - t
    for k in range(2, n + 1):
        v = perm.perm_layer_tile_order(n, t, k, value_bytes)
        pos = 0
        for kp, m in tiled_groups(n, t, k):
            c = comb(nh, m)
            slots = (c + 7) // 8 * 8
            seg = v[pos:pos + slots]
            pos += slots
            assert seg.size == slots, (n, k, kp)
            real = seg[seg != NO_TILE]
            assert real.size == c, (n, k, kp, real.size, c)
            assert real.max(initial=0) < (1 << nh)
            assert np.all(popcount(real) == m), (n, k, kp)
            assert np.unique(real).size == c, (n, k, kp)
            # each XCD (slot index mod 8) holds ceil(c / 8) slots, at most one
            # of them empty
            for x in range(8):
                assert np.count_nonzero(seg[x::8] == NO_TILE) <= 1
        assert pos == v.size, (n, k)


def test_first_family_is_the_lowest_z_set(perm):
    """The first family of a group is every m-subset of the lowest z high
    columns (the z-set with the most unprocessed subsets, lowest rank on
    ties), dealt to XCD 0 (the least-loaded, lowest index) in colex order."""
    n, t, k = 28, 12, 14
    nh = n - t
    v = perm.perm_layer_tile_order(n, t, k, 16)
    kp, m = tiled_groups(n, t, k)[3]  # k' = 6, m = 8: windows of C(12, 6) values
    pos = sum((comb(nh, mm) + 7) // 8 * 8 for _, mm in tiled_groups(n, t, k)[:3])
    seg = v[pos:pos + (comb(nh, m) + 7) // 8 * 8]
    # z: the largest with C(z, m - 1) windows of C(t, k') 16-byte values within 16 MiB
    z = max(c for c in range(m + 2, nh) if comb(c, m - 1) * comb(t, kp) * 16 <= 16 << 20)
    first = [sum(1 << c for c in S) for S in combinations(range(z), m)]
    first.sort()
    assert list(seg[0::8][:len(first)]) == first


def test_fallback_keeps_colex_runs(perm):
    """Groups with no room for a family (m + 2 > nh - 1) keep colex order in
    runs of the tuned XCD run length: XCD x takes runs x, x + 8, ..."""
    n, t, run = 28, 12, 256
    nh = n - t
    saved = perm.perm_tuning_get()
    try:
        tu = perm.perm_tuning_t.from_buffer_copy(saved)
        tu.layer_xcd_remap[n] = run
        perm.perm_tuning_set(tu)
        k = 22  # k' = 3..9 gives m = 13..19 > nh - 3 for k' <= 5
        v = perm.perm_layer_tile_order(n, t, k, 16)
    finally:
        perm.perm_tuning_set(saved)
    kp, m = tiled_groups(n, t, k)[0]
    assert m + 2 > nh - 1
    c = comb(nh, m)
    seg = v[:(c + 7) // 8 * 8]
    colex = sorted(sum(1 << x for x in S) for S in combinations(range(nh), m))
    want = [[] for _ in range(8)]
    for i, T in enumerate(colex):
        want[(i // run) % 8].append(T)
    L = (c + 7) // 8
    # lists longer than L give their tail to the shortest ones; compare the
    # untouched prefixes
    for x in range(8):
        got = [int(T) for T in seg[x::8] if T != NO_TILE]
        keep = min(len(want[x]), len(got))
        assert got[:keep] == want[x][:keep], x


def test_rejects_bad_arguments(perm):
    with pytest.raises(RuntimeError):
        perm.perm_layer_tile_order(34, 12, 10)  # 22 high columns: beyond the order's range
    with pytest.raises(RuntimeError):
        perm.perm_layer_tile_order(20, 12, 1)
    with pytest.raises(RuntimeError):
        perm.perm_layer_tile_order(20, 12, 10, 0)
