"""The C-ABI library loads and exports every entry point include/perm.h
declares; host-only behaviour that needs no GPU.  CPU only."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import exact

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "perm.h")


@pytest.fixture(scope="module")
def perm():
    from paper_1802_02779_amd import perm as p
    if not os.path.exists(p.LIB_PATH):
        from paper_1802_02779_amd import build
        build.build()
    p.lib()
    return p


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(perm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    fns = header_functions()
    for name in ("perm_solve", "perm_solve_batch", "perm_server_submit", "perm_server_poll",
                 "perm_workspace_bytes", "perm_last_error"):
        assert name in fns


def test_library_exports_every_declared_symbol(perm):
    L = perm.lib()
    missing = [f for f in header_functions() if not hasattr(L, f)]
    assert not missing, missing
    assert sorted(perm.EXPORTS) == header_functions()


def test_primes_match_oracle(perm):
    ours = [perm.perm_prime(i) for i in range(perm.PERM_MAX_PRIMES)]
    assert ours == exact.primes_61(perm.PERM_MAX_PRIMES)
    with pytest.raises(perm.PermError):
        perm.perm_prime(perm.PERM_MAX_PRIMES)


def test_workspace_bytes(perm):
    from math import comb
    for n in range(2, 35):
        b = perm.perm_workspace_bytes(perm.PERM_COMPLEX128, n)
        maxc = max(comb(n, k) for k in range(n + 1))
        tables = 2 * 16 * maxc
        assert b >= tables + 16 * n * n
        assert b < tables + 16 * n * n + 4096
        bi = perm.perm_workspace_bytes(perm.PERM_INT64, n)
        assert bi >= 2 * 3 * 8 * maxc
    assert perm.perm_workspace_bytes(perm.PERM_COMPLEX128, 35) == 0
    assert perm.perm_workspace_bytes(perm.PERM_COMPLEX128, -1) == 0
    assert perm.perm_workspace_bytes(7, 5) == 0
    # n = 28 complex: two layer tables of C(28,14) entries, about 1.28 GB
    assert abs(perm.perm_workspace_bytes(perm.PERM_COMPLEX128, 28) - 2 * 16 * comb(28, 14)) < 1e5


def test_argument_errors_before_any_device_work(perm):
    L = perm.lib()
    out = perm.perm_c128_t()
    a = np.zeros((35, 35), dtype=np.complex128)
    assert L.perm_solve(1, 35, a.ctypes.data, 35, ctypes.byref(out), None, 0, None) == perm.PERM_ERANGE
    assert "35" in perm.perm_last_error()
    assert L.perm_solve(1, -1, a.ctypes.data, 35, ctypes.byref(out), None, 0, None) == perm.PERM_EINVAL
    assert L.perm_solve(1, 3, None, 3, ctypes.byref(out), None, 0, None) == perm.PERM_EINVAL
    assert L.perm_solve(1, 3, a.ctypes.data, 2, ctypes.byref(out), None, 0, None) == perm.PERM_EINVAL
    assert L.perm_solve(5, 3, a.ctypes.data, 3, ctypes.byref(out), None, 0, None) == perm.PERM_EINVAL
    assert L.perm_solve(1, 5, a.ctypes.data, 5, ctypes.byref(out), None, 0, None) == perm.PERM_ENOMEM
    assert L.perm_solve_async(35, None, 35, None, None, 0, None) == perm.PERM_ERANGE
    assert L.perm_solve_async(3, None, 3, None, None, 0, None) == perm.PERM_EINVAL
    ns = np.array([3, 13], dtype=np.int32)
    offs = np.array([0, 9], dtype=np.int64)
    dummy = ctypes.c_char * 16
    buf = dummy()
    assert L.perm_solve_batch(1, 2, ns.ctypes.data, offs.ctypes.data, ctypes.addressof(buf),
                              ctypes.addressof(buf), ctypes.addressof(buf), 16, None, 0) == perm.PERM_ERANGE
    assert L.perm_solve_batch(1, 1, ns.ctypes.data, offs.ctypes.data, ctypes.addressof(buf),
                              ctypes.addressof(buf), ctypes.addressof(buf), 16, None, 0x80) == perm.PERM_EINVAL


def test_trivial_orders_without_device(perm):
    # n = 0 and n = 1 are answered on the host: empty product and a[0][0]
    L = perm.lib()
    out = perm.perm_c128_t()
    a = np.array([[2.5 - 1.0j]], dtype=np.complex128)
    assert L.perm_solve(1, 0, None, 1, ctypes.byref(out), None, 0, None) == 0
    assert (out.re, out.im) == (1.0, 0.0)
    assert L.perm_solve(1, 1, a.ctypes.data, 1, ctypes.byref(out), None, 0, None) == 0
    assert (out.re, out.im) == (2.5, -1.0)
    oi = perm.perm_int_t()
    ai = np.array([[-(2 ** 63)]], dtype=np.int64)
    assert L.perm_solve(0, 1, ai.ctypes.data, 1, ctypes.byref(oi), None, 0, None) == 0
    assert oi.value() == -(2 ** 63)
    assert L.perm_solve(0, 0, None, 1, ctypes.byref(oi), None, 0, None) == 0
    assert oi.value() == 1


def test_tuning_validation(perm):
    t = perm.perm_tuning_get()
    saved = perm.perm_tuning_t.from_buffer_copy(t)
    t.layer_t[20] = 16
    with pytest.raises(perm.PermError):
        perm.perm_tuning_set(t)
    t = perm.perm_tuning_t.from_buffer_copy(saved)
    t.batch_group[10] = 48
    with pytest.raises(perm.PermError):
        perm.perm_tuning_set(t)
    t = perm.perm_tuning_t.from_buffer_copy(saved)
    t.layer_flags[24] = 8  # only bits 0, 1 and 2 are defined
    with pytest.raises(perm.PermError):
        perm.perm_tuning_set(t)
    t = perm.perm_tuning_t.from_buffer_copy(saved)
    t.layer_t[28] = 13
    t.layer_flags[28] = 7
    t.batch_group[12] = 128
    perm.perm_tuning_set(t)
    assert perm.perm_tuning_get().layer_t[28] == 13
    assert perm.perm_tuning_get().layer_flags[28] == 7
    perm.perm_tuning_set(saved)


def test_perm_int_t_decoding(perm):
    v = perm.perm_int_t()
    v.sign = -1
    v.nlimbs = 2
    v.limb[0] = 5
    v.limb[1] = 3
    assert v.value() == -(3 * 2 ** 64 + 5)


def test_server_config_validation(perm):
    L = perm.lib()
    h = ctypes.c_void_p()
    cfg = perm.perm_server_config_t(None, 0, 0, 1, 1, 12, 1)
    assert L.perm_server_create(ctypes.byref(cfg), ctypes.byref(h)) == perm.PERM_EINVAL
    buf = (ctypes.c_char * 1024)()
    for bad in (dict(max_large_slots=0), dict(queue_capacity=0), dict(small_n_max=13),
                dict(max_small_batch=0), dict(budget_bytes=4096)):
        kw = dict(pool=ctypes.addressof(buf), pool_bytes=1024, budget_bytes=0, max_large_slots=1,
                  queue_capacity=4, small_n_max=12, max_small_batch=4)
        kw.update(bad)
        cfg = perm.perm_server_config_t(**kw)
        assert L.perm_server_create(ctypes.byref(cfg), ctypes.byref(h)) == perm.PERM_EINVAL, bad
    assert L.perm_server_create(None, ctypes.byref(h)) == perm.PERM_EINVAL
    assert L.perm_server_destroy(None) == perm.PERM_EINVAL
    assert L.perm_server_poll(None, 1, None, None) == perm.PERM_EINVAL


def test_tuning_file_optional_arrays(perm, tmp_path):
    # perm_tuning_load checks the device key first, so only the CPU-side
    # parser behaviour that needs no device is exercised here: a missing file
    assert perm.perm_tuning_load(str(tmp_path / "missing.json")) == perm.PERM_ENOTFOUND
