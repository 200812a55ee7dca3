"""Python binding of libpermgpu (include/perm.h): argument marshalling only.

Every function here has the name of the C entry point it calls and does no
arithmetic of its own: all work of the permanent runs in the library's HIP
kernels.  PyTorch provides device memory (workspaces, device matrices) and
streams.  If ``_lib/libpermgpu.so`` has not been built, :func:`lib` raises --
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libpermgpu.so")

PERM_INT64 = 0
PERM_COMPLEX128 = 1
PERM_N_MAX = 34
PERM_BATCH_N_MAX = 12
PERM_INT_LIMBS = 36
PERM_MULTI_N_MAX = 64
PERM_MAX_PRIMES = 40

PERM_OK = 0
PERM_PENDING = 1
PERM_EINVAL = -1
PERM_ERANGE = -2
PERM_ENOMEM = -3
PERM_EDEVICE = -4
PERM_EAGAIN = -5
PERM_ENOTFOUND = -6
PERM_ECANCELLED = -7

PERM_BATCH_SYNC = 1
PERM_BATCH_GRAPH = 2
PERM_BATCH_REUSE = 4

_NAMES = {0: "PERM_OK", 1: "PERM_PENDING", -1: "PERM_EINVAL", -2: "PERM_ERANGE", -3: "PERM_ENOMEM",
          -4: "PERM_EDEVICE", -5: "PERM_EAGAIN", -6: "PERM_ENOTFOUND", -7: "PERM_ECANCELLED"}

# every symbol the header declares
EXPORTS = [
    "perm_last_error", "perm_version", "perm_prime", "perm_workspace_bytes", "perm_solve",
    "perm_solve_async", "perm_ryser_workspace_bytes", "perm_ryser", "perm_ryser_async",
    "perm_batch_workspace_bytes", "perm_solve_batch", "perm_server_create",
    "perm_server_submit", "perm_server_poll", "perm_server_destroy", "perm_tuning_get",
    "perm_tuning_set", "perm_tuning_load", "perm_tuning_save", "perm_tuning_key",
    "perm_profile_enable", "perm_profile_read", "perm_multi_workspace_bytes", "perm_solve_multi",
    "perm_solve_multi_async", "perm_multi_plan_info", "perm_probe_fp64", "perm_solve_async_noalloc",
    "perm_probe_int", "perm_bunched_workspace_bytes", "perm_bunched_orientation", "perm_solve_bunched",
    "perm_layer_tile_order",
]


class perm_multi_plan_info_t(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int), ("states", ctypes.c_uint64), ("low_states", ctypes.c_uint64),
                ("max_layer", ctypes.c_uint32), ("tiles", ctypes.c_uint64), ("windows", ctypes.c_uint64),
                ("plan_bytes", ctypes.c_uint64), ("checked", ctypes.c_uint64)]


class PermError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class perm_c128_t(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class perm_int_t(ctypes.Structure):
    _fields_ = [("sign", ctypes.c_int32), ("nlimbs", ctypes.c_uint32),
                ("limb", ctypes.c_uint64 * PERM_INT_LIMBS)]

    def value(self) -> int:
        v = 0
        for i in range(self.nlimbs - 1, -1, -1):
            v = (v << 64) | int(self.limb[i])
        return -v if self.sign < 0 else v


class perm_server_config_t(ctypes.Structure):
    _fields_ = [("pool", ctypes.c_void_p), ("pool_bytes", ctypes.c_size_t),
                ("budget_bytes", ctypes.c_size_t), ("max_large_slots", ctypes.c_int),
                ("queue_capacity", ctypes.c_int), ("small_n_max", ctypes.c_int),
                ("max_small_batch", ctypes.c_int)]


class perm_req_stats_t(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double),
                ("n", ctypes.c_int), ("status", ctypes.c_int)]


class perm_tuning_t(ctypes.Structure):
    _fields_ = [("layer_t", ctypes.c_int * (PERM_N_MAX + 1)),
                ("layer_xcd_remap", ctypes.c_int * (PERM_N_MAX + 1)),
                ("layer_flags", ctypes.c_int * (PERM_N_MAX + 1)),
                ("layer_thin", ctypes.c_int * (PERM_N_MAX + 1)),
                ("batch_group", ctypes.c_int * (PERM_BATCH_N_MAX + 1))]


class perm_profile_t(ctypes.Structure):
    _fields_ = [("layer_c128_ms", ctypes.c_double), ("layer_c128_launches", ctypes.c_int64),
                ("layer_modp_ms", ctypes.c_double), ("layer_modp_launches", ctypes.c_int64),
                ("batch_ms", ctypes.c_double), ("batch_launches", ctypes.c_int64),
                ("ryser_ms", ctypes.c_double), ("ryser_launches", ctypes.c_int64),
                ("multi_c128_ms", ctypes.c_double), ("multi_c128_launches", ctypes.c_int64),
                ("multi_modp_ms", ctypes.c_double), ("multi_modp_launches", ctypes.c_int64),
                ("int_plain_layers", ctypes.c_int64)]


_lock = threading.Lock()
_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    """Load libpermgpu.so (built by ``python -m paper_1802_02779_amd.build``)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1802_02779_amd.build` (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i32, i64, u32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int64, ctypes.c_uint32
        L.perm_last_error.restype = ctypes.c_char_p
        L.perm_last_error.argtypes = []
        L.perm_version.restype = i32
        L.perm_prime.argtypes = [i32, ctypes.POINTER(ctypes.c_uint64)]
        L.perm_prime.restype = i32
        L.perm_workspace_bytes.argtypes = [i32, i32]
        L.perm_workspace_bytes.restype = sz
        L.perm_solve.argtypes = [i32, i32, vp, i64, vp, vp, sz, vp]
        L.perm_solve.restype = i32
        L.perm_solve_async.argtypes = [i32, vp, i64, vp, vp, sz, vp]
        L.perm_solve_async.restype = i32
        L.perm_bunched_workspace_bytes.argtypes = [i32, i32, vp, i32, vp]
        L.perm_bunched_workspace_bytes.restype = sz
        L.perm_bunched_orientation.argtypes = [i32, vp, i32, vp, ctypes.POINTER(ctypes.c_int)]
        L.perm_bunched_orientation.restype = i32
        L.perm_solve_bunched.argtypes = [i32, i32, vp, i32, vp, vp, i64, vp, vp, sz, vp]
        L.perm_solve_bunched.restype = i32
        L.perm_probe_int.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), vp]
        L.perm_probe_int.restype = i32
        L.perm_layer_tile_order.argtypes = [i32, i32, i32, i32, vp, sz, ctypes.POINTER(ctypes.c_size_t)]
        L.perm_layer_tile_order.restype = i32
        L.perm_solve_async_noalloc.argtypes = [i32, vp, i64, vp, vp]
        L.perm_solve_async_noalloc.restype = i32
        L.perm_ryser_workspace_bytes.argtypes = [i32, i32]
        L.perm_ryser_workspace_bytes.restype = sz
        L.perm_ryser.argtypes = [i32, i32, vp, i64, vp, vp, sz, vp]
        L.perm_ryser.restype = i32
        L.perm_ryser_async.argtypes = [i32, vp, i64, vp, vp, sz, vp]
        L.perm_ryser_async.restype = i32
        L.perm_multi_workspace_bytes.argtypes = [i32, i32, i32, vp]
        L.perm_multi_workspace_bytes.restype = sz
        L.perm_solve_multi.argtypes = [i32, i32, i32, vp, vp, i64, vp, vp, sz, vp]
        L.perm_solve_multi.restype = i32
        L.perm_solve_multi_async.argtypes = [i32, i32, vp, vp, i64, vp, vp, sz, vp]
        L.perm_solve_multi_async.restype = i32
        L.perm_multi_plan_info.argtypes = [i32, i32, vp, i32, ctypes.POINTER(perm_multi_plan_info_t)]
        L.perm_multi_plan_info.restype = i32
        L.perm_probe_fp64.argtypes = [ctypes.POINTER(ctypes.c_double), vp]
        L.perm_probe_fp64.restype = i32
        L.perm_batch_workspace_bytes.argtypes = [i32, i32, vp]
        L.perm_batch_workspace_bytes.restype = sz
        L.perm_solve_batch.argtypes = [i32, i32, vp, vp, vp, vp, vp, sz, vp, u32]
        L.perm_solve_batch.restype = i32
        L.perm_server_create.argtypes = [ctypes.POINTER(perm_server_config_t), ctypes.POINTER(vp)]
        L.perm_server_create.restype = i32
        L.perm_server_submit.argtypes = [vp, i32, i32, vp, i64, ctypes.POINTER(ctypes.c_uint64)]
        L.perm_server_submit.restype = i32
        L.perm_server_poll.argtypes = [vp, ctypes.c_uint64, vp, ctypes.POINTER(perm_req_stats_t)]
        L.perm_server_poll.restype = i32
        L.perm_server_destroy.argtypes = [vp]
        L.perm_server_destroy.restype = i32
        L.perm_tuning_get.argtypes = [ctypes.POINTER(perm_tuning_t)]
        L.perm_tuning_get.restype = i32
        L.perm_tuning_set.argtypes = [ctypes.POINTER(perm_tuning_t)]
        L.perm_tuning_set.restype = i32
        L.perm_tuning_load.argtypes = [ctypes.c_char_p]
        L.perm_tuning_load.restype = i32
        L.perm_tuning_save.argtypes = [ctypes.c_char_p]
        L.perm_tuning_save.restype = i32
        L.perm_tuning_key.argtypes = [ctypes.c_char_p, sz]
        L.perm_tuning_key.restype = i32
        L.perm_profile_enable.argtypes = [i32]
        L.perm_profile_enable.restype = i32
        L.perm_profile_read.argtypes = [ctypes.POINTER(perm_profile_t)]
        L.perm_profile_read.restype = i32
        _lib = L
        return L


def _check(rc: int) -> int:
    if rc < 0:
        raise PermError(rc, lib().perm_last_error().decode(errors="replace"))
    return rc


def perm_last_error() -> str:
    return lib().perm_last_error().decode(errors="replace")


def perm_version() -> int:
    return int(lib().perm_version())


def perm_prime(i: int) -> int:
    p = ctypes.c_uint64()
    _check(lib().perm_prime(i, ctypes.byref(p)))
    return int(p.value)


def perm_workspace_bytes(dtype: int, n: int) -> int:
    return int(lib().perm_workspace_bytes(dtype, n))


# ---------------------------------------------------------------- torch glue
def _torch():
    import torch  # imported lazily: the ABI checks on the CPU need no torch
    return torch


def _stream_ptr(stream) -> int:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def device_buffer(nbytes: int, device="cuda"):
    """A torch uint8 device tensor of at least nbytes (1 byte minimum)."""
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _dtype_of(A: np.ndarray) -> int:
    if np.issubdtype(A.dtype, np.complexfloating):
        return PERM_COMPLEX128
    if np.issubdtype(A.dtype, np.integer) or A.dtype == np.bool_:
        return PERM_INT64
    raise TypeError(f"unsupported dtype {A.dtype}")


def perm_solve(A, workspace=None, stream=None):
    """per(A) of a host matrix (int64 -> Python int, complex128 -> complex).

    ``workspace``: a torch device tensor of at least perm_workspace_bytes
    bytes (allocated here when None).
    """
    A = np.asarray(A)
    dt = _dtype_of(A)
    A = np.ascontiguousarray(A, dtype=np.int64 if dt == PERM_INT64 else np.complex128)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("square matrix expected")
    n = A.shape[0]
    need = perm_workspace_bytes(dt, n)
    ws = workspace if workspace is not None else (device_buffer(need) if n >= 2 else None)
    ws_ptr = ws.data_ptr() if ws is not None else None
    ws_bytes = ws.numel() * ws.element_size() if ws is not None else 0
    s = _stream_ptr(stream) if n >= 2 else None
    if dt == PERM_INT64:
        out = perm_int_t()
        _check(lib().perm_solve(dt, n, A.ctypes.data if n else None, max(n, 1), ctypes.byref(out),
                                ws_ptr, ws_bytes, s))
        return out.value()
    out = perm_c128_t()
    _check(lib().perm_solve(dt, n, A.ctypes.data if n else None, max(n, 1), ctypes.byref(out),
                            ws_ptr, ws_bytes, s))
    return complex(out.re, out.im)


def perm_solve_async(n: int, a_dev, lda: int, result_dev, workspace, stream=None) -> None:
    """Queue per(A) of a device complex128 matrix (torch tensor) into result_dev."""
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(lib().perm_solve_async(n, a_dev.data_ptr() if a_dev is not None else None, lda,
                                  result_dev.data_ptr(),
                                  workspace.data_ptr() if workspace is not None else None, ws_bytes,
                                  _stream_ptr(stream)))


PERM_NOALLOC_N_MAX = 22
PERM_NOALLOC_SCRATCH_BYTES = 24 << 20


def perm_solve_async_noalloc(n: int, a_dev, lda: int, result_dev, stream=None) -> None:
    """perm_solve_async without a workspace: the library's fixed device array
    holds the tables (n <= PERM_NOALLOC_N_MAX; calls on one device must not
    overlap)."""
    _check(lib().perm_solve_async_noalloc(n, a_dev.data_ptr() if a_dev is not None else None, lda,
                                          result_dev.data_ptr() if result_dev is not None else None,
                                          _stream_ptr(stream)))


def perm_ryser_workspace_bytes(dtype: int, n: int) -> int:
    return int(lib().perm_ryser_workspace_bytes(dtype, n))


def perm_ryser(A, workspace=None, stream=None):
    """per(A) of a host matrix by Ryser's formula (eq. 4): complex128 ->
    complex, int64 -> exact Python int."""
    A = np.asarray(A)
    dt = _dtype_of(A)
    A = np.ascontiguousarray(A, dtype=np.int64 if dt == PERM_INT64 else np.complex128)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("square matrix expected")
    n = A.shape[0]
    need = perm_ryser_workspace_bytes(dt, n)
    ws = workspace if workspace is not None else (device_buffer(need) if n >= 1 else None)
    ws_ptr = ws.data_ptr() if ws is not None else None
    ws_bytes = ws.numel() * ws.element_size() if ws is not None else 0
    s = _stream_ptr(stream) if n >= 1 else None
    if dt == PERM_INT64:
        out = perm_int_t()
        _check(lib().perm_ryser(dt, n, A.ctypes.data if n else None, max(n, 1), ctypes.byref(out),
                                ws_ptr, ws_bytes, s))
        return out.value()
    out = perm_c128_t()
    _check(lib().perm_ryser(dt, n, A.ctypes.data if n else None, max(n, 1), ctypes.byref(out),
                            ws_ptr, ws_bytes, s))
    return complex(out.re, out.im)


def perm_ryser_async(n: int, a_dev, lda: int, result_dev, workspace, stream=None) -> None:
    """Queue Ryser's per(A) of a device complex128 matrix into result_dev."""
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(lib().perm_ryser_async(n, a_dev.data_ptr() if a_dev is not None else None, lda,
                                  result_dev.data_ptr(),
                                  workspace.data_ptr() if workspace is not None else None, ws_bytes,
                                  _stream_ptr(stream)))


def _mult(mult) -> np.ndarray:
    t = np.ascontiguousarray(np.asarray(mult, dtype=np.int32))
    if t.ndim != 1:
        raise ValueError("one multiplicity per column")
    return t


def perm_multi_workspace_bytes(dtype: int, mult) -> int:
    """Workspace for a matrix whose column j is repeated mult[j] times (n = sum)."""
    t = _mult(mult)
    return int(lib().perm_multi_workspace_bytes(dtype, int(t.sum()), t.shape[0], t.ctypes.data))


def perm_solve_multi(A, mult, workspace=None, stream=None):
    """Permanent of the n x n matrix with column j of the host n x m matrix A
    repeated mult[j] times (int64 -> Python int, complex128 -> complex)."""
    A = np.asarray(A)
    dt = _dtype_of(A)
    A = np.ascontiguousarray(A, dtype=np.int64 if dt == PERM_INT64 else np.complex128)
    if A.ndim != 2:
        raise ValueError("matrix expected")
    t = _mult(mult)
    n, m = A.shape
    need = int(lib().perm_multi_workspace_bytes(dt, n, m, t.ctypes.data))
    ws = workspace if workspace is not None else (device_buffer(need) if n >= 2 and need else None)
    ws_ptr = ws.data_ptr() if ws is not None else None
    ws_bytes = ws.numel() * ws.element_size() if ws is not None else 0
    s = _stream_ptr(stream) if n >= 2 else None
    out = perm_int_t() if dt == PERM_INT64 else perm_c128_t()
    _check(lib().perm_solve_multi(dt, n, m, t.ctypes.data, A.ctypes.data if n else None, max(m, 1),
                                  ctypes.byref(out), ws_ptr, ws_bytes, s))
    return out.value() if dt == PERM_INT64 else complex(out.re, out.im)


def perm_solve_multi_async(n: int, mult, a_dev, lda: int, result_dev, workspace, stream=None) -> None:
    """Queue the repeated-column permanent of a device complex128 n x m matrix."""
    t = _mult(mult)
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(lib().perm_solve_multi_async(n, t.shape[0], t.ctypes.data, a_dev.data_ptr() if a_dev is not None else None,
                                        lda, result_dev.data_ptr(),
                                        workspace.data_ptr() if workspace is not None else None, ws_bytes,
                                        _stream_ptr(stream)))


def _mults(row_mult, col_mult):
    rm = np.ascontiguousarray(np.asarray(row_mult, dtype=np.int32))
    cm = np.ascontiguousarray(np.asarray(col_mult, dtype=np.int32))
    if rm.ndim != 1 or cm.ndim != 1:
        raise ValueError("multiplicities are 1-D")
    return rm, cm


def bunched_orientation(row_mult, col_mult) -> bool:
    """True when perm_solve_bunched compresses the rows (runs on the
    transpose): the library's rule, the side with fewer count vectors
    prod(mult + 1); ties keep the columns."""
    rm, cm = _mults(row_mult, col_mult)
    rows = ctypes.c_int()
    _check(lib().perm_bunched_orientation(rm.shape[0], rm.ctypes.data, cm.shape[0], cm.ctypes.data,
                                          ctypes.byref(rows)))
    return bool(rows.value)


def perm_bunched_workspace_bytes(dtype: int, row_mult, col_mult) -> int:
    rm, cm = _mults(row_mult, col_mult)
    return int(lib().perm_bunched_workspace_bytes(dtype, rm.shape[0], rm.ctypes.data, cm.shape[0], cm.ctypes.data))


def perm_solve_bunched(A, row_mult, col_mult, workspace=None, stream=None):
    """Permanent of the n x n matrix with row i of the r x c matrix A repeated
    row_mult[i] times and column j repeated col_mult[j] times (sum row_mult =
    sum col_mult = n); see perm_solve_bunched in include/perm.h."""
    rm, cm = _mults(row_mult, col_mult)
    A = np.asarray(A)
    if A.ndim != 2 or A.shape != (rm.shape[0], cm.shape[0]):
        raise ValueError("one multiplicity per row and per column of A")
    dt = _dtype_of(A)
    A = np.ascontiguousarray(A, dtype=np.complex128 if dt == PERM_COMPLEX128 else np.int64)
    if workspace is None:
        need = perm_bunched_workspace_bytes(dt, rm, cm)
        workspace = device_buffer(need) if need else None
    ws_ptr = workspace.data_ptr() if workspace is not None else None
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    r, c = A.shape
    out = perm_int_t() if dt == PERM_INT64 else perm_c128_t()
    _check(lib().perm_solve_bunched(dt, r, rm.ctypes.data, c, cm.ctypes.data, A.ctypes.data if A.size else None,
                                    max(c, 1), ctypes.byref(out), ws_ptr, ws_bytes, _stream_ptr(stream)))
    return out.value() if dt == PERM_INT64 else complex(out.re, out.im)


def perm_multi_plan_info(mult, check: bool = False) -> perm_multi_plan_info_t:
    """Host-only shape (and, with check, verification) of the plan for mult."""
    t = _mult(mult)
    out = perm_multi_plan_info_t()
    _check(lib().perm_multi_plan_info(int(t.sum()), t.shape[0], t.ctypes.data, 1 if check else 0,
                                      ctypes.byref(out)))
    return out


def perm_probe_fp64(stream=None) -> float:
    """FP64 TFLOP/s sustained by independent FMA chains (measurement probe)."""
    v = ctypes.c_double()
    _check(lib().perm_probe_fp64(ctypes.byref(v), _stream_ptr(stream)))
    return float(v.value)


def perm_probe_int(stream=None):
    """(mac_fold, add64) rates of the integer sweep's per-term arithmetic, in
    1e9 terms per second (measurement probe)."""
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(lib().perm_probe_int(ctypes.byref(a), ctypes.byref(b), _stream_ptr(stream)))
    return float(a.value), float(b.value)


def perm_layer_tile_order(n: int, t: int, k: int, value_bytes: int = 16) -> np.ndarray:
    """The cache-aware tile order of layer k (host only): high-part masks in
    workgroup order, 0xffffffff for padding slots."""
    ln = ctypes.c_size_t()
    _check(lib().perm_layer_tile_order(n, t, k, value_bytes, None, 0, ctypes.byref(ln)))
    out = np.zeros(ln.value, dtype=np.uint32)
    _check(lib().perm_layer_tile_order(n, t, k, value_bytes, out.ctypes.data if out.size else None, out.size,
                                       ctypes.byref(ln)))
    return out


def perm_batch_workspace_bytes(dtype: int, ns: np.ndarray) -> int:
    ns = np.ascontiguousarray(ns, dtype=np.int32)
    return int(lib().perm_batch_workspace_bytes(dtype, ns.shape[0], ns.ctypes.data))


def perm_solve_batch(dtype: int, ns, offsets, mats, results, workspace, stream=None, flags: int = 0):
    """Batched solve.  complex128: ``mats``/``results`` are torch device
    tensors; int64: ``mats`` is a host int64 numpy array and the return value
    is a list of Python ints (``results`` is ignored)."""
    ns = np.ascontiguousarray(ns, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    count = int(ns.shape[0])
    ws_bytes = workspace.numel() * workspace.element_size()
    if dtype == PERM_INT64:
        mats = np.ascontiguousarray(mats, dtype=np.int64)
        out = (perm_int_t * max(count, 1))()
        _check(lib().perm_solve_batch(dtype, count, ns.ctypes.data, offsets.ctypes.data, mats.ctypes.data,
                                      ctypes.addressof(out), workspace.data_ptr(), ws_bytes,
                                      _stream_ptr(stream), flags))
        return [out[i].value() for i in range(count)]
    _check(lib().perm_solve_batch(dtype, count, ns.ctypes.data, offsets.ctypes.data, mats.data_ptr(),
                                  results.data_ptr(), workspace.data_ptr(), ws_bytes,
                                  _stream_ptr(stream), flags))
    return results


# ------------------------------------------------------------------ server
def perm_server_create(pool, budget_bytes: int = 0, max_large_slots: int = 2, queue_capacity: int = 4096,
                       small_n_max: int = 12, max_small_batch: int = 4096):
    """Create a server carving its tables from the torch device tensor ``pool``."""
    cfg = perm_server_config_t(pool.data_ptr(), pool.numel() * pool.element_size(), budget_bytes,
                               max_large_slots, queue_capacity, small_n_max, max_small_batch)
    h = ctypes.c_void_p()
    _check(lib().perm_server_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h


def perm_server_submit(server, A) -> int:
    """Submit a host complex128 matrix; returns the ticket.  Raises PermError
    (code PERM_EAGAIN when the queue is full)."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    n = A.shape[0]
    ticket = ctypes.c_uint64()
    _check(lib().perm_server_submit(server, PERM_COMPLEX128, n, A.ctypes.data if n else None, max(n, 1),
                                    ctypes.byref(ticket)))
    return int(ticket.value)


def perm_server_poll(server, ticket: int):
    """None while pending, else (result complex, stats perm_req_stats_t)."""
    out = perm_c128_t()
    st = perm_req_stats_t()
    rc = lib().perm_server_poll(server, ticket, ctypes.byref(out), ctypes.byref(st))
    if rc == PERM_PENDING:
        return None
    _check(rc)
    return complex(out.re, out.im), st


def perm_server_destroy(server) -> None:
    _check(lib().perm_server_destroy(server))


# ----------------------------------------------------------- tuning/profile
def perm_tuning_get() -> perm_tuning_t:
    t = perm_tuning_t()
    _check(lib().perm_tuning_get(ctypes.byref(t)))
    return t


def perm_tuning_set(t: perm_tuning_t) -> None:
    _check(lib().perm_tuning_set(ctypes.byref(t)))


def perm_tuning_load(path: str) -> int:
    rc = lib().perm_tuning_load(path.encode())
    if rc == PERM_ENOTFOUND:
        return rc
    return _check(rc)


def perm_tuning_save(path: str) -> None:
    _check(lib().perm_tuning_save(path.encode()))


def perm_tuning_key() -> str:
    buf = ctypes.create_string_buffer(256)
    _check(lib().perm_tuning_key(buf, 256))
    return buf.value.decode()


def perm_profile_enable(on: bool) -> None:
    _check(lib().perm_profile_enable(1 if on else 0))


def perm_profile_read() -> perm_profile_t:
    p = perm_profile_t()
    _check(lib().perm_profile_read(ctypes.byref(p)))
    return p
