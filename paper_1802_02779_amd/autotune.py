"""Autotuner for libpermgpu's tile and schedule parameters.

    python -m paper_1802_02779_amd.autotune [--out FILE] [--layer-n 20,24,26,28,30] [--int-n 26,28,30] [--batch]

For each order n it times the candidates of one path on seeded synthetic
inputs through the C ABI and keeps the fastest candidate whose result is
bitwise equal to the result of the library's default configuration (every
parameter here only changes the schedule, so any difference would be a bug and
disqualifies the candidate):

* layer sweep (perm_solve_async, complex128): low-window width t, XCD chunk
  of the tile order, non-temporal output stores, per-thread threshold, and
  then, on the winning schedule, the cache-aware tile order (bit 2 of
  layer_flags, which the exact integer sweep of that order uses too);
* exact integer sweep (perm_solve, int64 Bernoulli input): whether its plain
  64-bit layers take one low column more than the complex sweep (bit 1 of
  layer_flags; the values must come out identical);
* batched kernel (perm_solve_batch, complex128): threads per matrix.

The winners go into the process-wide tuning table (perm_tuning_set) and are
written with perm_tuning_save, a JSON file keyed by GPU architecture, CU count
and HIP runtime version; perm_tuning_load ignores a file written for another
key.  All timing runs in the library's kernels; this module only drives them.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_FILE = os.path.join(HERE, "tuning", "gfx950.json")
HIGH_BITS = 22  # the library's largest tile high part: n - t above it is rejected
ORDER_HIGH_BITS = 18  # largest high part the cache-aware tile order covers


def _time_ms(fn, reps: int, sync) -> float:
    fn()
    sync()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        sync()
        ts.append((time.perf_counter() - t0) * 1000.0)
    return float(np.median(ts))


def _time_events_ms(fn, reps: int, torch, inner: int) -> float:
    """Median over reps of the mean device time of `inner` back-to-back calls
    of an asynchronous fn, from events on the current stream (host launch
    overhead and synchronization stay out of the figure)."""
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(inner):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / inner)
    return float(np.median(ts))


def _log(msg):
    print(msg, flush=True)


def tune_layer(perm, inputs, torch, n: int, log=_log, reps: int = 3):
    C = perm.PERM_COMPLEX128
    A = inputs.complex_gaussian(n, seed=n)
    d_a = torch.from_numpy(A).cuda()
    d_r = torch.zeros(1, dtype=torch.complex128, device="cuda")
    ws = perm.device_buffer(perm.perm_workspace_bytes(C, n))
    base = perm.perm_tuning_get()
    default = perm.perm_tuning_t.from_buffer_copy(base)
    default.layer_t[n] = 0
    default.layer_xcd_remap[n] = -1
    default.layer_flags[n] = base.layer_flags[n] & ~5  # bits 0 and 2 are this sweep's; bit 1 is kept
    default.layer_thin[n] = 0
    perm.perm_tuning_set(default)
    run = lambda: perm.perm_solve_async(n, d_a, n, d_r, ws)  # noqa: E731
    inner = 10 if n <= 28 else 4
    timed = lambda: _time_events_ms(run, reps, torch, inner)  # noqa: E731
    ref_ms = timed()
    ref = d_r.cpu().numpy().view(np.uint64).copy()
    best = (ref_ms, 0, -1, 0, 0)
    # above n = 30 one solve takes 40-400 ms: a smaller grid
    big = n > 30
    t_lo, t_hi = max(1, n - HIGH_BITS), min(14 if big else 15, n)
    for t in range(max(t_lo, 8), t_hi + 1):
        log(f"  n={n} t={t} ...")
        for chunk in ((64, 256) if big else (0, 16, 64, 256)):
            for nt in (0, 1):
                for thin in ((-1, 128) if big else (-1, 128, 512)):
                    cand = perm.perm_tuning_t.from_buffer_copy(default)
                    cand.layer_t[n] = t
                    cand.layer_xcd_remap[n] = chunk
                    cand.layer_flags[n] = default.layer_flags[n] | nt
                    cand.layer_thin[n] = thin
                    perm.perm_tuning_set(cand)
                    ms = timed()
                    same = (d_r.cpu().numpy().view(np.uint64) == ref).all()
                    if not same:
                        log(f"  n={n} t={t} chunk={chunk} nt={nt} thin={thin}: result differs, rejected")
                        continue
                    if ms < best[0]:
                        best = (ms, t, chunk, nt, thin)
    # the cache-aware tile order on the winning schedule
    order = 0
    t_eff = best[1] or min(12, max(6, n - 12))
    if n - t_eff <= ORDER_HIGH_BITS:
        cand = perm.perm_tuning_t.from_buffer_copy(default)
        (cand.layer_t[n], cand.layer_xcd_remap[n], cand.layer_thin[n]) = best[1], best[2], best[4]
        cand.layer_flags[n] = default.layer_flags[n] | best[3] | 4
        perm.perm_tuning_set(cand)
        ms = timed()
        same = (d_r.cpu().numpy().view(np.uint64) == ref).all()
        log(f"  n={n} cache-aware tile order: {ms:.3f} ms" + ("" if same else ", result differs, rejected"))
        if same and ms < best[0]:
            order = 4
            best = (ms,) + best[1:]
    final = perm.perm_tuning_t.from_buffer_copy(base)
    (final.layer_t[n], final.layer_xcd_remap[n], final.layer_thin[n]) = best[1], best[2], best[4]
    final.layer_flags[n] = (final.layer_flags[n] & ~5) | best[3] | order
    perm.perm_tuning_set(final)
    log(f"layer n={n}: default {ref_ms:.3f} ms -> t={best[1]} chunk={best[2]} nt={best[3]} "
        f"thin={best[4]} order={order >> 2} {best[0]:.3f} ms")
    return best


def tune_int_plain(perm, inputs, torch, n: int, log=_log, reps: int = 5):
    """Bit 1 of layer_flags[n]: whether the exact integer sweep's plain 64-bit
    layers take one low column more than layer_t.  Timed on a Bernoulli 0/1
    matrix (most layers plain); kept only if the value is unchanged."""
    B = inputs.bernoulli01(n, seed=n)
    ws = perm.device_buffer(perm.perm_workspace_bytes(perm.PERM_INT64, n))
    base = perm.perm_tuning_get()
    res = {}
    for bit in (0, 2):
        cand = perm.perm_tuning_t.from_buffer_copy(base)
        cand.layer_flags[n] = (cand.layer_flags[n] & ~2) | bit
        perm.perm_tuning_set(cand)
        out = []
        ms = _time_ms(lambda: out.append(perm.perm_solve(B, workspace=ws)), reps, torch.cuda.synchronize)  # noqa: B023
        res[bit] = (ms, out[-1])
    if res[0][1] != res[2][1]:
        raise RuntimeError(f"integer n={n}: values differ between the two widths")
    bit = 2 if res[2][0] < res[0][0] else 0
    final = perm.perm_tuning_t.from_buffer_copy(base)
    final.layer_flags[n] = (final.layer_flags[n] & ~2) | bit
    perm.perm_tuning_set(final)
    log(f"int n={n}: plain layers at layer_t {res[0][0]:.3f} ms, at layer_t + 1 {res[2][0]:.3f} ms "
        f"-> bit {bit >> 1}")
    del ws
    return bit


def tune_batch(perm, inputs, torch, n: int, count: int = 1 << 16, log=_log, reps: int = 7):
    C = perm.PERM_COMPLEX128
    U = inputs.haar_unitary(64, seed=2018)
    b = inputs.submatrix_batch(U, count, n, n, seed=n)
    d_mats = torch.from_numpy(b.mats).cuda()
    d_out = torch.zeros(count, dtype=torch.complex128, device="cuda")
    ws = perm.device_buffer(perm.perm_batch_workspace_bytes(C, b.ns))
    base = perm.perm_tuning_get()
    cand = perm.perm_tuning_t.from_buffer_copy(base)
    cand.batch_group[n] = 0
    perm.perm_tuning_set(cand)
    # each candidate plans its work list and captures its graph once (with the
    # tuning in force), then the graph replay alone is timed
    G, R, Y = perm.PERM_BATCH_GRAPH, perm.PERM_BATCH_REUSE, perm.PERM_BATCH_SYNC
    plan = lambda: perm.perm_solve_batch(C, b.ns, b.offsets, d_mats, d_out, ws, flags=G | Y)  # noqa: E731
    run = lambda: perm.perm_solve_batch(C, b.ns, b.offsets, d_mats, d_out, ws, flags=G | R | Y)  # noqa: E731
    plan()
    ref_ms = _time_ms(run, reps, torch.cuda.synchronize)
    ref = d_out.cpu().numpy().view(np.uint64).copy()
    best = (ref_ms, 0)
    for g in (16, 32, 64, 128, 256, 512):
        cand = perm.perm_tuning_t.from_buffer_copy(base)
        cand.batch_group[n] = g
        perm.perm_tuning_set(cand)
        plan()
        ms = _time_ms(run, reps, torch.cuda.synchronize)
        if not (d_out.cpu().numpy().view(np.uint64) == ref).all():
            log(f"  batch n={n} group={g}: result differs, rejected")
            continue
        if ms < best[0]:
            best = (ms, g)
    final = perm.perm_tuning_t.from_buffer_copy(base)
    final.batch_group[n] = best[1]
    perm.perm_tuning_set(final)
    log(f"batch n={n}: default {ref_ms:.3f} ms -> group={best[1]} {best[0]:.3f} ms "
        f"({count / best[0] * 1e3:.3e} perms/s)")
    return best


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_FILE)
    ap.add_argument("--layer-n", default="16,20,24,26,28,30")
    ap.add_argument("--int-n", default="",
                    help="orders whose integer plain-layer width is tuned (layer_flags bit 1)")
    ap.add_argument("--batch", action="store_true")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    import torch

    from paper_1802_02779_amd import inputs, perm
    torch.cuda.set_device(0)
    perm.lib()
    if os.path.exists(args.out):
        perm.perm_tuning_load(args.out)
    for n in [int(x) for x in args.layer_n.split(",") if x]:
        tune_layer(perm, inputs, torch, n)
        torch.cuda.empty_cache()
    for n in [int(x) for x in args.int_n.split(",") if x]:
        tune_int_plain(perm, inputs, torch, n)
        torch.cuda.empty_cache()
    if args.batch:
        for n in range(3, 13):
            tune_batch(perm, inputs, torch, n)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    perm.perm_tuning_save(args.out)
    print(f"key {perm.perm_tuning_key()} -> {args.out}")


if __name__ == "__main__":
    main()
