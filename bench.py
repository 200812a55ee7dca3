"""Benchmark of the Store-zechin permanent on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extras]

One step is one complete permanent of a 28x28 complex128 matrix (iid complex
Gaussian entries, parts N(0, 1/2)): ingest of the device-resident matrix,
layer 1, the 27 layer sweeps and the readout, all in the library's kernels
(perm_solve_async).  The timed region holds exactly K steps between two
device synchronizations; the input is already in HBM.  The JSON line on
stdout reports perms/s, the roofline of the dominant kernel (the complex
layer sweep) measured with HIP events on its own stream, and the oracle timed
on the host's cores.  Extra fields cover the other workloads: the 26x26
complex and 30x30 0/1 integer solves, the 10x10 integer solve, the batched
2^20 submatrix workload against a plain per-matrix loop, and the serving
trace, Ryser's eq. (4) at n = 28 and 34, n = 34 Store-zechin, and the
repeated-column (bunched-boson) solves.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "n=28 complex128 perm wall time; batched perms/s; p50/p99 latency vs plain"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
GOLDEN = os.path.join(ROOT, "tests", "golden", "large_configs.json")
COUNTERS = os.path.join(ROOT, "profiles", "layer_c128_n28_counters.json")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def layer_bytes(n: int, elem: int = 16) -> int:
    """Algorithmic HBM bytes of all layer sweeps of one order-n permanent:
    every stored value of layers 1..n-1 read once, of layers 2..n written once."""
    return elem * sum(math.comb(n, k - 1) + math.comb(n, k) for k in range(2, n + 1))


def plain_layers(A) -> int:
    """Layers 1..K whose stored values the integer path bounds below 2^63
    (the product over rows i < k of min(sum_j |a_ij|, (i+1) max_j |a_ij|));
    those run in plain 64-bit arithmetic, the rest in residues."""
    n = A.shape[0]
    B = 1
    K = 0
    for k in range(1, n + 1):
        row = [abs(int(x)) for x in A[k - 1]]
        B *= min(sum(row), k * max(row))
        if B > 2 ** 63 - 1:
            break
        K = k
    return K


def int_layer_bytes(n: int, K: int, R: int) -> int:
    """Algorithmic HBM bytes of the exact integer sweep with R residues:
    8-byte values read once and written once per layer, one plane for layers
    up to K, R planes above; plus the conversion of layer K (read once,
    written as R residues)."""
    def lb(k, planes):
        return 8 * planes * (math.comb(n, k - 1) + math.comb(n, k))
    tot = sum(lb(k, 1 if k <= K else R) for k in range(2, n + 1))
    if K >= 2:
        tot += 8 * (1 + R) * math.comb(n, K)
    return tot


def algorithmic_flops(n: int) -> int:
    """6 flops per complex multiplication, 2 per complex addition; a stored
    value of order k costs k multiplications and k-1 additions."""
    M = sum(k * math.comb(n, k) for k in range(2, n + 1))
    A = sum((k - 1) * math.comb(n, k) for k in range(2, n + 1))
    return 6 * M + 2 * A


def ryser_flops(n: int) -> int:
    """Algorithmic flops of eq. (4) over all 2^n subsets, one column change
    per subset: n complex additions (2n), n-1 complex multiplications
    (6 each) and one signed complex accumulation (2)."""
    return (1 << n) * (2 * n + 6 * (n - 1) + 2)


def ryser_issue_bound(n: int) -> float:
    """Fraction of the FP64 flop peak the instruction mix allows: per subset
    2n additions (1 flop, 1 instruction), n-1 products of 2 multiplications
    and 2 fused multiply-adds (6 flops, 4 instructions), 2 fused adds; the
    peak assumes 2 flops in every issue slot."""
    instr = 2 * n + 4 * (n - 1) + 2
    return ryser_flops(n) / (1 << n) / (2.0 * instr)


def source_hash() -> str:
    from paper_1802_02779_amd.profiling import source_hash as _h
    return _h(ROOT)


def int_source_hash() -> str:
    from paper_1802_02779_amd.profiling import int_source_hash as _h
    return _h(ROOT)


def bits(z):
    import numpy as np
    return tuple(int(x) for x in np.array([z.real, z.imag], dtype=np.float64).view(np.uint64))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--only", default="",
                    help="comma list of extra sections to run (n26, ryser, n34, h2h, compare, int30, multi, int10, batch, "
                         "serving); "
                         "default: all")
    ap.add_argument("--tune28", default="",
                    help="override the n = 28 row of the tuning table: 't,remap,flags' (layer_t, "
                         "layer_xcd_remap, layer_flags)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device to device (a plain copy kernel of known size, "
                         "the reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library runs a "
              "permanent on a single MI355X and has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1802_02779_amd import inputs, perm

    torch.cuda.set_device(0)
    perm.lib()
    C128 = perm.PERM_COMPLEX128
    tuning_file = os.path.join(ROOT, "paper_1802_02779_amd", "tuning", "gfx950.json")
    tuning = "library defaults"
    if os.path.exists(tuning_file):
        try:
            if perm.perm_tuning_load(tuning_file) == 0:
                tuning = os.path.relpath(tuning_file, ROOT)
        except perm.PermError as e:
            log(f"tuning file ignored: {e}")
    if args.tune28:
        t28, r28, f28 = (int(x) for x in args.tune28.split(","))
        tu = perm.perm_tuning_get()
        tu.layer_t[28], tu.layer_xcd_remap[28], tu.layer_flags[28] = t28, r28, f28
        perm.perm_tuning_set(tu)
        tuning += f" with n = 28 row t={t28}, remap={r28}, flags={f28}"
    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    golden = {}
    if os.path.exists(GOLDEN):
        with open(GOLDEN) as f:
            golden = json.load(f)

    # ------------------------------------------------ headline: n = 28
    n = 28
    A = inputs.complex_gaussian(n, seed=0)
    d_a = torch.from_numpy(A).cuda()
    d_res = torch.zeros(1, dtype=torch.complex128, device="cuda")
    ws = perm.device_buffer(perm.perm_workspace_bytes(C128, n))
    log(f"n={n} complex128: workspace {ws.numel() / 1e9:.2f} GB, warmup {args.warmup}")
    for _ in range(args.warmup):
        perm.perm_solve_async(n, d_a, n, d_res, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        perm.perm_solve_async(n, d_a, n, d_res, ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    z = complex(d_res.cpu().numpy()[0])
    key = "c128_n28_s0"
    verified = (bits(z) == (int(golden[key]["re_bits"], 16), int(golden[key]["im_bits"], 16))) \
        if key in golden else None
    log(f"n=28: {ms_per_step:.3f} ms/step over {args.steps} steps, verified={verified}")

    # per-kernel durations: HIP events around every layer launch on the
    # stream the library launches on (separate pass, same work)
    perm.perm_profile_enable(True)
    perm.perm_profile_read()
    for _ in range(args.steps):
        perm.perm_solve_async(n, d_a, n, d_res, ws)
    torch.cuda.synchronize()
    prof = perm.perm_profile_read()
    perm.perm_profile_enable(False)
    kernel, launches, kern_ms = "k_layer_c128", int(prof.layer_c128_launches), prof.layer_c128_ms
    counters_file = COUNTERS
    per_step = launches // args.steps
    avg_ms = kern_ms / max(launches, 1)
    # algorithmic bytes of one solve (every stored value written once and
    # read once), shared equally by the launches of a step
    bytes_per_launch = layer_bytes(n) / per_step
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    flops_per_step = algorithmic_flops(n)
    kern_ms_per_step = kern_ms / args.steps
    traffic = None
    if os.path.exists(counters_file):
        with open(counters_file) as f:
            cnt = json.load(f)
        if cnt.get("source_hash") == source_hash():
            traffic = cnt.get("hbm_bytes_per_launch")
    roofline = {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "traffic_source": os.path.relpath(counters_file, ROOT) + " (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                  "valid while the kernel sources and tuning row hash to its source_hash; "
                                  "null otherwise)",
                "avg_launch_ms": round(avg_ms, 5), "launches_per_step": per_step,
                "algorithmic_bytes_per_launch": int(bytes_per_launch),
                "fp64_tflops": round(flops_per_step / (kern_ms_per_step * 1e-3) / 1e12, 3),
                "fp64_frac": round(flops_per_step / (kern_ms_per_step * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)}
    # what the memory system delivers to a plain stream: a 1 GiB device-to-
    # device copy (read + write bytes over its time), next to the rate at
    # which the sweep moves its measured traffic
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * (1 << 30) * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    roofline["copy_gbs"] = round(copy_gbs, 1)
    if traffic:
        roofline["traffic_gbs"] = round(traffic / (avg_ms * 1e-3) / 1e9, 1)
        roofline["amplification"] = round(traffic / bytes_per_launch, 3)
    log(f"{kernel}: avg {avg_ms:.4f} ms/launch, {achieved:.0f} GB/s algorithmic; "
        f"measured traffic at {roofline.get('traffic_gbs')} GB/s, plain 1 GiB copy {copy_gbs:.0f} GB/s")

    result = {
        "metric": METRIC, "value": round(1000.0 / ms_per_step, 3), "unit": "perms/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "one 28x28 complex128 permanent per step, entries iid complex Gaussian "
                               "(parts N(0,1/2)), seed 0, device-resident input",
                   "n": n, "global_batch": 1, "parallelism": "single GPU", "tuning": tuning},
        "verified_bitwise_vs_oracle": verified,
        "roofline": roofline,
    }

    if not args.no_extras:
        only = {x.strip() for x in args.only.split(",") if x.strip()}
        result["extras"] = extras(perm, inputs, golden, np, torch, log, only)

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(inputs, log)
    print(json.dumps(result), flush=True)


def extras(perm, inputs, golden, np, torch, log, only=frozenset()):
    out = {}
    want = lambda name: not only or name in only  # noqa: E731
    if want("n26"):
        _extra_n26(perm, inputs, golden, torch, log, out)
    if want("ryser"):
        _extra_ryser(perm, inputs, torch, log, out)
    if want("n34"):
        _extra_n34(perm, inputs, torch, log, out)
    if want("h2h"):
        _extra_h2h(perm, inputs, out)
    if want("compare"):
        _extra_compare(perm, inputs, torch, log, out)
    if want("int30"):
        _extra_int30(perm, inputs, golden, log, out)
    if want("multi"):
        _extra_multi(perm, inputs, golden, torch, log, out)
    if want("int10"):
        _extra_int10(perm, inputs, np, out)
    if want("batch"):
        _extra_batch(perm, inputs, np, torch, log, out)
    if want("serving"):
        out["serving"] = serving(perm, inputs, np, torch, log)
    return out


def _extra_n26(perm, inputs, golden, torch, log, out):
    import numpy as np
    C128 = perm.PERM_COMPLEX128
    n = 26
    A = inputs.complex_gaussian(n, seed=0)
    d_a = torch.from_numpy(A).cuda()
    d_res = torch.zeros(1, dtype=torch.complex128, device="cuda")
    ws = perm.device_buffer(perm.perm_workspace_bytes(C128, n))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    perm.perm_solve_async(n, d_a, n, d_res, ws)  # cold: first call with a fresh workspace
    torch.cuda.synchronize()
    cold_ms = (time.perf_counter() - t0) * 1000.0
    perm.perm_solve_async(n, d_a, n, d_res, ws)
    torch.cuda.synchronize()
    ts = []
    for _ in range(10):
        t0 = time.perf_counter()
        perm.perm_solve_async(n, d_a, n, d_res, ws)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    ms = float(np.median(ts)) * 1000.0
    z = complex(d_res.cpu().numpy()[0])
    g = golden.get("c128_n26_s0")
    out["c128_n26"] = {"ms": round(ms, 4), "median_of": 10, "cold_ms": round(cold_ms, 4),
                       "roofline_ms_hbm": round(layer_bytes(26) / HBM_PEAK_GBS / 1e6, 4),
                       "verified": (bits(z) == (int(g["re_bits"], 16), int(g["im_bits"], 16))) if g else None}
    log(f"n=26 complex: {ms:.3f} ms")
    del ws


def _extra_ryser(perm, inputs, torch, log, out):
    """Ryser's formula (eq. 4), the paper's comparison method, at n = 28."""
    C128 = perm.PERM_COMPLEX128
    n = 28
    A28 = inputs.complex_gaussian(n, seed=0)
    d_a = torch.from_numpy(A28).cuda()
    d_r = torch.zeros(2, dtype=torch.complex128, device="cuda")
    ws = perm.device_buffer(perm.perm_ryser_workspace_bytes(C128, n))
    # FP64-bound launches: the clock settles only after a few of them
    for _ in range(10):
        perm.perm_ryser_async(n, d_a, n, d_r[0:1], ws)
    torch.cuda.synchronize()
    perm.perm_profile_enable(True)
    perm.perm_profile_read()
    for _ in range(20):
        perm.perm_ryser_async(n, d_a, n, d_r[0:1], ws)
    pr = perm.perm_profile_read()
    perm.perm_profile_enable(False)
    del ws
    wsz = perm.device_buffer(perm.perm_workspace_bytes(C128, n))
    perm.perm_solve_async(n, d_a, n, d_r[1:2], wsz)
    torch.cuda.synchronize()
    del wsz
    r = d_r.cpu().numpy()
    rms = pr.ryser_ms / max(1, pr.ryser_launches)
    rflops = ryser_flops(n)
    probe = perm.perm_probe_fp64()
    out["ryser_c128_n28"] = {"ms": round(rms, 4), "fp64_tflops": round(rflops / rms / 1e9, 3),
                             "fp64_frac": round(rflops / rms / 1e9 / FP64_PEAK_TFLOPS, 4),
                             "issue_bound_frac": round(ryser_issue_bound(n), 4),
                             "fp64_probe_tflops": round(probe, 2),
                             "fp64_frac_of_probe": round(rflops / rms / 1e9 / probe, 4),
                             "rel_diff_vs_store_zechin": float(abs(r[0] - r[1]) / abs(r[1]))}
    log(f"Ryser n=28: {rms:.3f} ms ({rflops / rms / 1e9:.1f} TFLOP/s; FMA probe {probe:.1f} TFLOP/s), "
        f"rel. diff. to Store-zechin {abs(r[0] - r[1]) / abs(r[1]):.2e}")


def _extra_n34(perm, inputs, torch, log, out):
    """The largest order: Store-zechin sweep (75 GB of layer tables) and
    Ryser's formula on the same 34x34 complex Gaussian matrix."""
    C128 = perm.PERM_COMPLEX128
    n = 34
    A = inputs.complex_gaussian(n, seed=n)
    d_a = torch.from_numpy(A).cuda()
    d_r = torch.zeros(2, dtype=torch.complex128, device="cuda")
    ws = perm.device_buffer(perm.perm_workspace_bytes(C128, n))
    perm.perm_solve_async(n, d_a, n, d_r[0:1], ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        perm.perm_solve_async(n, d_a, n, d_r[0:1], ws)
    torch.cuda.synchronize()
    sz_ms = (time.perf_counter() - t0) * 1000.0 / 3
    ws_gb = ws.numel() / 1e9
    del ws
    torch.cuda.empty_cache()
    wr = perm.device_buffer(perm.perm_ryser_workspace_bytes(C128, n))
    perm.perm_ryser_async(n, d_a, n, d_r[1:2], wr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    perm.perm_ryser_async(n, d_a, n, d_r[1:2], wr)
    torch.cuda.synchronize()
    ry_ms = (time.perf_counter() - t0) * 1000.0
    r = d_r.cpu().numpy()
    out["c128_n34"] = {"store_zechin_ms": round(sz_ms, 2), "workspace_gb": round(ws_gb, 1),
                       "roofline_ms_hbm": round(layer_bytes(n) / HBM_PEAK_GBS / 1e6, 2),
                       "ryser_ms": round(ry_ms, 2),
                       "ryser_fp64_frac": round(ryser_flops(n) / ry_ms / 1e9 / FP64_PEAK_TFLOPS, 4),
                       "rel_diff": float(abs(r[1] - r[0]) / abs(r[0]))}
    log(f"n=34 complex: Store-zechin {sz_ms:.1f} ms ({ws_gb:.0f} GB), Ryser {ry_ms:.1f} ms")


def _extra_compare(perm, inputs, torch, log, out):
    """The paper's comparison (Table 4: Store-zechin against Ryser's eq. (4)),
    measured: both methods on the same complex Gaussian matrices, n = 20..34,
    device-resident, median of 3 after one warm-up call."""
    C128 = perm.PERM_COMPLEX128
    rows = []
    for n in (20, 22, 24, 26, 28, 30, 32, 34):
        A = inputs.complex_gaussian(n, seed=n)
        d_a = torch.from_numpy(A).cuda()
        d_r = torch.zeros(2, dtype=torch.complex128, device="cuda")
        res = {}
        for name, wsb, call in (("store_zechin", perm.perm_workspace_bytes, perm.perm_solve_async),
                                ("ryser", perm.perm_ryser_workspace_bytes, perm.perm_ryser_async)):
            ws = perm.device_buffer(wsb(C128, n))
            slot = d_r[0:1] if name == "store_zechin" else d_r[1:2]
            call(n, d_a, n, slot, ws)
            torch.cuda.synchronize()
            ts = []
            for _ in range(3):
                t0 = time.perf_counter()
                call(n, d_a, n, slot, ws)
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t0) * 1000.0)
            res[name] = sorted(ts)[1]
            del ws
            torch.cuda.empty_cache()
        r = d_r.cpu().numpy()
        rows.append({"n": n, "store_zechin_ms": round(res["store_zechin"], 3), "ryser_ms": round(res["ryser"], 3),
                     "ryser_over_sz": round(res["ryser"] / res["store_zechin"], 3),
                     "rel_diff": float(abs(r[1] - r[0]) / abs(r[0]))})
        log(f"compare n={n}: Store-zechin {res['store_zechin']:.3f} ms, Ryser {res['ryser']:.3f} ms")
    out["store_zechin_vs_ryser"] = rows


def _extra_h2h(perm, inputs, out):
    """Host-to-host n = 28 (PCIe-inclusive, for the record)."""
    C128 = perm.PERM_COMPLEX128
    A28 = inputs.complex_gaussian(28, seed=0)
    ws = perm.device_buffer(perm.perm_workspace_bytes(C128, 28))
    perm.perm_solve(A28, workspace=ws)
    t0 = time.perf_counter()
    for _ in range(5):
        perm.perm_solve(A28, workspace=ws)
    out["c128_n28_host_to_host_ms"] = round((time.perf_counter() - t0) * 200.0, 4)
    del ws


def _extra_int30(perm, inputs, golden, log, out):
    """30x30 Bernoulli 0/1, exact (3 primes: 2 + 1 redundant)."""
    B = inputs.bernoulli01(30, seed=0)
    wsi = perm.device_buffer(perm.perm_workspace_bytes(perm.PERM_INT64, 30))
    v = perm.perm_solve(B, workspace=wsi)
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        v = perm.perm_solve(B, workspace=wsi)
        ts.append((time.perf_counter() - t0) * 1000.0)
    ms = sorted(ts)[2]  # median of 5
    g = golden.get("int_n30_bern_s0")
    # the library's own count of plain 64-bit layers, and the layer kernels'
    # time, from its event profile
    perm.perm_profile_enable(True)
    perm.perm_profile_read()
    for _ in range(3):
        perm.perm_solve(B, workspace=wsi)
    pr = perm.perm_profile_read()
    perm.perm_profile_enable(False)
    K = int(pr.int_plain_layers) // 3 + 1
    launches = int(pr.layer_modp_launches) // 3
    kern_ms = pr.layer_modp_ms / 3
    algo = int_layer_bytes(30, K, 3)
    achieved = algo / (kern_ms * 1e-3) / 1e9
    traffic = None
    cfile = os.path.join(ROOT, "profiles", "layer_modp_n30_counters.json")
    if os.path.exists(cfile):
        with open(cfile) as f:
            cnt = json.load(f)
        if cnt.get("source_hash") == int_source_hash():
            traffic = cnt.get("hbm_bytes_per_launch")
    # the per-term arithmetic: every row of a 0/1 matrix is binary, so every
    # nonzero term is one addition (64-bit on the plain layers, 128-bit per
    # prime on the residue layers); its rate from the probe on the same GPU
    mac_fold, add64 = perm.perm_probe_int()
    plain_terms = resid_terms = 0
    for k in range(2, 31):
        terms = int(B[k - 1].sum()) * math.comb(29, k - 1)
        if k <= K:
            plain_terms += terms
        else:
            resid_terms += 3 * terms
    alu_ms = (plain_terms + 2 * resid_terms) / (add64 * 1e9) * 1e3
    out["int_n30_bernoulli"] = {
        "ms": round(ms, 3), "value": str(v), "verified": (str(v) == g["value"]) if g else None,
        "plain_int64_layers": K, "residues": 3, "hbm_bytes": algo,
        "roofline": {"bound": "hbm", "kernel": "k_layer_modp", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "launches_per_solve": launches,
                     "avg_launch_ms": round(kern_ms / max(launches, 1), 5),
                     "algorithmic_bytes_per_launch": int(algo / max(launches, 1)),
                     "traffic_source": "profiles/layer_modp_n30_counters.json"},
        "alu": {"probe_add64_gops": round(add64, 1), "probe_mac128_fold_gops": round(mac_fold, 1),
                "plain_add_terms": plain_terms, "residue_add_terms": resid_terms,
                "floor_ms": round(alu_ms, 3), "frac": round(alu_ms / kern_ms, 4),
                "note": "128-bit additions counted as two 64-bit ones; the sweep's time goes to index "
                        "work and memory, not to this arithmetic"}}
    log(f"n=30 0/1 integer: {ms:.2f} ms, layer kernels {kern_ms:.2f} ms, {achieved:.0f} GB/s algorithmic; "
        f"ALU floor {alu_ms:.3f} ms (add64 probe {add64:.0f} G/s)")
    del wsi


def multi_layer_sizes(mult):
    """Count vectors per layer: coefficients of prod_j (1 + x + ... + x^mult[j])."""
    c = [1]
    for t in mult:
        d = [0] * (len(c) + int(t))
        for i, v in enumerate(c):
            for e in range(int(t) + 1):
                d[i + e] += v
        c = d
    return c


def multi_bytes(mult, elem: int = 16) -> int:
    """Algorithmic HBM bytes of the repeated-column sweep: every stored value
    of layers 1..n-1 read once, of layers 2..n written once."""
    w = multi_layer_sizes(mult)
    return elem * sum(w[k - 1] + w[k] for k in range(2, len(w)))


def _extra_multi(perm, inputs, golden, torch, log, out):
    """Repeated columns: 40 photons landing uniformly in 20 detectors (seed 0),
    the 40 x m block of a Haar unitary, complex128; and the 36-photon 0/1
    integer case."""
    import numpy as np
    C128 = perm.PERM_COMPLEX128
    n, M = 40, 20
    t = inputs.bunched_pattern(n, M, 0)
    A = inputs.bunched_output(n, t, 0)
    m = len(t)
    d_a = torch.from_numpy(A).cuda()
    d_r = torch.zeros(1, dtype=torch.complex128, device="cuda")
    ws = perm.device_buffer(perm.perm_multi_workspace_bytes(C128, t))
    t0 = time.perf_counter()
    perm.perm_solve_multi_async(n, t, d_a, m, d_r, ws)  # builds and uploads the plan
    torch.cuda.synchronize()
    first_ms = (time.perf_counter() - t0) * 1000.0
    for _ in range(3):
        perm.perm_solve_multi_async(n, t, d_a, m, d_r, ws)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        perm.perm_solve_multi_async(n, t, d_a, m, d_r, ws)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / reps
    perm.perm_profile_enable(True)
    perm.perm_profile_read()
    for _ in range(reps):
        perm.perm_solve_multi_async(n, t, d_a, m, d_r, ws)
    pr = perm.perm_profile_read()
    perm.perm_profile_enable(False)
    z = complex(d_r.cpu().numpy()[0])
    g = golden.get("multi_c128_n40_M20_s0")
    verified = (bits(z) == (int(g["re_bits"], 16), int(g["im_bits"], 16))) if g else None
    kern_ms = pr.multi_c128_ms / reps
    byts = multi_bytes(t)
    sizes = multi_layer_sizes(t)
    traffic = None
    cfile = os.path.join(ROOT, "profiles", "multi_c128_n40_counters.json")
    if os.path.exists(cfile):
        from paper_1802_02779_amd.profiling import multi_source_hash
        with open(cfile) as f:
            cnt = json.load(f)
        if cnt.get("source_hash") == multi_source_hash(ROOT) and cnt.get("mult") == [int(x) for x in t]:
            traffic = cnt.get("hbm_bytes_per_solve")
    out["multi_c128_n40_M20"] = {
        "ms": round(ms, 4), "first_call_ms": round(first_ms, 2), "kernel_ms": round(kern_ms, 4),
        "layer_launches": int(pr.multi_c128_launches // reps), "mult": [int(x) for x in t],
        "count_vectors": int(sum(sizes)), "largest_layer": int(max(sizes)), "algorithmic_bytes": byts,
        "achieved_gbs": round(byts / (kern_ms * 1e-3) / 1e9, 1),
        "hbm_frac": round(byts / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "traffic_bytes": traffic,
        "verified": verified}
    log(f"repeated columns n=40 M=20 (m={m}, {sum(sizes):.3g} count vectors): {ms:.3f} ms, kernels {kern_ms:.3f} ms, "
        f"{byts / (kern_ms * 1e-3) / 1e9:.0f} GB/s algorithmic, first call {first_ms:.1f} ms, verified={verified}")
    del ws
    ti = inputs.bunched_pattern(36, 18, 0)
    B = inputs.bernoulli01(36, seed=0)[:, :len(ti)]
    wsi = perm.device_buffer(perm.perm_multi_workspace_bytes(perm.PERM_INT64, ti))
    v = perm.perm_solve_multi(B, ti, workspace=wsi)
    t0 = time.perf_counter()
    for _ in range(3):
        v = perm.perm_solve_multi(B, ti, workspace=wsi)
    ims = (time.perf_counter() - t0) * 1000.0 / 3
    gi = golden.get("multi_int_n36_M18_bern_s0")
    out["multi_int_n36_M18_bernoulli"] = {"ms": round(ims, 3),
                                          "verified": (str(v) == gi["value"]) if gi else None}
    log(f"repeated columns 0/1 integer n=36 M=18: {ims:.2f} ms")
    del wsi


def _extra_int10(perm, inputs, np, out):
    """10x10 uniform {0..9} integer, host to host."""
    C = inputs.uniform_int(10, 0, 9, seed=0)
    wsc = perm.device_buffer(perm.perm_workspace_bytes(perm.PERM_INT64, 10))
    perm.perm_solve(C, workspace=wsc)
    ts = []
    for _ in range(1000):
        t0 = time.perf_counter()
        perm.perm_solve(C, workspace=wsc)
        ts.append(time.perf_counter() - t0)
    out["int_n10_us_median"] = round(float(np.median(ts)) * 1e6, 2)


def _extra_batch(perm, inputs, np, torch, log, out):
    """Batched: 2^20 submatrices of a 64x64 Haar unitary, n uniform in 3..12."""
    C128 = perm.PERM_COMPLEX128
    count = 1 << 20
    U = inputs.haar_unitary(64, seed=2018)
    t0 = time.perf_counter()
    b = inputs.submatrix_batch(U, count, 3, 12, seed=1)
    log(f"batch input generated in {time.perf_counter() - t0:.1f}s ({b.mats.nbytes / 1e9:.2f} GB)")
    d_mats = torch.from_numpy(b.mats).cuda()
    d_out = torch.zeros(count, dtype=torch.complex128, device="cuda")
    wsb = perm.device_buffer(perm.perm_batch_workspace_bytes(C128, b.ns))
    flags = perm.PERM_BATCH_GRAPH
    perm.perm_solve_batch(C128, b.ns, b.offsets, d_mats, d_out, wsb, flags=flags | perm.PERM_BATCH_SYNC)
    times = []
    for _ in range(10):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        perm.perm_solve_batch(C128, b.ns, b.offsets, d_mats, d_out, wsb,
                              flags=flags | perm.PERM_BATCH_REUSE | perm.PERM_BATCH_SYNC)
        times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    flops = 0
    cnts = np.bincount(b.ns, minlength=13)
    for n in range(3, 13):
        flops += int(cnts[n]) * algorithmic_flops(n)
    perm.perm_profile_enable(True)
    perm.perm_profile_read()
    perm.perm_solve_batch(C128, b.ns, b.offsets, d_mats, d_out, wsb,
                          flags=flags | perm.PERM_BATCH_REUSE | perm.PERM_BATCH_SYNC)
    pb = perm.perm_profile_read()
    perm.perm_profile_enable(False)
    # plain: the same matrices one perm_solve_async at a time (first 4096)
    nplain = 4096
    d_one = torch.zeros(1, dtype=torch.complex128, device="cuda")
    wsp = perm.device_buffer(perm.perm_workspace_bytes(C128, 12))
    views = [d_mats[int(b.offsets[i]):int(b.offsets[i]) + int(b.ns[i]) ** 2] for i in range(nplain)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(nplain):
        perm.perm_solve_async(int(b.ns[i]), views[i], int(b.ns[i]), d_one, wsp)
    torch.cuda.synchronize()
    plain_rate = nplain / (time.perf_counter() - t0)
    out["batch_2p20"] = {"perms_per_s": round(count / med, 1), "ms": round(med * 1000, 3),
                         "kernel_ms": round(pb.batch_ms, 3),
                         "fp64_tflops_kernel": round(flops / (pb.batch_ms * 1e-3) / 1e12, 3),
                         "fp64_frac_kernel": round(flops / (pb.batch_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
                         "plain_perm_solve_perms_per_s": round(plain_rate, 1),
                         "speedup_vs_plain": round(count / med / plain_rate, 1),
                         "launch": "graph replay of one persistent kernel"}
    log(f"batch 2^20: {med * 1000:.2f} ms ({count / med:.3e} perms/s); plain {plain_rate:.0f} perms/s")
    del d_mats, d_out, wsb


def _percentiles(lat):
    import numpy as np
    lat = np.sort(np.asarray(lat))
    if lat.size == 0:
        return {}
    q = lambda p: float(lat[min(lat.size - 1, int(np.ceil(p * lat.size)) - 1)]) * 1000.0  # noqa: E731
    return {"p50_ms": round(q(0.50), 3), "p99_ms": round(q(0.99), 3), "p999_ms": round(q(0.999), 3),
            "mean_ms": round(float(lat.mean()) * 1000.0, 3)}


def _serve_trace(perm, srv, trace, log):
    """Submit at the trace's arrival times; returns per-request (n, latency s)."""
    t0 = time.perf_counter()
    tickets = []
    for i in range(len(trace.ns)):
        while time.perf_counter() - t0 < trace.t_arrive[i]:
            pass
        while True:
            try:
                tickets.append((perm.perm_server_submit(srv, trace.mats[i]), int(trace.ns[i])))
                break
            except perm.PermError as e:
                if e.code != perm.PERM_EAGAIN:
                    raise
    out = []
    for t, n in tickets:
        while True:
            r = perm.perm_server_poll(srv, t)
            if r is not None:
                st = r[1]
                out.append((n, st.t_done - st.t_submit, st.t_submit, st.t_done))
                break
    return out


WARMUP_REQ = 1000     # served first at each load, left out of the statistics
MEASURED_REQ = 20000  # per load level (0.5, 0.8, 0.95 of saturation)
SIDE_REQ = 10000      # the constrained-budget run and the plain FIFO baseline


def serving(perm, inputs, np, torch, log):
    """Poisson arrivals of submatrix permanents of a 64x64 Haar unitary,
    n uniform in 5..12 with probability 0.8, else uniform in 20..28."""
    U = inputs.haar_unitary(64, seed=4242)
    pool = perm.device_buffer(48 << 30)
    res = {}
    # saturation: a burst of requests with the trace's size mix
    burst = inputs.poisson_trace(U, 2000, 1e9, seed=7)
    srv = perm.perm_server_create(pool, max_large_slots=3, queue_capacity=100000, small_n_max=12,
                                  max_small_batch=4096)
    try:
        t0 = time.perf_counter()
        done = _serve_trace(perm, srv, burst, log)
        sat = len(done) / (max(d[3] for d in done) - min(d[2] for d in done))
        log(f"serving saturation: {sat:.0f} requests/s ({time.perf_counter() - t0:.1f}s burst)")
        res["saturation_perms_per_s"] = round(sat, 1)
        for frac in (0.5, 0.8, 0.95):
            rate = frac * sat
            trace = inputs.poisson_trace(U, WARMUP_REQ + MEASURED_REQ, rate, seed=11)
            done = _serve_trace(perm, srv, trace, log)[WARMUP_REQ:]
            lat = [d[1] for d in done]
            span = max(d[3] for d in done) - min(d[2] for d in done)
            entry = {"offered_per_s": round(rate, 1), "perms_per_s": round(len(done) / span, 1)}
            entry.update(_percentiles(lat))
            entry["small_n"] = _percentiles([d[1] for d in done if d[0] <= 12])
            entry["large_n"] = _percentiles([d[1] for d in done if d[0] > 12])
            res[f"load_{frac}"] = entry
            log(f"serving at {rate:.0f}/s: p50 {entry['p50_ms']} ms p99 {entry['p99_ms']} ms")
    finally:
        perm.perm_server_destroy(srv)
    # the same 0.8-load trace with an 8 GiB budget (admission binds: n=28 charges 4 GiB)
    srv = perm.perm_server_create(pool, budget_bytes=8 << 30, max_large_slots=3, queue_capacity=100000,
                                  small_n_max=12, max_small_batch=4096)
    try:
        trace = inputs.poisson_trace(U, WARMUP_REQ + SIDE_REQ, 0.8 * sat, seed=11)
        done = _serve_trace(perm, srv, trace, log)[WARMUP_REQ:]
        entry = {"budget_bytes": 8 << 30, "requests": len(done)}
        entry.update(_percentiles([d[1] for d in done]))
        res["load_0.8_budget_8GiB"] = entry
    finally:
        perm.perm_server_destroy(srv)
    # plain: the same trace served first-in first-out by perm_solve, one at a time
    trace = inputs.poisson_trace(U, WARMUP_REQ + SIDE_REQ, 0.8 * sat, seed=11)
    ws = perm.device_buffer(perm.perm_workspace_bytes(perm.PERM_COMPLEX128, 28))
    lat = []
    t0 = time.perf_counter()
    for i in range(len(trace.ns)):
        while time.perf_counter() - t0 < trace.t_arrive[i]:
            pass
        perm.perm_solve(trace.mats[i], workspace=ws)
        lat.append(time.perf_counter() - t0 - trace.t_arrive[i])
    span = time.perf_counter() - t0
    plain = {"perms_per_s": round(len(lat) / span, 1), "requests": len(lat) - WARMUP_REQ}
    plain.update(_percentiles(lat[WARMUP_REQ:]))
    res["plain_fifo_perm_solve_load_0.8"] = plain
    log(f"plain FIFO: p50 {plain['p50_ms']} ms p99 {plain['p99_ms']} ms")
    return res


def cpu_baseline(inputs, log):
    from oracle import native
    native.build(force=False)
    A = inputs.complex_gaussian(28, seed=0)
    cores = native.max_threads()
    log(f"oracle (C, layers mode) on {cores} host threads, one 28x28 complex permanent ...")
    t0 = time.perf_counter()
    native.per_c128(A, mode=native.MODE_LAYERS, nthreads=0)
    dt = time.perf_counter() - t0
    log(f"oracle: {dt:.1f} s")
    # the 10x10 integer configuration, one core, beside the GPU's end-to-end latency
    C = inputs.uniform_int(10, 0, 9, seed=0)
    ts = []
    for _ in range(100):
        t0 = time.perf_counter()
        native.per_int(C)
        ts.append(time.perf_counter() - t0)
    ts.sort()
    int10_us = ts[len(ts) // 2] * 1e6
    log(f"oracle 10x10 integer: {int10_us:.0f} us")
    # one core: layers mode at n = 24 (1/16 of the n = 28 table), and the
    # paper's own order (memo: recursive development along the last row,
    # each minor stored at first use) at n = 22
    A24 = inputs.complex_gaussian(24, seed=0)
    t0 = time.perf_counter()
    native.per_c128(A24, mode=native.MODE_LAYERS, nthreads=1)
    one24 = time.perf_counter() - t0
    A22 = inputs.complex_gaussian(22, seed=0)
    t0 = time.perf_counter()
    native.per_c128(A22, mode=native.MODE_MEMO)
    memo22 = time.perf_counter() - t0
    log(f"oracle one core: n=24 layers {one24:.2f} s, n=22 memo {memo22:.2f} s")
    # context only: the paper's section 5.2 operation-rate model for n = 28,
    # with the Store-zechin counts M(n) = n(2^(n-1) - 1), A(n) = (n-2) 2^(n-1) + 1
    from oracle import exact
    m28, a28 = 28 * (2 ** 27 - 1), 26 * 2 ** 27 + 1
    paper = {mach: round(exact.machine_time_ms(m28, a28, mach) / 86400e3, 1) for mach in ("ENIAC", "TRADIC")}
    log(f"paper's rate model, n=28 Store-zechin: ENIAC {paper['ENIAC']} days, TRADIC {paper['TRADIC']} days")
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"value": round(1.0 / dt, 5), "unit": "perms/s", "cores": cores, "kind": "oracle",
            "host_cpu_model": model, "host_cpus_usable": usable,
            "paper_rate_model_n28_days": paper,
            "sample": "one full 28x28 complex128 permanent (all 2^28 stored sub-permanents), "
                      f"{dt:.1f} s wall",
            "int_n10_us_median": round(int10_us, 1),
            "one_core_n24_layers_s": round(one24, 3), "one_core_n22_memo_s": round(memo22, 3)}


if __name__ == "__main__":
    main()
