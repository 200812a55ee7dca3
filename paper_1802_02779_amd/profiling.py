"""Summarize a rocprofv3 --kernel-trace --stats results database as markdown.

    python -m paper_1802_02779_amd.profiling <results.db> "<command that produced it>" > profiles/<name>.md

Lists per-kernel totals (calls, total/average duration) and, for the complex
layer sweep, the per-layer durations of the last step with the algorithmic
bytes of each layer.
"""
import math
import re
import sqlite3
import sys


def main():
    db, cmd = sys.argv[1], sys.argv[2]
    mode = sys.argv[3] if len(sys.argv) > 3 else ""
    multi = mode == "multi"
    n = int(mode) if mode.isdigit() else 28
    cur = sqlite3.connect(db).cursor()
    print(f"command: `{cmd}`\n")
    print("| kernel | calls | total us | average us | % |")
    print("|---|---|---|---|---|")
    for name, calls, tot, avg, pct in cur.execute("select * from top_kernels"):
        short = re.sub(r"\(.*", "", name)
        print(f"| {short} | {calls} | {tot:.1f} | {avg:.3f} | {pct:.2f} |")
    longest = list(cur.execute("select name, duration, grid_x, workgroup_x from kernels "
                               "order by duration desc limit 8"))
    if longest:
        print("\nlongest dispatches:\n")
        print("| kernel | us | workgroups | threads per workgroup |")
        print("|---|---|---|---|")
        for name, d, g, wg in longest:
            print(f"| {re.sub(r'[(].*', '', name)} | {d / 1000:.1f} | {g // max(wg, 1)} | {wg} |")
    if multi:
        multi_layers(cur)
        return
    if mode == "int":
        int_layers(cur, 30)
        return
    rows = list(cur.execute("select duration, grid_x, workgroup_x, lds_size from kernels "
                            "where name like '%k_layer_c128%' order by start"))
    if len(rows) >= n - 1:
        print(f"\nlast step, complex layer sweep, n = {n}:\n")
        print("| layer k | us | workgroups | LDS bytes | algorithmic GB/s |")
        print("|---|---|---|---|---|")
        tot = 0
        for k, (d, g, wg, lds) in zip(range(2, n + 1), rows[-(n - 1):]):
            by = 16 * (math.comb(n, k - 1) + math.comb(n, k))
            tot += d
            print(f"| {k} | {d / 1000:.1f} | {g // wg} | {lds} | {by / d:.0f} |")
        print(f"\nsum of the step's layer launches: {tot / 1e6:.3f} ms")


def int_layers(cur, n):
    """Per-layer durations of the last exact integer solve of order n (one
    k_layer_modp launch per layer k = 2..n): RP residue planes of 8-byte
    values per launch, RP = 1 for the plain 64-bit layers."""
    rows = list(cur.execute("select name, duration, grid_x, workgroup_x from kernels "
                            "where name like '%k_layer_modp%' order by start"))
    if len(rows) < n - 1:
        return
    print(f"\nlast exact integer solve, n = {n}:\n")
    print("| layer k | kernel | us | workgroups | algorithmic GB/s |")
    print("|---|---|---|---|---|")
    tot = 0
    for k, (name, d, g, wg) in zip(range(2, n + 1), rows[-(n - 1):]):
        m = re.search(r"k_layer_modp<(\d+), *(\w+)>", name)
        rp = int(m.group(1)) if m else 1
        by = 8 * rp * (math.comb(n, k - 1) + math.comb(n, k))
        tot += d
        label = m.group(0) if m else "k_layer_modp"
        print(f"| {k} | {label} | {d / 1000:.1f} | {g // wg} | {by / d:.0f} |")
    print(f"\nsum of the solve's layer launches: {tot / 1e6:.3f} ms")


def multi_layers(cur):
    """Per-layer durations of the last complex solve of the repeated-column
    sweep over the 40-photon workload (20 detectors, seed 0)."""
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    from paper_1802_02779_amd import inputs
    t = inputs.bunched_pattern(40, 20, 0).tolist()
    W = multi_layer_sizes(t)
    n = sum(t)
    rows = list(cur.execute("select duration, grid_x, workgroup_x from kernels "
                            "where name like '%k_multi_layer_c128%' order by start"))
    if len(rows) < n - 1:
        return
    print(f"\nlast complex solve, repeated columns {t} (n = {n}):\n")
    print("| layer k | us | workgroups | count vectors | algorithmic GB/s |")
    print("|---|---|---|---|---|")
    tot = 0
    for k, (d, g, wg) in zip(range(2, n + 1), rows[-(n - 1):]):
        by = 16 * (W[k - 1] + W[k])
        tot += d
        print(f"| {k} | {d / 1000:.1f} | {g // wg} | {W[k]} | {by / d:.0f} |")
    print(f"\nsum of the solve's layer launches: {tot / 1e6:.3f} ms")


def source_hash(root: str, n: int = 28) -> str:
    """Hash of what decides the complex layer sweep's memory traffic at order
    n: its kernel sources, the host code that builds the cache-aware tile
    order, and the order-n entries of the shipped tuning file.  Counter data
    is valid only while this hash is unchanged (declarations in shared
    headers are not part of it)."""
    import hashlib
    import json
    import os
    h = hashlib.sha256()
    csrc = os.path.join(root, "paper_1802_02779_amd", "csrc")
    for f in ("perm_layers.hip", "perm_layer_c128.hip", "perm_order.cpp"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    tfile = os.path.join(root, "paper_1802_02779_amd", "tuning", "gfx950.json")
    if os.path.exists(tfile):
        with open(tfile) as fh:
            t = json.load(fh)
        row = [t.get(k, [0] * (n + 1))[n] for k in ("layer_t", "layer_xcd_remap", "layer_flags", "layer_thin")]
        h.update(repr(row).encode())
    return h.hexdigest()[:16]


def int_source_hash(root: str, n: int = 30) -> str:
    """Hash of what decides the integer sweep's memory traffic at order n:
    its kernel sources, the host code that builds the cache-aware tile order,
    and the order-n row of the shipped tuning file."""
    import hashlib
    import json
    import os
    h = hashlib.sha256()
    csrc = os.path.join(root, "paper_1802_02779_amd", "csrc")
    for f in ("perm_layers.hip", "perm_layer_modp.hip", "perm_order.cpp"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    tfile = os.path.join(root, "paper_1802_02779_amd", "tuning", "gfx950.json")
    if os.path.exists(tfile):
        with open(tfile) as fh:
            t = json.load(fh)
        row = [t.get(k, [0] * (n + 1))[n] for k in ("layer_t", "layer_xcd_remap", "layer_flags", "layer_thin")]
        h.update(repr(row).encode())
    return h.hexdigest()[:16]


def modp_counters(fetch_db: str, write_db: str, hit_db: str, cmd: str, root: str, n: int = 30):
    """HBM traffic of one exact integer solve (the last one in the run) of the
    order-n 0/1 workload: every k_layer_modp dispatch of that solve, scaled by
    the 1 GiB copy each run starts with.  Returns (markdown, json-able dict)."""
    def load(db):
        cur = sqlite3.connect(db).cursor()
        rows = list(cur.execute("select dispatch_id, kernel_name, grid_size, counter_name, value "
                                "from counters_collection order by dispatch_id"))
        cal, per = {}, {}
        for d, k, g, c, v in rows:
            if "copyBuffer" in k and g == 131072:
                cal[c] = v
            if "k_layer_modp" in k:
                per.setdefault(d, {})[c] = v
        return cal, [per[d] for d in sorted(per)][-(n - 1):]

    fcal, fl = load(fetch_db)
    wcal, wl = load(write_db)
    _, hl = load(hit_db)
    ff = 1048576.0 / fcal["FETCH_SIZE"]
    wf = 1048576.0 / wcal["WRITE_SIZE"]
    tf = sum(x["FETCH_SIZE"] for x in fl) * 1024 * ff
    tw = sum(x["WRITE_SIZE"] for x in wl) * 1024 * wf
    hits = sum(x["TCC_HIT_sum"] for x in hl)
    misses = sum(x["TCC_MISS_sum"] for x in hl)
    md = (f"commands:\n\n    {cmd}\n\n"
          f"calibration (1 GiB device copy): FETCH_SIZE factor {ff:.4f}, WRITE_SIZE factor {wf:.4f}\n\n"
          f"kernel `k_layer_modp`, the {len(fl)} layer launches of one {n}x{n} 0/1 solve: fetched "
          f"{tf / 1e9:.2f} GB, written {tw / 1e9:.2f} GB, L2 hit rate {hits / max(hits + misses, 1):.3f}\n")
    data = {"source_hash": int_source_hash(root, n), "n": n, "launches": len(fl),
            "hbm_bytes_per_launch": int((tf + tw) / max(len(fl), 1)), "fetch_bytes_per_solve": int(tf),
            "write_bytes_per_solve": int(tw), "fetch_factor": ff, "write_factor": wf}
    return md, data


def counters(fetch_db: str, write_db: str, cmd: str, root: str, n: int = 28, extra_dbs=()):
    """HBM traffic of the complex layer sweep from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE), each scaled by what the same counter reads
    for the 1 GiB device-to-device copy the run starts with.  Returns
    (markdown, json-able dict)."""
    import collections

    def load(db):
        cur = sqlite3.connect(db).cursor()
        rows = list(cur.execute("select dispatch_id, kernel_name, grid_size, counter_name, value, duration "
                                "from counters_collection order by dispatch_id"))
        cal, lay = {}, collections.OrderedDict()
        for d, k, g, c, v, dur in rows:
            if "copyBuffer" in k and g == 131072:
                cal[c] = v
            if "k_layer_c128" in k:
                lay.setdefault(d, {})[c] = v
        return cal, [lay[d] for d in list(lay)[: n - 1]]

    fcal, fl = load(fetch_db)
    wcal, wl = load(write_db)
    extra = [load(db)[1] for db in extra_dbs]
    ff = 1048576.0 / fcal["FETCH_SIZE"]
    wf = 1048576.0 / wcal["WRITE_SIZE"]
    lines = [f"commands:\n\n    {cmd}\n",
             f"calibration (1 GiB device copy): FETCH_SIZE reads {fcal['FETCH_SIZE']:.0f} KiB "
             f"(factor {ff:.4f}), WRITE_SIZE reads {wcal['WRITE_SIZE']:.0f} KiB (factor {wf:.4f})\n",
             "| layer k | algorithmic read MB | fetched MB | algorithmic write MB | written MB |"
             + (" L2 hit |" if extra else ""),
             "|---|---|---|---|---|" + ("---|" if extra else "")]
    tf = tw = ta = 0.0
    hits = misses = 0.0
    for i, k in enumerate(range(2, n + 1)):
        ar, aw = 16 * math.comb(n, k - 1), 16 * math.comb(n, k)
        f = fl[i]["FETCH_SIZE"] * 1024 * ff
        w = wl[i]["WRITE_SIZE"] * 1024 * wf
        tf, tw, ta = tf + f, tw + w, ta + ar + aw
        row = f"| {k} | {ar / 1e6:.1f} | {f / 1e6:.1f} | {aw / 1e6:.1f} | {w / 1e6:.1f} |"
        if extra and "TCC_HIT_sum" in extra[0][i]:
            h, m = extra[0][i]["TCC_HIT_sum"], extra[0][i]["TCC_MISS_sum"]
            hits, misses = hits + h, misses + m
            row += f" {h / max(h + m, 1):.3f} |"
        lines.append(row)
    lines.append(f"\nper step: fetched {tf / 1e9:.2f} GB, written {tw / 1e9:.2f} GB, algorithmic "
                 f"{ta / 1e9:.2f} GB, amplification {(tf + tw) / ta:.2f}"
                 + (f", L2 hit rate {hits / (hits + misses):.3f}" if hits + misses else ""))
    data = {"source_hash": source_hash(root), "n": n, "launches": n - 1,
            "hbm_bytes_per_launch": int((tf + tw) / (n - 1)), "fetch_bytes_per_step": int(tf),
            "write_bytes_per_step": int(tw), "algorithmic_bytes_per_step": int(ta),
            "fetch_factor": ff, "write_factor": wf}
    return "\n".join(lines) + "\n", data


def multi_source_hash(root: str) -> str:
    """Hash of what decides the repeated-column sweep's memory traffic: its
    kernel and plan sources."""
    import hashlib
    import os
    h = hashlib.sha256()
    csrc = os.path.join(root, "paper_1802_02779_amd", "csrc")
    for f in ("perm_multi.hip", "perm_multi.cpp", "perm_multi.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


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


def multi_counters(fetch_db: str, write_db: str, hit_db: str, cmd: str, root: str, mult):
    """HBM traffic of one repeated-column complex solve (the last one in the
    run) from three rocprofv3 --pmc runs, scaled by the 1 GiB copy the run
    starts with, per layer and in total.  Returns (markdown, json-able dict)."""
    import collections

    W = multi_layer_sizes(mult)
    n = len(W) - 1

    def load(db):
        cur = sqlite3.connect(db).cursor()
        rows = list(cur.execute("select dispatch_id, kernel_name, grid_size, counter_name, value "
                                "from counters_collection order by dispatch_id"))
        cal, lay = {}, collections.OrderedDict()
        for d, k, g, c, v in rows:
            if "copyBuffer" in k and g == 131072:
                cal[c] = v
            if "k_multi_layer_c128" in k:
                lay.setdefault(d, {})[c] = v
        return cal, list(lay.values())[-(n - 1):]

    fcal, fl = load(fetch_db)
    wcal, wl = load(write_db)
    _, hl = load(hit_db)
    ff = 1048576.0 / fcal["FETCH_SIZE"]
    wf = 1048576.0 / wcal["WRITE_SIZE"]
    lines = [f"commands:\n\n    {cmd}\n",
             f"workload: column multiplicities {list(map(int, mult))} (n = {n}, {sum(W)} count vectors)\n",
             f"calibration (1 GiB device copy): FETCH_SIZE factor {ff:.4f}, WRITE_SIZE factor {wf:.4f}\n",
             "| layer k | algorithmic read MB | fetched MB | algorithmic write MB | written MB | L2 hit |",
             "|---|---|---|---|---|---|"]
    tf = tw = ta = hits = misses = 0.0
    for i, k in enumerate(range(2, n + 1)):
        ar, aw = 16 * W[k - 1], 16 * W[k]
        f = fl[i]["FETCH_SIZE"] * 1024 * ff
        w = wl[i]["WRITE_SIZE"] * 1024 * wf
        h, m = hl[i]["TCC_HIT_sum"], hl[i]["TCC_MISS_sum"]
        tf, tw, ta, hits, misses = tf + f, tw + w, ta + ar + aw, hits + h, misses + m
        lines.append(f"| {k} | {ar / 1e6:.1f} | {f / 1e6:.1f} | {aw / 1e6:.1f} | {w / 1e6:.1f} | "
                     f"{h / max(h + m, 1):.3f} |")
    lines.append(f"\nper solve: fetched {tf / 1e9:.2f} GB, written {tw / 1e9:.2f} GB, algorithmic "
                 f"{ta / 1e9:.2f} GB, amplification {(tf + tw) / ta:.2f}, L2 hit rate {hits / (hits + misses):.3f}")
    data = {"source_hash": multi_source_hash(root), "mult": [int(x) for x in mult], "launches": n - 1,
            "hbm_bytes_per_solve": int(tf + tw), "fetch_bytes_per_solve": int(tf), "write_bytes_per_solve": int(tw),
            "algorithmic_bytes_per_solve": int(ta), "fetch_factor": ff, "write_factor": wf}
    return "\n".join(lines) + "\n", data


def kernel_counters(fetch_db: str, write_db: str, hit_db: str, cmd: str, kernel: str, launches: int,
                    algorithmic_bytes: int, what: str) -> str:
    """HBM traffic of the last `launches` dispatches of `kernel` (one solve)
    from three rocprofv3 --pmc runs, scaled by the 1 GiB copy each run
    starts with, against the solve's algorithmic bytes."""
    def load(db):
        cur = sqlite3.connect(db).cursor()
        rows = list(cur.execute("select dispatch_id, kernel_name, grid_size, counter_name, value "
                                "from counters_collection order by dispatch_id"))
        cal, per = {}, {}
        for d, k, g, c, v in rows:
            if "copyBuffer" in k and g == 131072:
                cal[c] = v
            if kernel in k:
                per.setdefault(d, {})[c] = v
        return cal, [per[d] for d in sorted(per)][-launches:]

    fcal, fl = load(fetch_db)
    wcal, wl = load(write_db)
    _, hl = load(hit_db)
    ff = 1048576.0 / fcal["FETCH_SIZE"]
    wf = 1048576.0 / wcal["WRITE_SIZE"]
    tf = sum(x["FETCH_SIZE"] for x in fl) * 1024 * ff
    tw = sum(x["WRITE_SIZE"] for x in wl) * 1024 * wf
    hits = sum(x["TCC_HIT_sum"] for x in hl)
    misses = sum(x["TCC_MISS_sum"] for x in hl)
    return (f"commands:\n\n    {cmd}\n\nworkload: {what}\n\n"
            f"calibration (1 GiB device copy): FETCH_SIZE factor {ff:.4f}, WRITE_SIZE factor {wf:.4f}\n\n"
            f"kernel `{kernel}`, {len(fl)} launches of one solve: fetched {tf / 1e9:.2f} GB, written "
            f"{tw / 1e9:.2f} GB, algorithmic {algorithmic_bytes / 1e9:.2f} GB, amplification "
            f"{(tf + tw) / algorithmic_bytes:.2f}, L2 hit rate {hits / max(hits + misses, 1):.3f}\n")


def batch_sq_counters(dbs, cmd: str) -> str:
    """SQ / GRBM counters of the persistent batched launch (the last
    k_batch_c128 dispatch with more than one workgroup) from one or more
    rocprofv3 --pmc runs, with the ratios that say where its cycles go."""
    vals = {}
    for db in dbs:
        cur = sqlite3.connect(db).cursor()
        rows = list(cur.execute("select dispatch_id, kernel_name, grid_size, counter_name, value "
                                "from counters_collection order by dispatch_id"))
        last = {}
        for d, k, g, c, v in rows:
            if "k_batch_c128" in k and g > 4096:  # the persistent launch, not a single-matrix one
                last.setdefault(d, {})[c] = v
        if last:
            vals.update(last[max(last)])
    lines = [f"commands:\n\n    {cmd}\n", "persistent k_batch_c128 launch over the 2^20 mixed batch:\n",
             "| counter | value |", "|---|---|"]
    for c in sorted(vals):
        lines.append(f"| {c} | {vals[c]:.4g} |")
    def ratio(a, b):
        return vals[a] / vals[b] if a in vals and b in vals and vals[b] else None
    derived = [("SQ_WAIT_ANY / SQ_WAVE_CYCLES (waves waiting on anything)", ratio("SQ_WAIT_ANY", "SQ_WAVE_CYCLES")),
               ("SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES", ratio("SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES")),
               ("SQ_ACTIVE_INST_LDS / SQ_WAVE_CYCLES", ratio("SQ_ACTIVE_INST_LDS", "SQ_WAVE_CYCLES")),
               ("SQ_LDS_BANK_CONFLICT / SQ_ACTIVE_INST_LDS", ratio("SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_LDS")),
               ("SQ_INSTS_LDS / SQ_INSTS_VALU", ratio("SQ_INSTS_LDS", "SQ_INSTS_VALU")),
               ("SQ_INSTS_VALU_FMA_F64 / SQ_INSTS_VALU", ratio("SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU")),
               ("SQ_WAVE_CYCLES / SQ_BUSY_CYCLES (resident waves per busy cycle)",
                ratio("SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES"))]
    lines.append("\n| ratio | value |\n|---|---|")
    for name, v in derived:
        if v is not None:
            lines.append(f"| {name} | {v:.3f} |")
    return "\n".join(lines) + "\n"


def layer_unit_counters(dbs, cmd: str, n: int = 28, k_lo: int = 12, k_hi: int = 16) -> str:
    """Unit counters (SQ, TA, TCP, TCC) of the middle layers k_lo..k_hi of the
    last n = 28 step's k_layer_c128 launches, summed over those launches,
    from one or more rocprofv3 --pmc runs, with the ratios that say which
    unit waits on which."""
    tot = {}
    for db in dbs:
        cur = sqlite3.connect(db).cursor()
        per = {}
        for d, k, c, v in cur.execute("select dispatch_id, kernel_name, counter_name, value "
                                      "from counters_collection order by dispatch_id"):
            if "k_layer_c128" in k:
                per.setdefault(d, {})[c] = per.get(d, {}).get(c, 0) + v
        last = sorted(per)[-(n - 1):]
        run = {}
        for d in last[k_lo - 2:k_hi - 1]:
            for c, v in per[d].items():
                run[c] = run.get(c, 0) + v
        for c, v in run.items():
            tot.setdefault(c, v)  # a counter taken in several runs (GRBM_GUI_ACTIVE) counts once
    lines = [f"commands:\n\n    {cmd}\n",
             f"k_layer_c128, layers {k_lo}..{k_hi} of the last {n}x{n} step (sums over those launches; "
             "GRBM_GUI_ACTIVE is summed over the 8 XCDs, TA_BUSY_avr and TCC_BUSY_avr are per-instance "
             "averages):\n", "| counter | value |", "|---|---|"]
    for c in sorted(tot):
        lines.append(f"| {c} | {tot[c]:.4g} |")

    def ratio(a, b, scale=1.0):
        return tot[a] / (tot[b] * scale) if a in tot and b in tot and tot[b] else None
    xcd_cycles = tot.get("GRBM_GUI_ACTIVE", 0) / 8.0
    derived = [
        ("SQ_WAIT_ANY / SQ_WAVE_CYCLES (waves waiting on a counter)", ratio("SQ_WAIT_ANY", "SQ_WAVE_CYCLES")),
        ("SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES", ratio("SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES")),
        ("SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES", ratio("SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES")),
        ("SQ_ACTIVE_INST_LDS / SQ_WAVE_CYCLES", ratio("SQ_ACTIVE_INST_LDS", "SQ_WAVE_CYCLES")),
        ("TA busy (TA_BUSY_avr / GPU cycles per XCD)",
         tot["TA_BUSY_avr"] / xcd_cycles if "TA_BUSY_avr" in tot and xcd_cycles else None),
        ("TCP stalled on data pending from L2 (TCP_PENDING_STALL_CYCLES_sum / 256 CUs / GPU cycles)",
         tot["TCP_PENDING_STALL_CYCLES_sum"] / 256 / xcd_cycles
         if "TCP_PENDING_STALL_CYCLES_sum" in tot and xcd_cycles else None),
        ("L1 -> L2 read latency, cycles (TCP_TCC_READ_REQ_LATENCY_sum / TCP_TCC_READ_REQ_sum)",
         ratio("TCP_TCC_READ_REQ_LATENCY_sum", "TCP_TCC_READ_REQ_sum")),
        ("L2 -> memory read latency, cycles (TCC_EA0_RDREQ_LEVEL_sum / TCC_EA0_RDREQ_sum)",
         ratio("TCC_EA0_RDREQ_LEVEL_sum", "TCC_EA0_RDREQ_sum")),
        ("TCC busy (TCC_BUSY_avr / GPU cycles per XCD)",
         tot["TCC_BUSY_avr"] / xcd_cycles if "TCC_BUSY_avr" in tot and xcd_cycles else None)]
    lines.append("\n| ratio | value |\n|---|---|")
    for name, v in derived:
        if v is not None:
            lines.append(f"| {name} | {v:.3f} |")
    return "\n".join(lines) + "\n"


if __name__ == "__main__" and len(sys.argv) > 1 and sys.argv[1] == "batch-sq":
    # "command" db [db ...]
    print(batch_sq_counters(sys.argv[3:], sys.argv[2]))


if __name__ == "__main__" and len(sys.argv) > 1 and sys.argv[1] == "kernel-counters":
    # fetch.db write.db hit.db "command" kernel launches algorithmic_bytes "workload"
    print(kernel_counters(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6], int(sys.argv[7]),
                          int(sys.argv[8]), sys.argv[9]))


if __name__ == "__main__" and len(sys.argv) > 1 and sys.argv[1] == "multi-counters":
    import json
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    from paper_1802_02779_amd import inputs
    md, data = multi_counters(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], root,
                              inputs.bunched_pattern(40, 20, 0))
    print(md)
    with open(os.path.join(root, "profiles", "multi_c128_n40_counters.json"), "w") as f:
        json.dump(data, f, indent=1)


if __name__ == "__main__" and len(sys.argv) > 1 and sys.argv[1] == "counters":
    import json
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    md, data = counters(sys.argv[2], sys.argv[3], sys.argv[4], root,
                        extra_dbs=sys.argv[5:])
    print(md)
    with open(os.path.join(root, "profiles", "layer_c128_n28_counters.json"), "w") as f:
        json.dump(data, f, indent=1)


if __name__ == "__main__" and len(sys.argv) > 1 and sys.argv[1] == "modp-counters":
    import json
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    md, data = modp_counters(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], root)
    print(md)
    with open(os.path.join(root, "profiles", "layer_modp_n30_counters.json"), "w") as f:
        json.dump(data, f, indent=1)


if __name__ == "__main__" and len(sys.argv) > 1 and sys.argv[1] == "layer-units":
    # "command" db [db ...]
    print(layer_unit_counters(sys.argv[3:], sys.argv[2]))


if __name__ == "__main__" and not (len(sys.argv) > 1 and sys.argv[1] in ("counters", "multi-counters",
                                                                       "kernel-counters", "modp-counters",
                                                                       "batch-sq", "layer-units")):
    main()
