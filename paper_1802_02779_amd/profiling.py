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
    n = int(sys.argv[3]) if len(sys.argv) > 3 else 28
    cur = sqlite3.connect(db).cursor()
    print(f"command: `{cmd}`\n")
    print("| kernel | calls | total us | average us | % |")
    print("|---|---|---|---|---|")
    for name, calls, tot, avg, pct in cur.execute("select * from top_kernels"):
        short = re.sub(r"\(.*", "", name)
        print(f"| {short} | {calls} | {tot:.1f} | {avg:.3f} | {pct:.2f} |")
    rows = list(cur.execute("select duration, grid_x, workgroup_x, lds_size from kernels "
                            "where name like '%k_layer_c128%' order by start"))
    if len(rows) >= n - 1:
        print(f"\nlast step, complex layer sweep, n = {n}:\n")
        print("| layer k | us | tiles | LDS bytes | algorithmic GB/s |")
        print("|---|---|---|---|---|")
        tot = 0
        for k, (d, g, wg, lds) in zip(range(2, n + 1), rows[-(n - 1):]):
            by = 16 * (math.comb(n, k - 1) + math.comb(n, k))
            tot += d
            print(f"| {k} | {d / 1000:.1f} | {g // wg} | {lds} | {by / d:.0f} |")
        print(f"\nsum of the step's layer launches: {tot / 1e6:.3f} ms")


if __name__ == "__main__":
    main()
