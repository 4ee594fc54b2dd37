"""Condense rocprofv3 CSV output into the short text tables kept with the
measurements.

    python -m paper_1608_05238_amd.profsum stats <dir>      # --kernel-trace --stats -f csv
    python -m paper_1608_05238_amd.profsum counters <dir>   # --pmc ... -f csv
    python -m paper_1608_05238_amd.profsum tail <dir> <n> <kernel>[,<kernel>...]

`stats` prints the kernel summary table (calls, total, average); `counters`
sums every counter per kernel over its dispatches and prints the per-dispatch
average, so a counter of a plain copy of known size can calibrate the others;
`tail` averages the durations of the last n dispatches of the named kernels
(from the per-dispatch kernel trace), e.g. the launches of a benchmark's
timed steps.  Only reads CSV files; no GPU work.
"""
from __future__ import annotations

import csv
import glob
import os
import re
import sys
from collections import defaultdict


def _short(name: str) -> str:
    name = name.replace("void ", "").replace("(anonymous namespace)::", "")
    name = re.sub(r"\(.*$", "", name)
    return name.strip()[:60]


def _find(root: str, suffix: str) -> list:
    return sorted(glob.glob(os.path.join(root, "**", f"*{suffix}"), recursive=True))


def stats(root: str) -> str:
    files = _find(root, "kernel_stats.csv")
    if not files:
        raise SystemExit(f"no *kernel_stats.csv under {root}")
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                rows.append((_short(r["Name"]), int(r["Calls"]), float(r["TotalDurationNs"]),
                             float(r["AverageNs"]), float(r["Percentage"])))
    rows.sort(key=lambda x: -x[2])
    out = ["| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for n, c, t, a, p in rows:
        out.append(f"| {n} | {c} | {t / 1e3:.1f} | {a / 1e3:.2f} | {p:.3f} |")
    return "\n".join(out)


def counters(root: str) -> str:
    files = _find(root, "counter_collection.csv")
    if not files:
        raise SystemExit(f"no *counter_collection.csv under {root}")
    tot = defaultdict(float)
    per = defaultdict(lambda: defaultdict(float))
    disp = defaultdict(set)
    for f in files:
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                k = _short(r["Kernel_Name"])
                d = (r.get("Agent_Id", ""), r["Dispatch_Id"])
                v = float(r["Counter_Value"])
                tot[(k, r["Counter_Name"])] += v
                per[(k, r["Counter_Name"])][d] += v
                disp[k].add(d)
    out = ["| kernel | counter | dispatches | sum | per dispatch | largest dispatch |", "|---|---|---|---|---|---|"]
    for (k, c), v in sorted(tot.items(), key=lambda x: -x[1]):
        n = len(disp[k])
        out.append(f"| {k} | {c} | {n} | {v:.6e} | {v / max(n, 1):.6e} | {max(per[(k, c)].values()):.6e} |")
    return "\n".join(out)


def tail(root: str, n: int, kernels: list) -> str:
    files = _find(root, "kernel_trace.csv")
    if not files:
        raise SystemExit(f"no *kernel_trace.csv under {root}")
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                k = _short(r["Kernel_Name"])
                if k in kernels:
                    rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), k))
    rows.sort()
    last = rows[-n:]
    if not last:
        raise SystemExit(f"no dispatch of {kernels} under {root}")
    dur = [e - b for b, e, _ in last]
    per = defaultdict(int)
    for _, _, k in last:
        per[k] += 1
    mix = ", ".join(f"{k}: {c}" for k, c in sorted(per.items()))
    return (f"last {len(last)} of {len(rows)} dispatches ({mix}): average {sum(dur) / len(dur) / 1e3:.2f} us, "
            f"total {sum(dur) / 1e3:.1f} us")


def main(argv) -> int:
    if len(argv) == 5 and argv[1] == "tail":
        print(tail(argv[2], int(argv[3]), argv[4].split(",")))
        return 0
    if len(argv) != 3 or argv[1] not in ("stats", "counters"):
        print(__doc__, file=sys.stderr)
        return 2
    print(stats(argv[2]) if argv[1] == "stats" else counters(argv[2]))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
