"""Condense rocprofv3 CSV output into the short text tables kept with the
measurements.

    python -m paper_1608_05238_amd.profsum stats <dir>      # --kernel-trace --stats -f csv
    python -m paper_1608_05238_amd.profsum counters <dir>   # --pmc ... -f csv
    python -m paper_1608_05238_amd.profsum tail <dir> <n> <kernel>[,<kernel>...] [<launches>]
    python -m paper_1608_05238_amd.profsum counters-tail <dir> <n> <kernel>[,<kernel>...] [<launches>]
    python -m paper_1608_05238_amd.profsum runs <dir>       # --kernel-trace, per Monte Carlo run

`stats` prints the kernel summary table (calls, total, average); `counters`
sums every counter per kernel over its dispatches and prints the per-dispatch
average, so a counter of a plain copy of known size can calibrate the others;
`tail` averages the durations of the last n dispatches of the named kernels
(from the per-dispatch kernel trace), e.g. the launches of a benchmark's
timed steps; `counters-tail` sums each counter over the last n dispatches of
the named kernels; `runs` cuts a kernel trace into Monte Carlo runs and sums
each run's generation, tile and finisher kernels.  Given <launches>, `tail`
and `counters-tail` also divide the totals by it: a benchmark's timer may
bracket fewer launches than the dispatches its steps make (a launch that
returns at once and is not timed), and the per-launch figures then match the
timer's count.  Only reads CSV files; no GPU work.
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


def counters_tail(root: str, n: int, kernels: list, launches: int = 0) -> str:
    """Each counter summed over the last n dispatches (by dispatch id) of the
    named kernels, and its average per dispatch: the launches of a
    benchmark's timed steps without its set-up runs."""
    files = _find(root, "counter_collection.csv")
    if not files:
        raise SystemExit(f"no *counter_collection.csv under {root}")
    vals = defaultdict(lambda: defaultdict(float))
    names = {}
    for f in files:
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                k = _short(r["Kernel_Name"])
                if k in kernels:
                    d = (int(r["Dispatch_Id"]), r.get("Agent_Id", ""))
                    vals[d][r["Counter_Name"]] += float(r["Counter_Value"])
                    names[d] = k
    last = sorted(vals)[-n:]
    if not last:
        raise SystemExit(f"no dispatch of {kernels} under {root}")
    per = defaultdict(int)
    for d in last:
        per[names[d]] += 1
    tot = defaultdict(float)
    for d in last:
        for c, v in vals[d].items():
            tot[c] += v
    kinds = ", ".join(f"{k}: {m}" for k, m in sorted(per.items()))
    if launches:
        out = [f"last {len(last)} dispatches ({kinds}), per launch over {launches} timed launches",
               "| counter | sum | per dispatch | per launch |", "|---|---|---|---|"]
        for c, v in sorted(tot.items()):
            out.append(f"| {c} | {v:.6e} | {v / len(last):.6e} | {v / launches:.6e} |")
    else:
        out = [f"last {len(last)} dispatches ({kinds})", "| counter | sum | per dispatch |", "|---|---|---|"]
        for c, v in sorted(tot.items()):
            out.append(f"| {c} | {v:.6e} | {v / len(last):.6e} |")
    return "\n".join(out)


def runs(root: str, first_kernel: str = "k_ctl_init") -> str:
    """The kernel trace cut into Monte Carlo runs (a run starts at each
    dispatch of first_kernel): per run its span from that dispatch to the end
    of its last transport dispatch, the summed durations of the generation
    kernels, of the tile kernel and of the finisher, and how many tile
    launches found work (longer than 6 us)."""
    files = _find(root, "kernel_trace.csv")
    if not files:
        raise SystemExit(f"no *kernel_trace.csv under {root}")
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), _short(r["Kernel_Name"])))
    rows.sort()
    out = ["| run | span ms | tile ms | busy / tile launches | generation kernels ms | finisher ms |",
           "|---|---|---|---|---|---|"]
    cur, k = None, 0
    def emit(run, k):
        tr = [x for x in run if x[2].startswith(("k_transport_tile", "k_finish", "k_gen_"))]
        if not tr:
            return
        span = (tr[-1][1] - run[0][0]) / 1e6
        tile = [(e - b) / 1e3 for b, e, n in run if n.startswith("k_transport_tile")]
        gen = sum((e - b) / 1e3 for b, e, n in run if n.startswith("k_gen_"))
        fin = sum((e - b) / 1e3 for b, e, n in run if n.startswith("k_finish"))
        busy = sum(1 for t in tile if t > 6.0)
        out.append(f"| {k} | {span:.1f} | {sum(tile) / 1e3:.1f} | {busy} / {len(tile)} | {gen / 1e3:.1f} | {fin / 1e3:.1f} |")
    for row in rows:
        if row[2] == first_kernel:
            if cur:
                emit(cur, k)
                k += 1
            cur = []
        if cur is not None:
            cur.append(row)
    if cur:
        emit(cur, k)
    return "\n".join(out)


def tail(root: str, n: int, kernels: list, launches: int = 0) -> str:
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
    line = (f"last {len(last)} of {len(rows)} dispatches ({mix}): average {sum(dur) / len(dur) / 1e3:.2f} us, "
            f"total {sum(dur) / 1e3:.1f} us")
    if launches:
        line += f", {sum(dur) / launches / 1e3:.2f} us per timed launch ({launches})"
    return line


def main(argv) -> int:
    if len(argv) in (5, 6) and argv[1] == "tail":
        print(tail(argv[2], int(argv[3]), argv[4].split(","), int(argv[5]) if len(argv) == 6 else 0))
        return 0
    if len(argv) == 3 and argv[1] == "runs":
        print(runs(argv[2]))
        return 0
    if len(argv) in (5, 6) and argv[1] == "counters-tail":
        print(counters_tail(argv[2], int(argv[3]), argv[4].split(","), int(argv[5]) if len(argv) == 6 else 0))
        return 0
    if len(argv) != 3 or argv[1] not in ("stats", "counters"):
        print(__doc__, file=sys.stderr)
        return 2
    print(stats(argv[2]) if argv[1] == "stats" else counters(argv[2]))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
