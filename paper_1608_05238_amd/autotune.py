"""Autotuner of the tiled transport: live packets, job size, visits per stay,
the pause rule of quiet jobs, the smallest job and the tile side (any other
mc_tuning field can be searched through the `space` argument).

`tune()` times short forward (or adjoint) runs of the caller's problem over
candidate tunings and returns the fastest (record it in an optional JSON
cache keyed by grid size, harmonic order and run kind); `tune_batch()` does
the same for a batch of problems (mc_run_batch) on a sample of it.  The
library keeps no tuning state: the caller passes the tuning it got to its
runs (`tuning=` of mc_forward, mc_adjoint, mc_run_batch).  The default search
is coordinate-wise: each knob in turn takes the candidate that runs fastest
with the others held at the best values found so far (19 trials); `grid=True`
tries every combination.  The tuning changes only the schedule (which packets
move together, how often they are sorted); the result of a run is the same
(bitwise while its FP64 sums are exact, see mc_forward in include/mcrad.h).

    python -m paper_1608_05238_amd.autotune      # tune the 256x256 disc workload
"""
from __future__ import annotations

import itertools
import json
import os
import sys
from typing import Callable, Iterable, Optional, Sequence

import torch

from . import rmc

DEFAULT_CANDIDATES = {
    "live_packets": (1 << 25, 1 << 26),
    "job_packets": (8192, 16384, 32768),
    "max_visits": (32, 64, 128),
    "tail_visits": (1, 2, 4),
    "quiet_percent": (35, 50, 75),
    "min_job_packets": (512, 1024, 2048),
    "tile": (16, 23),
}


def candidates(space: Optional[dict] = None) -> Iterable[dict]:
    space = space or DEFAULT_CANDIDATES
    keys = list(space)
    for vals in itertools.product(*(space[k] for k in keys)):
        yield dict(zip(keys, vals))


def _key(medium: rmc.Medium, n_harm: int, adjoint: bool) -> str:
    return f"{medium.nx}x{medium.nz}_N{n_harm}_{'adjoint' if adjoint else 'forward'}"


def _time(run: Callable[[dict], None], tuning: dict) -> float:
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    run(tuning)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3


def search(run: Callable[[dict], None], n_packets: int, space: Optional[dict] = None, log=None,
           grid: bool = False) -> dict:
    """Time `run(tuning)` (moving n_packets packets) under candidate tunings
    and return {"tuning": fastest, "packets_per_s": ..., "trials": [...]}."""
    space = space or DEFAULT_CANDIDATES
    base = rmc.default_tuning()
    trials = []
    run(base)   # warm-up (code, caches)

    def trial(cand: dict) -> float:
        t = _time(run, {**base, **cand})
        trials.append({"tuning": {**base, **cand}, "packets_per_s": n_packets / t})
        if log:
            log(f"{cand}: {n_packets / t:.4e} packets/s")
        return n_packets / t

    if grid:
        for cand in candidates(space):
            trial(cand)
    else:
        best: dict = {}
        for k, vals in space.items():
            rates = {v: trial({**best, k: v}) for v in vals}
            best[k] = max(rates, key=rates.get)
    top = max(trials, key=lambda r: r["packets_per_s"])
    return {"tuning": top["tuning"], "packets_per_s": top["packets_per_s"], "trials": trials}


def tune(medium: rmc.Medium, sources: Sequence, n_harm: int, trial_packets: int = 10_000_000,
         adjoint: bool = False, space: Optional[dict] = None, cache_path: Optional[str] = None, log=None,
         grid: bool = False) -> dict:
    """The fastest tuning for this problem: {"tuning": ..., "packets_per_s":
    ..., "trials": [...]} (from the cache when it holds this problem's key)."""
    key = _key(medium, n_harm, adjoint)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]
    fn = rmc.mc_adjoint if adjoint else rmc.mc_forward
    run = rmc.make_run(trial_packets, n_harm, seed=1, stream_tag=1 if adjoint else 0)
    out = search(lambda t: fn(medium, sources, run, ledger=False, tuning=t), trial_packets, space, log, grid)
    if cache_path:
        cache[key] = {"tuning": out["tuning"], "packets_per_s": out["packets_per_s"]}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return out


def tune_batch(problems: Sequence[rmc.Problem], every: int = 4, scale: float = 0.25,
               space: Optional[dict] = None, log=None, grid: bool = False) -> dict:
    """Tune for a batch on a sample of it: every `every`-th problem with its
    packet count scaled by `scale` (same grids, sources and seeds)."""
    sub = []
    for pr in problems[::every]:
        r = pr.run
        n = max(1, int(r.n_packets * scale))
        sub.append(rmc.Problem(pr.medium, pr.sources,
                               rmc.make_run(n, r.n_harm, r.seed, r.first_packet_id, r.stream_tag, r.w_threshold,
                                            r.roulette_m, r.flags), pr.adjoint))
    total = sum(p.run.n_packets for p in sub)
    return search(lambda t: rmc.mc_run_batch(sub, ledger=False, tuning=t), total, space, log, grid)


def main(argv=None) -> int:
    import argparse
    import numpy as np
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--dx", type=float, default=0.1)
    ap.add_argument("--trial-packets", type=float, default=1e7)
    ap.add_argument("--adjoint", action="store_true")
    ap.add_argument("--cache", default=None)
    args = ap.parse_args(argv)
    dev = torch.device("cuda", 0)
    n, dx = args.n, args.dx
    L = n * dx
    rng = np.random.default_rng(0)
    mua = np.full((n, n), 0.01, np.float32)
    mus = np.full((n, n), 10.0, np.float32)
    c = (np.arange(n) + 0.5) * dx
    X, Z = np.meshgrid(c, c)
    for _ in range(4):
        r = rng.uniform(1, 4)
        cx, cz = rng.uniform(r, L - r, 2)
        inside = (X - cx) ** 2 + (Z - cz) ** 2 <= r * r
        mua[inside] *= rng.uniform(2, 10)
        mus[inside] *= rng.uniform(0.5, 2)
    med = rmc.Medium(torch.as_tensor(mua, device=dev), torch.as_tensor(mus, device=dev),
                     torch.full((n, n), 0.9, dtype=torch.float32, device=dev), dx)
    if args.adjoint:
        q = torch.as_tensor(np.sin(X / 3.0) * np.cos(Z / 5.0) * 1e-3, device=dev)
        src = [rmc.Source("map", map=q)]
    else:
        src = [rmc.Source("line", 0.0, 0.0, L, 0.0, 0.0, 1.0, 0, 0.25), rmc.Source("line", 0.0, L, L, L, 0.0, -1.0, 0, 0.25),
               rmc.Source("line", 0.0, 0.0, 0.0, L, 1.0, 0.0, 0, 0.25), rmc.Source("line", L, 0.0, L, L, -1.0, 0.0, 0, 0.25)]
    res = tune(med, src, 16, int(args.trial_packets), args.adjoint, cache_path=args.cache,
               log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps({"best": res["tuning"], "packets_per_s": res["packets_per_s"],
                      "trials": len(res.get("trials", []))}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
