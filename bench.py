#!/usr/bin/env python3
"""Benchmark: one step = forward MC + residual + adjoint MC + gradient on the
256x256 disc phantom (four collimated line sources, 1e8 + 1e8 packets, N = 16
harmonics), on one MI355X.  Prints one JSON line.

The hot path follows Hochuli et al. (arXiv:1608.05238): forward radiance MC
with the harmonic tally (Sec. 3, 3.1), adjoint source q* = mua (Hmeas - H)
(Sec. 6), adjoint radiance MC (Sec. 4), gradients from harmonic products
(Sec. 5).  Inputs are synthetic and resident in HBM before timing starts.

Besides the throughput the line carries:
  roofline      the transport kernels' algorithmic tally bytes (272 B per pixel
                visit) per launch over their average launch time (HIP events on
                the launch stream), against the 8 TB/s of HBM3E, and the
                measured HBM traffic per launch (rocprofv3 counters, or null if
                the kernel source changed since they were taken);
  lds_roofline  the K LDS tally adds per visit per second against the
                random-address 64-bit LDS add rate measured in the same run;
  valu_roofline the transport launches' VALU wave-instructions per second
                (rocprofv3's count per visit for this kernel source, null once
                it changes) against one wave64 instruction per SIMD every 4
                cycles at 2.4 GHz;
  cpu_baseline  the FP64 oracle on the host's cores (and on one thread) on a
                bounded sample of the same workload.
Other modes: --time-to-error, --batch, --pencil32 (one JSON line each).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published

# HBM traffic of the transport launches from two rocprofv3 counter passes
# (FETCH_SIZE, then WRITE_SIZE, KiB summed over the launches of one benchmark
# step and divided by their number), each scaled by what the same counter
# reads for a plain 1 GiB device copy.  Valid only for the kernel source it
# was measured on: reported as null once that source changes.
TRAFFIC = {
    "source_sha256": "acb2c6d744c7990c7892e442ad93cc19e8cc09672bd7207f78f9c803cf6eaf7c",
    "fetch_kib_per_launch": 272942.70, "fetch_factor": 2.000,
    "write_kib_per_launch": 835908.56, "write_factor": 1.000,
    # VALU wave-instructions per pixel visit (rocprofv3 SQ_INSTS_VALU over the
    # k_transport_tile<16> and k_finish<16> dispatches of one benchmark step)
    "valu_per_visit": 13.023,
}


def traffic_bytes_per_launch():
    import hashlib
    src = os.path.join(ROOT, "paper_1608_05238_amd", "csrc", "mcrad.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != TRAFFIC["source_sha256"]:
            return None
    t = TRAFFIC
    return 1024.0 * (t["fetch_kib_per_launch"] * t["fetch_factor"] + t["write_kib_per_launch"] * t["write_factor"])


def valu_per_visit():
    """SQ_INSTS_VALU per pixel visit of the transport kernels, or None once
    the kernel source differs from the one it was counted on."""
    import hashlib
    src = os.path.join(ROOT, "paper_1608_05238_amd", "csrc", "mcrad.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != TRAFFIC["source_sha256"]:
            return None
    return TRAFFIC["valu_per_visit"]


def lds_atomic_ceiling(dev) -> float:
    """Lane-operations per second of random-address 64-bit integer LDS adds
    (the tally's atomic) on this device, measured now with the microbenchmark
    kernel in the transport's shape (512-thread workgroups, 64 KiB of LDS
    each); best of three launches."""
    import ctypes as C
    import torch
    from paper_1608_05238_amd import _lib as L
    lib = L.load()
    ncu = torch.cuda.get_device_properties(dev).multi_processor_count
    nblk, block, iters = ncu * 16, 512, 2048
    sink = torch.empty(nblk, dtype=torch.float64, device=dev)
    stream = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    best = float("inf")
    for _ in range(4):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        L.check("mb_lds_atomics", lib.mb_lds_atomics(L.MB_LDS_ADD_U64, 64 * 1024, block, nblk, iters, 7,
                                                     sink.data_ptr(), None, stream))
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    return nblk * block * iters / best


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(n_packets: int, threads: int) -> dict:
    """The FP64 oracle on a bounded sample of the same workload: forward,
    residual, adjoint and gradient with n_packets each, timed on host cores."""
    import numpy as np
    import oracle as O
    import phantoms as P
    c = P.config2()
    ph, true = c.phantom, c.extra["true"]
    om = O.medium_from(ph)
    # measured data: the oracle's own forward on the true phantom (untimed)
    ht, _ = O.run_mc(O.medium_from(true), O.sources_from(c.sources), O.Run(n_packets, 1, 16), n_threads=threads)
    hm = true.mua.astype(np.float64) * ht[0]
    t0 = time.perf_counter()
    fo, _ = O.run_mc(om, O.sources_from(c.sources), O.Run(n_packets, 0, 16), n_threads=threads)
    _, q = O.residual(om, fo, hm)
    ao, _ = O.run_mc(om, [O.Source(O.MAP, map=q)], O.Run(n_packets, 0, 16, stream_tag=1, adjoint=1),
                     n_threads=threads)
    O.gradient(om, 16, fo, ao, hm)
    dt = time.perf_counter() - t0
    # one host thread on a tenth of the sample: the oracle's single-core rate
    n1 = max(1, n_packets // 10)
    t1 = time.perf_counter()
    fo1, _ = O.run_mc(om, O.sources_from(c.sources), O.Run(n1, 0, 16), n_threads=1)
    _, q1 = O.residual(om, fo1, hm)
    ao1, _ = O.run_mc(om, [O.Source(O.MAP, map=q1)], O.Run(n1, 0, 16, stream_tag=1, adjoint=1), n_threads=1)
    O.gradient(om, 16, fo1, ao1, hm)
    dt1 = time.perf_counter() - t1
    return {"value": 2 * n_packets / dt, "unit": "packets/s", "cores": threads, "kind": "oracle",
            "sample": f"disc256 forward+adjoint+gradient, {n_packets}+{n_packets} packets, N=16, FP64, "
                      f"{dt:.1f} s",
            "single_thread": {"value": 2 * n1 / dt1, "unit": "packets/s", "cores": 1,
                              "sample": f"{n1}+{n1} packets, {dt1:.1f} s"}}


def time_to_error(args) -> dict:
    """Second half of the headline metric: wall time of one gradient evaluation
    (forward + residual + adjoint + gradient, N = 16) at the smallest packet
    count (doubling from 1e6, then three geometric bisection steps) whose
    gradients are within 5% (d eps/d mua) and 20% (d eps/d mus) relative L2
    error of a reference gradient from
    args.ref_packets + args.ref_packets packets, over pixels at least 10
    pixels from the boundary."""
    import torch
    import phantoms as P
    from paper_1608_05238_amd import rmc
    dev = torch.device("cuda", 0)
    c = P.config2()
    N = c.n_harm
    med = rmc.Medium.from_phantom(c.phantom, dev)
    tmed = rmc.Medium.from_phantom(c.extra["true"], dev)
    ht, _ = rmc.mc_forward(tmed, c.sources, rmc.make_run(int(args.hmeas_packets), N, seed=1), ledger=False)
    hmeas = rmc.mc_absorbed(tmed, ht)

    def gradient(n, seed):
        f, _ = rmc.mc_forward(med, c.sources, rmc.make_run(n, N, seed=seed), ledger=False)
        q, _ = rmc.mc_residual(med, f, hmeas)
        a, _ = rmc.mc_adjoint(med, [rmc.Source("map", map=q)], rmc.make_run(n, N, seed=seed, stream_tag=1),
                              ledger=False)
        return rmc.mc_gradient(med, N, f, a, hmeas)

    log(f"reference gradient: {args.ref_packets:.0e} + {args.ref_packets:.0e} packets")
    ra, rs = gradient(int(args.ref_packets), 100)
    m = 10
    ra, rs = ra[m:-m, m:-m], rs[m:-m, m:-m]
    rows = []

    def evaluate(n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ga, gs = gradient(n, 7)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ea = float((ga[m:-m, m:-m] - ra).norm() / ra.norm())
        es = float((gs[m:-m, m:-m] - rs).norm() / rs.norm())
        rows.append({"packets": n, "wall_ms": wall * 1e3, "err_dmua": ea, "err_dmus": es})
        log(f"{n:.2e} packets: {wall * 1e3:.1f} ms, error dmua {ea:.4f}, dmus {es:.4f}")
        return ea <= 0.05 and es <= 0.20

    # doubling from 1e6 packets, then three geometric bisection steps between
    # the last count that missed the targets and the first that met them
    n, lo = 1_000_000, None
    while not evaluate(n) and n < args.ref_packets // 4:
        lo, n = n, 2 * n
    hi = n
    if lo is not None and rows[-1]["err_dmua"] <= 0.05 and rows[-1]["err_dmus"] <= 0.20:
        for _ in range(3):
            mid = int(round(math.sqrt(lo * hi) / 1e4)) * 10_000
            if evaluate(mid):
                hi = mid
            else:
                lo = mid
    hit = next(r for r in rows if r["packets"] == hi)
    ok = hit["err_dmua"] <= 0.05 and hit["err_dmus"] <= 0.20
    return {"metric": "wall time to gradient at fixed rel. error (5% d eps/d mua, 20% d eps/d mus)",
            "value": hit["wall_ms"] if ok else None, "unit": "ms", "higher_is_better": False, "n_gpus": 1,
            "packets_forward": hit["packets"], "packets_adjoint": hit["packets"], "reached": ok,
            "reference_packets": int(args.ref_packets), "dtype": "f32", "data": "synthetic",
            "config": {"workload": "disc256: forward + residual + adjoint + gradient, N = 16, interior pixels "
                                   "(10-pixel margin)"},
            "sweep": rows}


def single_gradient(args) -> dict:
    """Wall time of one gradient evaluation on disc256 at args.gradient
    packets per run (the measured data from args.hmeas_packets packets), best
    of args.steps after args.warmup; the time-to-error search's unit of work
    at the packet count it settles on."""
    import torch
    import phantoms as P
    from paper_1608_05238_amd import rmc
    dev = torch.device("cuda", 0)
    c = P.config2()
    N = c.n_harm
    n = int(args.gradient)
    med = rmc.Medium.from_phantom(c.phantom, dev)
    tmed = rmc.Medium.from_phantom(c.extra["true"], dev)
    ht, _ = rmc.mc_forward(tmed, c.sources, rmc.make_run(int(args.hmeas_packets), N, seed=1), ledger=False)
    hmeas = rmc.mc_absorbed(tmed, ht)

    def gradient():
        f, _ = rmc.mc_forward(med, c.sources, rmc.make_run(n, N, seed=7), ledger=False)
        q, _ = rmc.mc_residual(med, f, hmeas)
        a, _ = rmc.mc_adjoint(med, [rmc.Source("map", map=q)], rmc.make_run(n, N, seed=7, stream_tag=1),
                              ledger=False)
        return rmc.mc_gradient(med, N, f, a, hmeas)

    walls = []
    for i in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gradient()
        torch.cuda.synchronize()
        if i >= args.warmup:
            walls.append((time.perf_counter() - t0) * 1e3)
        log(f"gradient at {n:.3g} packets: {(time.perf_counter() - t0) * 1e3:.1f} ms")
    return {"metric": "wall time of one gradient (forward + residual + adjoint + gradient, N=16)",
            "value": min(walls), "unit": "ms", "higher_is_better": False, "n_gpus": 1,
            "packets_forward": n, "packets_adjoint": n, "walls_ms": walls, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "disc256 gradient"}}


def batch_workload(args) -> dict:
    """64 problems in one packet pool: 16 sources x 4 wavelengths (mua scaled
    0.5, 1, 2, 4), grids drawn from {128, 192, 256, 512}^2 over the same
    25.6 mm square, packets per problem log-uniform in [args.batch_min,
    args.batch_max], N = 16.  Timed as one mc_run_batch call and as the same
    64 runs one after the other (the same packets), after autotuning on a
    sample of the batch when args.autotune is set."""
    import numpy as np
    import torch
    import phantoms as P
    from paper_1608_05238_amd import rmc
    rng = np.random.default_rng(3)
    dev = torch.device("cuda", 0)
    side = 25.6
    sizes = rng.choice([128, 192, 256, 512], size=16)      # one grid per source
    # 16 sources: four collimated segments along each side, inward
    segs = []
    for k in range(4):
        a, b = side * k / 4, side * (k + 1) / 4
        segs += [P.SourceSpec("line", a, 0.0, b, 0.0, 0.0, 1.0, 0, 1.0),
                 P.SourceSpec("line", a, side, b, side, 0.0, -1.0, 0, 1.0),
                 P.SourceSpec("line", 0.0, a, 0.0, b, 1.0, 0.0, 0, 1.0),
                 P.SourceSpec("line", side, a, side, b, -1.0, 0.0, 0, 1.0)]
    probs, meta = [], []
    for si in range(16):
        n = int(sizes[si])
        base = P.disc_phantom(n, side / n, 0.01, 10.0, 0.9, seed=100 + si)
        for wi, f in enumerate((0.5, 1.0, 2.0, 4.0)):
            ph = base.copy()
            ph.mua = (ph.mua * f).astype(np.float32)
            npk = int(np.exp(rng.uniform(np.log(args.batch_min), np.log(args.batch_max))))
            probs.append(rmc.Problem(rmc.Medium.from_phantom(ph, dev), [segs[si]],
                                     rmc.make_run(npk, 16, seed=1000 + 4 * si + wi)))
            meta.append((n, f, npk))
    total = sum(m[2] for m in meta)
    tuned = None
    if args.autotune:
        from paper_1608_05238_amd import autotune
        log("autotune on every 4th problem at a quarter of its packets")
        tuned = autotune.tune_batch(probs, every=4, scale=0.25, log=log)["tuning"]
    rmc.mc_run_batch(probs[:2], ledger=False)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rmc.mc_run_batch(probs, ledger=False)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    log(f"batch: {t_batch:.2f} s for {total:.3e} packets")
    t0 = time.perf_counter()
    for pr in probs:
        rmc.mc_forward(pr.medium, pr.sources, pr.run, ledger=False)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    log(f"one by one: {t_seq:.2f} s")
    return {"metric": "packets/s fwd MC, 64 problems in one packet pool (N=16 harmonics)",
            "value": total / t_batch, "unit": "packets/s", "higher_is_better": True, "n_gpus": 1,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": "64 problems: 16 segment sources x 4 wavelengths (mua x0.5-4), grids "
                                   "{128,192,256,512}^2 over 25.6 mm, disc phantoms",
                       "packets_total": total, "packets_per_problem": [args.batch_min, args.batch_max],
                       "grids": [int(x) for x in sizes]},
            "batch_s": t_batch, "one_by_one_s": t_seq, "one_by_one_packets_per_s": total / t_seq,
            "speedup": t_seq / t_batch, "tuning": tuned}


def pencil32(args) -> dict:
    """Forward MC on the 32x32 pencil-beam medium (0.5 mm pixels, mua 0.05,
    mus 5, g 0.8) at args.packets packets, N = 8 and N = 16 (at 1e8 packets
    both take the tiled transport; the whole-grid kernel serves small runs)."""
    import torch
    import phantoms as P
    from paper_1608_05238_amd import rmc
    c = P.config1()
    med = rmc.Medium.from_phantom(c.phantom)
    n = int(args.packets)
    res = {}
    for N in (8, 16):
        rmc.mc_forward(med, c.sources, rmc.make_run(min(n, 1_000_000), N), ledger=False)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, led = rmc.mc_forward(med, c.sources, rmc.make_run(n, N, seed=1))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        L = rmc.ledger_dict(led)
        whole = 32 * 32 * (2 * N + 1) * 8 <= 144 * 1024 and n <= rmc.mc_get_tuning()["grid_max_packets"]
        res[f"N{N}"] = {"packets_per_s": n / dt, "ms": dt * 1e3, "visits_per_packet": L["visits"] / n,
                        "mode": "whole-grid LDS tally" if whole else "tiled"}
        log(f"pencil32 N={N}: {n / dt:.3e} packets/s")
    out = {"metric": "packets/s fwd MC, 32x32 pencil beam", "value": res["N8"]["packets_per_s"],
           "unit": "packets/s", "higher_is_better": True, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "pencil32: 32x32 pixels of 0.5 mm, mua 0.05, mus 5, g 0.8, pencil beam",
                      "packets": n}, "runs": res}
    if args.cpu_packets > 0:   # the oracle on the configuration's own 1e5 packets, N = 8
        import oracle as O
        threads = min(16, os.cpu_count() or 1)
        t0 = time.perf_counter()
        O.run_mc(O.medium_from(c.phantom), O.sources_from(c.sources), O.Run(100_000, 0, 8), n_threads=threads)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1e5 / dt, "unit": "packets/s", "cores": threads, "kind": "oracle",
                               "sample": f"pencil32 forward, 100000 packets, N=8, FP64, {dt:.2f} s"}
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packets", type=float, default=1e8, help="packets per MC run (forward and adjoint each)")
    ap.add_argument("--cpu-packets", type=int, default=60_000, help="oracle sample size (0: skip)")
    ap.add_argument("--hmeas-packets", type=float, default=2e7)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this size first (calibrates HBM counters)")
    ap.add_argument("--time-to-error", action="store_true",
                    help="instead of the throughput line, measure the wall time to a gradient of fixed error")
    ap.add_argument("--ref-packets", type=float, default=1e9, help="packets of the reference gradient (each run)")
    ap.add_argument("--gradient", type=float, default=0,
                    help="time single gradients (forward + residual + adjoint + gradient) at this many packets "
                         "per run, without the reference and the search of --time-to-error")
    ap.add_argument("--batch", action="store_true",
                    help="instead of the throughput line, time the 64-problem batched workload")
    ap.add_argument("--batch-min", type=float, default=1e6)
    ap.add_argument("--batch-max", type=float, default=1e7)
    ap.add_argument("--autotune", action="store_true", help="with --batch: autotune before timing")
    ap.add_argument("--pencil32", action="store_true",
                    help="instead of the throughput line, time the 32x32 pencil-beam forward run (N = 8 and 16)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the Monte Carlo runs on a single MI355X; "
              "sharding packets over several GPUs is not built.", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import phantoms as P
    from paper_1608_05238_amd import rmc

    torch.cuda.set_device(0)
    if args.time_to_error:
        print(json.dumps(time_to_error(args)), flush=True)
        return 0
    if args.batch:
        print(json.dumps(batch_workload(args)), flush=True)
        return 0
    if args.gradient > 0:
        print(json.dumps(single_gradient(args)), flush=True)
        return 0
    if args.pencil32:
        print(json.dumps(pencil32(args)), flush=True)
        return 0
    dev = torch.device("cuda", 0)
    if args.copy_probe_mib > 0:
        a = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    c = P.config2()
    N = c.n_harm
    K = 2 * N + 1
    Np = int(args.packets)
    ph, true = c.phantom, c.extra["true"]
    med = rmc.Medium.from_phantom(ph, dev)
    # measured data Hmeas = mua Phi on the true phantom (untimed set-up)
    log(f"set-up: Hmeas from {int(args.hmeas_packets)} packets on the true phantom")
    tmed = rmc.Medium.from_phantom(true, dev)
    ht, _ = rmc.mc_forward(tmed, c.sources, rmc.make_run(int(args.hmeas_packets), N, seed=1), ledger=False)
    hmeas = (tmed.mua.double() * ht[0]).contiguous()
    ws_f = torch.empty(rmc.mc_workspace_bytes(med, c.sources, rmc.make_run(Np, N)) + 256, dtype=torch.uint8,
                       device=dev)
    fwd = torch.empty((K, ph.nz, ph.nx), dtype=torch.float64, device=dev)
    adj = torch.empty_like(fwd)
    torch.cuda.synchronize()

    ledgers = []

    def step(i: int, keep: bool):
        f, lf = rmc.mc_forward(med, c.sources, rmc.make_run(Np, N, seed=100 + i), out=fwd, workspace=ws_f)
        q, eps = rmc.mc_residual(med, f, hmeas)
        a, la = rmc.mc_adjoint(med, [P.SourceSpec("map", map=q)], rmc.make_run(Np, N, seed=100 + i, stream_tag=1),
                               out=adj)
        g = rmc.mc_gradient(med, N, f, a, hmeas)
        if keep:
            ledgers.append((lf, la))
        return g

    for i in range(args.warmup):
        log(f"warmup step {i}")
        step(i, False)
    torch.cuda.synchronize()
    rmc.mc_profile_read(reset=True)
    rmc.mc_profile_enable(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for i in range(args.steps):
        step(args.warmup + i, True)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rmc.mc_profile_enable(False)
    tr_ms, tr_launches = rmc.mc_profile_read(reset=True)
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    log(f"timed {args.steps} steps: {ms_step:.1f} ms/step (wall {wall:.2f} s)")

    visits = segments = scatters = 0
    for lf, la in ledgers:
        for l in (rmc.ledger_dict(lf), rmc.ledger_dict(la)):
            visits += l["visits"]
            segments += l["segments"]
            scatters += l["scatters"]
    # algorithmic bytes per pixel visit: the K-channel FP64 tally update the
    # method accumulates plus the two medium coefficients of the pixel
    bytes_per_visit = K * 8 + 8
    avg_launch_ms = tr_ms / max(tr_launches, 1)
    achieved = visits * bytes_per_visit / tr_launches / (avg_launch_ms * 1e-3) / 1e9 if tr_launches else 0.0
    value = 2 * Np * args.steps / (ms_total * 1e-3)
    out = {
        "metric": "packets/s fwd+adj MC (N=16 harmonics)",
        "value": value,
        "unit": "packets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "disc256: 256x256 pixels of 0.1 mm, 3-6 seeded disc inclusions, 4 line sources, "
                               "forward + adjoint + gradient",
                   "packets_forward": Np, "packets_adjoint": Np, "n_harm": N,
                   "tally": "64-bit fixed-point LDS tiles, FP64 map, packet migration"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_bytes_per_launch(),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                     "kernel": "k_transport_tile<16> + k_finish<16>", "avg_launch_ms": avg_launch_ms,
                     "launches": tr_launches, "algorithmic_bytes_per_launch": visits * bytes_per_visit / max(tr_launches, 1),
                     "bytes_per_visit": bytes_per_visit,
                     "visits_per_packet": visits / (2 * Np * args.steps),
                     "segments_per_packet": segments / (2 * Np * args.steps),
                     "scatters_per_packet": scatters / (2 * Np * args.steps),
                     "transport_share_of_step": tr_ms / ms_total},
    }
    # the tally's own ceiling: K LDS atomic adds per visit against the device's
    # random-address 64-bit LDS add rate, measured in this run
    ceiling = lds_atomic_ceiling(dev)
    lane_ops = visits * K / max(tr_launches, 1) / (avg_launch_ms * 1e-3) if tr_launches else 0.0
    out["lds_roofline"] = {"bound": "lds_atomics", "achieved": lane_ops, "peak": ceiling, "unit": "lane-ops/s",
                           "frac": lane_ops / ceiling, "kernel": "k_transport_tile<16> + k_finish<16>",
                           "peak_source": "ds_add_u64 at random LDS addresses, mb_lds_atomics, this run"}
    # the issue ceiling the loop actually meets: VALU wave-instructions (counted
    # once per source by rocprofv3) per launch over the live launch time, against
    # one wave64 VALU instruction per SIMD every 4 cycles at the 2.4 GHz peak clock
    vpv = valu_per_visit()
    ncu = torch.cuda.get_device_properties(dev).multi_processor_count
    vpeak = ncu * 4 * 2.4e9 / 4
    vach = vpv * visits / max(tr_launches, 1) / (avg_launch_ms * 1e-3) if (vpv and tr_launches) else None
    out["valu_roofline"] = {"bound": "alu", "achieved": vach, "peak": vpeak, "unit": "wave64 VALU instructions/s",
                            "frac": vach / vpeak if vach else None, "valu_per_visit": vpv,
                            "kernel": "k_transport_tile<16> + k_finish<16>",
                            "peak_source": f"{ncu} CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave64 instruction"}
    if args.cpu_packets > 0:
        threads = min(16, os.cpu_count() or 1)
        log(f"cpu baseline: oracle with {args.cpu_packets}+{args.cpu_packets} packets on {threads} threads")
        out["cpu_baseline"] = cpu_baseline(args.cpu_packets, threads)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
