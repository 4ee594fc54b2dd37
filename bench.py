#!/usr/bin/env python3
"""Benchmark: one step = forward MC + residual + adjoint MC + gradient on the
256x256 disc phantom (four collimated line sources, 1e8 + 1e8 packets, N = 16
harmonics), on one MI355X.  Prints one JSON line.

The hot path follows Hochuli et al. (arXiv:1608.05238): forward radiance MC
with the harmonic tally (Sec. 3, 3.1), adjoint source q* = mua (Hmeas - H)
(Sec. 6), adjoint radiance MC (Sec. 4), gradients from harmonic products
(Sec. 5).  Inputs are synthetic and resident in HBM before timing starts.

Besides the throughput the line carries:
  roofline      the transport kernels' algorithmic arithmetic (lane-operations
                the method itself demands per segment, scatter and launch,
                ALGO_OPS) per launch over their average launch time (HIP
                events on the launch stream), against the chip's vector issue
                rate in lane-operations (157.3 TFLOP/s of packed FP32 FMA =
                2 flops x 2 lanes per issued lane-operation: 3.93e13 /s);
  valu_issue    the VALU wave-instructions the compiled kernels actually issue
                (rocprofv3's count per visit for this kernel source, null once
                it changes) against one wave64 instruction per SIMD every 4
                cycles at 2.4 GHz: how busy the SIMDs are, method or not;
  lds_atomics   the K LDS tally adds per visit per second against the
                random-address 64-bit LDS add rate measured in the same run
                (addresses generated once per 33 adds, as in a tally flush);
  hbm           the transport launches' measured HBM traffic (rocprofv3
                FETCH_SIZE + WRITE_SIZE per launch, calibrated; null once the
                source changes) per average launch time against 8 TB/s;
  time_to_error the other half of the metric: wall time of one gradient
                (forward + residual + adjoint + gradient) at the smallest
                packet count whose gradient errors, averaged over 4 seeds, are
                within 5% (d eps/d mua) and 20% (d eps/d mus) relative L2 of a
                1e9 + 1e9-packet reference, with equal forward and adjoint
                packet counts; `split` holds the same search with
                FWD_ADJ_RATIO forward packets per adjoint packet;
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
# (FETCH_SIZE, then WRITE_SIZE, KiB summed over all 1116 transport dispatches
# of one benchmark step and divided by the 1114 launches the timer brackets:
# the two untimed finisher passes for unlaunched packets find none), each
# scaled by what the same counter reads for a plain 1 GiB device copy.  Valid
# only for the kernel source it was measured on: reported as null once that
# source changes.
TRAFFIC = {
    "source_sha256": "8bb39fd3887b04371c6d942347b4d62e84295b83b6cd1f108f5dbfd0a7129089",
    "fetch_kib_per_launch": 253160.5, "fetch_factor": 2.000,
    "write_kib_per_launch": 364187.4, "write_factor": 1.000,
    # VALU wave-instructions per pixel visit (rocprofv3 SQ_INSTS_VALU over the
    # same dispatches, divided by the step's pixel visits)
    "valu_per_visit": 13.147,
}

# Algorithmic arithmetic of the method, in lane-operations (one FMA, compare,
# logic or integer op, or one transcendental = 1), counted from the steps as
# the paper states them, independent of how the kernels are written:
#  per segment (free path through a pixel, Sec. 3; tally, Sec. 3.1, eq.
#  Fourier_terms): distances to the two pixel faces 4, their minimum 1,
#  optical depth and the scatter test 2, segment length 1, mua l 1, absorbed
#  fraction (1 - e^-x)/x 3, deposit T, weight loss and update 4, position 2,
#  remaining depth 1, pixel step 2, escape test 2; the harmonic tally
#  a_n += T cos n t, b_n += T sin n t: K = 2N+1 multiply-adds;
#  per scatter: Philox4x32-10 10 rounds x (2 products, 2 three-way XORs, 2 key
#  additions) = 60, three uniforms 9, free path -ln u 2, roulette test 2, HG
#  angle 2 atan(((1-g)/(1+g)) tan(pi (u - 1/2))) 6, new direction 3, harmonic
#  vector cos n t, sin n t by recurrence 2N;
#  per launched packet: one Philox block 69, source position and direction 20.
ALGO_OPS = {"segment_base": 23, "scatter_base": 82, "launch": 89}
ISSUE_PEAK_LANE_OPS = 157.3e12 / 4.0   # MI355X fp32 vector peak / (2 flops per FMA x 2 packed lanes)


def algo_ops(segments, scatters, packets, n_harm):
    """Lane-operations of the method for the given event counts."""
    K = 2 * n_harm + 1
    return ((ALGO_OPS["segment_base"] + K) * segments + (ALGO_OPS["scatter_base"] + 2 * n_harm) * scatters
            + ALGO_OPS["launch"] * packets)


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
    kernel in the transport's shape (1024-thread workgroups, 144 KiB of LDS
    each, one per CU), each lane adding to all 33 slots of a random row (one
    address per 33 adds, the pattern of a tally flush at N = 16); best of four
    launches."""
    import ctypes as C
    import torch
    from paper_1608_05238_amd import _lib as L
    lib = L.load()
    ncu = torch.cuda.get_device_properties(dev).multi_processor_count
    nblk, block, iters = ncu * 8, 1024, 128
    sink = torch.empty(nblk, dtype=torch.float64, device=dev)
    stream = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    best = float("inf")
    for _ in range(4):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        L.check("mb_lds_atomics", lib.mb_lds_atomics(L.MB_LDS_ADD_U64_ROW33, 144 * 1024, block, nblk, iters, 7,
                                                     sink.data_ptr(), None, stream))
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    return nblk * block * iters * 33 / best


def host_cpu() -> dict:
    """Threads the oracle may use on this host (the OpenMP thread count the
    environment sets, else every core this process may run on), the cores
    the OS shows, and the CPU model."""
    visible = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS", "")
    threads = min(int(env), visible) if env.isdigit() and int(env) > 0 else visible
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"threads": threads, "cores_visible": visible, "cpu_model": model}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(n_packets: int, threads: int, host: dict) -> dict:
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
    # one host thread on a twentieth of the sample: the oracle's single-core rate
    n1 = max(1, n_packets // 20)
    t1 = time.perf_counter()
    fo1, _ = O.run_mc(om, O.sources_from(c.sources), O.Run(n1, 0, 16), n_threads=1)
    _, q1 = O.residual(om, fo1, hm)
    ao1, _ = O.run_mc(om, [O.Source(O.MAP, map=q1)], O.Run(n1, 0, 16, stream_tag=1, adjoint=1), n_threads=1)
    O.gradient(om, 16, fo1, ao1, hm)
    dt1 = time.perf_counter() - t1
    return {"value": 2 * n_packets / dt, "unit": "packets/s", "cores": threads, "kind": "oracle",
            "sample": f"disc256 forward+adjoint+gradient, {n_packets}+{n_packets} packets, N=16, FP64, "
                      f"{dt:.1f} s",
            "cpu_model": host["cpu_model"], "cores_visible": host["cores_visible"],
            "single_thread": {"value": 2 * n1 / dt1, "unit": "packets/s", "cores": 1,
                              "sample": f"{n1}+{n1} packets, {dt1:.1f} s"}}


# Forward : adjoint packets of the second time-to-error search.  At these
# counts the d eps/d mus error is dominated by the product of the forward and
# adjoint noise (it falls about as 1 / sqrt(N_fwd N_adj)), so the cost
# c_fwd N_fwd + c_adj N_adj of a fixed error is least at N_fwd / N_adj =
# c_adj / c_fwd; an adjoint packet of disc256 costs about twice a forward one
# (1.57 against 0.71 s per 1e8 packets).
FWD_ADJ_RATIO = 2


def time_to_error(args, seeds: int = 4) -> dict:
    """Second half of the headline metric: wall time of one gradient evaluation
    (forward + residual + adjoint + gradient, N = 16) at the smallest packet
    count whose gradients, with their relative L2 errors averaged over `seeds`
    independent seeds, are within 5% (d eps/d mua) and 20% (d eps/d mus) of a
    reference gradient from args.ref_packets + args.ref_packets packets, over
    pixels at least 10 pixels from the boundary.  Search: doubling from
    5e5 packets until the mean errors meet both targets, then four geometric
    bisection steps between the last count that missed and the first that met
    them.  The reported time is the mean wall time of one gradient at that
    count (each timed alone, bracketed by device synchronisations).  The same
    search is then made with FWD_ADJ_RATIO forward packets per adjoint packet
    (`split`), doubling from a quarter of the first search's count."""
    import numpy as np
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

    def gradient(nf, na, seed):
        f, _ = rmc.mc_forward(med, c.sources, rmc.make_run(nf, N, seed=seed), ledger=False)
        q, _ = rmc.mc_residual(med, f, hmeas)
        a, _ = rmc.mc_adjoint(med, [rmc.Source("map", map=q)], rmc.make_run(na, N, seed=seed, stream_tag=1),
                              ledger=False)
        return rmc.mc_gradient(med, N, f, a, hmeas)

    log(f"time to error: reference gradient from {args.ref_packets:.0e} + {args.ref_packets:.0e} packets")
    t0 = time.perf_counter()
    ra, rs = gradient(int(args.ref_packets), int(args.ref_packets), 100)
    torch.cuda.synchronize()
    log(f"reference: {time.perf_counter() - t0:.1f} s")
    m = 10
    ra, rs = ra[m:-m, m:-m], rs[m:-m, m:-m]

    def evaluate(nf, na):
        ea, es, walls = [], [], []
        for k in range(seeds):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ga, gs = gradient(nf, na, 7 + 1000 * k)
            torch.cuda.synchronize()
            walls.append((time.perf_counter() - t0) * 1e3)
            ea.append(float((ga[m:-m, m:-m] - ra).norm() / ra.norm()))
            es.append(float((gs[m:-m, m:-m] - rs).norm() / rs.norm()))
        se = lambda v: float(np.std(v, ddof=1) / np.sqrt(len(v)))
        r = {"packets_forward": nf, "packets_adjoint": na, "wall_ms": float(np.mean(walls)),
             "wall_ms_min": float(np.min(walls)), "err_dmua": float(np.mean(ea)), "err_dmua_se": se(ea),
             "err_dmus": float(np.mean(es)), "err_dmus_se": se(es)}
        log(f"{nf:.3e} + {na:.3e} packets: {r['wall_ms']:.1f} ms, error dmua {r['err_dmua']:.4f} +- "
            f"{r['err_dmua_se']:.4f}, dmus {r['err_dmus']:.4f} +- {r['err_dmus_se']:.4f}")
        return r

    def search(ratio, start):
        rows = {}

        def hit(n):   # n adjoint packets, ratio * n forward
            if n not in rows:
                rows[n] = evaluate(ratio * n, n)
            return rows[n]["err_dmua"] <= 0.05 and rows[n]["err_dmus"] <= 0.20

        n, lo = start, None
        while not hit(n) and n < args.ref_packets // 8:
            lo, n = n, 2 * n
        hi = n
        ok = hit(hi)
        if ok and lo is not None:
            for _ in range(4):
                mid = int(round(math.sqrt(lo * hi) / 1e4)) * 10_000
                if mid in rows or mid <= lo or mid >= hi:
                    break
                if hit(mid):
                    hi = mid
                else:
                    lo = mid
        best = rows[hi]
        return {"value": best["wall_ms"] if ok else None, "reached": ok,
                "packets_forward": best["packets_forward"], "packets_adjoint": best["packets_adjoint"],
                "err_dmua": best["err_dmua"], "err_dmua_se": best["err_dmua_se"],
                "err_dmus": best["err_dmus"], "err_dmus_se": best["err_dmus_se"],
                "sweep": [rows[k] for k in sorted(rows)]}

    eq = search(1, 500_000)
    log(f"time to error, forward : adjoint packets {FWD_ADJ_RATIO} : 1")
    sp = search(FWD_ADJ_RATIO, max(10_000, int(round(eq["packets_adjoint"] / 4 / 1e4)) * 10_000))
    sp["ratio"] = FWD_ADJ_RATIO
    out = {"value": eq["value"], "unit": "ms", "higher_is_better": False, "reached": eq["reached"]}
    out.update({k: v for k, v in eq.items() if k not in ("value", "reached")})
    out.update({"targets": {"dmua": 0.05, "dmus": 0.20}, "seeds": seeds, "reference_packets": int(args.ref_packets),
                "pixels": "interior, 10-pixel margin", "split": sp})
    return out


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

    gens = []

    def gradient():
        f, lf = rmc.mc_forward(med, c.sources, rmc.make_run(n, N, seed=7))
        q, _ = rmc.mc_residual(med, f, hmeas)
        a, la = rmc.mc_adjoint(med, [rmc.Source("map", map=q)], rmc.make_run(n, N, seed=7, stream_tag=1))
        gens.append((lf, la))
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
    g_used = [[rmc.ledger_dict(x)["generations"] for x in pair] for pair in gens]
    return {"metric": "wall time of one gradient (forward + residual + adjoint + gradient, N=16)",
            "value": min(walls), "unit": "ms", "higher_is_better": False, "n_gpus": 1,
            "packets_forward": n, "packets_adjoint": n, "walls_ms": walls, "generations_fwd_adj": g_used,
            "dtype": "f32", "data": "synthetic", "config": {"workload": "disc256 gradient"}}


def batch_workload(args) -> dict:
    """Multi-wavelength gradients of 64 problems: 16 sources x 4 wavelengths
    (mua scaled 0.5, 1, 2, 4), grids drawn from {128, 192, 256, 512}^2 over
    the same 25.6 mm square, packets per problem log-uniform in
    [args.batch_min, args.batch_max], N = 16.  Each problem's gradient is its
    forward run, the residual against its measured data (a 1e6-packet run on
    a second phantom, untimed set-up), its adjoint run and the gradient.
    Timed two ways on the same problems and packets: batched (the 64 forward
    runs in one mc_run_batch call, then the 64 adjoint runs in another) and
    one problem after the other.  The batch moves each problem's packets
    exactly as its own run does, so both reach the same gradient error and
    the ratio of the wall times is the time to the same error.  The maps are
    the same bits while every pixel's FP64 sum is exact; at 1e7-1e8 packets
    the brightest pixels' sums pass 2^53 of their quanta and round in the
    order the atomics arrive, so the comparison reports the largest relative
    differences of the forward maps and of the gradients.  With
    args.autotune the batch first tunes on a sample of itself."""
    import numpy as np
    import torch
    import phantoms as P
    from paper_1608_05238_amd import rmc
    rng = np.random.default_rng(3)
    dev = torch.device("cuda", 0)
    side = 25.6
    N = 16
    sizes = rng.choice([128, 192, 256, 512], size=16)      # one grid per source
    # 16 sources: four collimated segments along each side, inward
    segs = []
    for k in range(4):
        a, b = side * k / 4, side * (k + 1) / 4
        segs += [P.SourceSpec("line", a, 0.0, b, 0.0, 0.0, 1.0, 0, 1.0),
                 P.SourceSpec("line", a, side, b, side, 0.0, -1.0, 0, 1.0),
                 P.SourceSpec("line", 0.0, a, 0.0, b, 1.0, 0.0, 0, 1.0),
                 P.SourceSpec("line", side, a, side, b, -1.0, 0.0, 0, 1.0)]
    probs, truth, meta = [], [], []
    for si in range(16):
        n = int(sizes[si])
        base = P.disc_phantom(n, side / n, 0.01, 10.0, 0.9, seed=100 + si)
        true = P.disc_phantom(n, side / n, 0.01, 10.0, 0.9, seed=500 + si)
        for wi, f in enumerate((0.5, 1.0, 2.0, 4.0)):
            ph, tp = base.copy(), true.copy()
            ph.mua = (ph.mua * f).astype(np.float32)
            tp.mua = (tp.mua * f).astype(np.float32)
            npk = int(np.exp(rng.uniform(np.log(args.batch_min), np.log(args.batch_max))))
            probs.append(rmc.Problem(rmc.Medium.from_phantom(ph, dev), [segs[si]],
                                     rmc.make_run(npk, N, seed=1000 + 4 * si + wi)))
            truth.append(rmc.Problem(rmc.Medium.from_phantom(tp, dev), [segs[si]],
                                     rmc.make_run(1_000_000, N, seed=3000 + 4 * si + wi)))
            meta.append((n, f, npk))
    total = sum(m[2] for m in meta)
    log(f"batch: measured data of 64 problems ({sum(n * n for n, _, _ in meta):.3e} pixels)")
    hmeas = [rmc.mc_absorbed(t.medium, o[0]) for t, o in zip(truth, rmc.mc_run_batch(truth, ledger=False))]
    tuned = None
    if args.autotune:
        from paper_1608_05238_amd import autotune
        log("autotune on every 4th problem at a quarter of its packets")
        tuned = autotune.tune_batch(probs, every=4, scale=0.25, log=log)["tuning"]

    def adjoint_problem(pr, q):
        r = pr.run
        return rmc.Problem(pr.medium, [rmc.Source("map", map=q)],
                           rmc.make_run(r.n_packets, N, seed=r.seed, stream_tag=1), True)

    def batched():
        fw = [o[0] for o in rmc.mc_run_batch(probs, ledger=False, tuning=tuned)]
        qs = [rmc.mc_residual(pr.medium, f, h)[0] for pr, f, h in zip(probs, fw, hmeas)]
        ad = [o[0] for o in rmc.mc_run_batch([adjoint_problem(pr, q) for pr, q in zip(probs, qs)], ledger=False,
                                             tuning=tuned)]
        return fw, [rmc.mc_gradient(pr.medium, N, f, a, h) for pr, f, a, h in zip(probs, fw, ad, hmeas)]

    def one_by_one():
        out, fws = [], []
        for k, (pr, h) in enumerate(zip(probs, hmeas)):
            if k % 16 == 0:
                log(f"one by one: problem {k}")
            f, _ = rmc.mc_forward(pr.medium, pr.sources, pr.run, ledger=False, tuning=tuned)
            fws.append(f)
            q, _ = rmc.mc_residual(pr.medium, f, h)
            ap = adjoint_problem(pr, q)
            a, _ = rmc.mc_adjoint(ap.medium, ap.sources, ap.run, ledger=False, tuning=tuned)
            out.append(rmc.mc_gradient(pr.medium, N, f, a, h))
        return fws, out

    rmc.mc_run_batch(probs[:2], ledger=False)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fb, gb = batched()
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    log(f"batched: {t_batch:.2f} s for {total:.3e} + {total:.3e} packets")
    t0 = time.perf_counter()
    fs, gs = one_by_one()
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    log(f"one by one: {t_seq:.2f} s")
    same = all(torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) for a, b in zip(gb, gs))
    rel = lambda a, b: float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))
    diff_f = max(rel(a, b) for a, b in zip(fb, fs))
    diff_g = max(max(rel(a[0], b[0]), rel(a[1], b[1])) for a, b in zip(gb, gs))
    return {"metric": "wall time to 64 multi-wavelength gradients (fwd + residual + adj + gradient each, N=16)",
            "value": t_batch, "unit": "s", "higher_is_better": False, "n_gpus": 1,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": "64 problems: 16 segment sources x 4 wavelengths (mua x0.5-4), grids "
                                   "{128,192,256,512}^2 over 25.6 mm, disc phantoms",
                       "packets_per_run_total": total, "packets_per_problem": [args.batch_min, args.batch_max],
                       "grids": [int(x) for x in sizes]},
            "batched_s": t_batch, "one_by_one_s": t_seq, "speedup": t_seq / t_batch,
            "packets_per_s_batched": 2 * total / t_batch, "packets_per_s_one_by_one": 2 * total / t_seq,
            "gradients_bitwise_equal": same, "max_rel_diff_forward_maps": diff_f, "max_rel_diff_gradients": diff_g,
            "tuning": tuned}


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
        whole = 32 * 32 * (2 * N + 1) * 8 <= 144 * 1024 and n <= rmc.default_tuning()["grid_max_packets"]
        res[f"N{N}"] = {"packets_per_s": n / dt, "ms": dt * 1e3, "visits_per_packet": L["visits"] / n,
                        "mode": "whole-grid LDS tally" if whole else "tiled"}
        log(f"pencil32 N={N}: {n / dt:.3e} packets/s")
    out = {"metric": "packets/s fwd MC, 32x32 pencil beam", "value": res["N8"]["packets_per_s"],
           "unit": "packets/s", "higher_is_better": True, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "pencil32: 32x32 pixels of 0.5 mm, mua 0.05, mus 5, g 0.8, pencil beam",
                      "packets": n}, "runs": res}
    if args.cpu_packets > 0:   # the oracle on the configuration's own 1e5 packets, N = 8
        import oracle as O
        host = host_cpu()
        threads = host["threads"]
        t0 = time.perf_counter()
        O.run_mc(O.medium_from(c.phantom), O.sources_from(c.sources), O.Run(100_000, 0, 8), n_threads=threads)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1e5 / dt, "unit": "packets/s", "cores": threads, "kind": "oracle",
                               "sample": f"pencil32 forward, 100000 packets, N=8, FP64, {dt:.2f} s",
                               "cpu_model": host["cpu_model"], "cores_visible": host["cores_visible"]}
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packets", type=float, default=1e8, help="packets per MC run (forward and adjoint each)")
    ap.add_argument("--cpu-packets", type=int, default=250_000, help="oracle sample size (0: skip)")
    ap.add_argument("--hmeas-packets", type=float, default=1e8)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this size first (calibrates HBM counters)")
    ap.add_argument("--time-to-error", action="store_true",
                    help="instead of the throughput line, measure only the wall time to a gradient of fixed error")
    ap.add_argument("--no-time-to-error", action="store_true",
                    help="leave the time-to-error measurement out of the throughput line")
    ap.add_argument("--tte-seeds", type=int, default=4, help="seeds averaged per packet count in time to error")
    ap.add_argument("--ref-packets", type=float, default=1e9, help="packets of the reference gradient (each run)")
    ap.add_argument("--gradient", type=float, default=0,
                    help="time single gradients (forward + residual + adjoint + gradient) at this many packets "
                         "per run, without the reference and the search of --time-to-error")
    ap.add_argument("--batch", action="store_true",
                    help="instead of the throughput line, time the 64-problem gradients batched and one by one")
    ap.add_argument("--batch-min", type=float, default=1e7)
    ap.add_argument("--batch-max", type=float, default=1e8)
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
        out = {"metric": "wall time to gradient at fixed rel. error (5% d eps/d mua, 20% d eps/d mus)",
               "n_gpus": 1, "dtype": "f32", "data": "synthetic",
               "config": {"workload": "disc256: forward + residual + adjoint + gradient, N = 16"}}
        out.update(time_to_error(args, args.tte_seeds))
        print(json.dumps(out), flush=True)
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
    # one workspace for both runs (the adjoint's map source adds its CDF)
    need = max(rmc.mc_workspace_bytes(med, c.sources, rmc.make_run(Np, N)),
               rmc.mc_workspace_bytes(med, [P.SourceSpec("map", map=torch.zeros_like(hmeas))],
                                      rmc.make_run(Np, N, stream_tag=1)))
    ws_f = torch.empty(need + 256, dtype=torch.uint8,
                       device=dev)
    fwd = torch.empty((K, ph.nz, ph.nx), dtype=torch.float64, device=dev)
    adj = torch.empty_like(fwd)
    torch.cuda.synchronize()

    ledgers = []
    timer = rmc.Timer()

    def step(i: int, keep: bool):
        tm = timer if keep else None
        f, lf = rmc.mc_forward(med, c.sources, rmc.make_run(Np, N, seed=100 + i), out=fwd, workspace=ws_f, timer=tm)
        q, eps = rmc.mc_residual(med, f, hmeas)
        a, la = rmc.mc_adjoint(med, [P.SourceSpec("map", map=q)], rmc.make_run(Np, N, seed=100 + i, stream_tag=1),
                               out=adj, workspace=ws_f, timer=tm)
        g = rmc.mc_gradient(med, N, f, a, hmeas)
        if keep:
            ledgers.append((lf, la))
        return g

    for i in range(args.warmup):
        log(f"warmup step {i}")
        step(i, False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for i in range(args.steps):
        step(args.warmup + i, True)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tr_ms, tr_launches = timer.read(reset=True)
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    log(f"timed {args.steps} steps: {ms_step:.1f} ms/step (wall {wall:.2f} s)")

    visits = segments = scatters = packets = 0
    gens = []
    for lf, la in ledgers:
        for l in (rmc.ledger_dict(lf), rmc.ledger_dict(la)):
            visits += l["visits"]
            segments += l["segments"]
            scatters += l["scatters"]
            packets += l["packets"]
            gens.append(l["generations"])
    avg_launch_ms = tr_ms / max(tr_launches, 1)
    per_launch = lambda v: v / max(tr_launches, 1)
    launch_s = avg_launch_ms * 1e-3
    ops = algo_ops(segments, scatters, packets, N)
    achieved = per_launch(ops) / launch_s if tr_launches else 0.0
    value = 2 * Np * args.steps / (ms_total * 1e-3)
    kern = "k_transport_tile<16> + k_finish<16>"
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
        # the method's arithmetic against the vector issue rate of the chip
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ISSUE_PEAK_LANE_OPS, "unit": "lane-ops/s",
                     "frac": achieved / ISSUE_PEAK_LANE_OPS, "traffic": None, "kernel": kern,
                     "avg_launch_ms": avg_launch_ms, "launches": tr_launches,
                     "algorithmic_ops_per_launch": per_launch(ops), "ops_per_visit": ops / max(visits, 1),
                     "ops_per_segment": ALGO_OPS["segment_base"] + K, "ops_per_scatter": ALGO_OPS["scatter_base"] + 2 * N,
                     "ops_per_launched_packet": ALGO_OPS["launch"],
                     "peak_source": "157.3 TFLOP/s fp32 vector / (2 flops per FMA x 2 packed lanes)",
                     "visits_per_packet": visits / (2 * Np * args.steps),
                     "segments_per_packet": segments / (2 * Np * args.steps),
                     "scatters_per_packet": scatters / (2 * Np * args.steps),
                     "generations_per_run": gens,
                     "transport_share_of_step": tr_ms / ms_total},
    }
    # HBM: measured traffic of a transport launch (counters of this source) over its time
    tb = traffic_bytes_per_launch()
    out["roofline"]["traffic"] = tb
    out["hbm"] = {"bound": "hbm", "achieved": tb / launch_s / 1e9 if (tb and tr_launches) else None,
                  "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": tb / launch_s / 1e9 / HBM_PEAK_GBS if (tb and tr_launches) else None,
                  "traffic": tb, "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                  "tally_update_bytes_per_launch": per_launch(visits) * (K * 8 + 8), "kernel": kern}
    # the tally's own ceiling: K LDS atomic adds per visit against the device's
    # random-address 64-bit LDS add rate, measured in this run
    ceiling = lds_atomic_ceiling(dev)
    lane_ops = per_launch(visits) * K / launch_s if tr_launches else 0.0
    out["lds_atomics"] = {"bound": "lds", "achieved": lane_ops, "peak": ceiling, "unit": "lane-ops/s",
                          "frac": lane_ops / ceiling, "kernel": kern,
                          "peak_source": "ds_add_u64 to all 33 slots of a random row, mb_lds_atomics, this run"}
    # issue: VALU wave-instructions (counted once per source by rocprofv3) per
    # launch over the live launch time, against one wave64 VALU instruction per
    # SIMD every 4 cycles at the 2.4 GHz peak clock
    vpv = valu_per_visit()
    ncu = torch.cuda.get_device_properties(dev).multi_processor_count
    vpeak = ncu * 4 * 2.4e9 / 4
    vach = vpv * per_launch(visits) / launch_s if (vpv and tr_launches) else None
    out["valu_issue"] = {"bound": "alu", "achieved": vach, "peak": vpeak, "unit": "wave64 VALU instructions/s",
                         "frac": vach / vpeak if vach else None, "valu_per_visit": vpv,
                         "method_share": (ops / max(visits, 1)) / (64 * vpv) if vpv else None, "kernel": kern,
                         "peak_source": f"{ncu} CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave64 instruction"}
    if not args.no_time_to_error:
        out["time_to_error"] = time_to_error(args, args.tte_seeds)
    if args.cpu_packets > 0:
        host = host_cpu()
        threads = host["threads"]
        log(f"cpu baseline: oracle with {args.cpu_packets}+{args.cpu_packets} packets on {threads} threads "
            f"({host['cpu_model']})")
        out["cpu_baseline"] = cpu_baseline(args.cpu_packets, threads, host)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
