"""Device ceilings the transport kernels are priced against (include/microbench.h).

    python -m paper_1608_05238_amd.microbench          # table + one JSON line
    python -m paper_1608_05238_amd.microbench --lds-only 1024   # LDS atomics in one shape only
                                                               # (for counter runs of rocprofv3)

Each kernel is launched once to warm up, then five times; the fastest launch
(HIP events on the launch stream) gives the rate.  Rates per CU per clock
use the shader clock measured inside the kernel (clock counter against the
constant-rate counter), so they do not assume the nominal 2.4 GHz.
"""
from __future__ import annotations

import ctypes as C
import json
import sys

import torch

from . import _lib as L


def _time(launch, reps: int = 5) -> float:
    launch()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        launch()
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    return best


def _check(name, st):
    if st != 0:
        raise L.MCError(name, st)


# Workgroup shapes of the LDS-atomic kernels: the tiled transport's (one
# 1024-thread workgroup with a 23x23-pixel tile per CU; 144 KiB of the
# kernel's 150 KiB here) and the earlier two 512-thread workgroups with 64 KiB
# each per CU.  Both hold 16 waves per CU, 4 per SIMD.
LDS_SHAPES = {1024: (1024, 144 * 1024, 8), 512: (512, 64 * 1024, 16)}   # block, LDS bytes, workgroups per CU


def run_all(dev: int = 0, lds_shapes=(1024, 512), lds_only: bool = False) -> dict:
    lib = L.load()
    torch.cuda.set_device(dev)
    d = torch.device("cuda", dev)
    stream = C.c_void_p(torch.cuda.current_stream(d).cuda_stream)
    props = torch.cuda.get_device_properties(d)
    ncu = props.multi_processor_count
    khz = C.c_int(0)
    _check("mb_wall_clock_khz", lib.mb_wall_clock_khz(dev, C.byref(khz)))
    clk = torch.zeros(4, dtype=torch.int64, device=d)

    def mhz():
        c = clk.cpu().tolist()
        return (c[1] - c[0]) / max(1, c[3] - c[2]) * khz.value / 1e3

    out = {"device": props.name, "cus": ncu, "wall_clock_khz": khz.value, "lds": [], "global_atomics": []}

    # LDS atomics in each shape (several workgroups per CU slot in turn)
    kinds = [(L.MB_LDS_ADD_F64, "ds_add_f64 random", 2048, 1), (L.MB_LDS_ADD_F32, "ds_add_f32 random", 2048, 1),
             (L.MB_LDS_ADD_U64, "ds_add_u64 random", 2048, 1), (L.MB_LDS_ADD_U32, "ds_add_u32 random", 2048, 1),
             (L.MB_LDS_ADD_F64_ROW33, "ds_add_f64 rows of 33", 64, 33),
             (L.MB_LDS_ADD_U64_ROW33, "ds_add_u64 rows of 33", 64, 33),
             (L.MB_LDS_ADD_U64_PRE, "ds_add_u64, 8 addresses drawn once", 256, 8)]
    for shape in lds_shapes:
        block, lds, per_cu = LDS_SHAPES[shape]
        nblk = ncu * per_cu
        sink = torch.empty(nblk, dtype=torch.float64, device=d)
        for kind, name, iters, per in kinds:   # the same threads per launch in both shapes
            t = _time(lambda: _check("mb_lds_atomics", lib.mb_lds_atomics(kind, lds, block, nblk, iters, 7,
                                                                           sink.data_ptr(), clk.data_ptr(), stream)))
            f = mhz()
            ops = nblk * block * iters * per
            out["lds"].append({"kind": name, "shape": f"{block} threads, {lds // 1024} KiB, {per_cu // 8} per CU",
                               "block": block, "lane_ops_per_launch": ops, "lane_ops_per_s": ops / t,
                               "shader_mhz": f, "lane_ops_per_clk_per_cu": ops / t / (f * 1e6) / ncu, "seconds": t})
        del sink
    if lds_only:
        return out

    # random-address FP64 atomics on the tally sizes of the 32x32 (N = 8) and 256x256 (N = 16) grids
    for label, n in (("1024 px x 17 (139 KB)", 1024 * 17), ("65536 px x 33 (17.3 MB)", 65536 * 33)):
        buf = torch.zeros(n, dtype=torch.float64, device=d)
        nb, iters = ncu * 8, 256
        t = _time(lambda: _check("mb_global_atomics_f64", lib.mb_global_atomics_f64(buf.data_ptr(), n, nb, iters, 3,
                                                                                     stream)))
        out["global_atomics"].append({"buffer": label, "atomics_per_s": nb * 256 * iters / t, "seconds": t})
        del buf
    # the finisher's flush: runs of 33 consecutive doubles of random pixels of the 256x256 (N = 16) tally
    buf = torch.zeros(65536 * 33, dtype=torch.float64, device=d)
    nb, iters = ncu * 8, 33 * 16
    t = _time(lambda: _check("mb_global_atomics_rows_f64", lib.mb_global_atomics_rows_f64(
        buf.data_ptr(), 65536, 33, nb, iters, 5, stream)))
    out["global_atomics_rows"] = {"buffer": "65536 px x 33 (17.3 MB), runs of 33", "atomics_per_s": nb * 256 * iters / t,
                                  "seconds": t}
    del buf

    # HBM: 1 GiB device copy
    n16 = 1 << 26
    a = torch.empty(n16 * 4, dtype=torch.float32, device=d).fill_(1.0)
    b = torch.empty_like(a)
    t = _time(lambda: _check("mb_copy", lib.mb_copy(a.data_ptr(), b.data_ptr(), n16, stream)))
    out["hbm_copy"] = {"bytes": 32 * n16, "gb_per_s": 32 * n16 / t / 1e9, "seconds": t}
    t = _time(lambda: b.copy_(a))   # the runtime's own device copy, for comparison
    out["hbm_copy_runtime"] = {"bytes": 32 * n16, "gb_per_s": 32 * n16 / t / 1e9, "seconds": t}
    del a, b

    # FP32 FMA issue rate (non-packed)
    nb, iters = ncu * 16, 16384
    fs = torch.empty(nb * 256, dtype=torch.float32, device=d)
    t = _time(lambda: _check("mb_fma_f32", lib.mb_fma_f32(fs.data_ptr(), nb, iters, clk.data_ptr(), stream)))
    f = mhz()
    flops = nb * 256 * iters * 8 * 2
    out["fma_f32"] = {"tflops": flops / t / 1e12, "shader_mhz": f,
                      "flops_per_clk_per_cu": flops / t / (f * 1e6) / ncu, "seconds": t}
    return out


def table(r: dict) -> str:
    rows = [f"{r['device']}, {r['cus']} CUs, constant counter {r['wall_clock_khz']} kHz", "",
            "| ceiling | rate | per CU per clock | shader clock (MHz) |", "|---|---|---|---|"]
    for e in r["lds"]:
        rows.append(f"| LDS {e['kind']} ({e['shape']}) | {e['lane_ops_per_s']:.3e} lane-ops/s | "
                    f"{e['lane_ops_per_clk_per_cu']:.2f} | {e['shader_mhz']:.0f} |")
    if "fma_f32" not in r:
        return "\n".join(rows)
    for e in r["global_atomics"]:
        rows.append(f"| global FP64 atomic, random, {e['buffer']} | {e['atomics_per_s']:.3e} /s | | |")
    e = r["global_atomics_rows"]
    rows.append(f"| global FP64 atomic, {e['buffer']} | {e['atomics_per_s']:.3e} /s | | |")
    rows.append(f"| HBM copy (1 GiB read + 1 GiB write) | {r['hbm_copy']['gb_per_s']:.0f} GB/s | | |")
    rows.append(f"| HBM copy, torch copy_ (same buffers) | {r['hbm_copy_runtime']['gb_per_s']:.0f} GB/s | | |")
    e = r["fma_f32"]
    rows.append(f"| FP32 FMA (non-packed) | {e['tflops']:.1f} TFLOP/s | {e['flops_per_clk_per_cu']:.1f} flops | "
                f"{e['shader_mhz']:.0f} |")
    return "\n".join(rows)


def main() -> int:
    if not torch.cuda.is_available():
        print("the microbenchmarks need the GPU", file=sys.stderr)
        return 2
    import argparse
    ap = argparse.ArgumentParser(description="device ceilings of the transport kernels")
    ap.add_argument("--lds-only", type=int, choices=sorted(LDS_SHAPES), default=None,
                    help="only the LDS atomics, in this workgroup size")
    a = ap.parse_args()
    r = run_all(lds_shapes=(a.lds_only,), lds_only=True) if a.lds_only else run_all()
    print(table(r), flush=True)
    print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
