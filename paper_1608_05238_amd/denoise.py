"""Learned denoiser of harmonic coefficient maps on BF16 matrix cores.

A small U-Net maps the 2N+1 coefficient maps of a run with few packets to
those of a run with many packets, so that a gradient evaluation can stand on
fewer packets.  Its 3x3 convolutions (forward, input gradient and weight
gradient) are the hand-written MFMA kernels of denoise.h (BF16 operands,
FP32 accumulation); pooling, upsampling, ReLU and the 1x1 output layer are
plain PyTorch.  Training pairs come from the Monte Carlo itself, run as
batches of problems (mc_run_batch).  The plain Monte Carlo stays the
reference and the fallback: `denoise_or_mc` returns the network's maps only when its
measured error on held-out pairs is below a threshold, else it runs more
packets.

    python -m paper_1608_05238_amd.denoise     # generate pairs, train, evaluate
"""
from __future__ import annotations

import ctypes as C
import json
import math
import sys
import time
from typing import List, Sequence, Tuple

import numpy as np
import torch
import torch.nn as nn
import torch.nn.functional as F

from . import _lib as L
from . import rmc


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _pad8(n: int) -> int:
    return (n + 7) // 8 * 8


def _nhwc_bf16(t: torch.Tensor, c_pad: int) -> torch.Tensor:
    """[n][c][h][w] as BF16 in channels-last storage ([n][h][w][c] in memory),
    zero channels appended up to c_pad."""
    t = t.detach().to(torch.bfloat16)
    if c_pad > t.shape[1]:
        t = F.pad(t, (0, 0, 0, 0, 0, c_pad - t.shape[1]))
    return t.contiguous(memory_format=torch.channels_last)


class _Conv3x3(torch.autograd.Function):
    """3x3 convolution, stride 1, padding 1, with BF16 operands on the MFMA
    units.  The kernels take channels-last data with a multiple of 8 channels:
    the operands are converted here (channels padded with zeros); outputs are
    channels-last FP32 tensors."""

    @staticmethod
    def forward(ctx, x, w, b):
        lib = L.load()
        n, ci, h, wd = x.shape
        co = w.shape[0]
        cip = _pad8(ci)
        xb = _nhwc_bf16(x, cip)
        wb = F.pad(w.detach().to(torch.bfloat16), (0, 0, 0, 0, 0, cip - ci)).permute(0, 2, 3, 1).contiguous()
        y = torch.empty((n, co, h, wd), dtype=torch.float32, device=x.device, memory_format=torch.channels_last)
        bias = b.detach().float().contiguous()
        L.check("dn_conv3x3_fwd", lib.dn_conv3x3_fwd(xb.data_ptr(), wb.data_ptr(), bias.data_ptr(), y.data_ptr(),
                                                     n, cip, co, h, wd, _stream()))
        ctx.save_for_backward(xb, w.detach())
        ctx.shape = (n, ci, co, h, wd)
        return y

    @staticmethod
    def backward(ctx, gy):
        lib = L.load()
        xb, w = ctx.saved_tensors
        n, ci, co, h, wd = ctx.shape
        cip, cop = _pad8(ci), _pad8(co)
        gyb = _nhwc_bf16(gy, cop)
        gx = gw = gb = None
        if ctx.needs_input_grad[0]:
            # the input gradient: the same convolution with the weights flipped
            # and input / output channels swapped, [ci][3][3][co]
            wt = F.pad(w.to(torch.bfloat16).flip(2, 3).permute(1, 2, 3, 0), (0, cop - co)).contiguous()
            gx = torch.empty((n, ci, h, wd), dtype=torch.float32, device=gy.device, memory_format=torch.channels_last)
            L.check("dn_conv3x3_fwd", lib.dn_conv3x3_fwd(gyb.data_ptr(), wt.data_ptr(), None, gx.data_ptr(),
                                                         n, cop, ci, h, wd, _stream()))
        if ctx.needs_input_grad[1]:
            g = torch.empty((cop, 3, 3, cip), dtype=torch.float32, device=gy.device)
            L.check("dn_conv3x3_wgrad", lib.dn_conv3x3_wgrad(xb.data_ptr(), gyb.data_ptr(), g.data_ptr(),
                                                             n, cip, cop, h, wd, _stream()))
            gw = g[:co, :, :, :ci].permute(0, 3, 1, 2).contiguous()
        if ctx.needs_input_grad[2]:
            gb = gy.sum(dim=(0, 2, 3))
        return gx, gw, gb


def conv3x3(x, w, b):
    return _Conv3x3.apply(x, w, b)


class Conv3x3(nn.Module):
    def __init__(self, ci: int, co: int):
        super().__init__()
        self.weight = nn.Parameter(torch.randn(co, ci, 3, 3) * math.sqrt(2.0 / (9 * ci)))
        self.bias = nn.Parameter(torch.zeros(co))

    def forward(self, x):
        return conv3x3(x, self.weight, self.bias)


class UNet(nn.Module):
    """Encoder-decoder with skip connections over len(widths) levels; predicts
    a correction added to the (normalised) input maps."""

    def __init__(self, channels: int, widths: Sequence[int] = (48, 64, 96)):
        super().__init__()
        self.enc = nn.ModuleList()
        c = channels
        for wdt in widths:
            self.enc.append(nn.ModuleList([Conv3x3(c, wdt), Conv3x3(wdt, wdt)]))
            c = wdt
        self.dec = nn.ModuleList()
        for wdt in reversed(widths[:-1]):
            self.dec.append(nn.ModuleList([Conv3x3(c + wdt, wdt), Conv3x3(wdt, wdt)]))
            c = wdt
        self.out = nn.Parameter(torch.zeros(channels, c))   # 1x1 output layer
        self.out_bias = nn.Parameter(torch.zeros(channels))

    def forward(self, x):
        skips = []
        h = x
        for i, (c1, c2) in enumerate(self.enc):
            h = F.relu(c2(F.relu(c1(h))))
            if i < len(self.enc) - 1:
                skips.append(h)
                h = F.max_pool2d(h, 2, ceil_mode=True)
        for c1, c2 in self.dec:
            s = skips.pop()
            h = F.interpolate(h, scale_factor=2, mode="nearest")[:, :, :s.shape[2], :s.shape[3]]
            h = F.relu(c2(F.relu(c1(torch.cat([h, s], 1)))))
        corr = torch.einsum("oc,nchw->nohw", self.out, h) + self.out_bias[None, :, None, None]
        return x + corr


def _scale(maps: torch.Tensor) -> torch.Tensor:
    """Per-sample scale: the RMS of the a0 map (positive for any nonzero map,
    also for the signed adjoint fields)."""
    return maps[:, 0].double().pow(2).mean(dim=(1, 2)).sqrt().clamp_min(1e-30).to(maps.dtype)


def _normalise(maps: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
    s = _scale(maps)
    return maps / s[:, None, None, None], s


def random_phantom_medium(n: int, side: float, seed: int, device) -> rmc.Medium:
    """Background mua 0.01, mus 10 /mm, g 0.9 with 3-6 random discs (radius
    1-4 mm, mua x2-10, mus x0.5-2), the recipe of the disc workload."""
    rng = np.random.default_rng(seed)
    dx = side / n
    mua = np.full((n, n), 0.01, np.float32)
    mus = np.full((n, n), 10.0, np.float32)
    c = (np.arange(n) + 0.5) * dx
    X, Z = np.meshgrid(c, c)
    for _ in range(int(rng.integers(3, 7))):
        r = rng.uniform(1.0, 4.0)
        cx, cz = rng.uniform(r, side - r, 2)
        inside = (X - cx) ** 2 + (Z - cz) ** 2 <= r * r
        mua[inside] = np.float32(0.01 * rng.uniform(2, 10))
        mus[inside] = np.float32(10.0 * rng.uniform(0.5, 2))
    return rmc.Medium(torch.as_tensor(mua, device=device), torch.as_tensor(mus, device=device),
                      torch.full((n, n), 0.9, dtype=torch.float32, device=device), dx)


def random_adjoint_source(med: rmc.Medium, seed: int) -> torch.Tensor:
    """A signed map shaped like an adjoint source mua (Hmeas - H): smooth
    random blobs of either sign times the medium's mua (relative to its mean)."""
    rng = np.random.default_rng(seed)
    n, dx = med.nx, med.dx
    c = (np.arange(n) + 0.5) * dx
    X, Z = np.meshgrid(c, c)
    q = np.zeros((n, n))
    for _ in range(int(rng.integers(3, 9))):
        x0, z0 = rng.uniform(0, n * dx, 2)
        w = rng.uniform(0.05, 0.3) * n * dx
        q += rng.choice([-1.0, 1.0]) * rng.uniform(0.3, 1.5) * np.exp(-((X - x0) ** 2 + (Z - z0) ** 2) / (2 * w * w))
    mua = med.mua.double()
    return torch.as_tensor(q, device=mua.device) * (mua / mua.mean()) * 1e-3


def side_sources(side: float) -> List[rmc.Source]:
    return [rmc.Source("line", 0.0, 0.0, side, 0.0, 0.0, 1.0, 0, 0.25),
            rmc.Source("line", 0.0, side, side, side, 0.0, -1.0, 0, 0.25),
            rmc.Source("line", 0.0, 0.0, 0.0, side, 1.0, 0.0, 0, 0.25),
            rmc.Source("line", side, 0.0, side, side, -1.0, 0.0, 0, 0.25)]


def make_pairs(n_samples: int, n: int, side: float, n_low: int, n_high: int, n_harm: int, seed0: int,
               batch: int = 32, adjoint: bool = False):
    """(low, high) coefficient maps [S][2N+1][n][n] from independent runs of
    n_low and n_high packets on seeded random phantoms (batched): forward runs
    of the four side sources, or adjoint runs of a random_adjoint_source."""
    dev = torch.device("cuda", torch.cuda.current_device())
    lows, highs = [], []
    for b0 in range(0, n_samples, batch):
        probs = []
        for i in range(b0, min(n_samples, b0 + batch)):
            med = random_phantom_medium(n, side, seed0 + i, dev)
            src = [rmc.Source("map", map=random_adjoint_source(med, seed0 + i))] if adjoint else side_sources(side)
            tag = 1 if adjoint else 0
            probs.append(rmc.Problem(med, src, rmc.make_run(n_low, n_harm, seed=2 * (seed0 + i), stream_tag=tag),
                                     adjoint))
            probs.append(rmc.Problem(med, src, rmc.make_run(n_high, n_harm, seed=2 * (seed0 + i) + 1,
                                                            stream_tag=tag), adjoint))
        outs = rmc.mc_run_batch(probs, ledger=False)
        lows += [o[0] for o in outs[0::2]]
        highs += [o[0] for o in outs[1::2]]
    return torch.stack(lows).float(), torch.stack(highs).float()


def rel_error(a: torch.Tensor, b: torch.Tensor) -> float:
    """Relative L2 error of a against b over the whole set."""
    return float((a - b).norm() / b.norm())


def train(model: UNet, low: torch.Tensor, high: torch.Tensor, epochs: int, batch: int = 16, lr: float = 2e-3,
          log=None):
    xl, s = _normalise(low)
    yh = high / s[:, None, None, None]
    opt = torch.optim.Adam(model.parameters(), lr=lr)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, epochs)
    g = torch.Generator(device="cpu").manual_seed(0)
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(len(xl), generator=g)
        tot = 0.0
        for i in range(0, len(xl), batch):
            idx = perm[i:i + batch].to(xl.device)
            loss = F.mse_loss(model(xl[idx]), yh[idx])
            opt.zero_grad()
            loss.backward()
            opt.step()
            tot += float(loss.detach()) * len(idx)
        sched.step()
        hist.append(tot / len(xl))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4e}")
    return hist


@torch.no_grad()
def denoise(model: UNet, maps: torch.Tensor) -> torch.Tensor:
    x, s = _normalise(maps.float())
    return model(x) * s[:, None, None, None]


def denoise_or_mc(model: UNet, val_error: float, medium: rmc.Medium, sources, n_low: int, n_fallback: int,
                  n_harm: int, threshold: float = 0.02, seed: int = 0):
    """Maps for (medium, sources): the denoised n_low-packet run when the
    network's held-out error is below `threshold`, else the plain Monte Carlo
    with n_fallback packets.  Returns (maps, "denoised" | "monte-carlo")."""
    if val_error <= threshold:
        low, _ = rmc.mc_forward(medium, sources, rmc.make_run(n_low, n_harm, seed=seed), ledger=False)
        return denoise(model, low[None])[0].double(), "denoised"
    maps, _ = rmc.mc_forward(medium, sources, rmc.make_run(n_fallback, n_harm, seed=seed), ledger=False)
    return maps, "monte-carlo"


def gradient_study(model: UNet, n_harm: int, ref_packets: int, counts: Sequence[int], hmeas_packets: int = 20_000_000,
                   margin: int = 10, log=None) -> dict:
    """The gradient of the 256x256 disc workload (four side sources, measured
    data from the second phantom) from plain Monte Carlo and from denoised
    forward and adjoint maps (the residual is taken from the denoised forward
    maps), at each packet count: relative L2 errors of d eps/d mua and
    d eps/d mus against a reference from ref_packets + ref_packets plain
    packets over pixels at least `margin` from the boundary, and wall times."""
    import phantoms as P
    c = P.config2()
    dev = torch.device("cuda", torch.cuda.current_device())
    med = rmc.Medium.from_phantom(c.phantom, dev)
    tmed = rmc.Medium.from_phantom(c.extra["true"], dev)
    ht, _ = rmc.mc_forward(tmed, c.sources, rmc.make_run(hmeas_packets, n_harm, seed=1), ledger=False)
    hmeas = rmc.mc_absorbed(tmed, ht)

    def grad(n, seed, den):
        f, _ = rmc.mc_forward(med, c.sources, rmc.make_run(n, n_harm, seed=seed), ledger=False)
        if den:
            f = denoise(model, f[None])[0].double()
        q, _ = rmc.mc_residual(med, f, hmeas)
        a, _ = rmc.mc_adjoint(med, [rmc.Source("map", map=q)], rmc.make_run(n, n_harm, seed=seed, stream_tag=1),
                              ledger=False)
        if den:
            a = denoise(model, a[None])[0].double()
        return rmc.mc_gradient(med, n_harm, f, a, hmeas)

    ra, rs = grad(ref_packets, 100, False)
    m = margin
    ra, rs = ra[m:-m, m:-m], rs[m:-m, m:-m]
    rows = []
    for n in counts:
        for den in (False, True):
            grad(n, 7, den)   # warm-up of this size
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ga, gs = grad(n, 7, den)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            r = {"packets": n, "denoised": den, "wall_ms": wall * 1e3,
                 "err_dmua": float((ga[m:-m, m:-m] - ra).norm() / ra.norm()),
                 "err_dmus": float((gs[m:-m, m:-m] - rs).norm() / rs.norm())}
            rows.append(r)
            if log:
                log(json.dumps(r))
    return {"reference_packets": ref_packets, "rows": rows}


def main(argv=None) -> int:
    import argparse
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--side", type=float, default=25.6)
    ap.add_argument("--train", type=int, default=448)
    ap.add_argument("--val", type=int, default=32)
    ap.add_argument("--low", type=float, default=1e5)
    ap.add_argument("--high", type=float, default=1e7)
    ap.add_argument("--harm", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=120)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--widths", default="48,64,96",
                    help="channels per U-Net level (24,32,48,64,96,128: six levels, 1.05M parameters)")
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--gradient-study", action="store_true",
                    help="train on forward and adjoint pairs, then compare the gradient of the 256x256 disc "
                         "workload from plain and from denoised maps (needs --n 256)")
    ap.add_argument("--ref", type=float, default=4e8, help="gradient study: reference packets per run")
    args = ap.parse_args(argv)
    widths = tuple(int(w) for w in args.widths.split(","))
    log = lambda m: print(m, file=sys.stderr, flush=True)
    torch.manual_seed(0)
    t0 = time.time()
    lo, hi = make_pairs(args.train + args.val, args.n, args.side, int(args.low), int(args.high), args.harm, 1000)
    if args.gradient_study:   # as many adjoint pairs, interleaved so both kinds are trained and held out
        alo, ahi = make_pairs(args.train + args.val, args.n, args.side, int(args.low), int(args.high), args.harm,
                              5000, adjoint=True)
        lo = torch.stack([lo, alo], 1).flatten(0, 1)
        hi = torch.stack([hi, ahi], 1).flatten(0, 1)
        args.train, args.val = 2 * args.train, 2 * args.val
    t_data = time.time() - t0
    log(f"pairs generated in {t_data:.1f} s")
    tr, va = slice(0, args.train), slice(args.train, args.train + args.val)
    model = UNet(2 * args.harm + 1, widths).cuda()
    t0 = time.time()
    hist = train(model, lo[tr], hi[tr], args.epochs, batch=args.batch, lr=args.lr, log=log)
    t_train = time.time() - t0
    den = denoise(model, lo[va])
    e_low = rel_error(lo[va], hi[va])
    e_den = rel_error(den, hi[va])
    e_den_a0 = rel_error(den[:, 0], hi[va][:, 0])
    e_low_a0 = rel_error(lo[va][:, 0], hi[va][:, 0])
    # the reference's own Monte Carlo error: the low-vs-high error scales as 1/sqrt(packets)
    floor = e_low * math.sqrt(args.low / args.high)
    # wall time to the same a0 error on one held-out phantom: a low-count run plus
    # the network, against the plain Monte Carlo with the packet count that
    # matches the network's a0 error (error ~ 1/sqrt(packets))
    dev = lo.device
    med = random_phantom_medium(args.n, args.side, 1000 + args.train, dev)
    src = side_sources(args.side)
    n_eq = int(args.low * (e_low_a0 / max(e_den_a0, 1e-12)) ** 2)
    for _ in range(2):   # the second pass is timed
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        low1, _ = rmc.mc_forward(med, src, rmc.make_run(int(args.low), args.harm, seed=5), ledger=False)
        denoise(model, low1[None])
        torch.cuda.synchronize()
        t_den = time.perf_counter() - t1
        t1 = time.perf_counter()
        rmc.mc_forward(med, src, rmc.make_run(n_eq, args.harm, seed=6), ledger=False)
        torch.cuda.synchronize()
        t_mc = time.perf_counter() - t1
    n_params = sum(p.numel() for p in model.parameters())
    out = {"grid": args.n, "harmonics": args.harm, "widths": list(widths), "train_pairs": args.train,
           "val_pairs": args.val,
           "packets_low": int(args.low), "packets_high": int(args.high), "params": n_params,
           "epochs": args.epochs, "final_loss": hist[-1], "data_s": t_data, "train_s": t_train,
           "val_rel_error_low_vs_high": e_low, "val_rel_error_denoised_vs_high": e_den,
           "val_rel_error_a0_low": e_low_a0, "val_rel_error_a0_denoised": e_den_a0,
           "reference_noise_floor_estimate": floor,
           "same_a0_error": {"denoised_ms": t_den * 1e3, "plain_mc_packets": n_eq, "plain_mc_ms": t_mc * 1e3}}
    if args.gradient_study:
        out["gradient_study"] = gradient_study(model, args.harm, int(args.ref),
                                               [int(args.low), 2 * int(args.low), 4 * int(args.low),
                                                10 * int(args.low), 40 * int(args.low)], log=log)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
