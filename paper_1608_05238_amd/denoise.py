"""Learned denoiser of harmonic coefficient maps on BF16 matrix cores.

A small U-Net maps the 2N+1 coefficient maps of a run with few packets to
those of a run with many packets, so that a gradient evaluation can stand on
fewer packets.  Its 3x3 convolutions (forward, input gradient and weight
gradient) are the hand-written MFMA kernels of denoise.h (BF16 operands,
FP32 accumulation); pooling, upsampling, ReLU and the 1x1 output layer are
plain PyTorch.  Training pairs come from the Monte Carlo itself, run as
batches of problems (mc_run_batch).  The plain Monte Carlo stays the
reference and the fallback: `denoise_or_mc` runs the low-count input as two
independent halves, predicts the error of that input's denoised maps from
how much the network's outputs for the halves differ plus a systematic part
calibrated on held-out pairs, and returns them only when the prediction is
within the threshold (2%), else it runs more packets.

    python -m paper_1608_05238_amd.denoise                 # generate pairs, train, evaluate
    python -m paper_1608_05238_amd.denoise --conv-bench    # TFLOP/s of the convolution kernels
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
               batch: int = 32, adjoint: bool = False, log=None):
    """Coefficient maps [S][2N+1][n][n] from independent runs on seeded random
    phantoms (batched; forward runs of the four side sources, or adjoint runs
    of a random_adjoint_source): the low-count input as two independent
    halves (n_low // 2 and the rest), their packet-weighted mean (an n_low-packet
    estimate) and the n_high-packet target.  Returns (low, high, half_a,
    half_b)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    na, nb = n_low // 2, n_low - n_low // 2
    lows, highs, has, hbs = [], [], [], []
    for b0 in range(0, n_samples, batch):
        probs = []
        for i in range(b0, min(n_samples, b0 + batch)):
            med = random_phantom_medium(n, side, seed0 + i, dev)
            src = [rmc.Source("map", map=random_adjoint_source(med, seed0 + i))] if adjoint else side_sources(side)
            tag = 1 if adjoint else 0
            for k, npk in enumerate((na, nb, n_high)):
                probs.append(rmc.Problem(med, src, rmc.make_run(npk, n_harm, seed=3 * (seed0 + i) + k,
                                                                stream_tag=tag), adjoint))
        outs = rmc.mc_run_batch(probs, ledger=False)
        for j in range(0, len(outs), 3):
            ha, hb, hi = outs[j][0], outs[j + 1][0], outs[j + 2][0]
            has.append(ha.float())
            hbs.append(hb.float())
            lows.append(((ha * na + hb * nb) / (na + nb)).float())
            highs.append(hi.float())
        if log:
            log(f"{'adjoint' if adjoint else 'forward'} pairs: {len(highs)} of {n_samples}")
    return torch.stack(lows), torch.stack(highs), torch.stack(has), torch.stack(hbs)


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


def _norms(t: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
    """Per-sample L2 norms of the a0 map and of all channels."""
    t = t.double()
    return t[:, 0].pow(2).sum(dim=(1, 2)).sqrt(), t.pow(2).sum(dim=(1, 2, 3)).sqrt()


@torch.no_grad()
def predicted_error(model: UNet, half_a: torch.Tensor, half_b: torch.Tensor, na: int, nb: int,
                    bias2=(0.0, 0.0)):
    """Denoise the packet-weighted mean of two independent half-runs and
    predict the relative L2 error of the result, per input, without a
    reference: the Monte Carlo noise left in the output is estimated from how
    much the network's outputs for the two halves differ (for noise that the
    network passes on linearly, |D(a) - D(b)|^2 = c (1/na + 1/nb) and the
    output's own share is c / (na + nb)); the network's systematic error is a
    fraction of the output's norm calibrated on held-out pairs (bias2: its
    square for the a0 map and for all channels).  Returns (denoised maps,
    predicted a0 error, predicted all-channel error), per sample."""
    low = (half_a.double() * na + half_b.double() * nb) / (na + nb)
    d = denoise(model, torch.cat([low.float(), half_a.float(), half_b.float()]))
    s = len(low)
    den, da, db = d[:s], d[s:2 * s], d[2 * s:]
    share = (1.0 / (na + nb)) / (1.0 / na + 1.0 / nb)
    n0, nall = _norms(da - db)
    d0, dall = _norms(den)
    p0 = (n0.pow(2) * share / d0.pow(2) + bias2[0]).sqrt()
    pall = (nall.pow(2) * share / dall.pow(2) + bias2[1]).sqrt()
    return den, p0, pall


@torch.no_grad()
def calibrate(model: UNet, half_a: torch.Tensor, half_b: torch.Tensor, high: torch.Tensor, n_low: int,
              n_high: int) -> dict:
    """Fit the systematic part of predicted_error on held-out pairs: the
    actual squared error of the denoised maps against the targets, less the
    targets' own noise (from the input-vs-target error and the packet ratio)
    and less the predicted noise part, averaged (not below zero)."""
    na, nb = n_low // 2, n_low - n_low // 2
    den, p0, pall = predicted_error(model, half_a, half_b, na, nb)
    low = (half_a.double() * na + half_b.double() * nb) / (na + nb)
    r = n_low / n_high
    out = {}
    for key, idx in (("a0", 0), ("all", 1)):
        h = _norms(high)[idx]
        act2 = (_norms(den - high)[idx] / h).pow(2)
        tgt2 = (_norms(low - high)[idx] / h).pow(2) * r / (1 + r)   # the targets' own noise
        pred2 = (p0 if idx == 0 else pall).pow(2)
        out[key] = float((act2 - tgt2 - pred2).clamp_min(0.0).mean())
    return {"bias2": (out["a0"], out["all"]), "samples": len(high)}


@torch.no_grad()
def judge_predictions(model: UNet, calib: dict, half_a: torch.Tensor, half_b: torch.Tensor, high: torch.Tensor,
                      n_low: int, n_high: int, threshold: float = 0.02) -> dict:
    """Predicted against actual a0 errors on held-out pairs not used by
    calibrate (actual: against the targets, their own noise removed), and
    the fallback decisions the threshold makes on them."""
    na, nb = n_low // 2, n_low - n_low // 2
    den, p0, pall = predicted_error(model, half_a, half_b, na, nb, calib["bias2"])
    low = (half_a.double() * na + half_b.double() * nb) / (na + nb)
    r = n_low / n_high
    h0 = _norms(high)[0]
    act = ((_norms(den - high)[0] / h0).pow(2) - (_norms(low - high)[0] / h0).pow(2) * r / (1 + r)).clamp_min(0).sqrt()
    ratio = (p0 / act.clamp_min(1e-12)).cpu().numpy()
    keep_p, keep_a = (p0 <= threshold).cpu().numpy(), (act <= threshold).cpu().numpy()
    pr = np.argsort(np.argsort(p0.cpu().numpy()))
    ar = np.argsort(np.argsort(act.cpu().numpy()))
    rho = float(np.corrcoef(pr, ar)[0, 1]) if len(pr) > 2 else float("nan")
    return {"samples": len(high), "threshold": threshold,
            "predicted_a0": [float(v) for v in p0.cpu()], "actual_a0": [float(v) for v in act.cpu()],
            "ratio_median": float(np.median(ratio)), "ratio_p10_p90": [float(np.percentile(ratio, 10)),
                                                                       float(np.percentile(ratio, 90))],
            "rank_correlation": rho,
            "denoised_and_within": int((keep_p & keep_a).sum()), "denoised_but_above": int((keep_p & ~keep_a).sum()),
            "fallback_but_within": int((~keep_p & keep_a).sum()), "fallback_and_above": int((~keep_p & ~keep_a).sum())}


def split_runs(medium: rmc.Medium, sources, n_low: int, n_harm: int, seed: int = 0, adjoint: bool = False):
    """Two independent half-runs (n_low // 2 and the rest packets) in one batch."""
    na, nb = n_low // 2, n_low - n_low // 2
    tag = 1 if adjoint else 0
    probs = [rmc.Problem(medium, sources, rmc.make_run(na, n_harm, seed=2 * seed, stream_tag=tag), adjoint),
             rmc.Problem(medium, sources, rmc.make_run(nb, n_harm, seed=2 * seed + 1, stream_tag=tag), adjoint)]
    outs = rmc.mc_run_batch(probs, ledger=False)
    return outs[0][0], outs[1][0], na, nb


def denoise_or_mc(model: UNet, calib: dict, medium: rmc.Medium, sources, n_low: int, n_fallback: int, n_harm: int,
                  threshold: float = 0.02, seed: int = 0, adjoint: bool = False):
    """Maps for (medium, sources), per input: the denoised n_low-packet run
    when its predicted a0 error (predicted_error, calibrated by calibrate) is
    at most `threshold`, else the plain Monte Carlo with n_fallback packets.
    Returns (maps, "denoised" | "monte-carlo", predicted a0 error)."""
    a, b, na, nb = split_runs(medium, sources, n_low, n_harm, seed, adjoint)
    den, p0, _ = predicted_error(model, a[None], b[None], na, nb, calib["bias2"])
    if float(p0[0]) <= threshold:
        return den[0].double(), "denoised", float(p0[0])
    run = rmc.make_run(n_fallback, n_harm, seed=seed, stream_tag=1 if adjoint else 0)
    maps, _ = (rmc.mc_adjoint if adjoint else rmc.mc_forward)(medium, sources, run, ledger=False)
    return maps, "monte-carlo", float(p0[0])


def gradient_study(model: UNet, n_harm: int, ref_packets: int, counts: Sequence[int], hmeas_packets: int = 20_000_000,
                   margin: int = 10, log=None, calib=None) -> dict:
    """The gradient of the 256x256 disc workload (four side sources, measured
    data from the second phantom) from plain Monte Carlo and from denoised
    forward and adjoint maps (the residual is taken from the denoised forward
    maps), at each packet count: relative L2 errors of d eps/d mua and
    d eps/d mus against a reference from ref_packets + ref_packets plain
    packets over pixels at least `margin` from the boundary, and wall times.
    With `calib`, the denoised runs go through the per-input path (two
    half-runs, predicted_error) and each row records the predicted a0 errors
    of its forward and adjoint maps, i.e. whether denoise_or_mc would have
    fallen back."""
    import phantoms as P
    c = P.config2()
    dev = torch.device("cuda", torch.cuda.current_device())
    med = rmc.Medium.from_phantom(c.phantom, dev)
    tmed = rmc.Medium.from_phantom(c.extra["true"], dev)
    ht, _ = rmc.mc_forward(tmed, c.sources, rmc.make_run(hmeas_packets, n_harm, seed=1), ledger=False)
    hmeas = rmc.mc_absorbed(tmed, ht)

    preds = {}

    def maps(n, seed, den, adjoint, src):
        run = rmc.make_run(n, n_harm, seed=seed, stream_tag=1 if adjoint else 0)
        if den and calib is not None:
            a, b, na, nb = split_runs(med, src, n, n_harm, seed, adjoint)
            d, p0, _ = predicted_error(model, a[None], b[None], na, nb, calib["bias2"])
            preds["adjoint" if adjoint else "forward"] = float(p0[0])
            return d[0].double()
        m, _ = (rmc.mc_adjoint if adjoint else rmc.mc_forward)(med, src, run, ledger=False)
        return denoise(model, m[None])[0].double() if den else m

    def grad(n, seed, den):
        f = maps(n, seed, den, False, c.sources)
        q, _ = rmc.mc_residual(med, f, hmeas)
        a = maps(n, seed, den, True, [rmc.Source("map", map=q)])
        return rmc.mc_gradient(med, n_harm, f, a, hmeas)

    if log:
        log(f"gradient study: reference from {ref_packets:.0e} + {ref_packets:.0e} packets")
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
            if den and calib is not None:
                r["predicted_a0"] = dict(preds)
            rows.append(r)
            if log:
                log(json.dumps(r))
    return {"reference_packets": ref_packets, "rows": rows}


def conv_bench(reps: int = 20, log=None) -> dict:
    """Achieved rate of the convolution kernels on the U-Net's layer shapes
    at 256x256 (batch 16, channels of the 6-level configuration and of the
    3-level one): forward, input gradient (the forward kernel on the flipped
    weights) and weight gradient, each the fastest of `reps` launches (HIP
    events), in dense BF16 TFLOP/s (2 flops per multiply-add of the 3x3
    convolution, padding channels not counted)."""
    lib = L.load()
    dev = torch.device("cuda", torch.cuda.current_device())
    st = _stream()
    shapes = [(16, 40, 48, 256, 256), (16, 48, 48, 256, 256), (16, 112, 48, 256, 256), (16, 64, 64, 128, 128),
              (16, 160, 64, 128, 128), (16, 96, 96, 64, 64)]
    rows = []
    for n, ci, co, h, w in shapes:
        g = torch.Generator(device="cpu").manual_seed(ci * co)
        x = torch.randn(n, h, w, ci, generator=g).to(dev, torch.bfloat16)
        wt = (torch.randn(co, 3, 3, ci, generator=g) / (3 * ci ** 0.5)).to(dev, torch.bfloat16)
        gy = torch.randn(n, h, w, co, generator=g).to(dev, torch.bfloat16)
        y = torch.empty(n, h, w, co, device=dev)
        gw = torch.empty(co, 3, 3, ci, device=dev)
        flops = 2.0 * 9 * ci * co * n * h * w

        def best(fn):
            fn()
            torch.cuda.synchronize()
            b = float("inf")
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                e1.synchronize()
                b = min(b, e0.elapsed_time(e1) * 1e-3)
            return b

        tf = best(lambda: L.check("dn_conv3x3_fwd", lib.dn_conv3x3_fwd(x.data_ptr(), wt.data_ptr(), None, y.data_ptr(),
                                                                        n, ci, co, h, w, st)))
        tg = best(lambda: L.check("dn_conv3x3_wgrad", lib.dn_conv3x3_wgrad(x.data_ptr(), gy.data_ptr(), gw.data_ptr(),
                                                                            n, ci, co, h, w, st)))
        r = {"shape": [n, ci, co, h, w], "gflop": flops / 1e9, "fwd_ms": tf * 1e3, "fwd_tflops": flops / tf / 1e12,
             "wgrad_ms": tg * 1e3, "wgrad_tflops": flops / tg / 1e12}
        rows.append(r)
        if log:
            log(json.dumps(r))
    return {"peak_tflops_bf16_dense": 2500.0, "rows": rows}


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
    ap.add_argument("--threshold", type=float, default=0.02, help="predicted a0 error above which the MC falls back")
    ap.add_argument("--gradient-study", action="store_true",
                    help="train on forward and adjoint pairs, then compare the gradient of the 256x256 disc "
                         "workload from plain and from denoised maps (needs --n 256)")
    ap.add_argument("--ref", type=float, default=4e8, help="gradient study: reference packets per run")
    ap.add_argument("--conv-bench", action="store_true", help="only time the convolution kernels (TFLOP/s)")
    args = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    if args.conv_bench:
        print(json.dumps(conv_bench(log=log)), flush=True)
        return 0
    widths = tuple(int(w) for w in args.widths.split(","))
    torch.manual_seed(0)
    t0 = time.time()
    n_low, n_high = int(args.low), int(args.high)
    lo, hi, ha, hb = make_pairs(args.train + args.val, args.n, args.side, n_low, n_high, args.harm, 1000, log=log)
    if args.gradient_study:   # as many adjoint pairs, interleaved so both kinds are trained and held out
        alo, ahi, aha, ahb = make_pairs(args.train + args.val, args.n, args.side, n_low, n_high, args.harm, 5000,
                                        adjoint=True, log=log)
        lo, hi, ha, hb = (torch.stack([u, v], 1).flatten(0, 1) for u, v in ((lo, alo), (hi, ahi), (ha, aha), (hb, ahb)))
        args.train, args.val = 2 * args.train, 2 * args.val
    t_data = time.time() - t0
    log(f"pairs generated in {t_data:.1f} s")
    tr = slice(0, args.train)
    # held out: the first half calibrates the error prediction, the second judges it
    half = args.val // 2
    vc, vt = slice(args.train, args.train + half), slice(args.train + half, args.train + args.val)
    va = slice(args.train, args.train + args.val)
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
    calib = calibrate(model, ha[vc], hb[vc], hi[vc], n_low, n_high)
    judged = judge_predictions(model, calib, ha[vt], hb[vt], hi[vt], n_low, n_high, args.threshold)
    log(f"error prediction: {json.dumps({k: v for k, v in judged.items() if not isinstance(v, list)})}")
    # the same held-out phantoms with 10x fewer packets, outside the training
    # distribution: the prediction has to see that their denoised error is larger
    n_few = max(2, n_low // 10)
    if args.gradient_study:   # the forward phantoms of the interleaved held-out set
        first, count, targets = (args.train + half) // 2, (args.val - half) // 2, hi[vt][0::2]
    else:
        first, count, targets = args.train + half, args.val - half, hi[vt]
    _, _, fa, fb = make_pairs(count, args.n, args.side, n_few, 2, args.harm, 1000 + first)
    judged_few = judge_predictions(model, calib, fa, fb, targets, n_few, n_high, args.threshold)
    log(f"error prediction, {n_few} packets: "
        f"{json.dumps({k: v for k, v in judged_few.items() if not isinstance(v, list)})}")
    # wall time to the same a0 error on one held-out phantom: the per-input
    # path (two half-runs, the network three times, the prediction) against
    # the plain Monte Carlo with the packet count that matches the network's
    # a0 error (error ~ 1/sqrt(packets))
    dev = lo.device
    med = random_phantom_medium(args.n, args.side, 1000 + args.train, dev)
    src = side_sources(args.side)
    n_eq = int(args.low * (e_low_a0 / max(e_den_a0, 1e-12)) ** 2)
    for _ in range(2):   # the second pass is timed
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, kind, pred = denoise_or_mc(model, calib, med, src, n_low, n_eq, args.harm, args.threshold, seed=5)
        torch.cuda.synchronize()
        t_den = time.perf_counter() - t1
        t1 = time.perf_counter()
        rmc.mc_forward(med, src, rmc.make_run(n_eq, args.harm, seed=6), ledger=False)
        torch.cuda.synchronize()
        t_mc = time.perf_counter() - t1
    n_params = sum(p.numel() for p in model.parameters())
    out = {"grid": args.n, "harmonics": args.harm, "widths": list(widths), "train_pairs": args.train,
           "val_pairs": args.val,
           "packets_low": n_low, "packets_high": n_high, "params": n_params,
           "epochs": args.epochs, "final_loss": hist[-1], "data_s": t_data, "train_s": t_train,
           "val_rel_error_low_vs_high": e_low, "val_rel_error_denoised_vs_high": e_den,
           "val_rel_error_a0_low": e_low_a0, "val_rel_error_a0_denoised": e_den_a0,
           "reference_noise_floor_estimate": floor,
           "error_prediction": {"bias_rel_a0": math.sqrt(calib["bias2"][0]),
                                "bias_rel_all": math.sqrt(calib["bias2"][1]),
                                "calibration_pairs": calib["samples"], **judged},
           "error_prediction_fewer_packets": {"packets_low": n_few, **judged_few},
           "same_a0_error": {"path": kind, "predicted_a0": pred, "denoised_ms": t_den * 1e3,
                             "plain_mc_packets": n_eq, "plain_mc_ms": t_mc * 1e3}}
    if args.gradient_study:
        out["gradient_study"] = gradient_study(model, args.harm, int(args.ref),
                                               [int(args.low), 2 * int(args.low), 4 * int(args.low),
                                                10 * int(args.low), 40 * int(args.low)], log=log, calib=calib)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
