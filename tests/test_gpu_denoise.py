"""BF16 matrix-core convolution kernels of the denoiser against PyTorch's FP64
convolution on the CPU, on the same BF16-rounded operands (the products are
exact in FP32; only the order of the FP32 sums differs), over channel counts
that need zero padding, several 32-channel chunks and 64-channel output
tiles, and images that end inside an 8 x 8 tile; and a short training run of
the U-Net built on them."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _mods():
    import torch
    import torch.nn.functional as F
    from paper_1608_05238_amd import denoise as D
    return torch, F, D


@pytest.mark.parametrize("shape", [(2, 33, 48, 17, 17), (1, 5, 70, 8, 13), (3, 64, 64, 32, 32), (1, 1, 1, 1, 1),
                                   (2, 160, 96, 19, 21), (1, 112, 48, 9, 64)])
def test_conv3x3_forward_and_gradients(shape):
    torch, F, D = _mods()
    n, ci, co, h, w = shape
    g = torch.Generator().manual_seed(sum(shape))
    x = torch.randn(n, ci, h, w, generator=g)
    wt = torch.randn(co, ci, 3, 3, generator=g) / (3 * ci ** 0.5)
    b = torch.randn(co, generator=g)
    gy = torch.randn(n, co, h, w, generator=g)
    # BF16-rounded operands, reference in FP64 on the CPU
    xr, wr, gyr = (t.to(torch.bfloat16).double() for t in (x, wt, gy))
    xr.requires_grad_(True)
    wr.requires_grad_(True)
    yr = F.conv2d(xr, wr, b.double(), padding=1)
    yr.backward(gyr)
    xd = x.cuda().requires_grad_(True)
    wd = wt.cuda().requires_grad_(True)
    bd = b.cuda().requires_grad_(True)
    y = D.conv3x3(xd, wd, bd)
    y.backward(gy.cuda())
    # the bias gradient is the plain FP32 sum of the (unrounded) upstream gradient
    for got, ref in ((y, yr), (xd.grad, xr.grad), (wd.grad, wr.grad), (bd.grad, gy.double().sum((0, 2, 3)))):
        got = got.detach().double().cpu()
        ref = ref.detach()
        err = float((got - ref).abs().max() / ref.abs().max().clamp_min(1e-30))
        assert err < 2e-5, (shape, len(ref.shape), err)


def test_unet_training_reduces_loss():
    """Denoise smooth random fields from noisy copies: the loss falls."""
    torch, F, D = _mods()
    torch.manual_seed(0)
    c, hw = 5, 24
    base = torch.randn(64, c, hw // 4, hw // 4)
    clean = F.interpolate(base, size=(hw, hw), mode="bilinear", align_corners=False).abs() + 1.0
    noisy = clean + 0.2 * torch.randn_like(clean)
    model = D.UNet(c, widths=(16, 24)).cuda()
    hist = D.train(model, noisy.cuda(), clean.cuda(), epochs=40, batch=16, lr=3e-3)
    assert hist[-1] < 0.7 * hist[0], hist
    den = D.denoise(model, noisy[:16].cuda())
    assert D.rel_error(den.cpu(), clean[:16]) < D.rel_error(noisy[:16], clean[:16])


def test_error_prediction_of_an_identity_network():
    """With the output layer at zero the U-Net is the identity, so the denoised
    maps are the packet-weighted mean of the two halves and their only error is
    the halves' noise: the split-half prediction must match the actual a0
    error (expected squared norms agree exactly; one sample fluctuates by
    ~1/sqrt(pixels)).  Calibration then finds (almost) no systematic part."""
    torch, F, D = _mods()
    torch.manual_seed(3)
    s, c, hw, sig = 24, 5, 32, 0.05
    base = torch.randn(s, c, hw // 4, hw // 4)
    clean = (F.interpolate(base, size=(hw, hw), mode="bilinear", align_corners=False).abs() + 1.0).cuda()
    na, nb = 3000, 5000   # unequal halves: noise variance ~ 1/packets
    ha = clean + sig * (8000 / na) ** 0.5 * torch.randn_like(clean)
    hb = clean + sig * (8000 / nb) ** 0.5 * torch.randn_like(clean)
    model = D.UNet(c, widths=(8, 8)).cuda()
    den, p0, pall = D.predicted_error(model, ha, hb, na, nb)
    mean = (ha * na + hb * nb) / (na + nb)
    assert torch.allclose(den, mean, rtol=1e-5, atol=1e-6)
    act0 = (den[:, 0] - clean[:, 0]).double().pow(2).sum((1, 2)).sqrt() / den[:, 0].double().pow(2).sum((1, 2)).sqrt()
    ratio = (p0 / act0).cpu().numpy()
    assert 0.93 < float(np.median(ratio)) < 1.07, ratio
    assert ratio.min() > 0.7 and ratio.max() < 1.4, ratio
    high = clean + 0.01 * sig * torch.randn_like(clean)
    cal = D.calibrate(model, ha, hb, high, na + nb, 100 * (na + nb))
    assert cal["bias2"][0] < (0.2 * float(act0.mean())) ** 2, cal


def test_denoise_or_mc_decides_per_input():
    """The per-input path: a threshold the prediction meets returns the
    denoised mean of the two half-runs; one it cannot meet returns exactly the
    plain run with the fallback packet count."""
    torch, F, D = _mods()
    from paper_1608_05238_amd import rmc
    import phantoms as P
    ph = P.disc_phantom(32, 0.5, 0.05, 5.0, 0.8, seed=4)
    med = rmc.Medium.from_phantom(ph)
    src = P.four_side_lines(ph)
    nh = 2
    model = D.UNet(2 * nh + 1, widths=(8, 8)).cuda()
    cal = {"bias2": (0.0, 0.0)}
    maps, kind, pred = D.denoise_or_mc(model, cal, med, src, 20_000, 50_000, nh, threshold=1.0, seed=9)
    assert kind == "denoised" and 0 < pred < 1.0
    a, b, na, nb = D.split_runs(med, src, 20_000, nh, seed=9)
    assert torch.allclose(maps.float(), ((a * na + b * nb) / (na + nb)).float(), rtol=1e-5, atol=1e-7)
    maps, kind, pred2 = D.denoise_or_mc(model, cal, med, src, 20_000, 50_000, nh, threshold=0.0, seed=9)
    assert kind == "monte-carlo" and pred2 == pred
    ref, _ = rmc.mc_forward(med, src, rmc.make_run(50_000, nh, seed=9), ledger=False)
    assert torch.equal(maps, ref)
