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
