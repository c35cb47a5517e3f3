"""The library's training loss (l1 + SSIM, eq. `loss` without its perceptual
term) and its gradient against the binary64 oracle (oracle/loss.py).

Tolerances, from the arithmetic: the kernels work in binary32.  The local
variance E[x^2] - mu^2 is a difference of two terms up to 1, so its rounding
error (a few ulp of 1, ~1e-7) is large next to c2 = 9e-4 where the image is
flat: a single SSIM value can be off by ~1.5e-4 there (measured 1.4e-4 for
a flat image against an fp32 evaluation of the oracle's formulas).  The
loss averages these (it moves by ~3e-8 in the same evaluation): the bar is
2e-6.  The gradient is a window blur of such coefficients: the bar is
5e-4 of its largest entry (measured 4e-5), or of 1/n, the l1 term's size,
when the gradient is zero.
"""
import numpy as np
import pytest
import torch

from oracle import loss as L
from paper_2508_03180_amd import _capi as capi

pytestmark = pytest.mark.gpu

LOSS_TOL = 2e-6
GRAD_RTOL = 5e-4


@pytest.fixture(scope="module")
def r():
    from paper_2508_03180_amd.renderer import Renderer
    if not torch.cuda.is_available():
        pytest.skip("needs a HIP device")
    return Renderer(0)


def smooth(rng, shape):
    """Blurred noise scaled to [0, 1]: locally flat regions, the hard case
    for the variance terms."""
    b = L.blur(rng.random(shape))
    return (b - b.min()) / (b.max() - b.min())


def check(r, x, y, lam):
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    yt = torch.tensor(y, dtype=torch.float32, device="cuda")
    loss, g = r.loss_l1_ssim(xt, yt, lam)
    torch.cuda.synchronize()
    # the oracle sees the same binary32 inputs
    lo, go, _ = L.l1_ssim_loss(xt.double().cpu().numpy(), yt.double().cpu().numpy(), lam)
    assert abs(float(loss) - lo) <= LOSS_TOL, (float(loss), lo)
    g = g.double().cpu().numpy()
    scale = max(np.abs(go).max(), 1.0 / x.size)
    err = np.abs(g - go).max()
    assert err <= GRAD_RTOL * scale, (err, scale)
    return float(loss), g


@pytest.mark.parametrize("shape", [(3, 16, 64), (3, 37, 53), (1, 1, 1), (2, 5, 7), (3, 130, 200), (1, 17, 129)])
def test_random_images(r, shape):
    """Whole tiles, ragged tiles, images smaller than the window's halo."""
    rng = np.random.default_rng(sum(shape))
    check(r, rng.random(shape), rng.random(shape), 0.2)


def test_smooth_images_close_to_the_target(r):
    rng = np.random.default_rng(11)
    x = smooth(rng, (3, 96, 160))
    check(r, x, np.clip(x + rng.normal(0, 0.01, x.shape), 0, 1), 0.2)


@pytest.mark.parametrize("lam", [0.0, 1.0, 0.5])
def test_lambda_extremes(r, lam):
    rng = np.random.default_rng(12)
    check(r, rng.random((3, 40, 70)), rng.random((3, 40, 70)), lam)


def test_identical_images(r):
    x = np.random.default_rng(13).random((3, 33, 65))
    loss, g = check(r, x, x.copy(), 0.2)
    assert abs(loss) <= LOSS_TOL


def test_full_hd_frame(r):
    """The differentiation workload's size: 3 x 1080 x 1920, a smooth image
    against a noisy copy."""
    rng = np.random.default_rng(14)
    x = smooth(rng, (3, 1080, 1920))
    check(r, x, np.clip(x + rng.normal(0, 0.02, x.shape), 0, 1), 0.2)


def test_loss_alone_and_repeatability(r):
    """Without a gradient the loss is the same; two calls are bit-identical
    (the sums are taken in a fixed order)."""
    rng = np.random.default_rng(15)
    xt = torch.tensor(rng.random((3, 70, 90)), dtype=torch.float32, device="cuda")
    yt = torch.tensor(rng.random((3, 70, 90)), dtype=torch.float32, device="cuda")
    l1, g1 = r.loss_l1_ssim(xt, yt, 0.2)
    l2, g2 = r.loss_l1_ssim(xt, yt, 0.2)
    l3, g3 = r.loss_l1_ssim(xt, yt, 0.2, grad=False)
    torch.cuda.synchronize()
    assert g3 is None
    assert float(l1) == float(l2) == float(l3)
    assert torch.equal(g1, g2)


def test_autograd_function(r):
    from paper_2508_03180_amd.renderer import L1SsimLoss
    rng = np.random.default_rng(16)
    x = torch.tensor(rng.random((3, 50, 80)), dtype=torch.float32, device="cuda", requires_grad=True)
    y = torch.tensor(rng.random((3, 50, 80)), dtype=torch.float32, device="cuda")
    loss = 3.0 * L1SsimLoss.apply(r, x, y, 0.2)
    loss.backward(retain_graph=True)
    _, g = r.loss_l1_ssim(x.detach(), y, 0.2)
    torch.cuda.synchronize()
    assert torch.allclose(x.grad, 3.0 * g, rtol=1e-6, atol=0)
    loss.backward()  # a retained graph walked again adds the same gradient
    torch.cuda.synchronize()
    assert torch.allclose(x.grad, 6.0 * g, rtol=1e-6, atol=0)


def test_invalid_arguments(r):
    x = torch.zeros((3, 8, 8), device="cuda")
    loss = torch.empty((), device="cuda")
    for args in [(3, 8, 8, 1.5), (3, 8, 8, -0.1), (0, 8, 8, 0.2), (3, 0, 8, 0.2), (3, 8, 40000, 0.2)]:
        st = capi.dgs_loss_l1_ssim(r.ctx, x.data_ptr(), x.data_ptr(), args[0], args[1], args[2], args[3],
                                   loss.data_ptr(), 0)
        assert st == capi.DGS_ERR_INVALID_ARG, args
    st = capi.dgs_loss_l1_ssim(r.ctx, x.data_ptr(), x.data_ptr(), 3, 8, 8, 0.2, 0, 0)
    assert st == capi.DGS_ERR_INVALID_ARG
