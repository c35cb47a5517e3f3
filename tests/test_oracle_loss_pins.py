"""Pins of the loss oracle (l1 + SSIM, eq. `loss`) against facts that do not
come from the oracle itself (CPU only)."""
import numpy as np
import pytest
from scipy.signal import convolve2d

from oracle import loss as L


def rand_pair(seed, shape):
    rng = np.random.default_rng(seed)
    return rng.random(shape), rng.random(shape)


def test_window_is_the_sigma_1_5_gaussian():
    g = L.window_1d()
    assert g.shape == (11,) and abs(g.sum() - 1) < 1e-15
    # ratio of neighbouring weights: exp(-((k+1)^2 - k^2) / (2 sigma^2))
    for k in range(5):
        assert g[6 + k] / g[5 + k] == pytest.approx(np.exp(-(2 * k + 1) / (2 * 1.5 ** 2)), rel=1e-13)
    assert np.allclose(g, g[::-1], rtol=0, atol=1e-17)


@pytest.mark.parametrize("shape", [(7, 9), (23, 40), (3, 3), (1, 1)])
def test_blur_is_the_zero_filled_2d_convolution(shape):
    """The separable blur equals scipy's 2-D convolution with the outer
    product window, 'same' size, zeros outside the image."""
    a = np.random.default_rng(1).random(shape)
    g = L.window_1d()
    ref = convolve2d(a, np.outer(g, g), mode="same", boundary="fill", fillvalue=0.0)
    assert np.abs(L.blur(a) - ref).max() < 1e-14


def test_identical_images_give_zero_loss_and_zero_gradient():
    x, _ = rand_pair(2, (3, 17, 29))
    loss, g, s = L.l1_ssim_loss(x, x.copy())
    assert np.abs(s - 1).max() < 1e-12
    assert abs(loss) < 1e-12
    assert np.abs(g).max() < 1e-15


def test_constant_images_closed_form_away_from_borders():
    """Constant planes a and b: away from the borders the window statistics
    are exact, the variances vanish and SSIM = (2ab + c1) / (a^2 + b^2 + c1)."""
    a, b = 0.7, 0.25
    x = np.full((1, 30, 30), a)
    y = np.full((1, 30, 30), b)
    s = L.ssim_map(x, y)[0, 5:-5, 5:-5]
    want = (2 * a * b + 0.01 ** 2) / (a * a + b * b + 0.01 ** 2)
    assert np.abs(s - want).max() < 1e-12
    # at the border the zero fill lowers the local means, so SSIM changes there
    assert abs(L.ssim_map(x, y)[0, 0, 0] - want) > 1e-3


def test_ssim_is_symmetric_and_bounded():
    x, y = rand_pair(3, (2, 19, 21))
    s1, s2 = L.ssim_map(x, y), L.ssim_map(y, x)
    assert np.abs(s1 - s2).max() < 1e-13
    assert s1.max() <= 1 + 1e-12 and s1.min() >= -1 - 1e-12


def test_lambda_zero_is_the_mean_absolute_error():
    x, y = rand_pair(4, (3, 8, 11))
    loss, g, _ = L.l1_ssim_loss(x, y, lam=0.0)
    assert loss == pytest.approx(np.abs(x - y).mean(), rel=1e-14)
    assert np.array_equal(g, np.sign(x - y) / x.size)


def test_lambda_one_is_one_minus_mean_ssim():
    x, y = rand_pair(5, (2, 12, 10))
    loss, _, s = L.l1_ssim_loss(x, y, lam=1.0)
    assert loss == pytest.approx(1 - s.mean(), rel=1e-14)


@pytest.mark.parametrize("lam", [0.2, 1.0])
def test_gradient_matches_central_differences(lam):
    """dL/dx against central differences of the loss (binary64, step 1e-6),
    at pixels in the interior, on the border and in a corner of every
    channel."""
    x, y = rand_pair(6, (2, 13, 16))
    # keep |x - y| away from 0 so that the l1 kink is not crossed by the step
    x = np.where(np.abs(x - y) < 0.05, y + 0.1, x)
    _, g, _ = L.l1_ssim_loss(x, y, lam=lam)
    h = 1e-6
    for (c, i, j) in [(0, 6, 7), (1, 0, 0), (1, 12, 15), (0, 0, 9), (1, 7, 15), (0, 12, 3)]:
        xp, xm = x.copy(), x.copy()
        xp[c, i, j] += h
        xm[c, i, j] -= h
        fd = (L.l1_ssim_loss(xp, y, lam=lam, grad=False)[0] - L.l1_ssim_loss(xm, y, lam=lam, grad=False)[0]) / (2 * h)
        assert g[c, i, j] == pytest.approx(fd, rel=2e-6, abs=1e-12), (c, i, j)


def test_channels_are_independent():
    """The window never mixes channels: the map of a stacked pair is the
    stack of the per-channel maps."""
    x, y = rand_pair(7, (3, 9, 14))
    s = L.ssim_map(x, y)
    for c in range(3):
        assert np.abs(s[c] - L.ssim_map(x[c:c + 1], y[c:c + 1])[0]).max() < 1e-15
