"""CPU oracle of the training loss: l1 plus SSIM (eq. `loss`), binary64.

TEST INFRASTRUCTURE ONLY: used by the test-suite, never by the library.  It
shares no code with the HIP kernels.

The paper's loss combines an l1 term, an SSIM term and a perceptual term
(eq. `loss`, Sec. "Perceptual Loss"), with lambda_1 = 0.2 for SSIM (Sec.
"Experimental Settings").  The perceptual term needs a pretrained network and
is left out, so the loss here is

    L = (1 - lam) * mean |x - y| + lam * (1 - mean SSIM(x, y)),

the mean taken over every channel and pixel.  SSIM follows its standard
definition (the paper cites it without restating it): per channel, local
means, variances and covariance from an 11 x 11 Gaussian window with
sigma = 1.5 (normalised to sum 1), the image treated as zero outside its
borders, and

    SSIM = (2 mu_x mu_y + c1) (2 s_xy + c2) / ((mu_x^2 + mu_y^2 + c1) (s_xx + s_yy + c2)),
    s_xx = E[x^2] - mu_x^2,  s_xy = E[xy] - mu_x mu_y,  c1 = 0.01^2,  c2 = 0.03^2.

The gradient with respect to x (y is the fixed target) is the analytic one,
written out step by step below.

Parity status: pinned (tests/test_oracle_loss_pins.py): identical images give
loss 0 and gradient 0, the window blur equals scipy's 2-D convolution with
zero fill, constant images give the closed-form SSIM away from the borders,
the SSIM map is symmetric in x and y, lam = 0 reduces to the mean absolute
error, and the gradient agrees with central finite differences.
"""
from __future__ import annotations

import numpy as np

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window_1d():
    """The 11 Gaussian weights (sigma 1.5) normalised to sum 1, binary64."""
    t = np.arange(WINDOW, dtype=np.float64) - WINDOW // 2
    g = np.exp(-0.5 * (t / SIGMA) ** 2)
    return g / g.sum()


def blur(a):
    """Window average of each [H, W] plane of a (leading axes are planes):
    the 2-D window is the outer product of the 1-D weights, applied as one
    pass along rows and one along columns, the plane zero outside."""
    g = window_1d()
    r = WINDOW // 2
    a = np.asarray(a, dtype=np.float64)
    H, W = a.shape[-2], a.shape[-1]
    pad = [(0, 0)] * (a.ndim - 2)
    ap = np.pad(a, pad + [(0, 0), (r, r)])
    rows = sum(g[i] * ap[..., :, i:i + W] for i in range(WINDOW))
    rp = np.pad(rows, pad + [(r, r), (0, 0)])
    return sum(g[i] * rp[..., i:i + H, :] for i in range(WINDOW))


def ssim_terms(x, y):
    """Local statistics and the pieces of the SSIM quotient, per pixel."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    mx, my = blur(x), blur(y)
    exx, eyy, exy = blur(x * x), blur(y * y), blur(x * y)
    sxx = exx - mx * mx
    syy = eyy - my * my
    sxy = exy - mx * my
    a1 = 2 * mx * my + C1
    a2 = 2 * sxy + C2
    b1 = mx * mx + my * my + C1
    b2 = sxx + syy + C2
    return dict(mx=mx, my=my, a1=a1, a2=a2, b1=b1, b2=b2)


def ssim_map(x, y):
    """SSIM of every channel and pixel of x against y ([C, H, W])."""
    t = ssim_terms(x, y)
    return (t["a1"] * t["a2"]) / (t["b1"] * t["b2"])


def l1_ssim_loss(x, y, lam=0.2, grad=True):
    """Loss value and (optionally) its gradient with respect to x.

    Returns (loss, dL/dx or None, SSIM map)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = x.size
    t = ssim_terms(x, y)
    s = (t["a1"] * t["a2"]) / (t["b1"] * t["b2"])
    loss = (1 - lam) * np.abs(x - y).sum() / n + lam * (1 - s.sum() / n)
    if not grad:
        return float(loss), None, s
    # dL/dS at every pixel: the SSIM term is lam (1 - mean S)
    dls = -lam / n
    mx, my = t["mx"], t["my"]
    # S = a1 a2 / (b1 b2) as a function of the window statistics of x:
    #   d a1/d mu_x = 2 mu_y, d a2/d mu_x = -2 mu_y (through s_xy),
    #   d b1/d mu_x = 2 mu_x, d b2/d mu_x = -2 mu_x (through s_xx),
    #   d b2/d E[x^2] = 1, d a2/d E[xy] = 2
    d_mx = dls * s * (2 * my / t["a1"] - 2 * my / t["a2"] - 2 * mx / t["b1"] + 2 * mx / t["b2"])
    d_exx = dls * s * (-1.0 / t["b2"])
    d_exy = dls * s * (2.0 / t["a2"])
    # mu_x = blur(x), E[x^2] = blur(x^2), E[xy] = blur(x y); the window is
    # symmetric, so the adjoint of the zero-filled blur is the same blur
    g = blur(d_mx) + 2 * x * blur(d_exx) + y * blur(d_exy)
    # l1: (1 - lam) / n sign(x - y), 0 where x == y
    g = g + (1 - lam) / n * np.sign(x - y)
    return float(loss), g, s
