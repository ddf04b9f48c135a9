"""The D-SSIM term of the loss of Sec. 4.5,
L = (1 - lambda_SSIM) L1 + lambda_SSIM L_SSIM, and its image gradient.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): plain float64, used
to check the HIP kernels.

SSIM is the measure the paper cites (Wang et al. 2004).  Readings (the paper
states neither the window nor lambda_SSIM): an 11 x 11 Gaussian window with
sigma 1.5 (normalised to sum 1), zero padding outside the image, C1 =
0.01^2 and C2 = 0.03^2 (data range 1), every colour channel separately;
L_SSIM = 1 - the mean of the SSIM map over the pixels and channels of all
views; L1 is the mean absolute difference over the same entries;
lambda_SSIM defaults to 0.2.
"""
from __future__ import annotations

import numpy as np
import torch

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2
LAMBDA_SSIM = 0.2


def gaussian_taps(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    """Normalised 1-D Gaussian taps; the 2-D window is their outer product."""
    x = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-x * x / (2.0 * sigma * sigma))
    return g / g.sum()


def ssim_map(X: torch.Tensor, Y: torch.Tensor) -> torch.Tensor:
    """SSIM map of one view, X and Y float64 [H, W, 3]: the local means,
    variances and covariance from the Gaussian window (zero padding), then
    ((2 mx my + C1)(2 sxy + C2)) / ((mx^2 + my^2 + C1)(sx^2 + sy^2 + C2))."""
    g = torch.tensor(gaussian_taps(), dtype=torch.float64)
    w2 = torch.outer(g, g)[None, None].repeat(3, 1, 1, 1)
    pad = WINDOW // 2

    def blur(Z):
        return torch.nn.functional.conv2d(Z.permute(2, 0, 1)[None], w2, padding=pad, groups=3)[0]

    mx, my = blur(X), blur(Y)
    sxx = blur(X * X) - mx * mx
    syy = blur(Y * Y) - my * my
    sxy = blur(X * Y) - mx * my
    num = (2.0 * mx * my + C1) * (2.0 * sxy + C2)
    den = (mx * mx + my * my + C1) * (sxx + syy + C2)
    return (num / den).permute(1, 2, 0)


def loss_and_grad(images, targets, lam: float = LAMBDA_SSIM):
    """Loss (1 - lam) L1 + lam (1 - mean SSIM) over views (lists of float
    [H, W, 3] arrays, any sizes) and its gradient per view (sign(0) = 0)."""
    Xs = [torch.tensor(np.asarray(x, dtype=np.float64), requires_grad=True) for x in images]
    Ys = [torch.tensor(np.asarray(y, dtype=np.float64)) for y in targets]
    n = sum(x.numel() for x in Xs)
    l1 = sum((x - y).abs().sum() for x, y in zip(Xs, Ys)) / n
    s = sum(ssim_map(x, y).sum() for x, y in zip(Xs, Ys)) / n
    loss = (1.0 - lam) * l1 + lam * (1.0 - s)
    grads = torch.autograd.grad(loss, Xs)
    return float(loss.detach()), [g_.numpy() for g_ in grads]


def ssim_brute(X: np.ndarray, Y: np.ndarray, i: int, j: int, c: int) -> float:
    """SSIM at one pixel and channel by explicit window sums (a pin of
    ssim_map)."""
    g = gaussian_taps()
    H, W = X.shape[:2]
    r = WINDOW // 2
    acc = np.zeros(5)
    for di in range(-r, r + 1):
        for dj in range(-r, r + 1):
            y, x = i + di, j + dj
            if 0 <= y < H and 0 <= x < W:
                w = g[di + r] * g[dj + r]
                a, b = X[y, x, c], Y[y, x, c]
                acc += w * np.array([a, b, a * a, b * b, a * b])
    mx, my, ex2, ey2, exy = acc
    sx, sy, sxy = ex2 - mx * mx, ey2 - my * my, exy - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sx + sy + C2))
