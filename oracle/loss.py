"""FP64 oracle of the training objective (TEST INFRASTRUCTURE ONLY).

Eq. 11: L = (1 - gamma) L1 + gamma L_SSIM with gamma = 0.2 (Sec. 4.1).
Readings (the paper cites SSIM without giving its window): L1 is the mean
absolute difference over all pixels; L_SSIM = 1 - the mean of the SSIM map
of Wang et al. over all pixels, each view's map computed on its own image
with an 11 x 11 Gaussian window of standard deviation 1.5 (normalised),
zero padding outside the image ("same" size), C1 = 0.01^2, C2 = 0.03^2
(dynamic range 1).  Where rendered and target pixels are equal the L1
subgradient is taken as 0.

``loss_and_grad`` returns L and dL/d(rendered image) for concatenated view
images; the SSIM adjoint is written out from the map's definition.
"""
from __future__ import annotations

import numpy as np

C1 = 0.01 ** 2
C2 = 0.03 ** 2
WINDOW = 11
SIGMA = 1.5


def window_1d(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    x = np.arange(size, dtype=np.float64) - (size - 1) / 2
    w = np.exp(-x * x / (2 * sigma * sigma))
    return w / w.sum()


def blur(img: np.ndarray, w: np.ndarray | None = None) -> np.ndarray:
    """Separable 2-D window sum at every pixel, zero outside the image."""
    w = window_1d() if w is None else w
    r = len(w) // 2
    h, wd = img.shape
    pad = np.zeros((h + 2 * r, wd + 2 * r))
    pad[r:r + h, r:r + wd] = img
    rows = np.zeros((h + 2 * r, wd))
    for k in range(len(w)):
        rows += w[k] * pad[:, k:k + wd]
    out = np.zeros((h, wd))
    for k in range(len(w)):
        out += w[k] * rows[k:k + h, :]
    return out


def ssim_stats(x: np.ndarray, y: np.ndarray):
    mx, my = blur(x), blur(y)
    exx, eyy, exy = blur(x * x), blur(y * y), blur(x * y)
    a1 = 2 * mx * my + C1
    a2 = 2 * (exy - mx * my) + C2
    b1 = mx * mx + my * my + C1
    b2 = (exx - mx * mx) + (eyy - my * my) + C2
    return mx, my, a1, a2, b1, b2


def ssim_map(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    _, _, a1, a2, b1, b2 = ssim_stats(np.asarray(x, np.float64), np.asarray(y, np.float64))
    return a1 * a2 / (b1 * b2)


def ssim_map_grad(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """d(sum of the SSIM map)/dx.  With m = blur(x), Exx = blur(x^2),
    Exy = blur(xy): dS/dm = S (2my/A1 - 2my/A2 - 2m/B1 + 2m/B2),
    dS/dExx = -S/B2, dS/dExy = 2S/A2, and each statistic's adjoint is the
    window sum again (symmetric window, zero padding)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my, a1, a2, b1, b2 = ssim_stats(x, y)
    s = a1 * a2 / (b1 * b2)
    dm = s * (2 * my / a1 - 2 * my / a2 - 2 * mx / b1 + 2 * mx / b2)
    dxx = -s / b2
    dxy = 2 * s / a2
    return blur(dm) + 2 * x * blur(dxx) + y * blur(dxy)


def loss_and_grad(image, target, sizes, gamma: float = 0.2):
    """Eq. 11 over concatenated views (row-major per view); sizes = [(w, h)]."""
    x = np.asarray(image, np.float64)
    y = np.asarray(target, np.float64)
    n = x.size
    d = x - y
    l1 = np.abs(d).sum() / n
    g = (1 - gamma) * np.sign(d) / n
    ssum = 0.0
    off = 0
    for w, h in sizes:
        xv = x[off:off + w * h].reshape(h, w)
        yv = y[off:off + w * h].reshape(h, w)
        ssum += ssim_map(xv, yv).sum()
        g[off:off + w * h] -= gamma / n * ssim_map_grad(xv, yv).reshape(-1)
        off += w * h
    loss = (1 - gamma) * l1 + gamma * (1 - ssum / n)
    return loss, g
