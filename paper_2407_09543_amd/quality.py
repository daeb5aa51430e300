"""Image-quality figures for reports (host side, not part of the compression path).

The paper evaluates decoded textures against the uncompressed ones with PSNR and SSIM (Sec. 4.3).
SSIM here is the usual structural similarity: a Gaussian window of standard deviation 1.5 truncated
to 11 x 11 texels, C1 = (0.01 L)^2 and C2 = (0.03 L)^2 with L = 255, averaged over every window that
lies inside the image and over the channels (the paper does not state its parameters; these are the
common defaults)."""
from __future__ import annotations

import numpy as np
from scipy.ndimage import gaussian_filter

SIGMA = 1.5
RADIUS = 5


def ssim(a, b, data_range: float = 255.0, k1: float = 0.01, k2: float = 0.03) -> float:
    """Mean SSIM of two images [H, W] or [H, W, C] (H, W > 10)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.shape != b.shape:
        raise ValueError(f"shapes differ: {a.shape} vs {b.shape}")
    if a.ndim == 2:
        a, b = a[..., None], b[..., None]
    r = RADIUS

    def win(z):  # windowed mean at every centre whose window lies inside the image
        return gaussian_filter(z, SIGMA, truncate=r / SIGMA, mode="constant")[r:-r, r:-r]

    c1, c2 = (k1 * data_range) ** 2, (k2 * data_range) ** 2
    vals = []
    for c in range(a.shape[2]):
        x, y = a[..., c], b[..., c]
        mx, my = win(x), win(y)
        sxx = win(x * x) - mx * mx
        syy = win(y * y) - my * my
        sxy = win(x * y) - mx * my
        m = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
        vals.append(float(m.mean()))
    return float(np.mean(vals))
