"""Image-quality figures for reports (host side, not part of the compression path).

The paper evaluates decoded textures against the uncompressed ones with PSNR and SSIM (Sec. 4.3).
PSNR is 10 log10(255^2 / MSE) over every texel and channel, with the squared error summed in float64
(an exact integer for 8-bit images: every term is at most 255^2 and the sums stay below 2^53); every
PSNR this package reports is computed here.  SSIM here is the usual structural similarity: a Gaussian window of standard deviation 1.5 truncated
to 11 x 11 texels, C1 = (0.01 L)^2 and C2 = (0.03 L)^2 with L = 255, averaged over every window that
lies inside the image and over the channels (the paper does not state its parameters; these are the
common defaults)."""
from __future__ import annotations

import numpy as np
from scipy.ndimage import gaussian_filter

SIGMA = 1.5
RADIUS = 5


def squared_error(a, b) -> float:
    """Sum of squared differences in float64 of two images of equal shape: NumPy arrays, or device
    tensors (then summed on the device in float64)."""
    if hasattr(a, "double") and hasattr(b, "double"):
        d = a.double() - b.double()
        return float((d * d).sum().item())
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    return float((d * d).sum())


def psnr_from_sse(sse: float, n_values: int, data_range: float = 255.0) -> float:
    """PSNR (dB) of a summed squared error over n_values values; +inf for zero error."""
    if sse == 0:
        return float("inf")
    return float(10.0 * np.log10(data_range ** 2 * n_values / sse))


def psnr(a, b, data_range: float = 255.0) -> float:
    """PSNR (dB) of image `a` against image `b` (same shape; NumPy arrays or device tensors)."""
    n = a.numel() if hasattr(a, "numel") else np.asarray(a).size
    return psnr_from_sse(squared_error(a, b), int(n), data_range)


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
