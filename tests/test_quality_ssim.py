"""SSIM of the reports (paper Sec. 4.3 metrics) against its definition written out with explicit
windows, plus closed forms."""
import numpy as np

from paper_2407_09543_amd import quality


def _brute(a, b, L=255.0):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if a.ndim == 2:
        a, b = a[..., None], b[..., None]
    r, s = quality.RADIUS, quality.SIGMA
    k = np.arange(-r, r + 1)
    g = np.exp(-k * k / (2 * s * s))
    w = np.outer(g, g)
    w /= w.sum()
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    per_channel = []
    for c in range(a.shape[2]):
        vals = []
        for i in range(r, a.shape[0] - r):
            for j in range(r, a.shape[1] - r):
                x = a[i - r:i + r + 1, j - r:j + r + 1, c]
                y = b[i - r:i + r + 1, j - r:j + r + 1, c]
                mx, my = (w * x).sum(), (w * y).sum()
                vx = (w * (x - mx) ** 2).sum()
                vy = (w * (y - my) ** 2).sum()
                cxy = (w * (x - mx) * (y - my)).sum()
                vals.append(((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2)))
        per_channel.append(np.mean(vals))
    return float(np.mean(per_channel))


def test_ssim_matches_windowed_definition():
    rng = np.random.default_rng(3)
    a = rng.integers(0, 256, (19, 23, 3))
    b = np.clip(a + rng.normal(0, 20, a.shape), 0, 255)
    assert abs(quality.ssim(a, b) - _brute(a, b)) < 1e-9
    c = rng.integers(0, 256, (17, 16))
    d = rng.integers(0, 256, (17, 16))
    assert abs(quality.ssim(c, d) - _brute(c, d)) < 1e-9


def test_ssim_closed_forms():
    rng = np.random.default_rng(4)
    a = rng.integers(0, 256, (24, 24, 3))
    assert abs(quality.ssim(a, a) - 1.0) < 1e-12
    # two constant images: only the luminance term remains
    x, y = np.full((16, 16), 100.0), np.full((16, 16), 140.0)
    c1 = (0.01 * 255) ** 2
    expect = (2 * 100 * 140 + c1) / (100 ** 2 + 140 ** 2 + c1)
    assert abs(quality.ssim(x, y) - expect) < 1e-12
    # symmetric
    b = rng.integers(0, 256, (24, 24, 3))
    assert abs(quality.ssim(a, b) - quality.ssim(b, a)) < 1e-12


def test_psnr_closed_forms_and_float64_sums():
    # reported PSNR (Sec. 4.3): 10 log10(255^2 / MSE), squared error summed in float64
    import torch
    a = np.full((64, 64, 3), 100, np.uint8)
    assert quality.psnr(a, a) == float("inf")
    b = a + 1                                                   # MSE 1
    assert abs(quality.psnr(b, a) - 20 * np.log10(255.0)) < 1e-12
    c = a.copy()
    c[0, 0, 0] = 0                                              # one error of 100 over 12,288 values
    assert abs(quality.psnr(c, a) - 10 * np.log10(255.0 ** 2 * a.size / 100 ** 2)) < 1e-12
    # a large image with a total squared error that float32 sums would round: exact in float64
    big = np.zeros((4096, 4096), np.uint8)
    noisy = big.copy()
    noisy[::2, ::3] = 255
    n255 = int((noisy == 255).sum())
    assert quality.squared_error(noisy, big) == n255 * 255.0 ** 2
    assert quality.squared_error(torch.from_numpy(noisy), torch.from_numpy(big)) == n255 * 255.0 ** 2
    assert quality.psnr(torch.from_numpy(noisy), torch.from_numpy(big)) == quality.psnr(noisy, big)
