"""Multi-resolution 2-D feature grids and their 8-bit quantisation (oracle; test infrastructure only).

Paper anchors: multi-resolution feature grids addressed by the normalised block index (s, t) in [0,1]
(Sec. 3.1 and Sec. 3.4), features of all levels concatenated; per-level asymmetric 8-bit quantisation
with min/max ranges recomputed every iteration (Sec. 3.3) using the uniform affine quantiser
(Sec. 2.3, Eqs. quantize, dequantize, quantizer, scaling_factor, zero_point).

Readings where the paper is silent or garbled:
  * Level l has res_l = base_res * 2^l vertices per side and res_l^2 vertices in all (the paper's
    stated storage sizes only come out with res^2 vertices per level).
  * Block (bx, by) of a Bw x Bh block grid samples level l at the cell-centred position
    p = (bx + 1/2) * res_l / Bw - 1/2 (likewise y), clamped to [0, res_l - 1]; corners i0 =
    min(floor(p), res_l - 2) and i0 + 1, fraction f = p - i0.  With p = num / (2 Bw),
    num = (2 bx + 1) res_l - Bw, the corner is an integer decision and f a dyadic fraction.
  * Bilinear weights (1-fx)(1-fy), fx(1-fy), (1-fx)fy, fx fy on the corners (i0,j0), (i0+1,j0),
    (i0,j0+1), (i0+1,j0+1).  Concatenation order: [level 0 features 0..F-1, level 1 ..., ...].
  * Storage: level-major, then row-major vertex index j*res + i (j = y), then feature.
  * Zero point: the printed z = round(alpha * s) is dimensionally wrong; the zero point that makes
    real 0 representable is z = clamp(round(-alpha / s), 0, 255).
  * Range: the zero point exists so that real 0 is an exact code (Sec. 2.3), which needs alpha <= 0 <=
    beta; a level whose values all share one sign has its range widened to include 0 (alpha = min(min,
    0), beta = max(max, 0)), so every value of the level stays inside [alpha, beta] and none is
    clamped.
  * The quantiser's gradient is 1 where the value is not clamped and 0 where it is (the printed
    "w" is read as 1); alpha and beta carry no gradient.
  * The half-way rounding is round-half-to-even.  s and z, and every code, are computed in float32
    (the GPU path's precision for these integer decisions).  A level whose min equals its max takes
    s = 1, z = 0.
"""
from __future__ import annotations

import numpy as np


def level_res(n_levels: int, base_res: int):
    return [base_res << l for l in range(n_levels)]


def level_offsets(n_levels: int, base_res: int):
    """Vertex offset of each level in the level-major storage, plus the total at the end."""
    offs = [0]
    for r in level_res(n_levels, base_res):
        offs.append(offs[-1] + r * r)
    return offs


def corner(b, blocks: int, res: int):
    """Integer corner index i0 and fraction numerator fnum (f = fnum / (2*blocks)) for block index b."""
    b = np.asarray(b, dtype=np.int64)
    den = 2 * blocks
    num = (2 * b + 1) * res - blocks
    hi = (res - 1) * den
    i0 = np.where(num <= 0, 0, np.where(num >= hi, res - 2, num // den))
    fnum = np.where(num <= 0, 0, np.where(num >= hi, den, num - i0 * den))
    return i0, fnum, den


def features(levels, bx, by, blocks_w: int, blocks_h: int):
    """Concatenated bilinear features [n, L*F] (float64) of blocks (bx, by).

    ``levels``: list of per-level vertex values, each [res*res, F] (real values, any float dtype)."""
    bx = np.asarray(bx, dtype=np.int64)
    by = np.asarray(by, dtype=np.int64)
    out = []
    for g in levels:
        g = np.asarray(g, dtype=np.float64)
        res = int(round(np.sqrt(g.shape[0])))
        i0, fxn, dx = corner(bx, blocks_w, res)
        j0, fyn, dy = corner(by, blocks_h, res)
        fx = (fxn / dx)[:, None]
        fy = (fyn / dy)[:, None]
        v00 = g[j0 * res + i0]
        v10 = g[j0 * res + i0 + 1]
        v01 = g[(j0 + 1) * res + i0]
        v11 = g[(j0 + 1) * res + i0 + 1]
        out.append((1 - fx) * (1 - fy) * v00 + fx * (1 - fy) * v10 + (1 - fx) * fy * v01 + fx * fy * v11)
    return np.concatenate(out, axis=1)


def features_backward(d_feat, bx, by, blocks_w: int, blocks_h: int, n_levels: int, base_res: int,
                      n_features: int, mask=None):
    """Scatter-add of d_feat [n, L*F] into a gradient grid [sum res^2, F] (float64).

    ``mask`` (optional, same shape as the grid) multiplies the result: the quantiser's pass-through."""
    offs = level_offsets(n_levels, base_res)
    grad = np.zeros((offs[-1], n_features), dtype=np.float64)
    bx = np.asarray(bx, dtype=np.int64)
    by = np.asarray(by, dtype=np.int64)
    for l, res in enumerate(level_res(n_levels, base_res)):
        d = np.asarray(d_feat[:, l * n_features:(l + 1) * n_features], dtype=np.float64)
        i0, fxn, dx = corner(bx, blocks_w, res)
        j0, fyn, dy = corner(by, blocks_h, res)
        fx = (fxn / dx)[:, None]
        fy = (fyn / dy)[:, None]
        base = offs[l]
        np.add.at(grad, base + j0 * res + i0, (1 - fx) * (1 - fy) * d)
        np.add.at(grad, base + j0 * res + i0 + 1, fx * (1 - fy) * d)
        np.add.at(grad, base + (j0 + 1) * res + i0, (1 - fx) * fy * d)
        np.add.at(grad, base + (j0 + 1) * res + i0 + 1, fx * fy * d)
    if mask is not None:
        grad = grad * mask
    return grad


def split_levels(grid, n_levels: int, base_res: int):
    offs = level_offsets(n_levels, base_res)
    return [grid[offs[l]:offs[l + 1]] for l in range(n_levels)]


# ------------------------------------------------------------------------------------------------
# 8-bit quantisation
# ------------------------------------------------------------------------------------------------
def qat_params(level_values):
    """(s, z) of one level from its real values: s float32, z int (float32 arithmetic), over the
    level's range widened to include 0."""
    v = np.asarray(level_values, dtype=np.float32)
    lo = min(np.float32(v.min()), np.float32(0.0))
    hi = max(np.float32(v.max()), np.float32(0.0))
    if hi == lo:
        return np.float32(1.0), 0
    s = np.float32(np.float32(hi - lo) / np.float32(255.0))
    z = np.float32(np.rint(np.float32(-lo) / s))
    z = int(min(max(z, np.float32(0.0)), np.float32(255.0)))
    return s, z


def quant_codes(values, s, z):
    """Unclamped t = rne(w/s) + z (float32 arithmetic) and the clamped uint8 code."""
    w = np.asarray(values, dtype=np.float32)
    t = np.rint(w / np.float32(s)).astype(np.float64) + z
    return t, np.clip(t, 0, 255).astype(np.uint8)


def dequant(codes, s, z):
    """Eq. dequantize: s * (q - z), in float64."""
    return np.float64(s) * (np.asarray(codes, dtype=np.float64) - z)


def fake_quant(values, s, z):
    """Eq. quantizer Q(w) (float64 result) and the pass-through mask (1 = not clamped)."""
    t, q = quant_codes(values, s, z)
    mask = ((t >= 0) & (t <= 255)).astype(np.float64)
    return dequant(q, s, z), mask


def quantise_grid(grid, n_levels: int, base_res: int):
    """Per-level (s, z) and uint8 codes of a real grid [sum res^2, F]."""
    scales, zeros, codes = [], [], []
    for g in split_levels(grid, n_levels, base_res):
        s, z = qat_params(g)
        scales.append(s)
        zeros.append(z)
        codes.append(quant_codes(g, s, z)[1])
    return (np.concatenate(codes, axis=0), np.array(scales, dtype=np.float32),
            np.array(zeros, dtype=np.int32))


def fake_quant_grid(grid, n_levels: int, base_res: int):
    """Q(grid) per level (float64) and the pass-through mask, both [sum res^2, F]."""
    vals, masks = [], []
    for g in split_levels(grid, n_levels, base_res):
        s, z = qat_params(g)
        v, m = fake_quant(g, s, z)
        vals.append(v)
        masks.append(m)
    return np.concatenate(vals, axis=0), np.concatenate(masks, axis=0)


def dequant_grid(codes, scales, zeros, n_levels: int, base_res: int):
    offs = level_offsets(n_levels, base_res)
    out = np.empty(codes.shape, dtype=np.float64)
    for l in range(n_levels):
        out[offs[l]:offs[l + 1]] = dequant(codes[offs[l]:offs[l + 1]], scales[l], int(zeros[l]))
    return out
