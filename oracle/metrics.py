"""Quality metrics and the tie classification (oracle; test infrastructure only).

PSNR against the uncompressed texture (Sec. 4.3): 10 log10(255^2 / MSE) over every texel and channel,
+inf when identical.  Block identity: the fraction of identical 64-bit words.

Tie classification of a block that differs between an implementation under test and the oracle: the
block is a quantisation-boundary tie when (1) packing the implementation's own head values with the
oracle's float32 packer reproduces its word bit for bit, and (2) the oracle's smallest decision margin
for that block (distance of an endpoint value to its rounding boundary, in y units; gap between the two
nearest squared palette distances) is within what the head difference d of the block, plus the
implementation's float32 rounding of the decision itself, can move it.  d = |Y_impl - Y_oracle|_inf
over the heads that decide this texture's word only (its endpoint values and its 16 predicted
colours), so a large difference in another texture's heads explains nothing here:
  * endpoint: d + 1.25e-7.  The implementation decides floor(fl(fl(y*m) + 0.5)) in float32; both
    roundings together move y*m by at most one ulp of values below m+1, i.e. 2^-23 * 2^ceil(log2(m+1)),
    which is < 1.25e-7 * m for m = 31, 63, 255;
  * index: 2*ch*d + 2e-6 for a ch-channel texel.  D_a - D_b changes by 2 sum_c (p_b,c - p_a,c) delta_c
    under a colour change delta (palette values lie in [0, 1]); float32 evaluation of each squared
    distance (a difference, ch squares, ch-1 sums, each within half an ulp, D <= 3) is off by < 1e-6.
"""
from __future__ import annotations

import numpy as np

from . import ntbc


def psnr(original, decoded):
    a = np.asarray(original, dtype=np.float64)
    b = np.asarray(decoded, dtype=np.float64)
    mse = ((a - b) ** 2).mean()
    return float("inf") if mse == 0 else 10.0 * np.log10(255.0 ** 2 / mse)


def identity(words_a, words_b):
    a = np.asarray(words_a, dtype=np.uint64)
    b = np.asarray(words_b, dtype=np.uint64)
    return float((a == b).mean())


def texture_head_difference(abs_diff, lay, t):
    """Per block, the largest |difference| among the heads that decide texture t's word: its endpoint
    values (6 for BC1, 2 for BC4) and its 16 x channels predicted colours.  abs_diff: [n, H]."""
    e = lay.ep_off[t]
    n_ep = 6 if lay.formats[t] == ntbc.BC1 else 2
    cols = lay.colour_index(t).ravel()
    sel = np.concatenate([np.arange(e, e + n_ep), cols])
    return abs_diff[:, sel].max(axis=1) if len(abs_diff) else np.zeros(0)


def classify_differences(Y_impl, words_impl, Y_oracle, words_oracle, formats, endpoint_slack=1.25e-7,
                         index_factor=2.0, index_slack=2e-6):
    """Per texture: number of differing blocks and how many of them are boundary ties.

    The allowances are those derived above (a block is a tie when its endpoint margin is at most
    d + endpoint_slack, or its index gap at most index_factor * ch * d + index_slack); they are
    arguments only so that a test can show that a wrong constant changes a verdict.
    Returns dict with 'differ', 'ties', 'repack_exact' (condition 1 over all blocks)."""
    lay = ntbc.Layout(formats)
    Y_impl = np.asarray(Y_impl)
    diff_all = np.abs(Y_impl.astype(np.float64) - np.asarray(Y_oracle, dtype=np.float64))
    out = {"differ": 0, "ties": 0, "repack_exact": True,
           "max_dy": float(diff_all.max()) if diff_all.size else 0.0, "non_ties": []}
    for t in range(len(lay.formats)):
        dy = texture_head_difference(diff_all, lay, t)
        repacked = ntbc.pack_texture(Y_impl, lay, t, "f32")
        if not np.array_equal(repacked, words_impl[t]):
            out["repack_exact"] = False
        diff = words_impl[t] != words_oracle[t]
        if not diff.any():
            continue
        _, ep_m, idx_m = ntbc.pack_texture(Y_oracle[diff], lay, t, "f64", return_margin=True)
        ch = lay.channels(t)
        tie = (ep_m <= dy[diff] + endpoint_slack) | (idx_m <= index_factor * ch * dy[diff] + index_slack)
        out["differ"] += int(diff.sum())
        out["ties"] += int(tie.sum())
        idx = np.nonzero(diff)[0]
        for i in np.nonzero(~tie)[0][:10]:
            out["non_ties"].append((t, int(idx[i]), float(dy[idx[i]]), float(ep_m[i]), float(idx_m[i])))
    return out


def model_bytes(grids, mlps, bytes_per_feature: int = 1, bytes_per_param: int = 2):
    """Stored size of a model: dense grids of res_l^2 vertices (res_l = base * 2^l) with
    ``bytes_per_feature`` per feature, plus MLP weights and biases at ``bytes_per_param`` each.

    grids: iterable of (n_levels, base_res, n_features); mlps: iterable of layer widths [in, ..., out]."""
    total = 0
    for n_levels, base_res, n_features in grids:
        total += sum((base_res << l) ** 2 for l in range(n_levels)) * n_features * bytes_per_feature
    for dims in mlps:
        total += sum(dims[i] * dims[i + 1] + dims[i + 1] for i in range(len(dims) - 1)) * bytes_per_param
    return total
