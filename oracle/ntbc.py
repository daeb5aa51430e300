"""Neural Texture Block Compression: heads -> BC blocks, and the training step (oracle).

Test infrastructure only.  Follows the paper's Sec. 3.2 (NTBC), Sec. 3.3 (grid quantisation),
Sec. 3.4 (configuration: Adam, learning rates, cosine annealing with warm-up, T = 0.01) and App. A
(straight-through estimator for the argmax).

One trunk maps the block position to a head vector Y in [0,1] (after the sigmoid):
  * endpoint head: per texture in order, BC1 -> (R0,G0,B0,R1,G1,B1), BC4 -> (e0,e1);
  * colour head: texel-major, [texel 0..15][channels of every texture in order] (BC1: 3, BC4: 1).
The endpoint head plays the paper's endpoint network (predicted endpoints e^) and the colour head the
colour network (predicted uncompressed colours c^ of the block's 16 texels).

Inference (Sec. 3.2, Eq. palette, Eq. dist):
  * endpoints quantise as q = floor(y (2^b - 1) + 1/2), clamped (b = 5/6/5 for BC1, 8 for BC4);
  * BC1: c0 = pack565(q(e0)), c1 = pack565(q(e1)); swapped when c0 < c1 (four-colour mode);
    c0 == c1 gives every code 0.  BC4: the mode follows the stored order (e0 > e1: eight values);
  * the palette is the decoded palette of the stored endpoints divided by 255;
  * each texel takes n = argmax_n -||c^ - c_n||, computed as the least squared distance (same argmax)
    with ties going to the smallest logical n, and stores the format's code for n.

Training (Sec. 3.2, Eqs. lossNTBC; App. A):
  * targets: reference endpoints e (8-bit decoded endpoints of the reference block / 255), texel
    colours c (/255) and the reference palette c_n = (1 - w_n) e0 + w_n e1 of Eq. palette (BC4
    six-value mode: the special entries 0 and 1 of Eq. weightBC4);
  * L_e = mean (e^ - e)^2, L_c = mean (c^ - c)^2;
  * endpoint branch: d_n = -||c - c^_n|| with the continuous palette of the predicted endpoints
    (BC4 mode from e^0 > e^1); colour branch: d_n = -||c^ - c_n|| with the reference palette;
  * both branches decode x = c_ref[argmax d] and add mean (x - c)^2;
  * backward through the argmax as through the softmax expectation x~ = sum_i softmax(d/T)_i c_ref,i:
    dx/dd_j = (1/T) s_j (c_ref,j - x~).  (App. A prints the weight form with "n" where the weight w_n
    belongs; the form used here is the correct derivative of the expectation in palette values.)
  * total loss L = L_e + L_c + L_cd(endpoint) + L_cd(colour), every term a mean over its elements.
"""
from __future__ import annotations

import math

import numpy as np

from . import bc
from . import grid as G
from . import mlp

BC1 = 1
BC4 = 4


class Layout:
    """Offsets of every texture's values inside the head vector."""

    def __init__(self, formats):
        self.formats = [int(f) for f in formats]
        self.ep_off, self.ch_off = [], []
        e = c = 0
        for f in self.formats:
            self.ep_off.append(e)
            self.ch_off.append(c)
            e += 6 if f == BC1 else 2
            c += 3 if f == BC1 else 1
        self.E, self.C = e, c
        self.H = e + 16 * c

    def channels(self, t):
        return 3 if self.formats[t] == BC1 else 1

    def colour_index(self, t):
        """[16, ch] positions of texture t's predicted colours in Y."""
        ch = self.channels(t)
        return self.E + np.arange(16)[:, None] * self.C + self.ch_off[t] + np.arange(ch)[None, :]


# ------------------------------------------------------------------------------------------------
# Inference: heads -> packed blocks
# ------------------------------------------------------------------------------------------------
def quant_endpoint(y, bits: int, precision: str = "f64"):
    mx = (1 << bits) - 1
    if precision == "f32":
        y32 = np.asarray(y, dtype=np.float32)
        t = np.floor((y32 * np.float32(mx)) + np.float32(0.5))
    else:
        t = np.floor(np.asarray(y, dtype=np.float64) * mx + 0.5)
    return np.clip(t, 0, mx).astype(np.int64)


def _palette_real(codes_pal, precision):
    if precision == "f32":
        return codes_pal.astype(np.float32) / np.float32(255.0)
    return codes_pal.astype(np.float64) / 255.0


def _sqdist(chat, pal, precision):
    """Squared distance of chat [n,16,ch] to pal [n,N,ch] -> [n,16,N], summed over channels in order."""
    if precision == "f32":
        d = chat.astype(np.float32)[:, :, None, :] - pal[:, None, :, :]
        acc = d[..., 0] * d[..., 0]
        for k in range(1, d.shape[-1]):
            acc = acc + d[..., k] * d[..., k]
        return acc
    d = chat.astype(np.float64)[:, :, None, :] - pal[:, None, :, :]
    return (d * d).sum(axis=-1)


def pack_texture(Y, lay: Layout, t: int, precision: str = "f64", return_margin: bool = False):
    """Packed words [n] of texture t from heads Y [n, H]; optionally the per-block decision margin."""
    e = lay.ep_off[t]
    chat = Y[:, lay.colour_index(t)]                                 # [n, 16, ch]
    if lay.formats[t] == BC1:
        q0 = np.stack([quant_endpoint(Y[:, e + 0], 5, precision), quant_endpoint(Y[:, e + 1], 6, precision),
                       quant_endpoint(Y[:, e + 2], 5, precision)], axis=-1)
        q1 = np.stack([quant_endpoint(Y[:, e + 3], 5, precision), quant_endpoint(Y[:, e + 4], 6, precision),
                       quant_endpoint(Y[:, e + 5], 5, precision)], axis=-1)
        c0 = bc.pack565(q0[:, 0], q0[:, 1], q0[:, 2])
        c1 = bc.pack565(q1[:, 0], q1[:, 1], q1[:, 2])
        swap = c0 < c1
        c0, c1 = np.where(swap, c1, c0), np.where(swap, c0, c1)
        order = np.broadcast_to(bc.BC1_CODE_OF_LOGICAL, (len(c0), 4))
        lpal = bc.bc1_palette(c0, c1)[:, bc.BC1_CODE_OF_LOGICAL, :]
        dist = _sqdist(chat, _palette_real(lpal, precision), precision)
        n = np.argmin(dist, axis=2)
        n[c0 == c1] = 0
        codes = np.take_along_axis(order, n, axis=1)
        words = bc.bc1_pack(c0, c1, codes)
    else:
        e0 = quant_endpoint(Y[:, e], 8, precision)
        e1 = quant_endpoint(Y[:, e + 1], 8, precision)
        order = bc.bc4_logical_order(e0, e1)
        lpal = np.take_along_axis(bc.bc4_palette(e0, e1), order, axis=1)[:, :, None]
        dist = _sqdist(chat, _palette_real(lpal, precision), precision)
        n = np.argmin(dist, axis=2)
        codes = np.take_along_axis(order, n, axis=1)
        words = bc.bc4_pack(e0, e1, codes)
    if not return_margin:
        return words
    # decision margins: endpoint rounding distance (in units of y) and index distance gap
    ys = Y[:, e:e + (6 if lay.formats[t] == BC1 else 2)].astype(np.float64)
    bits = np.array([5, 6, 5, 5, 6, 5] if lay.formats[t] == BC1 else [8, 8], dtype=np.float64)
    mx = 2.0 ** bits - 1
    ep_margin = (np.abs(ys * mx - (np.floor(ys * mx) + 0.5)) / mx).min(axis=1)
    srt = np.sort(dist.astype(np.float64), axis=2)
    idx_margin = (srt[:, :, 1] - srt[:, :, 0]).min(axis=1)
    return words, ep_margin, idx_margin


def pack(Y, formats, precision: str = "f64"):
    lay = Layout(formats)
    return np.stack([pack_texture(Y, lay, t, precision) for t in range(len(lay.formats))], axis=0)


def grid_levels(cfg, grid=None, codes=None, scales=None, zeros=None):
    """Real per-level vertex values from a float grid or from uint8 codes + (scale, zero point)."""
    if codes is not None:
        g = G.dequant_grid(codes, scales, zeros, cfg.n_levels, cfg.base_res)
    else:
        g = np.asarray(grid, dtype=np.float64)
    return G.split_levels(g, cfg.n_levels, cfg.base_res)


def heads(cfg, levels, layers, ids, precision: str = "f64", scales=None):
    ids = np.asarray(ids, dtype=np.int64)
    x = G.features(levels, ids % cfg.blocks_w, ids // cfg.blocks_w, cfg.blocks_w, cfg.blocks_h)
    y, _ = mlp.forward(layers, x, precision, scales)
    return y


def calibration_ids(n_positions: int, n_sample: int):
    """Block positions of an FP8 calibration sample: every stride-th block, stride = n_positions //
    n_sample (at least 1), the first min(n_sample, n_positions) of them."""
    n = min(int(n_sample), int(n_positions))
    stride = max(1, int(n_positions) // max(1, int(n_sample)))
    return np.arange(n, dtype=np.int64) * stride


def fp8_calibration(cfg, levels, layers, n_sample: int):
    """Per-layer (s_x, s_w) FP8 scales from the calibration sample's float64 forward."""
    ids = calibration_ids(cfg.n_positions, n_sample)
    x = G.features(levels, ids % cfg.blocks_w, ids // cfg.blocks_w, cfg.blocks_w, cfg.blocks_h)
    return mlp.fp8_scales(layers, x)


def infer_blocks(cfg, levels, layers, ids, precision: str = "f64", scales=None):
    """(words [T, n], Y [n, H]) for block positions ids."""
    y = heads(cfg, levels, layers, ids, precision, scales)
    return pack(y, cfg.formats), y


# ------------------------------------------------------------------------------------------------
# Training targets and losses
# ------------------------------------------------------------------------------------------------
def _bc1_weights():
    w = np.arange(4) / 3.0
    return 1.0 - w, w, np.zeros(4)


def _bc4_weights(eight):
    """Per logical n: coefficient on e0, on e1, and a constant (Eq. palette / Eq. weightBC4)."""
    if eight:
        w = np.arange(8) / 7.0
        return 1.0 - w, w, np.zeros(8)
    a = np.zeros(8)
    b = np.zeros(8)
    k = np.zeros(8)
    for n in range(1, 7):
        w = (n - 1) / 5.0
        a[n], b[n] = 1.0 - w, w
    k[7] = 1.0
    return a, b, k


def palette_real(e0, e1, fmt, eight=None):
    """Eq. palette (and Eq. weightBC4) over endpoints e0, e1 [n, ch] -> ([n,N,ch], a [n,N], b [n,N])."""
    n = e0.shape[0]
    if fmt == BC1:
        a, b, k = (np.broadcast_to(v, (n, 4)) for v in _bc1_weights())
    else:
        a8, b8, k8 = _bc4_weights(True)
        a6, b6, k6 = _bc4_weights(False)
        sel = np.asarray(eight)[:, None]
        a = np.where(sel, a8, a6)
        b = np.where(sel, b8, b6)
        k = np.where(sel, k8, k6)
    pal = a[:, :, None] * e0[:, None, :] + b[:, :, None] * e1[:, None, :] + k[:, :, None]
    return pal, a, b


class Targets:
    """Per block position: reference endpoints, colours and reference palettes of every texture."""

    def __init__(self, formats, ref_words, texel_blocks):
        self.lay = Layout(formats)
        npos = len(ref_words[0])
        self.e_ref = np.zeros((npos, self.lay.E))
        self.c = np.zeros((npos, 16, self.lay.C))
        self.pal_ref = []
        for t, f in enumerate(self.lay.formats):
            e = self.lay.ep_off[t]
            ch = self.lay.channels(t)
            cols = np.asarray(texel_blocks[t], dtype=np.float64).reshape(npos, 16, ch) / 255.0
            self.c[:, :, self.lay.ch_off[t]:self.lay.ch_off[t] + ch] = cols
            if f == BC1:
                c0, c1, _ = bc.bc1_fields(ref_words[t])
                e0 = bc.endpoint_rgb8(c0) / 255.0
                e1 = bc.endpoint_rgb8(c1) / 255.0
                self.e_ref[:, e:e + 3] = e0
                self.e_ref[:, e + 3:e + 6] = e1
                pal, _, _ = palette_real(e0, e1, BC1)
            else:
                b0, b1, _ = bc.bc4_fields(ref_words[t])
                e0 = (b0 / 255.0)[:, None]
                e1 = (b1 / 255.0)[:, None]
                self.e_ref[:, e] = e0[:, 0]
                self.e_ref[:, e + 1] = e1[:, 0]
                pal, _, _ = palette_real(e0, e1, BC4, b0 > b1)
            self.pal_ref.append(pal)


def _softmax(d, temp):
    z = d / temp
    z = z - z.max(axis=-1, keepdims=True)
    ez = np.exp(z)
    return ez / ez.sum(axis=-1, keepdims=True)


def _cd_branch(dist_delta, pal_ref, c, ncd, temp):
    """Shared part of the decoded-colour loss: hard argmax forward, softmax-expectation backward.

    dist_delta: [n,16,N,ch] differences whose norms are the distances (d = -norm).
    Returns (loss, dL/dd [n,16,N], norms [n,16,N])."""
    norm = np.sqrt((dist_delta ** 2).sum(axis=-1))
    d = -norm
    k = np.argmax(d, axis=2)                                           # first max: smallest n
    x = np.take_along_axis(pal_ref[:, None, :, :], k[:, :, None, None], axis=2)[:, :, 0, :]
    loss = ((x - c) ** 2).sum() / ncd
    gx = 2.0 * (x - c) / ncd                                           # [n,16,ch]
    s = _softmax(d, temp)                                              # [n,16,N]
    xs = (s[..., None] * pal_ref[:, None, :, :]).sum(axis=2)           # [n,16,ch]
    dd = (s / temp) * ((pal_ref[:, None, :, :] - xs[:, :, None, :]) * gx[:, :, None, :]).sum(axis=-1)
    return loss, dd, norm


def loss_and_grad(Y, tg: Targets, ids, temp: float = 0.01, terms=(1.0, 1.0, 1.0, 1.0)):
    """Losses (L_e, L_c, L_cd_e, L_cd_c) and dL/dY for heads Y [n, H] of block positions ids.

    ``terms`` weights the four losses in the returned gradient (all 1 in training)."""
    lay = tg.lay
    n = Y.shape[0]
    ids = np.asarray(ids, dtype=np.int64)
    e_hat = Y[:, :lay.E]
    c_hat = Y[:, lay.E:].reshape(n, 16, lay.C)
    e_ref = tg.e_ref[ids]
    c = tg.c[ids]
    w_e, w_c, w_cde, w_cdc = terms
    d_e = w_e * 2.0 * (e_hat - e_ref) / (n * lay.E)
    d_c = w_c * 2.0 * (c_hat - c) / (n * 16 * lay.C)
    l_e = ((e_hat - e_ref) ** 2).mean()
    l_c = ((c_hat - c) ** 2).mean()
    ncd = n * 16 * lay.C
    l_cde = l_cdc = 0.0
    for t, f in enumerate(lay.formats):
        e = lay.ep_off[t]
        ch = lay.channels(t)
        sl = slice(lay.ch_off[t], lay.ch_off[t] + ch)
        ct = c[:, :, sl]
        pal_ref = tg.pal_ref[t][ids]                                    # [n,N,ch]
        if f == BC1:
            e0h, e1h = e_hat[:, e:e + 3], e_hat[:, e + 3:e + 6]
            pal_h, a, b = palette_real(e0h, e1h, BC1)
        else:
            e0h, e1h = e_hat[:, e:e + 1], e_hat[:, e + 1:e + 2]
            pal_h, a, b = palette_real(e0h, e1h, BC4, e0h[:, 0] > e1h[:, 0])
        # endpoint branch: d_n = -||c - c^_n||
        delta = ct[:, :, None, :] - pal_h[:, None, :, :]
        loss, dd, norm = _cd_branch(delta, pal_ref, ct, ncd, temp)
        l_cde += loss
        with np.errstate(invalid="ignore", divide="ignore"):
            unit = np.where(norm[..., None] > 0, delta / norm[..., None], 0.0)
        g_pal = w_cde * dd[..., None] * unit                                    # dL/dc^_n  [n,16,N,ch]
        d_e[:, e:e + ch] += (g_pal * a[:, None, :, None]).sum(axis=(1, 2))
        d_e[:, e + ch:e + 2 * ch] += (g_pal * b[:, None, :, None]).sum(axis=(1, 2))
        # colour branch: d_n = -||c^ - c_n||
        ch_hat = c_hat[:, :, sl]
        delta = ch_hat[:, :, None, :] - pal_ref[:, None, :, :]
        loss, dd, norm = _cd_branch(delta, pal_ref, ct, ncd, temp)
        l_cdc += loss
        with np.errstate(invalid="ignore", divide="ignore"):
            unit = np.where(norm[..., None] > 0, delta / norm[..., None], 0.0)
        d_c[:, :, sl] += (-w_cdc * dd[..., None] * unit).sum(axis=2)
    dY = np.concatenate([d_e, d_c.reshape(n, -1)], axis=1)
    return np.array([l_e, l_c, l_cde, l_cdc]), dY


# ------------------------------------------------------------------------------------------------
# Optimiser and schedule (Sec. 3.4)
# ------------------------------------------------------------------------------------------------
def learning_rate(step: int, lr0: float, total_steps: int, warmup: int = 10):
    """Linear warm-up lr0*(step+1)/warmup, then cosine annealing to 0 at total_steps."""
    if step < warmup:
        return lr0 * (step + 1) / warmup
    return lr0 * 0.5 * (1.0 + math.cos(math.pi * (step - warmup) / max(1, total_steps - warmup)))


def adam(p, g, m, v, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-15):
    """One bias-corrected Adam update (t counts from 1); returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


class TrainState:
    def __init__(self, grid, layers):
        self.grid = np.asarray(grid, dtype=np.float64).copy()
        self.layers = [(np.asarray(w, np.float64).copy(), np.asarray(b, np.float64).copy())
                       for w, b in layers]
        self.m_grid = np.zeros_like(self.grid)
        self.v_grid = np.zeros_like(self.grid)
        self.m_layers = [(np.zeros_like(w), np.zeros_like(b)) for w, b in self.layers]
        self.v_layers = [(np.zeros_like(w), np.zeros_like(b)) for w, b in self.layers]


def gradients(cfg, grid, layers, tg: Targets, ids, qat: bool, temp: float = 0.01,
              terms=(1.0, 1.0, 1.0, 1.0), precision: str = "f64"):
    """Losses and gradients (d grid, [(dW, db)]) at the given parameters for batch ids.  precision
    "bf16" evaluates the MLP forward and backward with bfloat16 product operands (mlp.forward and
    mlp.backward); the losses, the grid and its scatter stay float64."""
    ids = np.asarray(ids, dtype=np.int64)
    if qat:
        gvals, mask = G.fake_quant_grid(grid, cfg.n_levels, cfg.base_res)
    else:
        gvals, mask = np.asarray(grid, dtype=np.float64), None
    levels = G.split_levels(gvals, cfg.n_levels, cfg.base_res)
    bx, by = ids % cfg.blocks_w, ids // cfg.blocks_w
    x = G.features(levels, bx, by, cfg.blocks_w, cfg.blocks_h)
    y, cache = mlp.forward(layers, x, precision)
    losses, dy = loss_and_grad(y, tg, ids, temp, terms)
    dws, dbs, dx = mlp.backward(layers, cache, dy, y, precision)
    dgrid = G.features_backward(dx, bx, by, cfg.blocks_w, cfg.blocks_h, cfg.n_levels, cfg.base_res,
                                cfg.n_features, mask)
    return losses, dgrid, list(zip(dws, dbs)), y


def train_step(cfg, st: TrainState, tg: Targets, ids, step: int, total_steps: int, qat: bool,
               lr_grid: float = 0.01, lr_mlp: float = 0.005, temp: float = 0.01):
    """One training iteration: forward, losses, backward, Adam on grid and MLP; returns the losses."""
    losses, dgrid, dlayers, _ = gradients(cfg, st.grid, st.layers, tg, ids, qat, temp)
    t = step + 1
    lg = learning_rate(step, lr_grid, total_steps)
    lm = learning_rate(step, lr_mlp, total_steps)
    st.grid, st.m_grid, st.v_grid = adam(st.grid, dgrid, st.m_grid, st.v_grid, t, lg)
    for k, ((w, b), (dw, db)) in enumerate(zip(st.layers, dlayers)):
        (mw, mb), (vw, vb) = st.m_layers[k], st.v_layers[k]
        w, mw, vw = adam(w, dw, mw, vw, t, lm)
        b, mb, vb = adam(b, db, mb, vb, t, lm)
        st.layers[k] = (w, b)
        st.m_layers[k] = (mw, mb)
        st.v_layers[k] = (vw, vb)
    return losses
