"""The naive approach (oracle; test infrastructure only): the paper's comparison method (Sec. 3.1, "Naive
Approach"; Fig. naive network) in this project's one-trunk form.

NTBC's colour head predicts each texel's uncompressed colour and picks the palette entry nearest to it
(Eq. dist).  The naive approach instead predicts each texel's interpolation weight:

Heads Y [n, H]: the endpoint head as NTBC (per texture in order: BC1 -> R0 G0 B0 R1 G1 B1, BC4 -> e0 e1;
E values), then the weight head, texel-major [texel 0..15][one weight per texture in order]:
H = E + 16 T for T textures.

Inference (Sec. 3.1: the floating-point weights w_f are quantised to the block's weights w_n):
  * endpoints quantise, order and choose the BC4 mode exactly as NTBC's (oracle.ntbc, reading 6);
  * BC1 (four-colour mode): n = argmin over n = 0..3 of |w' - n/3|, where w' = 1 - w when the
    endpoints were swapped (the stored c0 is then the predicted endpoint 1, so the weight axis turns
    round); c0 == c1: every code 0;
  * BC4 eight-value mode (e0 > e1): n = argmin |w - n/7| over n = 0..7; six-value mode: n = argmin
    |w - (n-1)/5| over n = 1..6 (the interpolated weights; the constant entries 0 and 1 carry no
    weight);
  * the decision is taken in float32 (w' = 1 - w and |w' - w_n| with w_n = float32(n) / float32(m));
    ties go to the smallest n; the stored code is the format's code of logical n (oracle.bc).

Training (Sec. 3.1, two stages):
  * stage 1 (the first 80% of the iterations): decoded colours from the predicted endpoints and the
    floating-point weights, x = (1 - w) e0^ + w e1^ per channel (Eq. palette with the continuous
    weight), L = mean over texels and channels of (x - c)^2 against the uncompressed texels c;
  * stage 2 (the rest): the same loss with w replaced by the nearest weight w_n of the block's mode
    (BC1: n/3; BC4 from e0^ > e1^: n/7, or (n-1)/5 for n = 1..6; the predicted endpoints stay
    continuous and unswapped; float32 decision as at inference), so only the endpoints receive a
    gradient; and the weight network is frozen.  One trunk serves both heads here, so "the weight
    network frozen" reads as: stage 2 updates only the endpoint head's own parameters (its rows of
    the last layer's weights and biases); the grid, the hidden layers and the weight head keep their
    values.
"""
from __future__ import annotations

import numpy as np

from . import bc
from .ntbc import BC1, BC4, Layout, quant_endpoint


class NaiveLayout:
    """Offsets inside the naive head vector."""

    def __init__(self, formats):
        self.base = Layout(formats)
        self.formats = self.base.formats
        self.ep_off = self.base.ep_off
        self.E = self.base.E
        self.T = len(self.formats)
        self.H = self.E + 16 * self.T

    def weight_index(self, t):
        """[16] positions of texture t's predicted weights in Y."""
        return self.E + np.arange(16) * self.T + t


def _grid_weights(m: int, first: int, count: int):
    """float32 weights (n - first) / m of logical n = first .. first+count-1."""
    n = np.arange(first, first + count)
    return (np.float32(1) * (n - first).astype(np.float32)) / np.float32(m)


def nearest_weight_index(w, fmt, eight):
    """Logical index n [.., 16] of the nearest quantised weight to w [.., 16] (float32 decision; ties
    to the smallest n).  BC1: weights n/3; BC4: n/7 (eight) or (n-1)/5 for n = 1..6 (six)."""
    w32 = np.asarray(w, dtype=np.float32)
    if fmt == BC1:
        d = np.abs(w32[..., None] - _grid_weights(3, 0, 4))
        return np.argmin(d, axis=-1)
    d8 = np.abs(w32[..., None] - _grid_weights(7, 0, 8))
    d6 = np.abs(w32[..., None] - _grid_weights(5, 1, 6))
    n8 = np.argmin(d8, axis=-1)
    n6 = np.argmin(d6, axis=-1) + 1
    return np.where(np.asarray(eight)[..., None], n8, n6)


def pack(Y, formats):
    """Packed words [T, n] of naive heads Y [n, H] (inference, float32 decisions)."""
    lay = NaiveLayout(formats)
    out = []
    for t, f in enumerate(lay.formats):
        e = lay.ep_off[t]
        w = np.asarray(Y[:, lay.weight_index(t)], dtype=np.float32)     # [n, 16]
        if f == BC1:
            q0 = np.stack([quant_endpoint(Y[:, e + k], b, "f32") for k, b in ((0, 5), (1, 6), (2, 5))], axis=-1)
            q1 = np.stack([quant_endpoint(Y[:, e + 3 + k], b, "f32") for k, b in ((0, 5), (1, 6), (2, 5))], axis=-1)
            c0 = bc.pack565(q0[:, 0], q0[:, 1], q0[:, 2])
            c1 = bc.pack565(q1[:, 0], q1[:, 1], q1[:, 2])
            swap = c0 < c1
            c0, c1 = np.where(swap, c1, c0), np.where(swap, c0, c1)
            w = np.where(swap[:, None], np.float32(1) - w, w)
            n = nearest_weight_index(w, BC1, None)
            n[c0 == c1] = 0
            out.append(bc.bc1_pack(c0, c1, bc.BC1_CODE_OF_LOGICAL[n]))
        else:
            e0 = quant_endpoint(Y[:, e], 8, "f32")
            e1 = quant_endpoint(Y[:, e + 1], 8, "f32")
            n = nearest_weight_index(w, BC4, e0 > e1)
            codes = np.take_along_axis(bc.bc4_logical_order(e0, e1), n, axis=1)
            out.append(bc.bc4_pack(e0, e1, codes))
    return np.stack(out, axis=0)


def _stage2_weight(w, fmt, eight):
    """The quantised weight w_n (float64 value n/3, n/7 or (n-1)/5) that stage 2 decodes with."""
    n = nearest_weight_index(w, fmt, eight)
    if fmt == BC1:
        return n / 3.0
    return np.where(np.asarray(eight)[..., None], n / 7.0, (n - 1) / 5.0)


def loss_and_grad(Y, tg, ids, stage: int):
    """(L, dL/dY) of naive heads Y [n, H] for block positions ids against the texels of tg (an
    oracle.ntbc.Targets: tg.c [positions, 16, C] in NTBC's channel layout).  stage 1: continuous
    weights; stage 2: quantised weights, no gradient to the weights."""
    lay = NaiveLayout(tg.lay.formats)
    n = Y.shape[0]
    ids = np.asarray(ids, dtype=np.int64)
    c = tg.c[ids]
    N = n * 16 * tg.lay.C
    dY = np.zeros_like(np.asarray(Y, dtype=np.float64))
    loss = 0.0
    for t, f in enumerate(lay.formats):
        e = lay.ep_off[t]
        ch = 3 if f == BC1 else 1
        ct = c[:, :, tg.lay.ch_off[t]:tg.lay.ch_off[t] + ch]               # [n, 16, ch]
        e0 = Y[:, e:e + ch].astype(np.float64)
        e1 = Y[:, e + ch:e + 2 * ch].astype(np.float64)
        wi = lay.weight_index(t)
        w = Y[:, wi].astype(np.float64)                                     # [n, 16]
        if stage == 2:
            w = _stage2_weight(Y[:, wi], f, e0[:, 0] > e1[:, 0] if f == BC4 else None)
        x = (1.0 - w)[:, :, None] * e0[:, None, :] + w[:, :, None] * e1[:, None, :]
        r = x - ct
        loss += (r * r).sum() / N
        g = 2.0 * r / N                                                     # dL/dx [n, 16, ch]
        dY[:, e:e + ch] += (g * (1.0 - w)[:, :, None]).sum(axis=1)
        dY[:, e + ch:e + 2 * ch] += (g * w[:, :, None]).sum(axis=1)
        if stage == 1:
            dY[:, wi] += (g * (e1 - e0)[:, None, :]).sum(axis=2)
    return loss, dY


def endpoint_rows(formats):
    """Stage 2's trainable rows of the last layer (weights [out][in] and biases [out]): the endpoint
    head's outputs 0 .. E-1."""
    return np.arange(NaiveLayout(formats).E)


def gradients(cfg, grid, layers, tg, ids, qat: bool, stage: int, precision: str = "f64"):
    """(L, d grid, [(dW, db)], Y) of the naive loss of the given stage at the given parameters for batch
    ids (the forward and backward of oracle.ntbc.gradients with this loss)."""
    from . import grid as G
    from . import mlp
    ids = np.asarray(ids, dtype=np.int64)
    if qat:
        gvals, mask = G.fake_quant_grid(grid, cfg.n_levels, cfg.base_res)
    else:
        gvals, mask = np.asarray(grid, dtype=np.float64), None
    levels = G.split_levels(gvals, cfg.n_levels, cfg.base_res)
    bx, by = ids % cfg.blocks_w, ids // cfg.blocks_w
    x = G.features(levels, bx, by, cfg.blocks_w, cfg.blocks_h)
    y, cache = mlp.forward(layers, x, precision)
    loss, dy = loss_and_grad(y, tg, ids, stage)
    dws, dbs, dx = mlp.backward(layers, cache, dy, y, precision)
    dgrid = G.features_backward(dx, bx, by, cfg.blocks_w, cfg.blocks_h, cfg.n_levels, cfg.base_res,
                                cfg.n_features, mask)
    return loss, dgrid, list(zip(dws, dbs)), y


def train_step(cfg, st, tg, ids, step: int, total_steps: int, qat: bool, stage: int,
               lr_grid: float = 0.01, lr_mlp: float = 0.005):
    """One naive training iteration on an oracle.ntbc.TrainState (float64): forward, the stage's loss,
    backward, Adam with the schedule of Sec. 3.4.  Stage 1 updates every parameter; stage 2 only the
    endpoint head's rows of the last layer (the rest keep their values and their moments)."""
    from .ntbc import adam, learning_rate
    loss, dgrid, dlayers, _ = gradients(cfg, st.grid, st.layers, tg, ids, qat, stage)
    t = step + 1
    lg = learning_rate(step, lr_grid, total_steps)
    lm = learning_rate(step, lr_mlp, total_steps)
    last = len(st.layers) - 1
    if stage == 1:
        st.grid, st.m_grid, st.v_grid = adam(st.grid, dgrid, st.m_grid, st.v_grid, t, lg)
    rows = endpoint_rows(tg.lay.formats)
    for k, (dw, db) in enumerate(dlayers):
        if stage == 2 and k != last:
            continue
        (w, b), (mw, mb), (vw, vb) = st.layers[k], st.m_layers[k], st.v_layers[k]
        if stage == 1:
            w, mw, vw = adam(w, dw, mw, vw, t, lm)
            b, mb, vb = adam(b, db, mb, vb, t, lm)
        else:
            w, mw, vw = w.copy(), mw.copy(), vw.copy()
            b, mb, vb = b.copy(), mb.copy(), vb.copy()
            w[rows], mw[rows], vw[rows] = adam(w[rows], dw[rows], mw[rows], vw[rows], t, lm)
            b[rows], mb[rows], vb[rows] = adam(b[rows], db[rows], mb[rows], vb[rows], t, lm)
        st.layers[k], st.m_layers[k], st.v_layers[k] = (w, b), (mw, mb), (vw, vb)
    return loss
