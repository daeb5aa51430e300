"""The paper's own NTBC network layout (oracle; test infrastructure only): separate endpoint and colour
networks with SELU hidden layers, half-precision MLPs, and the conservative / aggressive ways of
covering a material's RGB and single-channel textures (Sec. 3.2, Sec. 3.4, Sec. 4.1, Tab. inferPerf).

Model configuration (Sec. 3.4):
  * endpoint network: the normalised block index (s, t) -> a multi-resolution grid of 7 levels,
    coarsest 16, finest 1,024, 2 features per level (14 inputs) -> three hidden layers of 64 SELU
    units -> sigmoid outputs (the endpoints of every texture it covers);
  * colour network: the texture coordinate (u, v) of a texel -> a grid of 8 levels, 16 .. 2,048,
    2 features (16 inputs) -> three hidden layers of 64 SELU units -> sigmoid outputs (the predicted
    uncompressed colour of every texture it covers, at that texel);
  * half-precision weights and layer inputs; 8-bit grids (Sec. 3.3).
Material layouts (Sec. 4.1), with N_RGB BC1 and N_SC BC4 textures:
  * conservative: two models, one trained with BC1 (endpoint outputs 6 N_RGB, colour outputs
    3 N_RGB) and one with BC4 (2 N_SC and N_SC);
  * aggressive: one model for all textures (endpoint outputs 6 N_RGB + 2 N_SC, colour outputs
    3 N_RGB + N_SC), trained with eight distance nodes of which BC1 uses the first four (the other
    four are dummies with zero gradient).
A block decodes exactly as in oracle.ntbc: its endpoints come from one endpoint-network run and its
16 texels' colours from 16 colour-network runs, and the index of each texel is the palette entry
nearest to its predicted colour (Eq. dist).  So the heads of a block are assembled in oracle.ntbc's
head layout and packed by oracle.ntbc.pack.
Training (Sec. 3.2, Sec. 3.4) assembles the same heads for a batch of blocks, takes the NTBC losses
and their straight-through gradient on them (oracle.ntbc.loss_and_grad: the aggressive layout's
dummy distance nodes change neither value nor gradient), and back-propagates the endpoint part through
the endpoint network to its grid and the 16 colour parts of each block through the colour network to
its grid; Adam with the warm-up / cosine schedule updates both networks and both grids.

Readings where the paper is silent:
  * SELU with the published constants of Klambauer et al. (2017): lambda = 1.0507009873554805,
    alpha = 1.6732632423543772: selu(x) = lambda x (x > 0), lambda alpha (e^x - 1) (x <= 0).
  * The colour grid is addressed at texel centres with the block grid's convention (oracle.grid):
    texel (x, y) of a W x H texture is the "block" (x, y) of a W x H grid of cells.
  * Storage: the 8-bit grids, eight bytes of (scale, zero point) per grid level and the FP16 weights
    and biases of both MLPs, in MiB (2^20 bytes), which is how the paper's 13.37 / 26.74 come out.
  * Per-block cost: network executions (the inference table's measure) = 1 endpoint + 16 colour runs
    per model and block; "four network executions" of the conservative layout count each network of
    each model once.
  * Training: the colour network of a batch of n blocks sees the 16 n texels of those blocks; the
    losses are normalised per block batch as in oracle.ntbc (so a texel's colour error weighs as in
    the one-trunk model); SELU's derivative is lambda (z > 0) and lambda alpha e^z (z <= 0, the left
    branch at z = 0, as the forward's case split); grids in FP32 master form, fake-quantised per level
    when QAT is on (oracle.grid), as in oracle.ntbc.
"""
from __future__ import annotations

import numpy as np

from . import grid as G
from . import lowp
from . import metrics
from . import ntbc as N

SELU_LAMBDA = 1.0507009873554805
SELU_ALPHA = 1.6732632423543772

ENDPOINT_GRID = dict(n_levels=7, base_res=16, n_features=2)   # 16 .. 1,024
COLOUR_GRID = dict(n_levels=8, base_res=16, n_features=2)     # 16 .. 2,048
HIDDEN, N_HIDDEN = 64, 3


def selu(x):
    x = np.asarray(x, dtype=np.float64)
    return np.where(x > 0.0, SELU_LAMBDA * x, SELU_LAMBDA * SELU_ALPHA * np.expm1(np.minimum(x, 0.0)))


def grid_inputs(g) -> int:
    return g["n_levels"] * g["n_features"]


def grid_vertices(g) -> int:
    return sum(r * r for r in G.level_res(g["n_levels"], g["base_res"]))


def layer_dims(n_in: int, n_out: int):
    dims = [n_in] + [HIDDEN] * N_HIDDEN + [n_out]
    return [(dims[i], dims[i + 1]) for i in range(len(dims) - 1)]


def output_nodes(formats):
    """(endpoint outputs, colour outputs) of one model covering `formats` (BC1: 6 and 3, BC4: 2 and 1)."""
    e = sum(6 if f == N.BC1 else 2 for f in formats)
    c = sum(3 if f == N.BC1 else 1 for f in formats)
    return e, c


def models_of(formats, layout: str):
    """The texture groups of each model: aggressive -> one model over all textures, conservative ->
    the BC1 textures and the BC4 textures (each only if present), in head order."""
    if layout == "aggressive":
        return [list(range(len(formats)))]
    groups = [[i for i, f in enumerate(formats) if f == N.BC1], [i for i, f in enumerate(formats) if f == N.BC4]]
    return [g for g in groups if g]


def n_parameters(formats) -> int:
    """MLP weights and biases of one model (endpoint and colour networks)."""
    e, c = output_nodes(formats)
    return sum(i * o + o for i, o in layer_dims(grid_inputs(ENDPOINT_GRID), e)) + \
        sum(i * o + o for i, o in layer_dims(grid_inputs(COLOUR_GRID), c))


def model_bytes(formats) -> int:
    """Stored bytes of one model: uint8 grids and FP16 weights (oracle.metrics.model_bytes), plus the
    (scale, zero point) of every grid level (eight bytes each)."""
    e, c = output_nodes(formats)
    grids = [tuple(g[k] for k in ("n_levels", "base_res", "n_features")) for g in (ENDPOINT_GRID, COLOUR_GRID)]
    mlps = [[grid_inputs(ENDPOINT_GRID)] + [HIDDEN] * N_HIDDEN + [e],
            [grid_inputs(COLOUR_GRID)] + [HIDDEN] * N_HIDDEN + [c]]
    return metrics.model_bytes(grids, mlps) + 8 * (ENDPOINT_GRID["n_levels"] + COLOUR_GRID["n_levels"])


def material_bytes(formats, layout: str) -> int:
    return sum(model_bytes([formats[i] for i in grp]) for grp in models_of(formats, layout))


def executions_per_block(formats, layout: str) -> int:
    """Network runs per block: one endpoint run and 16 colour runs per model."""
    return 17 * len(models_of(formats, layout))


def mlp_forward(layers, x, precision: str = "fp16"):
    """SELU trunk, sigmoid outputs; "fp16" rounds every layer input and weight to IEEE half (the
    paper's network precision) with float64 accumulation, "f64" is exact."""
    h = np.asarray(x, dtype=np.float64)
    for k, (w, b) in enumerate(layers):
        w = np.asarray(w, dtype=np.float64)
        if precision == "fp16":
            z = lowp.round_fp16(h) @ lowp.round_fp16(w).T + np.asarray(b, dtype=np.float64)
        else:
            z = h @ w.T + np.asarray(b, dtype=np.float64)
        if k < len(layers) - 1:
            h = selu(z)
        else:
            with np.errstate(over="ignore"):
                h = 1.0 / (1.0 + np.exp(-z))
    return h


def block_heads(formats, ep_levels, ep_layers, col_levels, col_layers, bx, by, blocks_w: int, blocks_h: int,
                precision: str = "fp16"):
    """Heads [n, E + 16 C] in oracle.ntbc's layout for blocks (bx, by) of one model: the endpoint
    network at the block, the colour network at each of the block's 16 texel centres (texel i = 4y + x
    of the block is texel (4 bx + x, 4 by + y) of the texture)."""
    bx = np.asarray(bx, dtype=np.int64)
    by = np.asarray(by, dtype=np.int64)
    n = len(bx)
    e_dim, c_dim = output_nodes(formats)
    ye = mlp_forward(ep_layers, G.features(ep_levels, bx, by, blocks_w, blocks_h), precision)
    i = np.arange(16)
    tx = (4 * bx[:, None] + (i % 4)[None, :]).ravel()
    ty = (4 * by[:, None] + (i // 4)[None, :]).ravel()
    yc = mlp_forward(col_layers, G.features(col_levels, tx, ty, 4 * blocks_w, 4 * blocks_h), precision)
    return np.concatenate([ye, yc.reshape(n, 16 * c_dim)], axis=1)


def infer_blocks(formats, models, bx, by, blocks_w: int, blocks_h: int, layout: str, precision: str = "fp16"):
    """Packed words [T, n] of every texture: each model's heads packed by oracle.ntbc.pack, the words
    placed at their textures' positions.  models: per texture group of models_of(formats, layout),
    (endpoint levels, endpoint layers, colour levels, colour layers)."""
    groups = models_of(formats, layout)
    out = np.zeros((len(formats), len(np.asarray(bx))), dtype=np.uint64)
    for grp, (el, ew, cl, cw) in zip(groups, models):
        fm = [formats[i] for i in grp]
        y = block_heads(fm, el, ew, cl, cw, bx, by, blocks_w, blocks_h, precision)
        words = N.pack(y, fm, "f32" if precision != "f64" else "f64")
        for k, t in enumerate(grp):
            out[t] = words[k]
    return out


# ------------------------------------------------------------------------------------------------
# Training (Sec. 3.2, Sec. 3.4)
# ------------------------------------------------------------------------------------------------
def selu_grad(z):
    """d selu / dz: lambda for z > 0, lambda alpha e^z otherwise."""
    z = np.asarray(z, dtype=np.float64)
    return np.where(z > 0.0, SELU_LAMBDA, SELU_LAMBDA * SELU_ALPHA * np.exp(np.minimum(z, 0.0)))


def mlp_forward_cache(layers, x):
    """Exact (float64) forward with the layer inputs and pre-activations kept for the backward."""
    h = np.asarray(x, dtype=np.float64)
    hs, zs = [h], []
    for k, (w, b) in enumerate(layers):
        z = h @ np.asarray(w, dtype=np.float64).T + np.asarray(b, dtype=np.float64)
        zs.append(z)
        if k < len(layers) - 1:
            h = selu(z)
            hs.append(h)
    with np.errstate(over="ignore"):
        y = 1.0 / (1.0 + np.exp(-zs[-1]))
    return y, (hs, zs)


def mlp_backward(layers, cache, d_y, y):
    """(dW list, db list, dx) of a scalar loss from dL/dY by the chain rule: dZ_out = dL/dY Y (1 - Y),
    dW_k = dZ_k^T h_k, db_k = column sums of dZ_k, dh_k = dZ_k W_k, dZ_{k-1} = dh_k selu'(z_{k-1})."""
    hs, zs = cache
    dz = np.asarray(d_y, dtype=np.float64) * y * (1.0 - y)
    dws, dbs = [None] * len(layers), [None] * len(layers)
    dx = None
    for k in range(len(layers) - 1, -1, -1):
        dws[k] = dz.T @ hs[k]
        dbs[k] = dz.sum(axis=0)
        dh = dz @ np.asarray(layers[k][0], dtype=np.float64)
        if k > 0:
            dz = dh * selu_grad(zs[k - 1])
        else:
            dx = dh
    return dws, dbs, dx


def texel_coords(bx, by):
    """Texture coordinates (tx, ty) of the 16 texels of each block, block-major (texel i = 4y + x)."""
    bx = np.asarray(bx, dtype=np.int64)
    by = np.asarray(by, dtype=np.int64)
    i = np.arange(16)
    tx = (4 * bx[:, None] + (i % 4)[None, :]).ravel()
    ty = (4 * by[:, None] + (i // 4)[None, :]).ravel()
    return tx, ty


def _grid_values(grid, g, qat):
    if qat:
        return G.fake_quant_grid(grid, g["n_levels"], g["base_res"])
    return np.asarray(grid, dtype=np.float64), None


def gradients(formats, ep_grid, ep_layers, col_grid, col_layers, tg, ids, blocks_w: int, blocks_h: int,
              qat: bool = False, temp: float = 0.01, terms=(1.0, 1.0, 1.0, 1.0), ep_cfg=None, col_cfg=None):
    """Losses and gradients of one model of the layout at the given parameters for the block batch ids:
    (losses, d_ep_grid, [(dW, db)] of the endpoint network, d_col_grid, [(dW, db)] of the colour
    network, heads).  Grids [vertices][2] (FP32 master values), tg: oracle.ntbc.Targets of `formats`."""
    ep_cfg = ep_cfg or ENDPOINT_GRID
    col_cfg = col_cfg or COLOUR_GRID
    ids = np.asarray(ids, dtype=np.int64)
    n = len(ids)
    e_dim, c_dim = output_nodes(formats)
    bx, by = ids % blocks_w, ids // blocks_w
    ge, me = _grid_values(ep_grid, ep_cfg, qat)
    gc, mc = _grid_values(col_grid, col_cfg, qat)
    xe = G.features(G.split_levels(ge, ep_cfg["n_levels"], ep_cfg["base_res"]), bx, by, blocks_w, blocks_h)
    ye, ce = mlp_forward_cache(ep_layers, xe)
    tx, ty = texel_coords(bx, by)
    xc = G.features(G.split_levels(gc, col_cfg["n_levels"], col_cfg["base_res"]), tx, ty, 4 * blocks_w, 4 * blocks_h)
    yc, cc = mlp_forward_cache(col_layers, xc)
    y = np.concatenate([ye, yc.reshape(n, 16 * c_dim)], axis=1)
    losses, dy = N.loss_and_grad(y, tg, ids, temp, terms)
    dwe, dbe, dxe = mlp_backward(ep_layers, ce, dy[:, :e_dim], ye)
    dwc, dbc, dxc = mlp_backward(col_layers, cc, dy[:, e_dim:].reshape(16 * n, c_dim), yc)
    dge = G.features_backward(dxe, bx, by, blocks_w, blocks_h, ep_cfg["n_levels"], ep_cfg["base_res"],
                              ep_cfg["n_features"], me)
    dgc = G.features_backward(dxc, tx, ty, 4 * blocks_w, 4 * blocks_h, col_cfg["n_levels"], col_cfg["base_res"],
                              col_cfg["n_features"], mc)
    return losses, dge, list(zip(dwe, dbe)), dgc, list(zip(dwc, dbc)), y


class TrainState:
    """Parameters and Adam moments of one model of the layout (float64)."""

    def __init__(self, ep_grid, ep_layers, col_grid, col_layers):
        cp = lambda layers: [(np.asarray(w, np.float64).copy(), np.asarray(b, np.float64).copy()) for w, b in layers]
        self.params = [np.asarray(ep_grid, np.float64).copy(), cp(ep_layers),
                       np.asarray(col_grid, np.float64).copy(), cp(col_layers)]
        zeros = lambda p: np.zeros_like(p) if isinstance(p, np.ndarray) else [(np.zeros_like(w), np.zeros_like(b))
                                                                             for w, b in p]
        self.m = [zeros(p) for p in self.params]
        self.v = [zeros(p) for p in self.params]


def train_step(formats, st: TrainState, tg, ids, blocks_w: int, blocks_h: int, step: int, total_steps: int,
               qat: bool = False, lr_grid: float = 0.01, lr_mlp: float = 0.005, temp: float = 0.01,
               ep_cfg=None, col_cfg=None):
    """One iteration: gradients of both networks and grids, then Adam (grids at lr_grid, networks at
    lr_mlp, both on oracle.ntbc's warm-up / cosine schedule); returns the losses."""
    out = gradients(formats, st.params[0], st.params[1], st.params[2], st.params[3], tg, ids, blocks_w, blocks_h,
                    qat, temp, ep_cfg=ep_cfg, col_cfg=col_cfg)
    grads = out[1:5]
    t = step + 1
    lg = N.learning_rate(step, lr_grid, total_steps)
    lm = N.learning_rate(step, lr_mlp, total_steps)
    for k in range(4):
        if k % 2 == 0:
            st.params[k], st.m[k], st.v[k] = N.adam(st.params[k], grads[k], st.m[k], st.v[k], t, lg)
            continue
        for j, ((w, b), (dw, db)) in enumerate(zip(st.params[k], grads[k])):
            (mw, mb), (vw, vb) = st.m[k][j], st.v[k][j]
            w, mw, vw = N.adam(w, dw, mw, vw, t, lm)
            b, mb, vb = N.adam(b, db, mb, vb, t, lm)
            st.params[k][j] = (w, b)
            st.m[k][j] = (mw, mb)
            st.v[k][j] = (vw, vb)
    return out[0]
