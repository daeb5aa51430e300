"""Seeded model/material cases shared by the GPU tests (inputs only; expected values come from the
oracle)."""
import numpy as np

from oracle import grid as G
from oracle import ntbc as ON
from paper_2407_09543_amd import synth


def model_inputs(cfg, seed, u8=None, grid_scale=0.7):
    """(flat fp32 weights, grid arrays) with O(1) features so outputs spread over (0, 1)."""
    layers = synth.init_weights(cfg, seed)
    rng = np.random.default_rng(seed + 101)
    layers = [(w, (0.3 * rng.standard_normal(len(b))).astype(np.float32)) for w, b in layers]
    flat = synth.flatten_weights(layers)
    use_u8 = cfg.grid_u8 if u8 is None else u8
    if use_u8:
        codes, scale, zero = synth.random_u8_grid(cfg, seed)
        # rescale so features are O(1): s * (q - z) with q - z ~ +-128
        scale = (np.full(cfg.n_levels, grid_scale / 128.0) * (1 + 0.1 * np.arange(cfg.n_levels))).astype(np.float32)
        zero = np.full(cfg.n_levels, 128, dtype=np.int32) - np.arange(cfg.n_levels, dtype=np.int32)
        return flat, layers, dict(codes=codes, scale=scale, zero=zero)
    grid = synth.random_grid(cfg, seed, grid_scale)
    return flat, layers, dict(grid=grid)


def oracle_levels(cfg, g):
    if "codes" in g:
        return ON.grid_levels(cfg, codes=g["codes"], scales=g["scale"], zeros=g["zero"])
    return ON.grid_levels(cfg, grid=g["grid"])


def exact_model_inputs(cfg, seed):
    """Parameters on which float32 accumulation is exact (so the BF16 and FP32 paths can only differ
    from the oracle in the final sigmoid): grid values k/8 on a float grid; every weight row has four
    nonzero entries +-1 (hidden layers) or +-2^-6 (head); biases k/8.  The block grid must be a power
    of two so the bilinear fractions are dyadic.  Returns (flat, layers, grid dict)."""
    rng = np.random.default_rng(seed + 555)
    layers = []
    dims = cfg.layer_dims()
    for k, (fan_in, fan_out) in enumerate(dims):
        w = np.zeros((fan_out, fan_in), dtype=np.float32)
        mag = 1.0 if k < len(dims) - 1 else 2.0 ** -6
        for r in range(fan_out):
            cols = rng.choice(fan_in, min(4, fan_in), replace=False)
            w[r, cols] = mag * rng.choice([-1.0, 1.0], len(cols))
        b = (rng.integers(-8, 9, fan_out) / 8.0).astype(np.float32)
        layers.append((w, b))
    grid = (rng.integers(-8, 9, (cfg.grid_vertices, cfg.n_features)) / 8.0).astype(np.float32)
    return synth.flatten_weights(layers), layers, dict(grid=grid)


def assert_exact_in_float32(cfg, layers, g, ids):
    """Host check of the construction: the float64 forward equals a float32 forward at every layer."""
    from oracle import grid as OG, lowp
    lv = oracle_levels(cfg, g)
    ids = np.asarray(ids)
    x = OG.features(lv, ids % cfg.blocks_w, ids // cfg.blocks_w, cfg.blocks_w, cfg.blocks_h)
    assert np.array_equal(x, x.astype(np.float32).astype(np.float64))
    h = x
    for k, (w, b) in enumerate(layers):
        hb = lowp.round_bf16(h)
        z = hb @ w.astype(np.float64).T + b
        assert np.abs(z).max() < 2.0 ** 12
        assert np.array_equal(z, z.astype(np.float32).astype(np.float64))
        h = np.maximum(z, 0.0)


class TrainProblem:
    """A material, its reference blocks on both sides (each side encodes its own), and parameters."""

    def __init__(self, cfg, material, seed, grid_scale=0.5):
        import torch
        from oracle import bc as OB
        from paper_2407_09543_amd import ntbc
        self.cfg = cfg
        self.mat = material
        self.desc = ntbc.desc_from_config(cfg)
        blocks = [OB.image_to_blocks(t.texels) for t in material.textures]
        ref_or = [OB.bc1_encode_ref(b) if t.fmt == 1 else OB.bc4_encode_ref(b[..., 0])
                  for b, t in zip(blocks, material.textures)]
        self.tg_oracle = ON.Targets(cfg.formats, ref_or, blocks)
        tex = [torch.from_numpy(t.texels).cuda() for t in material.textures]
        ref_gpu = torch.stack([ntbc.encode_ref(t, f) for t, f in zip(tex, cfg.formats)])
        self.tg_gpu = ntbc.Targets(ref_gpu, tex)
        layers = synth.init_weights(cfg, seed)
        rng = np.random.default_rng(seed + 7)
        self.layers = [(w, (0.1 * rng.standard_normal(len(b))).astype(np.float32)) for w, b in layers]
        self.flat = synth.flatten_weights(self.layers)
        self.grid = synth.random_grid(cfg, seed, grid_scale)
        self.grid_d = torch.from_numpy(self.grid).cuda()
        self.flat_d = torch.from_numpy(self.flat).cuda()

    def ids(self, seed, n):
        import torch
        ids = synth.batch_ids(seed, 0, n, self.cfg.n_positions)
        return ids, torch.from_numpy(ids).cuda()


def near_tie_positions(pb, y, ids, gap=1e-6):
    """Positions where some texel's two smallest decoded-colour distances (either branch) differ by
    less than `gap` but are not equal (equal distances to equal palette entries are harmless): there
    the float32 and float64 argmax may differ."""
    lay, tg = pb.tg_oracle.lay, pb.tg_oracle
    n = len(ids)
    bad = np.zeros(n, dtype=bool)
    c_hat = y[:, lay.E:].reshape(n, 16, lay.C)
    for t, f in enumerate(lay.formats):
        e, ch = lay.ep_off[t], lay.channels(t)
        sl = slice(lay.ch_off[t], lay.ch_off[t] + ch)
        c = tg.c[ids][:, :, sl]
        pr = tg.pal_ref[t][ids]
        e0, e1 = y[:, e:e + ch], y[:, e + ch:e + 2 * ch]
        ph, _, _ = ON.palette_real(e0, e1, f, e0[:, 0] > e1[:, 0])
        for dist in (np.sqrt(((c[:, :, None, :] - ph[:, None]) ** 2).sum(-1)),
                     np.sqrt(((c_hat[:, :, None, sl] - pr[:, None]) ** 2).sum(-1))):
            s = np.sort(dist, axis=2)
            g = s[:, :, 1] - s[:, :, 0]
            bad |= ((g > 0) & (g < gap)).any(axis=1)
        if f == 4:
            bad |= np.abs(e0[:, 0] - e1[:, 0]) < gap          # BC4 mode switch of the prediction
    return bad
