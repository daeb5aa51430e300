"""Seeded synthetic inputs shared by the GPU path's tests, the benchmark and the oracle's tests.

This module holds no arithmetic of the compression method itself. It produces:

* procedural materials (value-noise textures, uint8) standing in for the 4096^2 scanned materials of
  the paper's dataset (Sec. 4.2), which are not available here;
* model descriptions (grid levels, feature counts, MLP widths) for the named workloads;
* initial parameters: He-normal MLP weights (Sec. 3.4), zero biases, grids uniform in +-1e-4 (Sec. 3.4);
* training batches of block ids, drawn from SplitMix64 (Steele, Lea & Flood, "Fast splittable
  pseudorandom number generators", OOPSLA 2014).

Everything is a pure function of its seed.  The procedural textures use only +, -, *, /, sqrt and floor (all correctly rounded) on
IEEE doubles, so they are bit-reproducible on any host.
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence, Tuple

import numpy as np

BC1 = 1
BC4 = 4

_M64 = (1 << 64) - 1


# --------------------------------------------------------------------------------------------------
# SplitMix64
# --------------------------------------------------------------------------------------------------
def splitmix64(x):
    """One SplitMix64 output for state value(s) ``x`` (the state already advanced by the golden gamma).

    Works on Python ints and on numpy uint64 arrays (wrap-around multiply)."""
    if isinstance(x, (int, np.integer)):
        z = int(x) & _M64
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        return z ^ (z >> 31)
    z = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


_GAMMA = 0x9E3779B97F4A7C15


def splitmix64_stream(seed: int, n: int) -> np.ndarray:
    """The first ``n`` outputs of a SplitMix64 generator whose state starts at ``seed``."""
    idx = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        states = np.uint64(seed & _M64) + idx * np.uint64(_GAMMA)
    return splitmix64(states)


def _key(*parts: int) -> int:
    """Mixes a tuple of small integers into one 64-bit key (a chain of SplitMix64 finalisations)."""
    h = 0
    for p in parts:
        h = splitmix64((h ^ (int(p) & _M64)) + _GAMMA)
    return h


def batch_ids(seed: int, step: int, batch: int, n_positions: int) -> np.ndarray:
    """Training batch ``step``: ``batch`` block-position ids drawn uniformly with replacement.

    id = (top 32 bits of a SplitMix64 output) * n_positions >> 32."""
    z = splitmix64_stream(_key(seed, 0xBA7C4, step), batch)
    hi = (z >> np.uint64(32)).astype(np.uint64)
    return ((hi * np.uint64(n_positions)) >> np.uint64(32)).astype(np.int32)


# --------------------------------------------------------------------------------------------------
# Value noise
# --------------------------------------------------------------------------------------------------
def _lattice(seed: int, octave: int, channel: int, freq: int) -> np.ndarray:
    """(freq+1)^2 lattice values in [0,1): top 53 bits of SplitMix64 / 2^53, periodic in ``freq``."""
    base = _key(seed, octave, channel)
    j, i = np.meshgrid(np.arange(freq + 1), np.arange(freq + 1), indexing="ij")
    cell = ((j % freq).astype(np.uint64) << np.uint64(32)) | (i % freq).astype(np.uint64)
    with np.errstate(over="ignore"):
        z = splitmix64(splitmix64(np.uint64(base) ^ cell) + np.uint64(_GAMMA))
    return (z >> np.uint64(11)).astype(np.float64) / float(1 << 53)


def _axis_weights(n: int, freq: int):
    u = (np.arange(n, dtype=np.float64) + 0.5) * (freq / n)
    i = np.floor(u).astype(np.int64)
    t = u - i
    s = t * t * (3.0 - 2.0 * t)
    return i, s


def value_noise(n: int, seed: int, channel: int, base_freq: int, octaves: int) -> np.ndarray:
    """Fractal value noise on an n x n image: octave o has frequency base_freq*2^o and amplitude 0.5^o;
    smoothstep-weighted bilinear blend of lattice values; normalised by the sum of amplitudes."""
    out = np.zeros((n, n), dtype=np.float64)
    total = 0.0
    for o in range(octaves):
        freq = base_freq << o
        amp = 0.5 ** o
        lat = _lattice(seed, o, channel, freq)
        ix, sx = _axis_weights(n, freq)
        iy, sy = _axis_weights(n, freq)
        rows0 = lat[iy]        # [n, freq+1]
        rows1 = lat[iy + 1]
        a = rows0[:, ix] * (1.0 - sx)[None, :] + rows0[:, ix + 1] * sx[None, :]
        b = rows1[:, ix] * (1.0 - sx)[None, :] + rows1[:, ix + 1] * sx[None, :]
        out += amp * (a * (1.0 - sy)[:, None] + b * sy[:, None])
        total += amp
    return out / total


def _to_u8(v: np.ndarray) -> np.ndarray:
    return np.floor(np.clip(v, 0.0, 1.0) * 255.0 + 0.5).astype(np.uint8)


# --------------------------------------------------------------------------------------------------
# Materials
# --------------------------------------------------------------------------------------------------
@dataclasses.dataclass
class Texture:
    name: str
    fmt: int                 # BC1 (RGB) or BC4 (single channel)
    texels: np.ndarray       # uint8 [H][W][3] for BC1, [H][W] for BC4

    @property
    def channels(self) -> int:
        return 3 if self.fmt == BC1 else 1


@dataclasses.dataclass
class Material:
    size: int
    textures: List[Texture]

    @property
    def formats(self) -> List[int]:
        return [t.fmt for t in self.textures]


def material_small(size: int = 256, seed: int = 1) -> Material:
    """Two textures: RGB diffuse (3-octave value noise per channel, f=8) as BC1 and single-channel
    roughness (2-octave, f=8) as BC4."""
    diffuse = np.stack([value_noise(size, seed, c, 8, 3) for c in range(3)], axis=-1)
    rough = value_noise(size, seed, 7, 8, 2)
    return Material(size, [Texture("diffuse", BC1, _to_u8(diffuse)),
                           Texture("roughness", BC4, _to_u8(rough))])


def _box5(h: np.ndarray, stride: int) -> np.ndarray:
    """Mean of the 5x5 taps at offsets {-2..2}*stride (periodic)."""
    acc = np.zeros_like(h)
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            acc += np.roll(np.roll(h, dy * stride, axis=0), dx * stride, axis=1)
    return acc / 25.0


def material_five(size: int, seed: int) -> Material:
    """Five correlated textures from one height field h (8-octave value noise, f=8):
    diffuse and normal as BC1; roughness, ambient occlusion and displacement as BC4."""
    h = value_noise(size, seed, 0, 8, 8)
    rng = np.random.default_rng(seed)
    col_a = rng.uniform(0.1, 0.5, size=3)
    col_b = rng.uniform(0.5, 0.9, size=3)
    diffuse = col_a[None, None, :] * (1.0 - h[..., None]) + col_b[None, None, :] * h[..., None]
    for c in range(3):
        diffuse[..., c] += 0.1 * (value_noise(size, seed, 10 + c, 32, 4) - 0.5)
    # normal map from central differences of h (periodic), slopes measured per 1/256 of the texture
    gx = (np.roll(h, -1, axis=1) - np.roll(h, 1, axis=1)) * (0.5 * size / 256.0)
    gy = (np.roll(h, -1, axis=0) - np.roll(h, 1, axis=0)) * (0.5 * size / 256.0)
    nx, ny, nz = -8.0 * gx, -8.0 * gy, np.ones_like(h)
    inv = 1.0 / np.sqrt(nx * nx + ny * ny + nz * nz)
    normal = np.stack([nx * inv, ny * inv, nz * inv], axis=-1) * 0.5 + 0.5
    rough = 0.3 + 0.5 * value_noise(size, seed, 20, 8, 4)
    ao = np.clip(1.0 - 30.0 * np.maximum(0.0, _box5(h, max(1, size // 256)) - h), 0.0, 1.0)
    disp = np.clip(1.4 * h - 0.2, 0.0, 1.0)
    return Material(size, [Texture("diffuse", BC1, _to_u8(diffuse)),
                           Texture("normal", BC1, _to_u8(normal)),
                           Texture("roughness", BC4, _to_u8(rough)),
                           Texture("ao", BC4, _to_u8(ao)),
                           Texture("displacement", BC4, _to_u8(disp))])


def texture_blocks(tex: Texture) -> np.ndarray:
    """Texels regrouped per 4x4 block: [H/4 * W/4, 16, C] (block id = by*(W/4)+bx, texel i = 4y+x)."""
    t = tex.texels if tex.texels.ndim == 3 else tex.texels[..., None]
    h, w, c = t.shape
    b = t.reshape(h // 4, 4, w // 4, 4, c).transpose(0, 2, 1, 3, 4).reshape(-1, 16, c)
    return b


def random_blocks(rng: np.random.Generator, n: int, channels: int, kind: str = "mixed") -> np.ndarray:
    """Adversarial tiny-block inputs for encoder tests: uniform, few-colour, flat, extremes."""
    if kind == "uniform":
        return rng.integers(0, 256, size=(n, 16, channels)).astype(np.uint8)
    out = np.empty((n, 16, channels), dtype=np.uint8)
    for b in range(n):
        mode = rng.integers(0, 5)
        if mode == 0:
            out[b] = rng.integers(0, 256, size=(16, channels))
        elif mode == 1:
            pal = rng.integers(0, 256, size=(rng.integers(1, 4), channels))
            out[b] = pal[rng.integers(0, len(pal), size=16)]
        elif mode == 2:
            out[b] = rng.integers(0, 256, size=(1, channels))
        elif mode == 3:
            base = rng.integers(0, 256, size=(1, channels)).astype(np.int64)
            out[b] = np.clip(base + rng.integers(-6, 7, size=(16, channels)), 0, 255)
        else:
            out[b] = rng.choice(np.array([0, 1, 2, 253, 254, 255]), size=(16, channels))
    return out


# --------------------------------------------------------------------------------------------------
# Model descriptions and initial parameters
# --------------------------------------------------------------------------------------------------
@dataclasses.dataclass
class ModelConfig:
    n_levels: int
    base_res: int
    n_features: int
    grid_u8: bool            # True: uint8 grids with per-level (scale, zero point)
    hidden: int
    n_hidden: int            # number of hidden layers
    formats: Tuple[int, ...]
    blocks_w: int
    blocks_h: int
    variant: str = "ntbc"    # "ntbc" (colour head) or "naive" (weight head, Sec. 3.1)

    @property
    def in_dim(self) -> int:
        return self.n_levels * self.n_features

    @property
    def endpoint_dim(self) -> int:
        return sum(6 if f == BC1 else 2 for f in self.formats)

    @property
    def colour_channels(self) -> int:
        return sum(3 if f == BC1 else 1 for f in self.formats)

    @property
    def head_dim(self) -> int:
        if self.variant == "naive":
            return self.endpoint_dim + 16 * len(self.formats)
        return self.endpoint_dim + 16 * self.colour_channels

    @property
    def level_res(self) -> List[int]:
        return [self.base_res << l for l in range(self.n_levels)]

    @property
    def grid_vertices(self) -> int:
        return sum(r * r for r in self.level_res)

    @property
    def n_positions(self) -> int:
        return self.blocks_w * self.blocks_h

    def layer_dims(self) -> List[Tuple[int, int]]:
        """(fan_in, fan_out) of each linear layer, input to output."""
        dims = [self.in_dim] + [self.hidden] * self.n_hidden + [self.head_dim]
        return [(dims[i], dims[i + 1]) for i in range(len(dims) - 1)]

    @property
    def n_weights(self) -> int:
        return sum(i * o + o for i, o in self.layer_dims())


def config_small(size: int = 256) -> ModelConfig:
    """Two textures (BC1 + BC4); 4 levels 8..64 x 4 FP32 features; MLP 16->64->64->heads."""
    return ModelConfig(4, 8, 4, False, 64, 2, (BC1, BC4), size // 4, size // 4)


def config_mid(size: int = 1024) -> ModelConfig:
    """Five textures; 6 levels 8..256 x 8 uint8 features; MLP 48->128->128->128->heads."""
    return ModelConfig(6, 8, 8, True, 128, 3, (BC1, BC1, BC4, BC4, BC4), size // 4, size // 4)


def config_paper_scale(size: int = 4096) -> ModelConfig:
    """Five textures; 8 levels 8..1024 x 8 uint8 features; MLP 64->256x3->heads."""
    return ModelConfig(8, 8, 8, True, 256, 3, (BC1, BC1, BC4, BC4, BC4), size // 4, size // 4)


def init_weights(cfg: ModelConfig, seed: int) -> List[Tuple[np.ndarray, np.ndarray]]:
    """He-normal weights (std sqrt(2/fan_in)) as float32 [out][in]; zero biases."""
    rng = np.random.default_rng(_key(seed, 0x3E1))
    layers = []
    for fan_in, fan_out in cfg.layer_dims():
        w = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=(fan_out, fan_in)).astype(np.float32)
        layers.append((w, np.zeros(fan_out, dtype=np.float32)))
    return layers


def flatten_weights(layers: Sequence[Tuple[np.ndarray, np.ndarray]]) -> np.ndarray:
    """Canonical flat layout: W1 (row-major [out][in]), b1, W2, b2, ..., W_out, b_out."""
    parts = []
    for w, b in layers:
        parts.append(np.asarray(w, dtype=np.float32).reshape(-1))
        parts.append(np.asarray(b, dtype=np.float32).reshape(-1))
    return np.concatenate(parts)


def unflatten_weights(cfg: ModelConfig, flat: np.ndarray):
    layers, off = [], 0
    for fan_in, fan_out in cfg.layer_dims():
        w = flat[off:off + fan_in * fan_out].reshape(fan_out, fan_in)
        off += fan_in * fan_out
        b = flat[off:off + fan_out]
        off += fan_out
        layers.append((w, b))
    return layers


def init_grid(cfg: ModelConfig, seed: int) -> np.ndarray:
    """float32 [sum_l res_l^2][F], uniform in [-1e-4, 1e-4]; level-major, row-major (y, x) per level."""
    rng = np.random.default_rng(_key(seed, 0x621D))
    return rng.uniform(-1e-4, 1e-4, size=(cfg.grid_vertices, cfg.n_features)).astype(np.float32)


def random_grid(cfg: ModelConfig, seed: int, scale: float = 1.0) -> np.ndarray:
    """A grid with O(1) values (used to exercise inference with non-trivial features)."""
    rng = np.random.default_rng(_key(seed, 0x9A1D))
    return (scale * rng.standard_normal(size=(cfg.grid_vertices, cfg.n_features))).astype(np.float32)


def random_u8_grid(cfg: ModelConfig, seed: int):
    """uint8 codes with per-level scale (float32) and zero point (int32), for inference tests."""
    rng = np.random.default_rng(_key(seed, 0x8008))
    codes = rng.integers(0, 256, size=(cfg.grid_vertices, cfg.n_features)).astype(np.uint8)
    scale = rng.uniform(0.002, 0.02, size=cfg.n_levels).astype(np.float32)
    zero = rng.integers(0, 256, size=cfg.n_levels).astype(np.int32)
    return codes, scale, zero
