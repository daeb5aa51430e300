"""GPU parity of the paper's own network layout (ntbc_faithful_infer: endpoint network + per-texel colour
network, SELU, half-precision operands) against its oracle (oracle.faithful).

Heads against the oracle's half-precision emulation (every layer input and weight rounded to IEEE half,
float64 accumulation): float32 accumulation noise now and then moves an activation across a half
rounding boundary (one half ulp, 2^-11 relative), as for the one-trunk FP16 path: max 2e-3, p99 4e-4,
median 1e-6.  Packing bit-exact on the kernel's own heads.  Both material layouts, uint8 and FP32 grids,
ragged block ranges, single blocks at either end of the grid, the largest heads."""
import numpy as np
import pytest
import torch

from util import ensure_built, log, u64
from oracle import faithful as F
from oracle import grid as G
from oracle import ntbc as ON
from oracle.ntbc import BC1, BC4
from paper_2407_09543_amd import ntbc

pytestmark = pytest.mark.gpu

SIX = [BC1, BC1, BC4, BC4, BC4, BC4]


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    assert torch.cuda.is_available()


def _net(rng, n_in, n_out):
    layers = []
    for i, o in F.layer_dims(n_in, n_out):
        w = (rng.standard_normal((o, i)) * np.sqrt(2.0 / i)).astype(np.float32)
        b = (0.2 * rng.standard_normal(o)).astype(np.float32)
        layers.append((w, b))
    return layers


def _flat(layers):
    return np.concatenate([np.concatenate([w.ravel(), b]) for w, b in layers]).astype(np.float32)


def _grid(rng, levels, u8):
    nv = sum((16 << l) ** 2 for l in range(levels))
    if not u8:
        g = rng.uniform(-1.0, 1.0, (nv, 2)).astype(np.float32)
        return g, None, None, G.split_levels(g.astype(np.float64), levels, 16)
    codes = rng.integers(0, 256, (nv, 2), dtype=np.uint8)
    scale = rng.uniform(0.004, 0.01, levels).astype(np.float32)
    zero = rng.integers(100, 156, levels).astype(np.int32)
    lv = G.split_levels(G.dequant_grid(codes, scale, zero, levels, 16), levels, 16)
    return codes, scale, zero, lv


def _model(rng, formats, bw, bh, u8):
    e, c = F.output_nodes(formats)
    ew, cw = _net(rng, 14, e), _net(rng, 16, c)
    ec, es, ez, el = _grid(rng, 7, u8)
    cc, cs, cz, cl = _grid(rng, 8, u8)
    t = lambda a: None if a is None else torch.from_numpy(a).cuda()
    m = ntbc.FaithfulModel(formats, bw, bh, t(ec), t(cc), t(_flat(ew)), t(_flat(cw)),
                           ep_scale=t(es), ep_zero=t(ez), col_scale=t(cs), col_zero=t(cz))
    assert m.n_ep_weights == sum(i * o + o for i, o in F.layer_dims(14, e))
    assert m.n_col_weights == sum(i * o + o for i, o in F.layer_dims(16, c))
    return m, (el, ew, cl, cw)


@pytest.mark.parametrize("layout", ["aggressive", "conservative"])
@pytest.mark.parametrize("u8", [True, False])
def test_paper_layout_matches_oracle(layout, u8):
    rng = np.random.default_rng(5 + int(u8))
    bw = bh = 64                                            # a 256^2 material
    first, n = 37, bw * bh - 37 - 21                        # ragged at both ends
    ids = np.arange(first, first + n)
    bx, by = ids % bw, ids // bw
    dys = []
    for grp in F.models_of(SIX, layout):
        fm = [SIX[i] for i in grp]
        m, (el, ew, cl, cw) = _model(rng, fm, bw, bh, u8)
        words, heads = m.infer(first, n, heads=True)
        words, heads = u64(words), heads.cpu().numpy()
        # packing: the oracle's float32 packer on the kernel's own heads
        assert np.array_equal(words, ON.pack(heads, fm, "f32"))
        y_or = F.block_heads(fm, el, ew, cl, cw, bx, by, bw, bh, "fp16")
        dy = np.abs(heads - y_or)
        dys.append(dy.ravel())
        log(f"paper layout {layout} u8={u8} {len(fm)} textures: max|dY| {dy.max():.3g} p99 "
            f"{np.percentile(dy, 99):.3g} median {np.median(dy):.3g}")
    dy = np.concatenate(dys)
    assert dy.max() <= 2e-3 and np.percentile(dy, 99) <= 4e-4 and np.median(dy) <= 1e-6


def test_paper_layout_rejects_bad_shapes():
    rng = np.random.default_rng(9)
    with pytest.raises(ntbc.NtbcError):          # 9 levels: 18 inputs exceed one K-step
        ntbc.FaithfulModel(SIX, 64, 64, torch.zeros((10, 2), dtype=torch.uint8, device="cuda"),
                           torch.zeros((10, 2), dtype=torch.uint8, device="cuda"),
                           torch.zeros(10, device="cuda"), torch.zeros(10, device="cuda"), ep_levels=9)
    m, _ = _model(rng, [BC1], 64, 64, False)
    with pytest.raises(ntbc.NtbcError):          # beyond the block grid
        m.infer(4000, 200)


@pytest.mark.parametrize("formats,first,n", [([BC4], 4095, 1), ([BC1], 0, 1), ([BC1] * 8, 100, 65), ([BC4] * 8, 0, 4096)])
def test_paper_layout_edge_ranges(formats, first, n):
    # one block at either end of the grid, the largest endpoint head (eight BC1 textures: 48 outputs, two
    # head tiles; 24 colour outputs) and eight single-channel textures, against the oracle
    rng = np.random.default_rng(len(formats) + first)
    bw = bh = 64
    m, (el, ew, cl, cw) = _model(rng, formats, bw, bh, True)
    words, heads = m.infer(first, n, heads=True)
    words, heads = u64(words), heads.cpu().numpy()
    assert np.array_equal(words, ON.pack(heads, formats, "f32"))
    ids = np.arange(first, first + n)
    y_or = F.block_heads(formats, el, ew, cl, cw, ids % bw, ids // bw, bw, bh, "fp16")
    dy = np.abs(heads - y_or)
    log(f"paper layout {len(formats)} textures, blocks [{first}, {first + n}): max|dY| {dy.max():.3g}")
    assert dy.max() <= 2e-3 and np.median(dy) <= 1e-6
