"""GPU parity of the reference encoder, decoder, per-block SSE and fallback against the oracle
(bit-exact)."""
import ctypes

import numpy as np
import pytest
import torch

from util import ensure_built, log, u64
from oracle import bc
from paper_2407_09543_amd import ntbc, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    assert torch.cuda.is_available()
    ntbc.lib()


def _encode_both(tex: np.ndarray, fmt: int):
    dev = torch.from_numpy(np.ascontiguousarray(tex)).cuda()
    words, sse = ntbc.encode_ref(dev, fmt, return_sse=True)
    torch.cuda.synchronize()
    blocks = bc.image_to_blocks(tex)
    enc = bc.bc1_encode_ref if fmt == 1 else bc.bc4_encode_ref
    ow, osse = enc(blocks if fmt == 1 else blocks[..., 0], return_sse=True)
    return u64(words), sse.cpu().numpy(), ow, osse


@pytest.mark.parametrize("size,seed", [(256, 1), (1024, 2)])
def test_encode_materials_bit_exact(size, seed):
    m = synth.material_small(size, seed) if size == 256 else synth.material_five(size, seed)
    for t in m.textures:
        log(f"encode {t.name} {size} fmt {t.fmt}")
        gw, gs, ow, osse = _encode_both(t.texels, t.fmt)
        assert np.array_equal(gw, ow), f"{t.name}: {(gw != ow).sum()} blocks differ"
        assert np.array_equal(gs, osse)


@pytest.mark.parametrize("fmt", [1, 4])
def test_encode_adversarial_blocks(fmt):
    rng = np.random.default_rng(11 + fmt)
    ch = 3 if fmt == 1 else 1
    blocks = synth.random_blocks(rng, 64 * 48, ch)
    tex = bc.blocks_to_image(blocks, 4 * 48, 4 * 64)
    tex = tex if fmt == 1 else tex[..., 0]
    gw, gs, ow, osse = _encode_both(tex, fmt)
    assert np.array_equal(gw, ow)
    assert np.array_equal(gs, osse)


def test_encode_single_colour_blocks():
    # one-colour blocks take REF-BC1's optimal single-colour step: every grey level, every value of
    # each channel alone, and random colours; mixed with non-uniform blocks in the same texture
    rng = np.random.default_rng(31)
    cols = [np.repeat(np.arange(256)[:, None], 3, axis=1)]
    for c in range(3):
        one = np.full((256, 3), 128)
        one[:, c] = np.arange(256)
        cols.append(one)
    cols.append(rng.integers(0, 256, (256, 3)))
    col = np.concatenate(cols)
    blocks = np.repeat(col[:, None, :], 16, axis=1).astype(np.uint8)
    blocks[1::7, 5] ^= 1  # some blocks one texel off uniform
    tex = bc.blocks_to_image(blocks, 4 * 40, 4 * 32)
    gw, gs, ow, osse = _encode_both(tex, 1)
    assert np.array_equal(gw, ow)
    assert np.array_equal(gs, osse)


@pytest.mark.parametrize("h,w", [(4, 4), (8, 12), (36, 20)])
def test_encode_ragged_sizes(h, w):
    rng = np.random.default_rng(h * 100 + w)
    for fmt in (1, 4):
        tex = rng.integers(0, 256, (h, w, 3) if fmt == 1 else (h, w)).astype(np.uint8)
        gw, gs, ow, osse = _encode_both(tex, fmt)
        assert np.array_equal(gw, ow)


def test_encode_row_pitch():
    rng = np.random.default_rng(3)
    tex = rng.integers(0, 256, (16, 40, 3)).astype(np.uint8)   # pitch 120 bytes, width 32 texels
    dev = torch.from_numpy(tex).cuda()
    out = torch.empty(4 * 8, dtype=torch.int64, device="cuda")
    st = ntbc.lib().ntbc_bc_encode_ref(ctypes.c_void_p(dev.data_ptr()), 32, 16, 120, 1,
                                       ctypes.c_void_p(out.data_ptr()), None, ntbc._stream())
    assert st == 0
    ow = bc.bc1_encode_ref(bc.image_to_blocks(np.ascontiguousarray(tex[:, :32])))
    assert np.array_equal(u64(out), ow)


def test_encode_paper_scale_sampled():
    m = synth.material_five(4096, 3)
    for t in m.textures[:3]:
        log(f"encode 4096 {t.name}")
        dev = torch.from_numpy(t.texels).cuda()
        words = u64(ntbc.encode_ref(dev, t.fmt))
        blocks = bc.image_to_blocks(t.texels)
        idx = np.random.default_rng(5).choice(len(blocks), 20000, replace=False)
        enc = bc.bc1_encode_ref if t.fmt == 1 else bc.bc4_encode_ref
        ow = enc(blocks[idx] if t.fmt == 1 else blocks[idx, :, 0])
        assert np.array_equal(words[idx], ow)


def _random_words(rng, n, fmt):
    if fmt == 1:
        c0 = rng.integers(0, 65536, n)
        c1 = rng.integers(0, 65536, n)
        c1[: n // 8] = c0[: n // 8]                      # equal endpoints
        return bc.bc1_pack(c0, c1, rng.integers(0, 4, (n, 16)))
    e0 = rng.integers(0, 256, n)
    e1 = rng.integers(0, 256, n)
    e1[: n // 8] = e0[: n // 8]
    return bc.bc4_pack(e0, e1, rng.integers(0, 8, (n, 16)))


@pytest.mark.parametrize("fmt", [1, 4])
def test_decode_all_modes_bit_exact(fmt):
    rng = np.random.default_rng(20 + fmt)
    bw, bh = 37, 23
    words = _random_words(rng, bw * bh, fmt)
    dev = torch.from_numpy(words.view(np.int64)).cuda()
    tex = ntbc.decode(dev, 4 * bw, 4 * bh, fmt).cpu().numpy()
    ref = bc.bc1_decode(words) if fmt == 1 else bc.bc4_decode(words)[..., None]
    want = bc.blocks_to_image(ref, 4 * bh, 4 * bw)
    assert np.array_equal(tex.reshape(want.shape), want)


@pytest.mark.parametrize("fmt", [1, 4])
def test_block_sse_and_fallback(fmt):
    rng = np.random.default_rng(30 + fmt)
    bw, bh = 32, 16
    ch = 3 if fmt == 1 else 1
    tex = rng.integers(0, 256, (4 * bh, 4 * bw, ch) if fmt == 1 else (4 * bh, 4 * bw)).astype(np.uint8)
    words = _random_words(rng, bw * bh, fmt)
    dev_tex = torch.from_numpy(tex).cuda()
    dev_w = torch.from_numpy(words.view(np.int64)).cuda()
    sse = ntbc.block_sse(dev_w, dev_tex, fmt).cpu().numpy()
    want = bc.block_sse(words, bc.image_to_blocks(tex), fmt)
    assert np.array_equal(sse, want)
    ref_w, ref_sse = ntbc.encode_ref(dev_tex, fmt, return_sse=True)
    sse_dev = torch.from_numpy(sse).cuda()
    out, count = ntbc.fallback(dev_w, ref_w, sse_dev, ref_sse, 1.5, 10.0)
    rs = ref_sse.cpu().numpy()
    repl = sse.astype(np.float32) > np.float32(1.5) * rs.astype(np.float32) + np.float32(10.0)
    assert np.array_equal(u64(out), np.where(repl, u64(ref_w), words))
    assert int(count.item()) == int(repl.sum())


@pytest.mark.parametrize("fmt", [1, 4])
def test_texels_to_blocks_bit_exact(fmt):
    # the block-major copy of the training targets equals the oracle's block split (rectangular texture)
    rng = np.random.default_rng(12 + fmt)
    shape = (40, 72, 3) if fmt == 1 else (40, 72)
    tex = rng.integers(0, 256, shape, dtype=np.uint8)
    got = ntbc.texels_to_blocks(torch.from_numpy(tex).cuda(), fmt).cpu().numpy()
    want = bc.image_to_blocks(tex)
    assert got.shape == (10 * 18, 16, 3 if fmt == 1 else 1)
    assert np.array_equal(got.reshape(want.shape), want)
