"""Pins of the BC1/BC4 oracle against the format definition, hand-decoded blocks, brute force and
round-trip invariants (no GPU)."""
import numpy as np
import pytest

from conftest import read_golden
from oracle import bc
from paper_2407_09543_amd import synth


def test_palettes_match_hand_decoded():
    for row in read_golden("bc_palettes.txt"):
        if row[0] == "bc1":
            c0, c1, code = int(row[1], 16), int(row[2], 16), int(row[3])
            pal = bc.bc1_palette(np.array([c0]), np.array([c1]))[0]
            assert pal[code].tolist() == [int(v) for v in row[4:7]], row
        else:
            e0, e1 = int(row[1]), int(row[2])
            pal = bc.bc4_palette(np.array([e0]), np.array([e1]))[0]
            assert pal.tolist() == [int(v) for v in row[3:11]], row


def test_words_decode_to_hand_values():
    for row in read_golden("bc_words.txt"):
        w = np.array([int(row[1], 16)], dtype=np.uint64)
        if row[0] == "bc1":
            expect = [[int(x) for x in t.split(",")] for t in row[2:18]]
            assert bc.bc1_decode(w)[0].tolist() == expect
        else:
            assert bc.bc4_decode(w)[0].tolist() == [int(x) for x in row[2:18]]


def test_six_value_mode_contains_zero_and_one():
    # Eq. weightBC4: the first and last weights reach c = 0 and c = 1 (paper, Sec. 3)
    rng = np.random.default_rng(0)
    e0 = rng.integers(0, 256, 500)
    e1 = np.maximum(e0, rng.integers(0, 256, 500))
    pal = bc.bc4_palette(e0, e1)
    assert (pal[:, 6] == 0).all() and (pal[:, 7] == 255).all()


def test_endpoint_expansion_exhaustive():
    # every 16-bit c0 with all codes 0 decodes to its endpoint in every texel (c1 = 0 keeps c0 > c1
    # except c0 = 0, which is three-colour mode whose code 0 is still c0)
    c0 = np.arange(65536, dtype=np.uint64)
    words = c0  # c1 = 0, codes 0
    tex = bc.bc1_decode(words)
    assert (tex == tex[:, :1, :]).all()
    r, g, b = c0 >> np.uint64(11), (c0 >> np.uint64(5)) & np.uint64(63), c0 & np.uint64(31)
    # bit replication stays within one unit of the exact rescale v*255/(2^b-1), hits 0 and 255
    for chan, v, mx in ((0, r, 31), (1, g, 63), (2, b, 31)):
        got = tex[:, 0, chan].astype(np.float64)
        exact = v.astype(np.float64) * 255.0 / mx
        assert np.abs(got - exact).max() < 1.0
    assert tex[0, 0].tolist() == [0, 0, 0] and tex[65535, 0].tolist() == [255, 255, 255]


def test_expansion_differs_from_rounding_only_at_known_codes():
    v = np.arange(32)
    diff5 = np.nonzero(bc.expand5(v) != np.floor(v * 255 / 31 + 0.5))[0].tolist()
    assert diff5 == [3, 7, 24, 28]
    # requantising an expanded code gives the code back (5 and 6 bits)
    assert (bc.quant565(np.stack([bc.expand5(v), bc.expand6(v), bc.expand5(v)], -1))[:, 0] == v).all()
    v6 = np.arange(64)
    assert ((bc.expand6(v6) * 63 + 127) // 255 == v6).all()


def test_pack_unpack_roundtrip():
    rng = np.random.default_rng(1)
    c0, c1 = rng.integers(0, 65536, 1000), rng.integers(0, 65536, 1000)
    codes = rng.integers(0, 4, (1000, 16))
    w = bc.bc1_pack(c0, c1, codes)
    a, b, c = bc.bc1_fields(w)
    assert (a == c0).all() and (b == c1).all() and (c == codes).all()
    e0, e1 = rng.integers(0, 256, 1000), rng.integers(0, 256, 1000)
    codes = rng.integers(0, 8, (1000, 16))
    w = bc.bc4_pack(e0, e1, codes)
    a, b, c = bc.bc4_fields(w)
    assert (a == e0).all() and (b == e1).all() and (c == codes).all()


def _random_valid_bc1(rng, n):
    """Four-colour blocks using codes 0 and 1, endpoints >= 2 codes apart in every differing channel."""
    out = []
    while len(out) < n:
        q0 = rng.integers(0, [32, 64, 32])
        q1 = rng.integers(0, [32, 64, 32])
        d = np.abs(q0 - q1)
        if ((d == 1)).any() or (d == 0).all():
            continue
        c0, c1 = int(bc.pack565(*q0)), int(bc.pack565(*q1))
        if c0 <= c1:
            c0, c1 = c1, c0
        if c0 == c1:
            continue
        codes = rng.integers(0, 4, 16)
        codes[rng.choice(16, 2, replace=False)] = [0, 1]
        out.append(int(bc.bc1_pack(c0, c1, codes)))
    return np.array(out, dtype=np.uint64)


def test_bc1_roundtrip_invariant():
    rng = np.random.default_rng(2)
    w = _random_valid_bc1(rng, 400)
    tex = bc.bc1_decode(w)
    w2, sse = bc.bc1_encode_ref(tex, return_sse=True)
    assert (sse == 0).all()
    assert (bc.bc1_decode(w2) == tex).all()


def test_bc4_roundtrip_invariant():
    rng = np.random.default_rng(3)
    n = 400
    e0 = rng.integers(1, 255, n)
    e1 = rng.integers(1, 255, n)
    codes = rng.integers(0, 8, (n, 16))
    codes[:, 0], codes[:, 1] = 0, 1
    w = bc.bc4_pack(e0, e1, codes)
    keep = e0 != e1
    tex = bc.bc4_decode(w[keep])
    w2, sse = bc.bc4_encode_ref(tex, return_sse=True)
    assert (sse == 0).all()
    assert (bc.bc4_decode(w2) == tex).all()


def _exhaustive_codes_bc1(words, texels):
    """Per texel: the code of least squared error over the block's decoded palette, ties to the
    smallest logical n (order 0,2,3,1) -- by trying every code in the word itself."""
    c0, c1, _ = bc.bc1_fields(words)
    best = np.zeros(texels.shape[:2], dtype=np.int64)
    best_err = np.full(texels.shape[:2], 1 << 60)
    for code in (0, 2, 3, 1):
        trial = bc.bc1_pack(c0, c1, np.full(texels.shape[:2], code))
        col = bc.bc1_decode(trial).astype(np.int64)
        err = ((col - texels.astype(np.int64)) ** 2).sum(-1)
        better = err < best_err
        best = np.where(better, code, best)
        best_err = np.where(better, err, best_err)
    return np.where((c0 == c1)[:, None], 0, best)


def test_bc1_codes_are_bruteforce_argmin():
    rng = np.random.default_rng(4)
    blocks = synth.random_blocks(rng, 600, 3)
    w = bc.bc1_encode_ref(blocks)
    _, _, codes = bc.bc1_fields(w)
    assert (codes == _exhaustive_codes_bc1(w, blocks)).all()


def test_bc4_codes_are_bruteforce_argmin():
    rng = np.random.default_rng(5)
    blocks = synth.random_blocks(rng, 600, 1)[..., 0]
    w = bc.bc4_encode_ref(blocks)
    e0, e1, codes = bc.bc4_fields(w)
    order = bc.bc4_logical_order(e0, e1)
    best = np.zeros((600, 16), dtype=np.int64)
    best_err = np.full((600, 16), 1 << 60)
    for k in range(8):
        code = order[:, k][:, None]
        trial = bc.bc4_pack(e0, e1, np.broadcast_to(code, (600, 16)))
        err = (bc.bc4_decode(trial).astype(np.int64) - blocks) ** 2
        better = err < best_err
        best = np.where(better, code, best)
        best_err = np.where(better, err, best_err)
    assert (codes == best).all()


def _bc4_optimum(v):
    """Least SSE over all 65,536 endpoint pairs with per-texel optimal codes."""
    e0, e1 = np.meshgrid(np.arange(256), np.arange(256), indexing="ij")
    pal = bc.bc4_palette(e0.ravel(), e1.ravel())                    # [65536, 8]
    err = (pal[:, None, :] - v[None, :, None].astype(np.int64)) ** 2
    return err.min(axis=2).sum(axis=1).min()


def test_bc4_against_exhaustive_search():
    rng = np.random.default_rng(6)
    blocks = synth.random_blocks(rng, 60, 1)[..., 0]
    _, sse = bc.bc4_encode_ref(blocks, return_sse=True)
    gaps = []
    for b in range(len(blocks)):
        opt = _bc4_optimum(blocks[b])
        assert sse[b] >= opt
        gaps.append(sse[b] - opt)
    # representable blocks (decoded from some BC4 word) must reach the optimum 0
    e0 = rng.integers(1, 255, 30)
    e1 = rng.integers(1, 255, 30)
    codes = rng.integers(0, 8, (30, 16))
    codes[:, 0], codes[:, 1] = 0, 1
    tex = bc.bc4_decode(bc.bc4_pack(e0, e1, codes))
    _, sse2 = bc.bc4_encode_ref(tex, return_sse=True)
    assert (sse2[e0 != e1] == 0).all()
    assert np.median(gaps) <= 16


def _bc1_lattice_optimum(tex):
    """Least SSE over the coarse endpoint lattice (every 4th 5-bit and 8th 6-bit code), c0 > c1."""
    r = np.arange(0, 32, 4)
    g = np.arange(0, 64, 8)
    R, G, B = np.meshgrid(r, g, r, indexing="ij")
    codes = bc.pack565(R.ravel(), G.ravel(), B.ravel())
    c0, c1 = np.meshgrid(codes, codes, indexing="ij")
    sel = c0 > c1
    c0, c1 = c0[sel], c1[sel]
    pal = bc.bc1_palette(c0, c1)                                    # [P, 4, 3]
    best = None
    for k in range(0, len(c0), 16384):
        p = pal[k:k + 16384]
        err = ((p[:, None, :, :] - tex[None, :, None, :].astype(np.int64)) ** 2).sum(-1)
        val = err.min(axis=2).sum(axis=1).min()
        best = val if best is None else min(best, val)
    return best


def test_bc1_against_coarse_lattice():
    rng = np.random.default_rng(7)
    # lattice-generated blocks: palette colours of a lattice endpoint pair -> optimum 0
    r = rng.integers(0, 8, (20, 2)) * 4
    g = rng.integers(0, 8, (20, 2)) * 8
    b = rng.integers(0, 8, (20, 2)) * 4
    c0 = bc.pack565(r[:, 0], g[:, 0], b[:, 0])
    c1 = bc.pack565(r[:, 1], g[:, 1], b[:, 1])
    keep = c0 != c1
    hi, lo = np.maximum(c0, c1)[keep], np.minimum(c0, c1)[keep]
    codes = rng.integers(0, 4, (len(hi), 16))
    codes[:, 0], codes[:, 1] = 0, 1
    tex = bc.bc1_decode(bc.bc1_pack(hi, lo, codes))
    for t in tex[:6]:
        assert _bc1_lattice_optimum(t) == 0
    _, sse = bc.bc1_encode_ref(tex, return_sse=True)
    assert (sse == 0).all()
    # tiny blocks of 2-3 distinct colours: the reference is never worse than the coarse lattice
    worse = 0
    for _ in range(12):
        pal = rng.integers(0, 256, (rng.integers(2, 4), 3))
        t = pal[rng.integers(0, len(pal), 16)].astype(np.uint8)
        _, s = bc.bc1_encode_ref(t[None], return_sse=True)
        worse += int(s[0] > _bc1_lattice_optimum(t))
    assert worse == 0


def _reachable(bits):
    """Every value a BC1 palette entry can take in one channel of `bits` bits: the endpoints E(a), and
    the four-colour points (2 E(a) + E(b) + 1) // 3 and (E(a) + 2 E(b) + 1) // 3 of every pair."""
    e = [(a << 3) | (a >> 2) if bits == 5 else (a << 2) | (a >> 4) for a in range(1 << bits)]
    vals = set(e)
    for x in e:
        for y in e:
            vals.add((2 * x + y + 1) // 3)
            vals.add((x + 2 * y + 1) // 3)
    return sorted(vals)


def test_single_colour_table_is_optimal():
    # step 8 of REF-BC1: the table's 2/3 point is as near to every value as any value a four-colour
    # palette entry can take (enumerated as a set, independently of the table's argmin and tie rule)
    for bits in (5, 6):
        reach = np.array(_reachable(bits))
        t = bc.single_colour_table(bits)
        e = bc.expand5(np.arange(1 << bits)) if bits == 5 else bc.expand6(np.arange(1 << bits))
        pt = (2 * e[t[:, 0]] + e[t[:, 1]] + 1) // 3
        best = np.abs(reach[None, :] - np.arange(256)[:, None]).min(axis=1)
        assert np.array_equal(np.abs(pt - np.arange(256)), best)
        # every value is within one of a reachable one (136 values reachable with 5 bits, 246 with 6)
        assert best.max() == 1
    assert len(_reachable(5)) == 136 and len(_reachable(6)) == 246


def test_single_colour_blocks():
    # a one-colour block: its SSE is 16 times the sum over channels of the least squared error any
    # palette entry can reach (a lower bound for every BC1 block that REF-BC1 must meet)
    rng = np.random.default_rng(8)
    col = np.concatenate([rng.integers(0, 256, (300, 3)), np.repeat(np.arange(256)[:, None], 3, axis=1)])
    tex = np.repeat(col[:, None, :], 16, axis=1).astype(np.uint8)
    w, sse = bc.bc1_encode_ref(tex, return_sse=True)
    r5, r6 = np.array(_reachable(5)), np.array(_reachable(6))
    err = [np.abs(r[None, :] - col[:, c][:, None]).min(axis=1) for c, r in ((0, r5), (1, r6), (2, r5))]
    assert np.array_equal(sse, 16 * sum(e_ * e_ for e_ in err))
    assert np.array_equal(bc.block_sse(w, tex, 1), sse)
    # blocks of two colours are not one-colour blocks: step 8 leaves them alone (their words come from
    # steps 1-7 only, which put a grey step 0/1 on the two endpoints exactly)
    two = np.zeros((1, 16, 3), np.uint8)
    two[0, 8:] = 8
    w2, s2 = bc.bc1_encode_ref(two, return_sse=True)
    assert s2[0] == 0
    v = rng.integers(0, 256, 100)
    w4, sse4 = bc.bc4_encode_ref(np.repeat(v[:, None], 16, axis=1).astype(np.uint8), return_sse=True)
    assert (sse4 == 0).all() and (bc.bc4_decode(w4) == v[:, None]).all()


def test_reference_encoder_quality_on_material():
    m = synth.material_small(128, 5)
    blocks = [bc.image_to_blocks(t.texels) for t in m.textures]
    w1, s1 = bc.bc1_encode_ref(blocks[0], return_sse=True)
    w4, s4 = bc.bc4_encode_ref(blocks[1], return_sse=True)
    assert (bc.block_sse(w1, blocks[0], 1) == s1).all()
    assert (bc.block_sse(w4, blocks[1], 4) == s4).all()
    # the encoder is never worse than either of its own starting candidates' bounding-box endpoints
    assert 10 * np.log10(255 ** 2 / (s1.sum() / (len(s1) * 48))) > 33
    assert 10 * np.log10(255 ** 2 / (s4.sum() / (len(s4) * 16))) > 45
