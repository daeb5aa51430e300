"""Pins of the oracle parts that drive the parity verdicts: the tie classification (decision margins
and the rule that turns a head difference into an allowed word difference), the real-valued training
palette of Eq. palette / Eq. weightBC4, the training targets, and the four NTBC losses on hand-built
blocks (no GPU)."""
from fractions import Fraction

import numpy as np
import pytest

from conftest import read_golden
from oracle import bc, metrics, ntbc


# ------------------------------------------------------------------------------------ tie classification
def _bc4_row(e0, e1, colours):
    """Heads [1, 18] of one BC4 texture: endpoint values e0, e1 and 16 colours (all in [0,1])."""
    y = np.zeros((1, 18))
    y[0, 0], y[0, 1] = e0, e1
    y[0, 2:] = colours
    return y


# Reference heads: e0 * 255 = 100.2 (quantises to 100, 0.3 from its boundary 100.5), e1 * 255 = 30.7
# (31, 0.2 from 30.5).  Eight-value palette of (100, 31) in weight order, by the format definition
# round(((7-j) 100 + 31 j) / 7): 100, 90 (90.14), 80 (80.29), 70 (70.43), 61 (60.57), 51 (50.71),
# 41 (40.86), 31.  Texel i predicts palette entry i % 8 exactly, so its best squared distance is 0 and
# the second best is the squared spacing to the nearest neighbour: 81/255^2 at 70 and 61 (spacing 9),
# 100/255^2 elsewhere.
PAL_100_31 = np.array([100, 90, 80, 70, 61, 51, 41, 31]) / 255.0
Y_REF = _bc4_row(100.2 / 255, 30.7 / 255, PAL_100_31[np.arange(16) % 8])
EP_MARGIN = 0.2 / 255
IDX_MARGIN = 81.0 / 255 ** 2


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_margins_of_hand_built_block(precision):
    lay = ntbc.Layout([4])
    words, ep_m, idx_m = ntbc.pack_texture(Y_REF, lay, 0, precision, return_margin=True)
    e0, e1, codes = bc.bc4_fields(words)
    assert (int(e0[0]), int(e1[0])) == (100, 31)
    assert np.isclose(ep_m[0], EP_MARGIN, rtol=1e-6, atol=0)
    assert np.isclose(idx_m[0], IDX_MARGIN, rtol=1e-5, atol=0)
    # texel i takes palette entry i % 8 (stored codes 0, 2..7, 1 in weight order)
    assert codes[0].tolist() == [[0, 2, 3, 4, 5, 6, 7, 1][i % 8] for i in range(16)]


def test_margin_of_an_index_near_tie():
    # texel 0 predicts 65.6/255, between 70 and 61: squared distances 4.4^2 and 4.6^2 (/255^2), gap
    # (4.6^2 - 4.4^2)/255^2 = 1.8/255^2
    y = Y_REF.copy()
    y[0, 2] = 65.6 / 255
    _, _, idx_m = ntbc.pack_texture(y, ntbc.Layout([4]), 0, "f64", return_margin=True)
    assert np.isclose(idx_m[0], 1.8 / 255 ** 2, rtol=1e-6)


def _classify(y_impl, words_impl, y_ref, formats):
    words_ref = ntbc.pack(y_ref, formats)
    return metrics.classify_differences(y_impl, words_impl, y_ref, words_ref, formats)


def _flipped(words):
    """The same words with one index bit of texture 0 changed: a word that differs."""
    w = words.copy()
    w[0, 0] ^= np.uint64(1) << np.uint64(40)
    return w


def test_endpoint_flip_beyond_the_margin_is_a_tie():
    # e1 moved down by 0.25/255 crosses 30.5: e1 -> 30, so the word differs; d = 0.25/255 >= margin
    y = Y_REF.copy()
    y[0, 1] -= 0.25 / 255
    words = ntbc.pack(y, [4], "f32")
    res = _classify(y, words, Y_REF, [4])
    assert res["repack_exact"] and res["differ"] == 1 and res["ties"] == 1


def test_difference_within_every_margin_is_not_a_tie():
    # d = 0.15/255 = 5.9e-4: below the endpoint margin (7.8e-4) and 2*d + 2e-6 = 1.18e-3 below the
    # index gap 81/255^2 = 1.25e-3, so a word difference is not explained by the heads
    y = Y_REF.copy()
    y[0, 1] -= 0.15 / 255
    res = _classify(y, _flipped(ntbc.pack(Y_REF, [4])), Y_REF, [4])
    assert res["differ"] == 1 and res["ties"] == 0 and not res["repack_exact"]
    # planted mistake: an endpoint allowance of a third of a code would call it a tie
    words_ref = ntbc.pack(Y_REF, [4])
    res = metrics.classify_differences(y, _flipped(words_ref), Y_REF, words_ref, [4], endpoint_slack=1.0 / 3 / 255)
    assert res["ties"] == 1


def test_index_rule_counts_both_sides_of_the_gap():
    # d = 7e-4 on a colour: 2*1*d + 2e-6 = 1.40e-3 >= 1.25e-3 (tie); a rule with half the factor
    # (d + 2e-6 = 7.02e-4) would call it a non-tie.  The endpoint margin 7.8e-4 > d + 1.25e-7.
    y = Y_REF.copy()
    y[0, 5] += 7e-4
    res = _classify(y, _flipped(ntbc.pack(Y_REF, [4])), Y_REF, [4])
    assert res["ties"] == 1
    # a classifier with the factor halved (a planted mistake) gives the other verdict on this block
    words_ref = ntbc.pack(Y_REF, [4])
    res = metrics.classify_differences(y, _flipped(words_ref), Y_REF, words_ref, [4], index_factor=1.0)
    assert res["ties"] == 0
    # just outside: 2*d + 2e-6 < 1.2457e-3
    y = Y_REF.copy()
    y[0, 5] += 6.1e-4
    res = _classify(y, _flipped(ntbc.pack(Y_REF, [4])), Y_REF, [4])
    assert res["ties"] == 0


def _bc1_row(s):
    """Heads [1, 54] of one BC1 texture with endpoints pure red / pure blue (y = 1 or 0: half a code,
    0.5/31 or 0.5/63 for green, from any rounding boundary) and 16 texels at palette entries, except
    texel 0 at the bisector of entries 0 (255,0,0) and 1 (170,0,85) moved by (s, 0, -s) towards entry
    0: its squared distances are 2(1/6 - s)^2 and 2(1/6 + s)^2, a gap of (4/3) s."""
    y = np.zeros((1, 54))
    y[0, 0:6] = [1, 0, 0, 0, 0, 1]
    pal = np.array([[255, 0, 0], [170, 0, 85], [85, 0, 170], [0, 0, 255]]) / 255.0
    cols = pal[np.arange(16) % 4].copy()
    cols[0] = np.array([212.5, 0, 42.5]) / 255.0 + np.array([s, 0.0, -s])
    y[0, 6:] = cols.ravel()
    return y


def test_index_rule_scales_with_the_channel_count():
    # BC1 (three channels): gap (4/3) 1e-3 = 1.333e-3; d = 4e-4 gives 2*3*d + 2e-6 = 2.40e-3 (tie), a
    # rule without the channel count would give 8.0e-4 (non-tie)
    y_ref = _bc1_row(1e-3)
    _, ep_m, idx_m = ntbc.pack_texture(y_ref, ntbc.Layout([1]), 0, "f64", return_margin=True)
    assert np.isclose(idx_m[0], 4.0 / 3.0 * 1e-3, rtol=1e-6)
    assert np.isclose(ep_m[0], 0.5 / 63, rtol=1e-9)
    y = y_ref.copy()
    y[0, 6 + 3 * 5] += 4e-4
    res = _classify(y, _flipped(ntbc.pack(y_ref, [1])), y_ref, [1])
    assert res["ties"] == 1
    # planted mistake: the channel count left out of the rule (factor 2 instead of 2 * 3)
    words_ref = ntbc.pack(y_ref, [1])
    res = metrics.classify_differences(y, _flipped(words_ref), y_ref, words_ref, [1], index_factor=2.0 / 3.0)
    assert res["ties"] == 0
    y = y_ref.copy()
    y[0, 6 + 3 * 5] += 2.0e-4   # 2*3*d + 2e-6 = 1.202e-3 < 1.333e-3
    res = _classify(y, _flipped(ntbc.pack(y_ref, [1])), y_ref, [1])
    assert res["ties"] == 0


def test_head_difference_is_taken_per_texture():
    # two textures: BC1 first (heads 0..5 and colour channels 0..2 of every texel), then the BC4 block of
    # Y_REF.  The BC1 heads differ by 0.05 (its word is left equal); the BC4 word differs with only
    # 0.15/255 on its own heads: a non-tie, which a difference taken over the whole head row would hide.
    lay = ntbc.Layout([1, 4])
    y_ref = np.zeros((1, lay.H))
    y_ref[0, 0:6] = [1, 0, 0, 0, 0, 1]
    y_ref[0, 6:8] = Y_REF[0, 0:2]
    bc1_cols = lay.colour_index(0)
    bc4_cols = lay.colour_index(1)
    y_ref[0, bc1_cols.ravel()] = 0.5
    y_ref[0, bc4_cols.ravel()] = Y_REF[0, 2:]
    y = y_ref.copy()
    y[0, bc1_cols[3, 1]] += 0.05
    y[0, 7] -= 0.15 / 255
    words = ntbc.pack(y_ref, [1, 4])
    words[1, 0] ^= np.uint64(1) << np.uint64(40)
    res = metrics.classify_differences(y, words, y_ref, ntbc.pack(y_ref, [1, 4]), [1, 4])
    assert res["differ"] == 1 and res["ties"] == 0
    assert np.isclose(res["max_dy"], 0.05)
    d = metrics.texture_head_difference(np.abs(y - y_ref), lay, 1)
    assert np.isclose(d[0], 0.15 / 255)


# ------------------------------------------------------------------------------- Eq. palette (training)
# Weight order n of the stored codes, from the format definition: BC1 four-colour c0, (2c0+c1)/3,
# (c0+2c1)/3, c1 are codes 0, 2, 3, 1; BC4 eight values e0, then the six interpolants, then e1 are codes
# 0, 2..7, 1; BC4 six values start at the special 0 (code 6), then e0, the four interpolants, e1, and
# end at the special 1 (code 7).
BC1_CODE = [0, 2, 3, 1]
BC4_CODE8 = [0, 2, 3, 4, 5, 6, 7, 1]
BC4_CODE6 = [6, 0, 2, 3, 4, 5, 1, 7]


def test_palette_real_matches_hand_decoded_palettes():
    # the real-valued Eq. palette of the decoded endpoints, times 255, is within 1/2 of every decoded
    # (rounded) palette entry of the hand-decoded golden, and the six-value specials are exactly 0, 1
    rows = read_golden("bc_palettes.txt")
    bc1 = {}
    for r in rows:
        if r[0] == "bc1" and int(r[1], 16) > int(r[2], 16):     # four-colour blocks (training targets)
            bc1.setdefault((r[1], r[2]), {})[int(r[3])] = [int(v) for v in r[4:7]]
    assert len(bc1) == 2
    for dec in bc1.values():
        e0 = np.array([dec[0]], dtype=np.float64) / 255.0
        e1 = np.array([dec[1]], dtype=np.float64) / 255.0
        pal, a, b = ntbc.palette_real(e0, e1, ntbc.BC1)
        for n in range(4):
            assert np.abs(pal[0, n] * 255.0 - dec[BC1_CODE[n]]).max() <= 0.5, (dec, n)
            assert np.isclose(a[0, n], 1.0 - n / 3.0) and np.isclose(b[0, n], n / 3.0)
    n_bc4 = 0
    for r in rows:
        if r[0] != "bc4":
            continue
        e0i, e1i = int(r[1]), int(r[2])
        dec = [int(v) for v in r[3:11]]
        eight = e0i > e1i
        pal, a, b = ntbc.palette_real(np.array([[e0i / 255.0]]), np.array([[e1i / 255.0]]), ntbc.BC4,
                                      np.array([eight]))
        order = BC4_CODE8 if eight else BC4_CODE6
        for n in range(8):
            assert abs(pal[0, n, 0] * 255.0 - dec[order[n]]) <= 0.5, (r, n)
        if eight:
            assert np.allclose(b[0], np.arange(8) / 7.0)
        else:
            assert pal[0, 0, 0] == 0.0 and pal[0, 7, 0] == 1.0
            assert a[0, 0] == b[0, 0] == 0.0 and a[0, 7] == b[0, 7] == 0.0
            assert np.allclose(b[0, 1:7], np.arange(6) / 5.0)
        n_bc4 += 1
    assert n_bc4 == 4


def test_targets_of_hand_decoded_words():
    # The two hand-decoded words of the golden: reference endpoints decode to 8-bit / 255, texels / 255
    # land in the texture's channels, and the reference palettes follow the stored endpoints' mode.
    rows = {r[0]: r for r in read_golden("bc_words.txt")}
    w1 = np.array([int(rows["bc1"][1], 16)], dtype=np.uint64)
    w4 = np.array([int(rows["bc4"][1], 16)], dtype=np.uint64)
    tex1 = np.array([[int(x) for x in t.split(",")] for t in rows["bc1"][2:18]], dtype=np.uint8)[None]
    tex4 = np.array([int(x) for x in rows["bc4"][2:18]], dtype=np.uint8)[None, :, None]
    tg = ntbc.Targets([1, 4], [w1, w4], [tex1, tex4])
    # BC1 c0 = 0xA50A -> (165, 162, 82), c1 = 0x18FC -> (24, 28, 231); BC4 e0 = 200, e1 = 10
    assert np.allclose(tg.e_ref[0] * 255.0, [165, 162, 82, 24, 28, 231, 200, 10], rtol=0, atol=1e-12)
    assert np.allclose(tg.c[0, :, 0:3] * 255.0, tex1[0], rtol=0, atol=1e-12)
    assert np.allclose(tg.c[0, :, 3] * 255.0, tex4[0, :, 0], rtol=0, atol=1e-12)
    bc1_dec = {0: [165, 162, 82], 1: [24, 28, 231], 2: [118, 117, 132], 3: [71, 73, 181]}
    for n in range(4):
        assert np.abs(tg.pal_ref[0][0, n] * 255.0 - bc1_dec[BC1_CODE[n]]).max() <= 0.5
    bc4_dec = [200, 10, 173, 146, 119, 91, 64, 37]
    for n in range(8):
        assert abs(tg.pal_ref[1][0, n, 0] * 255.0 - bc4_dec[BC4_CODE8[n]]) <= 0.5


# ------------------------------------------------------------------------------------- the four losses
def _expand(field):
    """Golden list: comma-separated numbers or 'Nxa:b:c' (N copies of the tuple a, b, c)."""
    out = []
    for item in field.split(","):
        if "x" in item:
            k, tup = item.split("x", 1)
            out.extend([float(v) for v in tup.split(":")] * int(k))
        else:
            out.append(float(item))
    return out


def _value(s):
    return float(Fraction(s)) if "/" in s else float(s)


@pytest.mark.parametrize("case", ["A", "B", "C"])
def test_losses_of_hand_computed_blocks(case):
    row = {r[0]: r for r in read_golden("loss_hand.txt")}[case]
    fmt = int(row[1])
    ch = 3 if fmt == 1 else 1
    word = np.array([int(row[2], 16)], dtype=np.uint64)
    texels = np.array(_expand(row[3]), dtype=np.float64).reshape(1, 16, ch).astype(np.uint8)
    heads = np.array(_expand(row[4]), dtype=np.float64)[None]
    want = [_value(v) for v in row[5:9]]
    tg = ntbc.Targets([fmt], [word], [texels])
    assert heads.shape[1] == tg.lay.H
    losses, dy = ntbc.loss_and_grad(heads, tg, np.array([0]), 0.01)
    assert np.allclose(losses, want, rtol=1e-12, atol=1e-15), (losses, want)
    # the smooth terms' gradient alone: 2 (y - target) / (number of elements of the term)
    _, dy_s = ntbc.loss_and_grad(heads, tg, np.array([0]), 0.01, terms=(1.0, 1.0, 0.0, 0.0))
    E = tg.lay.E
    assert np.allclose(dy_s[0, :E], 2.0 * (heads[0, :E] - tg.e_ref[0]) / E, rtol=1e-12, atol=1e-15)
    assert np.allclose(dy_s[0, E:], 2.0 * (heads[0, E:] - tg.c[0].ravel()) / (16 * ch), rtol=1e-12, atol=1e-15)
