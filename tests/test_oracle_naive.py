"""Pins of the naive-approach oracle (Sec. 3.1): hand-decoded packed blocks in both BC4 modes and the
BC1 swap, a brute-force nearest-entry check through the format's decoder, hand-computed stage-1 and
stage-2 losses, finite differences of the stage-1 gradient, and the frozen parameters of stage 2
(no GPU)."""
from types import SimpleNamespace

import numpy as np

from oracle import bc, naive, ntbc
from oracle.ntbc import BC1, BC4


def _heads(formats, n, rng):
    lay = naive.NaiveLayout(formats)
    return rng.uniform(0.0, 1.0, (n, lay.H)), lay


def _set_bc4(Y, lay, t, e0, e1, w):
    Y[:, lay.ep_off[t]] = e0 / 255.0
    Y[:, lay.ep_off[t] + 1] = e1 / 255.0
    Y[:, lay.weight_index(t)] = w


def test_bc4_hand_blocks_both_modes():
    lay = naive.NaiveLayout([BC4])
    Y = np.zeros((2, lay.H))
    _set_bc4(Y[0:1], lay, 0, 200, 100, 0.3)      # eight values: nearest n/7 to 0.3 is 2/7
    _set_bc4(Y[1:2], lay, 0, 100, 200, 0.33)     # six values: nearest (n-1)/5 to 0.33 is 0.4 (n = 3)
    words = naive.pack(Y, [BC4])[0]
    dec = bc.bc4_decode(words)
    # eight-value palette entry 2/7 of the way: code 3, (5*200 + 2*100 + 3) // 7 = 171
    assert (bc.bc4_fields(words[:1])[2] == 3).all() and (dec[0] == 171).all()
    # six-value entry 2/5 of the way: code 3, (3*100 + 2*200 + 2) // 5 = 140
    assert (bc.bc4_fields(words[1:])[2] == 3).all() and (dec[1] == 140).all()


def test_bc1_swapped_endpoints_turn_the_weight_round():
    lay = naive.NaiveLayout([BC1])
    Y = np.zeros((1, lay.H))
    Y[0, 0:3] = 0.0                                   # predicted e0 black
    Y[0, 3:6] = 1.0                                   # predicted e1 white -> c0 < c1, swapped
    Y[0, lay.weight_index(0)] = 0.2                   # 80% black
    w = naive.pack(Y, [BC1])[0]
    c0, c1, codes = bc.bc1_fields(w)
    assert c0[0] == 0xFFFF and c1[0] == 0
    # stored c0 is white: the entry 1/3 white + 2/3 black is code 3 = (c0 + 2 c1) / 3
    assert (codes == 3).all()
    assert (bc.bc1_decode(w)[0] == 85).all()
    # not swapped: white to black predicted, w = 0.2 -> entry (2 c0 + c1) / 3 = code 2, value 170
    Y[0, 0:3], Y[0, 3:6] = 1.0, 0.0
    assert (bc.bc1_decode(naive.pack(Y, [BC1])[0])[0] == 170).all()


def test_bc1_equal_endpoints_give_code_zero():
    lay = naive.NaiveLayout([BC1])
    Y = np.random.default_rng(3).uniform(0, 1, (4, lay.H))
    Y[:, 3:6] = Y[:, 0:3]
    _, _, codes = bc.bc1_fields(naive.pack(Y, [BC1])[0])
    assert (codes == 0).all()


def _ideal_bc1(c0, c1):
    """Real-valued entries by stored code of four-colour BC1 blocks (the palette before rounding)."""
    a, b = bc.endpoint_rgb8(c0).astype(np.float64), bc.endpoint_rgb8(c1).astype(np.float64)
    return np.stack([a, b, (2 * a + b) / 3, (a + 2 * b) / 3], axis=1)         # [n, code, 3]


def _ideal_bc4(e0, e1):
    """Real-valued entries by stored code and whether the code is an interpolated one."""
    a, b = e0.astype(np.float64), e1.astype(np.float64)
    eight = a > b
    vals = np.zeros((len(a), 8))
    ok = np.ones((len(a), 8), dtype=bool)
    vals[:, 0], vals[:, 1] = a, b
    for j in range(1, 7):
        v8 = ((7 - j) * a + j * b) / 7
        v6 = ((5 - j) * a + j * b) / 5 if j <= 4 else np.zeros_like(a)
        vals[:, j + 1] = np.where(eight, v8, v6)
        if j > 4:
            ok[:, j + 1] = eight
    return vals, ok


def test_brute_force_nearest_entry_on_the_segment():
    """Each texel's stored code is the one whose (unrounded) palette entry lies nearest to the continuous
    colour (1 - w) e0 + w e1 of the predicted quantised endpoints, found by trying every code."""
    rng = np.random.default_rng(11)
    formats = [BC1, BC4, BC1, BC4]
    Y, lay = _heads(formats, 3000, rng)
    words = naive.pack(Y, formats)
    checked = 0
    for t, f in enumerate(formats):
        e = lay.ep_off[t]
        w = Y[:, lay.weight_index(t)]
        if f == BC1:
            q = [ntbc.quant_endpoint(Y[:, e + k], b) for k, b in enumerate((5, 6, 5, 5, 6, 5))]
            p0 = bc.endpoint_rgb8(bc.pack565(q[0], q[1], q[2])).astype(np.float64)
            p1 = bc.endpoint_rgb8(bc.pack565(q[3], q[4], q[5])).astype(np.float64)
            c0, c1, codes = bc.bc1_fields(words[t])
            ideal = _ideal_bc1(c0, c1)
            x = (1 - w)[:, :, None] * p0[:, None, :] + w[:, :, None] * p1[:, None, :]
            d = ((x[:, :, None, :] - ideal[:, None, :, :]) ** 2).sum(-1)         # [n,16,4]
            valid = (c0 != c1)[:, None].repeat(16, 1)
        else:
            e0, e1, codes = bc.bc4_fields(words[t])
            assert (e0 == ntbc.quant_endpoint(Y[:, e], 8)).all()
            vals, ok = _ideal_bc4(e0, e1)
            x = (1 - w) * e0[:, None] + w * e1[:, None]
            d = (x[:, :, None] - vals[:, None, :]) ** 2
            d = np.where(ok[:, None, :], d, np.inf)
            valid = (e0 != e1)[:, None].repeat(16, 1)
        srt = np.sort(d, axis=2)
        clear = valid & (srt[:, :, 1] - srt[:, :, 0] > 1e-6 * (1 + srt[:, :, 1]))
        got = np.take_along_axis(d, codes[:, :, None], axis=2)[:, :, 0]
        assert np.array_equal(got[clear], srt[:, :, 0][clear]), t
        checked += clear.sum()
    assert checked > 0.9 * 4 * 3000 * 16


def _targets(formats, c):
    return SimpleNamespace(lay=ntbc.Layout(formats), c=c)


def test_hand_losses_one_bc4_block():
    """e0^ = 0.8, e1^ = 0.2, w = 0.25 on all 16 texels, texels 0.5.
    stage 1: x = 0.65, L = 0.15^2 = 0.0225; dL/de0^ = 2 * 0.15 * 0.75 = 0.225, dL/de1^ = 0.075,
    dL/dw = 2 * 0.15 * (0.2 - 0.8) / 16 = -0.01125 per texel.
    stage 2: eight-value mode, w_n = 2/7: x = (5 * 0.8 + 2 * 0.2) / 7 = 4.4/7, r = 0.9/7,
    L = 0.81/49; dL/de0^ = 2 r 5/7, dL/de1^ = 2 r 2/7, no weight gradient."""
    lay = naive.NaiveLayout([BC4])
    Y = np.zeros((1, lay.H))
    Y[0, 0], Y[0, 1] = 0.8, 0.2
    Y[0, lay.weight_index(0)] = 0.25
    tg = _targets([BC4], np.full((1, 16, 1), 0.5))
    L1, g1 = naive.loss_and_grad(Y, tg, [0], 1)
    assert abs(L1 - 0.0225) < 1e-15
    assert abs(g1[0, 0] - 0.225) < 1e-15 and abs(g1[0, 1] - 0.075) < 1e-15
    assert np.allclose(g1[0, lay.weight_index(0)], -0.01125, rtol=0, atol=1e-16)
    L2, g2 = naive.loss_and_grad(Y, tg, [0], 2)
    r = 0.9 / 7
    assert abs(L2 - 0.81 / 49) < 1e-15
    assert abs(g2[0, 0] - 2 * r * 5 / 7) < 1e-15 and abs(g2[0, 1] - 2 * r * 2 / 7) < 1e-15
    assert (g2[0, lay.weight_index(0)] == 0).all()


def test_stage1_gradient_against_finite_differences():
    rng = np.random.default_rng(5)
    formats = [BC1, BC4]
    Y, lay = _heads(formats, 3, rng)
    tg = _targets(formats, rng.uniform(0, 1, (3, 16, 4)))
    _, g = naive.loss_and_grad(Y, tg, np.arange(3), 1)
    h = 1e-6
    for j in range(lay.H):
        Yp, Ym = Y.copy(), Y.copy()
        Yp[1, j] += h
        Ym[1, j] -= h
        fd = (naive.loss_and_grad(Yp, tg, np.arange(3), 1)[0] - naive.loss_and_grad(Ym, tg, np.arange(3), 1)[0]) / (2 * h)
        assert abs(fd - g[1, j]) < 1e-8, j


def test_stage2_gradient_against_finite_differences_on_endpoints():
    """Stage 2 is piecewise: away from weight boundaries and the BC4 mode switch, the endpoints'
    finite differences match, and the weights get no gradient."""
    rng = np.random.default_rng(6)
    formats = [BC1, BC4]
    Y, lay = _heads(formats, 4, rng)
    Y[:, 7] = Y[:, 6] + 0.3 * np.sign(rng.standard_normal(4))    # BC4 endpoints well apart
    Y = np.clip(Y, 0.01, 0.99)
    tg = _targets(formats, rng.uniform(0, 1, (4, 16, 4)))
    _, g = naive.loss_and_grad(Y, tg, np.arange(4), 2)
    h = 1e-7
    for j in range(lay.E):
        Yp, Ym = Y.copy(), Y.copy()
        Yp[2, j] += h
        Ym[2, j] -= h
        fd = (naive.loss_and_grad(Yp, tg, np.arange(4), 2)[0] - naive.loss_and_grad(Ym, tg, np.arange(4), 2)[0]) / (2 * h)
        assert abs(fd - g[2, j]) < 1e-8, j
    assert (g[:, lay.E:] == 0).all()


def test_planted_mistake_without_the_swap_flip_fails_the_brute_force():
    """A packer that forgets to turn the weight round on swapped BC1 blocks stores the mirrored entry."""
    rng = np.random.default_rng(12)
    lay = naive.NaiveLayout([BC1])
    Y = rng.uniform(0, 1, (200, lay.H))
    Y[:, 0:3] *= 0.3
    Y[:, 3:6] = 0.7 + 0.3 * Y[:, 3:6]                 # every block swapped
    good = naive.pack(Y, [BC1])[0]
    Yw = Y.copy()
    Yw[:, lay.weight_index(0)] = 1 - Y[:, lay.weight_index(0)]
    wrong = naive.pack(Yw, [BC1])[0]                  # what the unflipped decision would store
    assert (bc.bc1_fields(good)[2] != bc.bc1_fields(wrong)[2]).mean() > 0.5


def test_stage2_freezes_all_but_the_endpoint_head():
    from paper_2407_09543_amd import synth
    cfg = synth.config_small(32)
    rng = np.random.default_rng(7)
    nh = naive.NaiveLayout(cfg.formats).H
    dims = cfg.layer_dims()[:-1] + [(cfg.hidden, nh)]           # naive heads: E + 16 T outputs
    layers = [(rng.standard_normal((o, i)) * 0.2, rng.standard_normal(o) * 0.1) for i, o in dims]
    nv = sum((cfg.base_res << l) ** 2 for l in range(cfg.n_levels))
    grid = rng.uniform(-0.5, 0.5, (nv, cfg.n_features))
    st = ntbc.TrainState(grid, layers)
    c = rng.uniform(0, 1, (cfg.n_positions, 16, ntbc.Layout(cfg.formats).C))
    tg = _targets(cfg.formats, c)
    ids = rng.choice(cfg.n_positions, 32, replace=False)
    naive.train_step(cfg, st, tg, ids, 0, 10, False, 1)
    g1 = st.grid.copy()
    l1 = [(w.copy(), b.copy()) for w, b in st.layers]
    naive.train_step(cfg, st, tg, ids, 1, 10, False, 2)
    assert np.array_equal(st.grid, g1)
    E = naive.NaiveLayout(cfg.formats).E
    for k, ((w, b), (w0, b0)) in enumerate(zip(st.layers, l1)):
        if k < len(l1) - 1:
            assert np.array_equal(w, w0) and np.array_equal(b, b0)
        else:
            assert np.array_equal(w[E:], w0[E:]) and np.array_equal(b[E:], b0[E:])
            assert not np.array_equal(w[:E], w0[:E]) and not np.array_equal(b[:E], b0[:E])
