"""Pins of the NTBC oracle: MLP closed forms, endpoint quantisation, hand-packed heads, brute-force
index selection, and the training gradients against finite differences (no GPU)."""
import numpy as np
import pytest

from conftest import read_golden
from oracle import bc, mlp, ntbc
from oracle import grid as G
from paper_2407_09543_amd import synth


# ------------------------------------------------------------------------------------------------ MLP
def test_mlp_zero_weights_give_sigmoid_of_bias():
    layers = [(np.zeros((5, 3)), np.zeros(5)), (np.zeros((2, 5)), np.array([0.0, np.log(3.0)]))]
    y, _ = mlp.forward(layers, np.random.default_rng(0).standard_normal((7, 3)))
    assert np.allclose(y, [[0.5, 0.75]] * 7, rtol=0, atol=1e-15)


def test_mlp_relu_closed_form():
    # identity hidden layer: Y = sigmoid(sum(relu(x)) + b)
    layers = [(np.eye(4), np.zeros(4)), (np.ones((1, 4)), np.array([-1.0]))]
    x = np.array([[1.0, -2.0, 0.5, -0.1], [-1.0, -1.0, -1.0, -1.0]])
    y, _ = mlp.forward(layers, x)
    assert np.allclose(y[:, 0], 1.0 / (1.0 + np.exp(-np.array([0.5, -1.0]))), rtol=1e-15)


def test_mlp_backward_against_finite_differences():
    rng = np.random.default_rng(1)
    layers = [(rng.standard_normal((8, 5)), rng.standard_normal(8)),
              (rng.standard_normal((6, 8)), rng.standard_normal(6)),
              (rng.standard_normal((3, 6)), rng.standard_normal(3))]
    x = rng.standard_normal((9, 5))
    g = rng.standard_normal((9, 3))
    y, cache = mlp.forward(layers, x)
    dws, dbs, dx = mlp.backward(layers, cache, g, y)

    def f(ls, xx):
        return (mlp.forward(ls, xx)[0] * g).sum()
    h = 1e-6
    for k in range(3):
        for _ in range(4):
            i, j = rng.integers(0, layers[k][0].shape[0]), rng.integers(0, layers[k][0].shape[1])
            lp = [(w.copy(), b.copy()) for w, b in layers]
            lp[k][0][i, j] += h
            lm = [(w.copy(), b.copy()) for w, b in layers]
            lm[k][0][i, j] -= h
            assert np.isclose((f(lp, x) - f(lm, x)) / (2 * h), dws[k][i, j], rtol=1e-5, atol=1e-8)
    i, j = 3, 2
    xp, xm = x.copy(), x.copy()
    xp[i, j] += h
    xm[i, j] -= h
    assert np.isclose((f(layers, xp) - f(layers, xm)) / (2 * h), dx[i, j], rtol=1e-5, atol=1e-8)


# --------------------------------------------------------------------------------------- quantise/pack
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_endpoint_codes_requantise(precision):
    for bits, expand in ((5, bc.expand5), (6, bc.expand6)):
        q = np.arange(1 << bits)
        y = expand(q) / 255.0
        assert (ntbc.quant_endpoint(y, bits, precision) == q).all()
    q = np.arange(256)
    assert (ntbc.quant_endpoint(q / 255.0, 8, precision) == q).all()
    assert ntbc.quant_endpoint(np.array([-0.3, 1.7]), 8, precision).tolist() == [0, 255]


def _hand_heads(case):
    lay = ntbc.Layout([1, 4])
    y = np.zeros((1, lay.H))
    bc4_8 = np.array([200, 10, 173, 146, 119, 91, 64, 37]) / 255.0
    bc4_6 = np.array([10, 200, 48, 86, 124, 162, 0, 255]) / 255.0
    if case == "C":
        y[0, 0:6] = 0.5
        y[0, 6:8] = 0.5
        y[0, lay.E:] = 0.5
        return y
    y[0, 0:6] = [1, 0, 0, 0, 0, 1] if case == "A" else [0, 0, 1, 1, 0, 0]
    y[0, 6:8] = [200 / 255.0, 10 / 255.0] if case == "A" else [10 / 255.0, 200 / 255.0]
    pal = np.array([[255, 0, 0], [170, 0, 85], [85, 0, 170], [0, 0, 255]]) / 255.0   # logical order
    for i in range(16):
        y[0, lay.E + i * 4:lay.E + i * 4 + 3] = pal[i % 4] + [0.01, 0, 0]
        v = bc4_8[i % 8] - 0.001 if case == "A" else bc4_6[i % 8]
        y[0, lay.E + i * 4 + 3] = v
    return y


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_hand_heads_pack(precision):
    for row in read_golden("pack_hand.txt"):
        y = _hand_heads(row[0])
        words = ntbc.pack(y, [1, 4], precision)
        assert int(words[0, 0]) == int(row[1], 16), row
        assert int(words[1, 0]) == int(row[2], 16), row


def _bruteforce_codes(words, chat, fmt):
    """Per texel the stored code whose decoded colour/255 is nearest to chat (ties: smallest logical)."""
    n = len(words)
    if fmt == 1:
        c0, c1, _ = bc.bc1_fields(words)
        order = [0, 2, 3, 1]
        dec = lambda code: bc.bc1_decode(bc.bc1_pack(c0, c1, np.full((n, 16), code))) / 255.0
    else:
        e0, e1, _ = bc.bc4_fields(words)
        order_arr = bc.bc4_logical_order(e0, e1)
    best = np.zeros((n, 16), dtype=np.int64)
    best_d = np.full((n, 16), np.inf)
    for k in range(4 if fmt == 1 else 8):
        if fmt == 1:
            code = np.full((n, 16), order[k])
            col = dec(order[k])
        else:
            code = np.broadcast_to(order_arr[:, k][:, None], (n, 16))
            col = (bc.bc4_decode(bc.bc4_pack(e0, e1, code)) / 255.0)[..., None]
        d = ((col - chat) ** 2).sum(-1)
        better = d < best_d
        best = np.where(better, code, best)
        best_d = np.where(better, d, best_d)
    if fmt == 1:
        best[c0 == c1] = 0
    return best


def test_pack_indices_are_bruteforce_argmin():
    rng = np.random.default_rng(3)
    formats = [1, 1, 4, 4, 4]
    lay = ntbc.Layout(formats)
    y = rng.uniform(0, 1, (800, lay.H))
    y[:100, :lay.E] = 0.5 + rng.uniform(-0.02, 0.02, (100, lay.E))   # near-equal endpoints
    words = ntbc.pack(y, formats)
    for t, f in enumerate(formats):
        chat = y[:, lay.colour_index(t)]
        if f == 1:
            _, _, codes = bc.bc1_fields(words[t])
        else:
            _, _, codes = bc.bc4_fields(words[t])
        assert (codes == _bruteforce_codes(words[t], chat, f)).all()


# ------------------------------------------------------------------------------------------ training
def _small_problem(seed=0, n=48):
    cfg = synth.config_small(64)
    m = synth.material_small(64, seed + 1)
    blocks = [bc.image_to_blocks(t.texels) for t in m.textures]
    refw = [bc.bc1_encode_ref(blocks[0]), bc.bc4_encode_ref(blocks[1])]
    tg = ntbc.Targets(cfg.formats, refw, blocks)
    layers = [(w.astype(np.float64), b.astype(np.float64) + 0.01)
              for w, b in synth.init_weights(cfg, seed)]
    grid = synth.random_grid(cfg, seed, 0.3).astype(np.float64)
    ids = synth.batch_ids(seed, 0, n, cfg.n_positions)
    return cfg, tg, layers, grid, ids


def test_smooth_loss_gradients_against_finite_differences():
    cfg, tg, layers, grid, ids = _small_problem()
    terms = (1.0, 1.0, 0.0, 0.0)
    _, dgrid, dl, _ = ntbc.gradients(cfg, grid, layers, tg, ids, qat=False, terms=terms)

    def loss(gr, ls):
        l, *_ = ntbc.gradients(cfg, gr, ls, tg, ids, qat=False, terms=terms)
        return l[0] + l[1]
    rng = np.random.default_rng(5)
    h = 1e-6
    checked = 0
    for _ in range(12):
        k = rng.integers(0, len(layers))
        i, j = rng.integers(0, layers[k][0].shape[0]), rng.integers(0, layers[k][0].shape[1])
        lp = [(w.copy(), b.copy()) for w, b in layers]
        lp[k][0][i, j] += h
        lm = [(w.copy(), b.copy()) for w, b in layers]
        lm[k][0][i, j] -= h
        fd = (loss(grid, lp) - loss(grid, lm)) / (2 * h)
        assert np.isclose(fd, dl[k][0][i, j], rtol=1e-5, atol=1e-10), (k, i, j, fd, dl[k][0][i, j])
        checked += 1
    # grid vertices actually touched by the batch
    touched = np.nonzero(np.abs(dgrid).sum(axis=1) > 0)[0]
    for v in rng.choice(touched, 10, replace=False):
        f = rng.integers(0, grid.shape[1])
        gp, gm = grid.copy(), grid.copy()
        gp[v, f] += h
        gm[v, f] -= h
        fd = (loss(gp, layers) - loss(gm, layers)) / (2 * h)
        assert np.isclose(fd, dgrid[v, f], rtol=1e-5, atol=1e-10)
        checked += 1
    assert checked == 22


def _soft_functional(y, tg, ids, branch, g_fixed, temp=0.01):
    """G(Y) = sum g * x_soft where x_soft = sum_n softmax(d/T)_n c_ref,n with d of the given branch."""
    lay = tg.lay
    n = y.shape[0]
    c_hat = y[:, lay.E:].reshape(n, 16, lay.C)
    total = 0.0
    for t, f in enumerate(lay.formats):
        e = lay.ep_off[t]
        ch = lay.channels(t)
        sl = slice(lay.ch_off[t], lay.ch_off[t] + ch)
        c = tg.c[ids][:, :, sl]
        pal_ref = tg.pal_ref[t][ids]
        if branch == "endpoint":
            e0, e1 = y[:, e:e + ch], y[:, e + ch:e + 2 * ch]
            pal, _, _ = ntbc.palette_real(e0, e1, f, e0[:, 0] > e1[:, 0])
            d = -np.sqrt(((c[:, :, None, :] - pal[:, None, :, :]) ** 2).sum(-1))
        else:
            d = -np.sqrt(((c_hat[:, :, None, sl] - pal_ref[:, None, :, :]) ** 2).sum(-1))
        z = d / temp
        s = np.exp(z - z.max(-1, keepdims=True))
        s /= s.sum(-1, keepdims=True)
        xs = (s[..., None] * pal_ref[:, None, :, :]).sum(2)
        total += (g_fixed[t] * xs).sum()
    return total


def _hard_grad_x(y, tg, ids, branch):
    """g = dL_cd/dx at the hard forward decode (held fixed by the straight-through estimator)."""
    lay = tg.lay
    n = y.shape[0]
    c_hat = y[:, lay.E:].reshape(n, 16, lay.C)
    out = []
    for t, f in enumerate(lay.formats):
        e = lay.ep_off[t]
        ch = lay.channels(t)
        sl = slice(lay.ch_off[t], lay.ch_off[t] + ch)
        c = tg.c[ids][:, :, sl]
        pal_ref = tg.pal_ref[t][ids]
        if branch == "endpoint":
            e0, e1 = y[:, e:e + ch], y[:, e + ch:e + 2 * ch]
            pal, _, _ = ntbc.palette_real(e0, e1, f, e0[:, 0] > e1[:, 0])
            dist = ((c[:, :, None, :] - pal[:, None, :, :]) ** 2).sum(-1)
        else:
            dist = ((c_hat[:, :, None, sl] - pal_ref[:, None, :, :]) ** 2).sum(-1)
        k = dist.argmin(-1)
        x = np.take_along_axis(pal_ref[:, None, :, :], k[:, :, None, None], axis=2)[:, :, 0, :]
        out.append(2.0 * (x - c) / (n * 16 * lay.C))
    return out


@pytest.mark.parametrize("branch", ["endpoint", "colour"])
def test_straight_through_gradient_is_softmax_expectation_gradient(branch):
    cfg, tg, layers, grid, ids = _small_problem(1, 24)
    y = ntbc.heads(cfg, G.split_levels(grid, cfg.n_levels, cfg.base_res), layers, ids)
    # keep BC4 endpoint order away from the mode switch for a clean finite difference
    lay = tg.lay
    e = lay.ep_off[1]
    y[:, e] = np.maximum(y[:, e], y[:, e + 1] + 0.05)
    terms = (0, 0, 1, 0) if branch == "endpoint" else (0, 0, 0, 1)
    _, dy = ntbc.loss_and_grad(y, tg, ids, 0.01, terms)
    g = _hard_grad_x(y, tg, ids, branch)
    rng = np.random.default_rng(7)
    cols = list(range(lay.E)) if branch == "endpoint" else list(range(lay.E, lay.H))
    h = 1e-7
    for _ in range(25):
        i = rng.integers(0, y.shape[0])
        j = cols[rng.integers(0, len(cols))]
        yp, ym = y.copy(), y.copy()
        yp[i, j] += h
        ym[i, j] -= h
        fd = (_soft_functional(yp, tg, ids, branch, g) - _soft_functional(ym, tg, ids, branch, g)) / (2 * h)
        assert np.isclose(fd, dy[i, j], rtol=1e-4, atol=1e-9), (i, j, fd, dy[i, j])


def test_expected_weight_derivative_reading():
    # App. A: w^ = sum_i w_i softmax(d/T)_i; its derivative is (1/T) s_j (w_j - w^).  The printed final
    # form uses n in place of w_n, which disagrees for j >= 1 (BC1: w_n = n/3).
    rng = np.random.default_rng(9)
    temp = 0.01
    w = np.arange(4) / 3.0
    for _ in range(10):
        d = -rng.uniform(0, 0.05, 4)

        def what(dd):
            z = dd / temp
            s = np.exp(z - z.max())
            s /= s.sum()
            return (w * s).sum(), s
        wh, s = what(d)
        for j in range(4):
            dp, dm = d.copy(), d.copy()
            dp[j] += 1e-8
            dm[j] -= 1e-8
            fd = (what(dp)[0] - what(dm)[0]) / 2e-8
            assert np.isclose(fd, s[j] * (w[j] - wh) / temp, rtol=1e-5, atol=1e-9)
            if j >= 1 and abs(s[j]) > 1e-3:
                assert not np.isclose(fd, s[j] * (j - wh) / temp, rtol=1e-3)


def test_qat_gradient_is_pass_through():
    cfg, tg, layers, grid, ids = _small_problem(2, 32)
    _, dq, _, _ = ntbc.gradients(cfg, grid, layers, tg, ids, qat=True)
    fq, mask = G.fake_quant_grid(grid, cfg.n_levels, cfg.base_res)
    _, d_at_q, _, _ = ntbc.gradients(cfg, fq, layers, tg, ids, qat=False)
    assert np.allclose(dq, d_at_q * mask, rtol=1e-12, atol=0)


def test_adam_first_step_and_schedule():
    g = np.array([3.0, -0.2, 1e-3])
    p, m, v = ntbc.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-9)
    assert ntbc.learning_rate(0, 0.01, 100) == pytest.approx(0.001)
    assert ntbc.learning_rate(9, 0.01, 100) == pytest.approx(0.01)
    assert ntbc.learning_rate(10, 0.01, 100) == pytest.approx(0.01)
    assert ntbc.learning_rate(55, 0.01, 100) == pytest.approx(0.005)
    assert ntbc.learning_rate(100, 0.01, 100) == pytest.approx(0.0, abs=1e-15)


def test_training_lowers_the_loss():
    cfg = synth.config_small(256)
    m = synth.material_small(256, 1)
    blocks = [bc.image_to_blocks(t.texels) for t in m.textures]
    tg = ntbc.Targets(cfg.formats, [bc.bc1_encode_ref(blocks[0]), bc.bc4_encode_ref(blocks[1])], blocks)
    st = ntbc.TrainState(synth.init_grid(cfg, 1), synth.init_weights(cfg, 1))
    losses = []
    for step in range(60):
        ids = synth.batch_ids(1, step, 512, cfg.n_positions)
        losses.append(ntbc.train_step(cfg, st, tg, ids, step, 60, qat=False).sum())
    assert losses[-1] < 0.2 * losses[0]
