"""Pins of the oracle of the paper's own network layout (separate endpoint and colour networks, SELU,
half precision; conservative and aggressive layouts): the configuration's node counts, the printed
model sizes, SELU's defining fixed point, the texel-centre addressing of the colour grid, and the
assembly of a block's heads from one endpoint run and 16 colour runs (no GPU)."""
import numpy as np
import pytest

from conftest import read_golden
from oracle import faithful as F
from oracle import grid as G
from oracle import ntbc as N
from oracle.ntbc import BC1, BC4

SIX = [BC1, BC1, BC4, BC4, BC4, BC4]      # the storage fixture's material: N_RGB = 2, N_SC = 4


def test_node_counts_of_the_configuration():
    # Sec. 3.4: 14 inputs for the endpoint network, 16 for the colour network; Sec. 4.1: outputs
    assert F.grid_inputs(F.ENDPOINT_GRID) == 14 and F.grid_inputs(F.COLOUR_GRID) == 16
    assert G.level_res(7, 16)[-1] == 1024 and G.level_res(8, 16)[-1] == 2048
    # closed form sum_l (16 2^l)^2 = 256 (4^L - 1) / 3
    assert F.grid_vertices(F.ENDPOINT_GRID) == 256 * (4 ** 7 - 1) // 3 == 1398016
    assert F.grid_vertices(F.COLOUR_GRID) == 256 * (4 ** 8 - 1) // 3 == 5592320
    n_rgb, n_sc = 2, 4
    assert F.output_nodes(SIX) == (6 * n_rgb + 2 * n_sc, 3 * n_rgb + n_sc)
    assert F.models_of(SIX, "aggressive") == [[0, 1, 2, 3, 4, 5]]
    assert F.models_of(SIX, "conservative") == [[0, 1], [2, 3, 4, 5]]
    assert F.output_nodes([BC1, BC1]) == (6 * n_rgb, 3 * n_rgb)
    assert F.output_nodes([BC4] * 4) == (2 * n_sc, n_sc)
    # one layer 14 -> 64, two 64 -> 64, one 64 -> 20 (with biases), and 16 -> 64 ... -> 10
    assert F.n_parameters(SIX) == (14 * 64 + 64) + 2 * (64 * 64 + 64) + (64 * 20 + 20) + \
        (16 * 64 + 64) + 2 * (64 * 64 + 64) + (64 * 10 + 10)


def test_storage_matches_the_printed_sizes():
    want = {r[0]: float(r[1]) for r in read_golden("storage.txt")}
    mib = 2.0 ** 20
    assert round(F.material_bytes(SIX, "aggressive") / mib, 2) == want["aggressive"]
    assert round(F.material_bytes(SIX, "conservative") / mib, 2) == want["conservative"]
    # the printed sizes hold for other mixes of six textures too (the MLPs are ~0.3% of a model)
    for fm in ([BC1, BC1, BC1, BC4, BC4, BC4], [BC1, BC1, BC1, BC1, BC4, BC4]):
        assert round(F.material_bytes(fm, "aggressive") / mib, 2) == want["aggressive"]
        assert round(F.material_bytes(fm, "conservative") / mib, 2) == want["conservative"]
    # a material of RGB textures only has one model in both layouts
    assert F.material_bytes([BC1, BC1], "conservative") == F.material_bytes([BC1, BC1], "aggressive")


def test_network_executions_per_block():
    # Tab. inferPerf: the conservative layout runs twice the networks of the aggressive one when the
    # material mixes RGB and single-channel textures, the same when it holds RGB textures only
    assert F.executions_per_block(SIX, "conservative") == 2 * F.executions_per_block(SIX, "aggressive") == 34
    assert F.executions_per_block([BC1, BC1], "conservative") == F.executions_per_block([BC1, BC1], "aggressive")


def test_selu_fixed_point_and_closed_forms():
    # the constants are the ones for which a standard normal input keeps mean 0 and variance 1
    from scipy.integrate import quad
    phi = lambda t: np.exp(-0.5 * t * t) / np.sqrt(2.0 * np.pi)
    moment = lambda k, fn: sum(quad(lambda t: float(fn(t)) ** k * phi(t), a, b, epsabs=1e-13)[0]
                               for a, b in ((-np.inf, 0.0), (0.0, np.inf)))
    assert abs(moment(1, F.selu)) < 1e-6
    assert abs(moment(2, F.selu) - 1.0) < 1e-6
    assert F.selu(0.0) == 0.0 and F.selu(1.0) == F.SELU_LAMBDA
    assert F.selu(-60.0) == pytest.approx(-F.SELU_LAMBDA * F.SELU_ALPHA, rel=1e-15)
    # planted mistake: the two constants exchanged miss the fixed point
    swapped = lambda t: F.SELU_ALPHA * t if t > 0 else F.SELU_ALPHA * F.SELU_LAMBDA * np.expm1(t)
    assert abs(moment(1, swapped)) > 1e-2 or abs(moment(2, swapped) - 1.0) > 1e-2


def test_colour_grid_samples_texel_centres():
    # at the level whose resolution equals the texture width, texel (x, y) sits exactly on vertex (x, y)
    W = 32
    levels = [np.zeros((r * r, 2)) for r in G.level_res(2, 16)]
    i, j = np.meshgrid(np.arange(32), np.arange(32))
    levels[1][:, 0] = (j * 32 + i).ravel() * 1.0
    levels[1][:, 1] = (i - j).ravel() * 0.5
    tx, ty = np.array([0, 5, 31, 17]), np.array([0, 9, 31, 2])
    f = G.features(levels, tx, ty, W, W)
    assert np.array_equal(f[:, 2], ty * 32.0 + tx) and np.array_equal(f[:, 3], (tx - ty) * 0.5)


def _layers(rng, n_in, n_out, scale=0.3):
    return [(rng.standard_normal((o, i)) * scale, rng.standard_normal(o) * 0.1)
            for i, o in F.layer_dims(n_in, n_out)]


def _levels(rng, g, scale=0.5):
    return [rng.uniform(-scale, scale, (r * r, g["n_features"])) for r in G.level_res(g["n_levels"], g["base_res"])]


def test_block_heads_assembly():
    rng = np.random.default_rng(3)
    fm = [BC1, BC4]
    e, c = F.output_nodes(fm)
    el, ew = _levels(rng, F.ENDPOINT_GRID), _layers(rng, 14, e)
    cl, cw = _levels(rng, F.COLOUR_GRID), _layers(rng, 16, c)
    bw = bh = 256                                           # a 1024^2 texture
    bx, by = np.array([0, 7, 255, 100]), np.array([0, 3, 255, 200])
    y = F.block_heads(fm, el, ew, cl, cw, bx, by, bw, bh, "f64")
    lay = N.Layout(fm)
    assert y.shape == (4, lay.H) and lay.H == e + 16 * c
    for k in range(4):
        ye = F.mlp_forward(ew, G.features(el, bx[k:k + 1], by[k:k + 1], bw, bh), "f64")
        assert np.allclose(y[k, :e], ye[0], rtol=0, atol=1e-13)
        for t in (0, 5, 15):
            xx, yy = 4 * bx[k] + t % 4, 4 * by[k] + t // 4
            yc = F.mlp_forward(cw, G.features(cl, np.array([xx]), np.array([yy]), 4 * bw, 4 * bh), "f64")
            assert np.allclose(y[k, lay.colour_index(0)[t]], yc[0, 0:3], rtol=0, atol=1e-13)
            assert np.allclose(y[k, lay.colour_index(1)[t]], yc[0, 3:4], rtol=0, atol=1e-13)
    # half precision stays within its rounding of the exact heads
    y16 = F.block_heads(fm, el, ew, cl, cw, bx, by, bw, bh, "fp16")
    assert np.abs(y16 - y).max() < 5e-3


def test_zero_weights_give_the_sigmoid_of_the_biases_and_layouts_place_words():
    fm = [BC1, BC4, BC4]
    rng = np.random.default_rng(4)
    models = []
    for grp in F.models_of(fm, "conservative"):
        e, c = F.output_nodes([fm[i] for i in grp])
        ew = [(np.zeros((o, i)), np.zeros(o)) for i, o in F.layer_dims(14, e)]
        cw = [(np.zeros((o, i)), np.zeros(o)) for i, o in F.layer_dims(16, c)]
        ew[-1] = (ew[-1][0], rng.standard_normal(e))
        cw[-1] = (cw[-1][0], rng.standard_normal(c))
        models.append((_levels(rng, F.ENDPOINT_GRID), ew, _levels(rng, F.COLOUR_GRID), cw))
    bx, by = np.arange(6), np.arange(6)[::-1]
    words = F.infer_blocks(fm, models, bx, by, 64, 64, "conservative", "f64")
    for grp, (el, ew, cl, cw) in zip(F.models_of(fm, "conservative"), models):
        sub = [fm[i] for i in grp]
        y = F.block_heads(sub, el, ew, cl, cw, bx, by, 64, 64, "f64")
        sig_e = 1.0 / (1.0 + np.exp(-ew[-1][1]))
        assert np.allclose(y[:, :len(sig_e)], sig_e[None, :], rtol=0, atol=1e-15)
        assert np.array_equal(words[grp], N.pack(y, sub, "f64"))


def test_dummy_distance_nodes_change_nothing():
    # aggressive layout (Sec. 4.1): eight distance nodes, BC1 uses the first four and the other four
    # are dummies with zero gradient -- a dummy never wins the argmax (d = -inf) and has softmax weight
    # 0, so the decoded-colour term equals the four-node one of oracle.ntbc, value and gradient
    rng = np.random.default_rng(9)
    n = 50
    c = rng.uniform(0, 1, (n, 16, 3))
    pal = rng.uniform(0, 1, (n, 4, 3))
    delta4 = c[:, :, None, :] - pal[:, None, :, :]
    l4, dd4, _ = N._cd_branch(delta4, pal, c, n * 16 * 3, 0.01)
    # eight nodes: the dummies sit infinitely far away (their reference colours are irrelevant)
    pal8 = np.concatenate([pal, rng.uniform(0, 1, (n, 4, 3))], axis=1)
    delta8 = np.concatenate([delta4, np.full((n, 16, 4, 3), np.inf)], axis=2)
    with np.errstate(invalid="ignore"):
        l8, dd8, _ = N._cd_branch(delta8, pal8, c, n * 16 * 3, 0.01)
    assert l8 == l4
    assert np.allclose(dd8[..., :4], dd4, rtol=1e-9, atol=1e-15) and (dd8[..., 4:] == 0).all()


# ------------------------------------------------------------------------------------------ training
TINY_EP = dict(n_levels=3, base_res=2, n_features=2)    # 2 .. 8
TINY_COL = dict(n_levels=3, base_res=4, n_features=2)   # 4 .. 16


def _train_problem(seed=0, n=24):
    """A 64^2 BC1 + BC4 material (16 x 16 blocks), small grids of both networks, random parameters."""
    from oracle import bc
    from paper_2407_09543_amd import synth
    m = synth.material_small(64, seed + 1)
    fm = [BC1, BC4]
    blocks = [bc.image_to_blocks(t.texels) for t in m.textures]
    tg = N.Targets(fm, [bc.bc1_encode_ref(blocks[0]), bc.bc4_encode_ref(blocks[1])], blocks)
    rng = np.random.default_rng(seed)
    e, c = F.output_nodes(fm)
    ew, cw = _layers(rng, 6, e, 0.3), _layers(rng, 6, c, 0.3)
    eg = rng.uniform(-0.5, 0.5, (F.grid_vertices(TINY_EP), 2))
    cg = rng.uniform(-0.5, 0.5, (F.grid_vertices(TINY_COL), 2))
    ids = rng.choice(256, n, replace=False)
    return fm, tg, eg, ew, cg, cw, ids


def test_selu_derivative_closed_form():
    z = np.array([-6.0, -1.3, -0.2, -1e-3, 1e-3, 0.4, 3.0])
    h = 1e-6
    fd = (F.selu(z + h) - F.selu(z - h)) / (2 * h)
    assert np.allclose(F.selu_grad(z), fd, rtol=1e-7, atol=0)
    # the left branch at 0 (the forward's case split): lambda alpha
    assert F.selu_grad(0.0) == F.SELU_LAMBDA * F.SELU_ALPHA


def _fd_check(fm, tg, eg, ew, cg, cw, ids, rng, grads):
    """Central differences of L_e + L_c (the smooth terms) against the analytic gradients at a sample
    of weights, biases and touched grid vertices of both networks; returns the largest mismatch."""
    terms = (1.0, 1.0, 0.0, 0.0)

    def loss(p):
        l = F.gradients(fm, p[0], p[1], p[2], p[3], tg, ids, 16, 16, terms=terms, ep_cfg=TINY_EP, col_cfg=TINY_COL)[0]
        return l[0] + l[1]
    params = [eg, ew, cg, cw]
    h = 1e-6
    worst = 0.0
    for k in range(4):
        for _ in range(8 if k % 2 else 5):
            pp = [x.copy() if isinstance(x, np.ndarray) else [(w.copy(), b.copy()) for w, b in x] for x in params]
            pm = [x.copy() if isinstance(x, np.ndarray) else [(w.copy(), b.copy()) for w, b in x] for x in params]
            if k % 2 == 0:
                touched = np.nonzero(np.abs(grads[k]).sum(axis=1) > 0)[0]
                v, f = rng.choice(touched), rng.integers(0, 2)
                pp[k][v, f] += h
                pm[k][v, f] -= h
                an = grads[k][v, f]
            else:
                layer = rng.integers(0, len(params[k]))
                w = params[k][layer][0]
                if rng.integers(0, 3) == 0:
                    i = rng.integers(0, w.shape[0])
                    pp[k][layer][1][i] += h
                    pm[k][layer][1][i] -= h
                    an = grads[k][layer][1][i]
                else:
                    i, j = rng.integers(0, w.shape[0]), rng.integers(0, w.shape[1])
                    pp[k][layer][0][i, j] += h
                    pm[k][layer][0][i, j] -= h
                    an = grads[k][layer][0][i, j]
            fd = (loss(pp) - loss(pm)) / (2 * h)
            worst = max(worst, abs(fd - an) / max(abs(fd), 1e-6))
    return worst


def test_training_gradients_against_finite_differences():
    # both networks and both grids, through the head assembly, the SELU layers and the texel-centre
    # scatter of the colour grid
    fm, tg, eg, ew, cg, cw, ids = _train_problem()
    out = F.gradients(fm, eg, ew, cg, cw, tg, ids, 16, 16, terms=(1.0, 1.0, 0.0, 0.0), ep_cfg=TINY_EP,
                      col_cfg=TINY_COL)
    worst = _fd_check(fm, tg, eg, ew, cg, cw, ids, np.random.default_rng(7), out[1:5])
    assert worst < 1e-5, worst


def test_training_gradient_planted_selu_mistake_fails(monkeypatch):
    # the ReLU-style derivative (lambda on both sides) is a plausible slip: the check catches it
    fm, tg, eg, ew, cg, cw, ids = _train_problem(1)
    monkeypatch.setattr(F, "selu_grad", lambda z: np.full(np.shape(z), F.SELU_LAMBDA))
    out = F.gradients(fm, eg, ew, cg, cw, tg, ids, 16, 16, terms=(1.0, 1.0, 0.0, 0.0), ep_cfg=TINY_EP,
                      col_cfg=TINY_COL)
    worst = _fd_check(fm, tg, eg, ew, cg, cw, ids, np.random.default_rng(8), out[1:5])
    assert worst > 1e-3, worst


def test_training_heads_are_the_inference_heads():
    # the training forward assembles the same heads as the inference oracle (float64)
    fm, tg, eg, ew, cg, cw, ids = _train_problem(2)
    y = F.gradients(fm, eg, ew, cg, cw, tg, ids, 16, 16, ep_cfg=TINY_EP, col_cfg=TINY_COL)[5]
    el = G.split_levels(eg, TINY_EP["n_levels"], TINY_EP["base_res"])
    cl = G.split_levels(cg, TINY_COL["n_levels"], TINY_COL["base_res"])
    y_inf = F.block_heads(fm, el, ew, cl, cw, ids % 16, ids // 16, 16, 16, "f64")
    assert np.allclose(y, y_inf, rtol=0, atol=1e-14)


def test_train_step_first_adam_update_is_signed_learning_rate():
    # Adam's first bias-corrected step moves every parameter by lr g / (|g| + eps), i.e. by lr sign(-g)
    # where |g| >> eps (lr of the warm-up's first step: lr0 / 10), grids at lr_grid and networks at
    # lr_mlp; untouched vertices stay
    fm, tg, eg, ew, cg, cw, ids = _train_problem(3)
    st = F.TrainState(eg, ew, cg, cw)
    grads = F.gradients(fm, eg, ew, cg, cw, tg, ids, 16, 16, ep_cfg=TINY_EP, col_cfg=TINY_COL)[1:5]
    F.train_step(fm, st, tg, ids, 16, 16, 0, 100, lr_grid=0.01, lr_mlp=0.005, ep_cfg=TINY_EP, col_cfg=TINY_COL)
    for k, lr in ((0, 0.001), (1, 0.0005), (2, 0.001), (3, 0.0005)):
        if k % 2 == 0:
            pairs = [(st.params[k], (eg, cg)[k // 2], grads[k])]
        else:
            pairs = [(a, b, c) for (a, _), (b, _), (c, _) in zip(st.params[k], (ew, cw)[k // 2], grads[k])]
        for new, old, g in pairs:
            big = np.abs(g) > 1e-6
            assert big.mean() > 0.5
            assert np.allclose((new - old)[big], -lr * np.sign(g[big]), rtol=1e-8, atol=0)
            assert (new[g == 0] == old[g == 0]).all()
