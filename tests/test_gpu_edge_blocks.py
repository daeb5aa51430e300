"""The BC format's edge cases forced through ntbc_infer_blocks (Sec. 2.1, Eq. palette, Eq. weightBC4;
Sec. 3.2 inference): a network whose head weights are zero, so every block's heads are the sigmoid of
the head biases, chosen so that each texture hits one edge case:

  BC1 c0 == c1 (every code 0), BC1 c0 < c1 before the swap, BC1 endpoints at black and white in both
  orders, BC4 e0 == e1 (six-value mode with the 0 and 255 specials), BC4 eight-value and six-value
  modes over the full 0..255 range, and exact ties between equal palette entries (value 0 as the
  special entry and as e0 = 0; 255 as e1 and as the special) that the smallest logical index decides.

Endpoint values sit at the centres of their quantisation cells (y (2^b - 1) an integer) and texel
colours at decoded palette values, so float32 and float64 take the same decisions.  The GPU blocks
must equal the oracle's bit for bit (FP32, BF16 and FP16 networks; register-resident and LDS-staged
epilogues), and the oracle's blocks must show each edge case."""
import dataclasses

import numpy as np
import pytest
import torch

from util import ensure_built, log, u64
from oracle import bc as OB
from oracle import ntbc as ON
from paper_2407_09543_amd import ntbc, synth

pytestmark = pytest.mark.gpu

BIG = 30.0  # sigmoid(+-30) is 0 or 1 to float32 (and within 1e-13 in float64)


def _logit(y):
    if y <= 0.0:
        return -BIG
    if y >= 1.0:
        return BIG
    return float(np.log(y / (1.0 - y)))


def _bc1_case(q0, q1, n_cycle=True):
    """Endpoint head values for BC1 endpoints q0, q1 (5/6/5-bit) and 16 texel colours at the decoded
    logical palette entries of the stored block, cycling n = i % 4."""
    ep = [q0[0] / 31, q0[1] / 63, q0[2] / 31, q1[0] / 31, q1[1] / 63, q1[2] / 31]
    c0, c1 = int(OB.pack565(*q0)), int(OB.pack565(*q1))
    c0, c1 = max(c0, c1), min(c0, c1)
    pal = OB.bc1_palette(np.array([c0]), np.array([c1]))[0][OB.BC1_CODE_OF_LOGICAL]  # logical order
    cols = np.array([pal[i % 4] for i in range(16)], dtype=np.float64) / 255.0
    return ep, cols


def _bc4_case(e0, e1, cols8):
    """Endpoint head values for BC4 endpoints e0, e1 and the given 16 texel values (0..255)."""
    return [e0 / 255, e1 / 255], np.asarray(cols8, dtype=np.float64)[:, None] / 255.0


def _bc4_at_entries(e0, e1):
    pal = OB.bc4_palette(np.array([e0]), np.array([e1]))[0]
    order = OB.bc4_logical_order(np.array([e0]), np.array([e1]))[0]
    return [int(pal[order[i % 8]]) for i in range(16)]


# two models of the five-texture layout (BC1, BC1, BC4, BC4, BC4)
CASES = {
    "A": [_bc1_case((10, 20, 5), (10, 20, 5)),                      # c0 == c1
          _bc1_case((5, 10, 5), (25, 50, 25)),                      # c0 < c1: swapped
          _bc4_case(100, 100, [0, 255, 100, 40, 180] * 3 + [0]),    # e0 == e1: six-value, specials
          _bc4_case(200, 40, _bc4_at_entries(200, 40)),             # eight-value
          _bc4_case(30, 220, _bc4_at_entries(30, 220))],            # six-value, distinct endpoints
    "B": [_bc1_case((31, 63, 31), (0, 0, 0)),                       # white > black
          _bc1_case((0, 0, 0), (31, 63, 31)),                       # black < white: swapped
          _bc4_case(255, 0, _bc4_at_entries(255, 0)),               # eight-value, full range
          _bc4_case(0, 255, [0, 255, 51, 102, 153, 204] * 2 + [0, 255, 0, 255]),  # ties 0/e0, e1/255
          _bc4_case(0, 0, [0, 255, 60, 200] * 4)],                  # e0 == e1 == 0
}


def _model(cfg, case, seed):
    lay = ON.Layout(cfg.formats)
    layers = synth.init_weights(cfg, seed)
    rng = np.random.default_rng(seed)
    layers = [(w, (0.3 * rng.standard_normal(len(b))).astype(np.float32)) for w, b in layers]
    w_head = np.zeros_like(layers[-1][0])
    b_head = np.zeros(cfg.head_dim, dtype=np.float64)
    for t, (ep, cols) in enumerate(case):
        e = lay.ep_off[t]
        b_head[e:e + len(ep)] = [_logit(v) for v in ep]
        idx = lay.colour_index(t)
        b_head[idx] = np.vectorize(_logit)(cols)
    layers[-1] = (w_head, b_head.astype(np.float32))
    return layers


def _expect_edges(name, words):
    """The oracle's blocks show the edge case each texture was built for."""
    w = [words[t][0] for t in range(5)]
    assert all(np.all(words[t] == w[t]) for t in range(5)), "heads are constant: every block is the same"
    f = [OB.bc1_fields(np.array([w[0]])), OB.bc1_fields(np.array([w[1]]))]
    g = [OB.bc4_fields(np.array([w[t]])) for t in (2, 3, 4)]
    if name == "A":
        assert f[0][0][0] == f[0][1][0] and np.all(f[0][2] == 0)             # c0 == c1 -> codes 0
        assert f[1][0][0] == OB.pack565(25, 50, 25) and f[1][1][0] == OB.pack565(5, 10, 5)  # swapped
        assert set(f[1][2][0].tolist()) == {0, 1, 2, 3}
        assert g[0][0][0] == g[0][1][0] == 100 and {6, 7, 0} <= set(g[0][2][0].tolist())
        assert g[1][0][0] == 200 and g[1][1][0] == 40 and set(g[1][2][0].tolist()) == set(range(8))
        assert g[2][0][0] == 30 and g[2][1][0] == 220 and set(g[2][2][0].tolist()) == set(range(8))
    else:
        assert f[0][0][0] == 0xFFFF and f[0][1][0] == 0 and set(f[0][2][0].tolist()) == {0, 1, 2, 3}
        assert f[1][0][0] == 0xFFFF and f[1][1][0] == 0
        assert g[0][0][0] == 255 and g[0][1][0] == 0 and set(g[0][2][0].tolist()) == set(range(8))
        codes = g[1][2][0].tolist()
        # value 0: the special entry (logical 0, code 6) beats e0 = 0 (logical 1, code 0); value 255:
        # e1 (logical 6, code 1) beats the special (logical 7, code 7)
        assert g[1][0][0] == 0 and g[1][1][0] == 255
        assert codes[0] == 6 and codes[1] == 1 and 0 not in codes and 7 not in codes
        assert g[2][0][0] == g[2][1][0] == 0 and g[2][2][0].tolist() == [6, 7, 6, 7] * 4


@pytest.mark.parametrize("epilogue", ["register", "staged"])
@pytest.mark.parametrize("name", ["A", "B"])
def test_forced_bc_edge_cases(name, epilogue):
    ensure_built()
    cfg = dataclasses.replace(synth.config_mid(64), grid_u8=False)
    if epilogue == "staged":
        cfg = dataclasses.replace(cfg, hidden=64, n_hidden=2)
    layers = _model(cfg, CASES[name], 5)
    grid = synth.random_grid(cfg, 5, 0.7)
    ids = np.arange(cfg.n_positions)
    y_or = ON.heads(cfg, ON.grid_levels(cfg, grid=grid), layers, ids)
    w_or = ON.pack(y_or, cfg.formats)
    _expect_edges(name, w_or)
    m = ntbc.Model(ntbc.desc_from_config(cfg), torch.from_numpy(synth.flatten_weights(layers)).cuda(),
                   torch.from_numpy(grid).cuda())
    for precision in (ntbc.FP32, ntbc.BF16, ntbc.FP16):
        words = u64(m.infer(precision))
        same = [bool(np.array_equal(words[t], w_or[t])) for t in range(5)]
        log(f"edge cases {name} ({epilogue}) precision {precision}: textures equal {same}")
        assert all(same)
