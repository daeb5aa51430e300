"""Pins of the grid oracle: closed forms of the bilinear sampling, the adjoint of the scatter, the
8-bit quantiser identities, and the paper's printed storage sizes (no GPU)."""
import numpy as np
import pytest

from conftest import read_golden
from oracle import grid as G
from oracle import metrics


def test_constant_grid_gives_constant():
    levels = [np.full((r * r, 3), 0.375) for r in (4, 8, 16)]
    bx = np.arange(64)
    by = (bx * 7) % 32
    x = G.features(levels, bx, by, 64, 32)
    assert (x == 0.375).all()


def test_affine_grid_reproduced_exactly():
    # g(i, j) = a i + b j + c is reproduced at the (clamped) sample point p = (b + 1/2) r / B - 1/2
    a, b, c = 0.25, -0.5, 3.0
    blocks = 32
    for r in (2, 4, 8, 16, 32):
        j, i = np.meshgrid(np.arange(r), np.arange(r), indexing="ij")
        lvl = (a * i + b * j + c).reshape(-1, 1)
        bx = np.arange(blocks)
        by = np.arange(blocks)[::-1]
        x = G.features([lvl], bx, by, blocks, blocks)[:, 0]
        px = np.clip((bx + 0.5) * r / blocks - 0.5, 0, r - 1)
        py = np.clip((by + 0.5) * r / blocks - 0.5, 0, r - 1)
        assert np.array_equal(x, a * px + b * py + c)


def test_finest_level_hits_one_vertex():
    blocks = 16
    lvl = np.random.default_rng(0).standard_normal((blocks * blocks, 2))
    bx, by = np.meshgrid(np.arange(blocks), np.arange(blocks))
    bx, by = bx.ravel(), by.ravel()
    x = G.features([lvl], bx, by, blocks, blocks)
    assert np.array_equal(x, lvl[by * blocks + bx])


def test_corner_is_integer_and_fraction_dyadic():
    for blocks, r in ((1024, 8), (1024, 1024), (64, 16), (256, 512)):
        b = np.arange(blocks)
        i0, fnum, den = G.corner(b, blocks, r)
        assert ((i0 >= 0) & (i0 <= r - 2)).all()
        p = np.clip((b + 0.5) * r / blocks - 0.5, 0, r - 1)
        assert np.array_equal(i0 + fnum / den, p)


def test_scatter_is_adjoint_of_gather():
    rng = np.random.default_rng(1)
    n_levels, base, F, bw, bh = 4, 4, 3, 40, 24
    offs = G.level_offsets(n_levels, base)
    g = rng.standard_normal((offs[-1], F))
    ids = rng.integers(0, bw * bh, 300)
    bx, by = ids % bw, ids // bw
    x = G.features(G.split_levels(g, n_levels, base), bx, by, bw, bh)
    d = rng.standard_normal(x.shape)
    back = G.features_backward(d, bx, by, bw, bh, n_levels, base, F)
    assert np.isclose((x * d).sum(), (g * back).sum(), rtol=1e-12)


def test_quantiser_identities():
    rng = np.random.default_rng(2)
    for scale in (1e-4, 0.3, 7.0):
        w = (rng.standard_normal(5000) * scale + rng.uniform(-scale, scale)).astype(np.float32)
        s, z = G.qat_params(w)
        assert 0 <= z <= 255 and float(s) > 0
        q, mask = G.fake_quant(w, s, z)
        assert mask.all()                                   # nothing inside [min, max] is clamped
        assert np.abs(q - w.astype(np.float64)).max() <= float(s) / 2 * (1 + 1e-5)
        q2, _ = G.fake_quant(q.astype(np.float32), s, z)
        assert np.array_equal(q, q2)                        # Q(Q(w)) = Q(w)
        zero, _ = G.fake_quant(np.zeros(1, np.float32), s, z)
        if w.min() <= 0 <= w.max():
            assert zero[0] == 0.0                           # real zero is representable
        _, codes = G.quant_codes(w, s, z)
        assert codes.min() <= 1 and codes.max() >= 254      # the range spans the 8-bit codes
    # a flat level (every value 0, so the range widened to contain 0 is empty): s = 1, z = 0
    s, z = G.qat_params(np.zeros(10, np.float32))
    assert float(s) == 1.0 and z == 0
    # clamped values get no gradient
    w = np.array([-1.0, 0.0, 1.0], np.float32)
    s, z = G.qat_params(w)
    _, mask = G.fake_quant(np.array([-3.0, 0.5, 3.0], np.float32), s, z)
    assert mask.tolist() == [0.0, 1.0, 0.0]


@pytest.mark.parametrize("lo,hi", [(0.5, 2.0), (-3.0, -1.0), (0.25, 0.25)])
def test_one_signed_level_keeps_its_range(lo, hi):
    # Sec. 2.3: the zero point makes real 0 an exact code, so the range [alpha, beta] must contain 0.
    # A level whose values all share one sign is quantised over [min(alpha, 0), max(beta, 0)]: for
    # values in [0.5, 2] that is s = 2/255, z = 0; for [-3, -1] s = 3/255, z = 255.  No value of the
    # level is clamped and every one is within s/2 of its quantised value.
    w = np.linspace(lo, hi, 257).astype(np.float32)
    s, z = G.qat_params(w)
    span = max(hi, 0.0) - min(lo, 0.0)
    assert float(s) == pytest.approx(span / 255.0, rel=1e-6)
    assert z == (0 if lo >= 0 else 255)
    q, mask = G.fake_quant(w, s, z)
    assert mask.all()
    assert np.abs(q - w.astype(np.float64)).max() <= float(s) / 2 * (1 + 1e-5)
    zero, _ = G.fake_quant(np.zeros(1, np.float32), s, z)
    assert zero[0] == 0.0


def test_storage_matches_paper():
    want = {r[0]: float(r[1]) for r in read_golden("storage.txt")}
    mib = 2.0 ** 20
    ep_grid = (7, 16, 2)
    col_grid = (8, 16, 2)
    agg = metrics.model_bytes([ep_grid, col_grid], [[14, 64, 64, 64, 20], [16, 64, 64, 64, 10]])
    cons = (metrics.model_bytes([ep_grid, col_grid], [[14, 64, 64, 64, 12], [16, 64, 64, 64, 6]])
            + metrics.model_bytes([ep_grid, col_grid], [[14, 64, 64, 64, 8], [16, 64, 64, 64, 4]]))
    assert round(agg / mib, 2) == want["aggressive"]
    assert round(cons / mib, 2) == want["conservative"]
    assert round(4096 * 4096 // 16 * 8 / mib, 2) == want["bc_texture_4k"]
    # the (res+1)^2-vertex convention would not reproduce the printed size
    alt = sum((16 * 2 ** l + 1) ** 2 for l in range(7)) * 2 + sum((16 * 2 ** l + 1) ** 2 for l in range(8)) * 2
    assert round((alt + 41276) / mib, 2) != want["aggressive"]
