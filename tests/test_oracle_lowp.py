"""Pins of the reduced-precision rounding against NumPy's and PyTorch's own casts and the E4M3 code table."""
import numpy as np
import torch

from oracle import lowp


def test_bf16_matches_torch_cast():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        [0.0, 1.0, -1.0, 3.0e38, 1e-40]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(lowp.round_bf16(x.astype(np.float64)), ref)


def test_bf16_ties_to_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: rounds to 1 (even); 1 + 3*2^-8 rounds up
    assert lowp.round_bf16(np.array([1 + 2.0 ** -8]))[0] == 1.0
    assert lowp.round_bf16(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6


def test_e4m3_table_and_cast():
    vals = lowp.e4m3_values()
    assert len(vals) == 253 and vals.max() == 448.0 and vals[vals > 0].min() == 2.0 ** -9
    assert np.array_equal(lowp.round_e4m3(vals), vals)
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(20000) * 10.0 ** rng.integers(-3, 3, 20000)).astype(np.float32)
    x = x[np.abs(x) < 440]
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(lowp.round_e4m3(x.astype(np.float64)), ref)
    # saturation
    assert lowp.round_e4m3(np.array([1e6, -500.0, 470.0]))[:].tolist() == [448.0, -448.0, 448.0]
    # every rounding lands on the nearest table value
    y = rng.uniform(-448, 448, 5000)
    r = lowp.round_e4m3(y)
    nearest = np.abs(vals[None, :] - y[:, None]).min(axis=1)
    assert np.allclose(np.abs(r - y), nearest)


def test_fp16_matches_numpy_cast():
    # NumPy's float64 -> float16 conversion rounds to nearest even, with subnormals and overflow to inf
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-9, 6, 20000),
                        [0.0, 1.0, -1.0, 65504.0, 65519.0, 65520.0, -70000.0, 2.0 ** -24, 2.0 ** -26, 1e-9]])
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(lowp.round_fp16(x), ref)


def test_fp16_ties_to_even_and_limits():
    # 1 + 2^-11 is halfway between 1 and 1 + 2^-10: rounds to 1 (even); 1 + 3*2^-11 rounds up
    assert lowp.round_fp16(np.array([1 + 2.0 ** -11]))[0] == 1.0
    assert lowp.round_fp16(np.array([1 + 3 * 2.0 ** -11]))[0] == 1 + 2.0 ** -9
    # smallest subnormal 2^-24; half of it ties to zero (even)
    assert lowp.round_fp16(np.array([2.0 ** -24, 2.0 ** -25, 1.5 * 2.0 ** -25])).tolist() == [2.0 ** -24, 0.0, 2.0 ** -24]
    # 65520 is halfway between 65504 and the next step 65536 (not finite): rounds to inf
    assert np.isinf(lowp.round_fp16(np.array([65520.0]))[0]) and lowp.round_fp16(np.array([65519.0]))[0] == 65504.0


def test_pow2_scale_closed_form():
    from oracle import mlp
    assert mlp.pow2_scale(448.0) == 1.0 and mlp.pow2_scale(448.0001) == 2.0
    assert mlp.pow2_scale(224.0) == 0.5 and mlp.pow2_scale(224.0001) == 1.0
    assert mlp.pow2_scale(0.0) == 1.0 and mlp.pow2_scale(float("inf")) == 1.0
    rng = np.random.default_rng(3)
    for m in 10.0 ** rng.uniform(-20, 20, 2000):
        s = mlp.pow2_scale(m)
        assert np.frexp(s)[0] == 0.5                       # a power of two
        assert m / s <= 448.0 < m / (s / 2)                 # the smallest such


def test_fp8_emulation_is_exact_on_representable_operands():
    # operands that are E4M3 values times the power-of-two scales pass through unrounded, so the middle
    # layer's fp8 product equals the float64 one; a dropped or doubled rescale would not.  The first
    # layer and the head take bfloat16 operands: inputs that bfloat16 holds but E4M3 does not pass
    # through the first layer unrounded.
    from oracle import mlp
    rng = np.random.default_rng(4)
    vals = lowp.e4m3_values()
    small = vals[np.abs(vals) <= 8]
    x = rng.choice(small[small >= 0], (16, 8)) * 0.25
    ident = (np.eye(8), np.zeros(8))                      # h_1 = relu(x) = x: E4M3 values again
    layers = [ident,
              (rng.choice(small, (12, 8)) * 2.0 ** -5, rng.standard_normal(12) * 0.1),
              (rng.choice(small, (5, 12)) * 2.0 ** -4, rng.standard_normal(5) * 0.1)]
    scales = mlp.fp8_scales(layers, x)
    for (sx, sw) in scales:
        assert np.frexp(sx)[0] == 0.5 and np.frexp(sw)[0] == 0.5
    y64, (hs, z64) = mlp.forward(layers, x, "f64")
    _, (_, z8) = mlp.forward(layers, x, "fp8", scales)
    assert np.array_equal(z8[0], z64[0]) and np.array_equal(z8[1], z64[1])
    # and every scaled layer input stays inside the E4M3 range
    for h, (sx, _) in zip(hs, scales):
        assert np.abs(h / sx).max() <= 448.0
    # bfloat16-exact inputs with more than four significant bits: exact through the first layer and the
    # head, rounded by the E4M3 middle layer
    xb = np.full((2, 8), 1.0 + 2.0 ** -6)
    _, (_, zb) = mlp.forward(layers, xb, "fp8", mlp.fp8_scales(layers, xb))
    assert np.array_equal(zb[0], xb @ np.eye(8))
    _, (_, zf) = mlp.forward(layers, xb, "f64")
    assert not np.array_equal(zb[1], zf[1])


def test_bf16_backward_emulation():
    # the bfloat16 backward rounds every product operand (dZ, W, h) and sums the rounded dZ for the
    # bias: (1) on operands that are bfloat16 values with exact float64 sums it equals the float64
    # backward; (2) a dZ that is not a bfloat16 value enters every product rounded: moving one dZ entry
    # by less than half a bfloat16 step changes none of the gradients, while the float64 backward moves
    from oracle import mlp
    rng = np.random.default_rng(5)
    x = rng.integers(-4, 5, (6, 4)) / 4.0
    layers = [(rng.integers(-3, 4, (5, 4)) / 8.0, rng.integers(-2, 3, 5) / 4.0),
              (rng.integers(-3, 4, (3, 5)) / 8.0, rng.integers(-2, 3, 3) / 4.0)]
    y, cache = mlp.forward(layers, x, "bf16")
    _, cache64 = mlp.forward(layers, x, "f64")
    assert all(np.array_equal(a, b) for a, b in zip(cache[1], cache64[1]))
    dy = rng.integers(-8, 9, y.shape) / 64.0
    # choose dL/dY so that dZ = dy exactly: divide out y (1 - y) in the caller's float64
    d_y = dy / (y * (1.0 - y))
    g16 = mlp.backward(layers, cache, d_y, y, "bf16")
    g64 = mlp.backward(layers, cache64, d_y, y, "f64")
    dz_exact = d_y * y * (1.0 - y)
    assert np.allclose(dz_exact, dy, rtol=0, atol=1e-15)
    for a, b in zip(g16[0] + g16[1] + [g16[2]], g64[0] + g64[1] + [g64[2]]):
        assert np.allclose(a, b, rtol=1e-12, atol=1e-15)
    # (2): perturb one head dZ by a third of a bfloat16 ulp
    bump = np.zeros_like(d_y)
    bump[2, 1] = (abs(dz_exact[2, 1]) * 2.0 ** -8 / 3.0 + 1e-300) / (y[2, 1] * (1.0 - y[2, 1]))
    h16 = mlp.backward(layers, cache, d_y + bump, y, "bf16")
    h64 = mlp.backward(layers, cache64, d_y + bump, y, "f64")
    assert all(np.array_equal(a, b) for a, b in zip(h16[0] + h16[1], g16[0] + g16[1]))
    assert not np.array_equal(h64[1][1], g64[1][1])
