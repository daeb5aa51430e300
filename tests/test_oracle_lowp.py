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
    # operands that are E4M3 values times the power-of-two scales pass through unrounded, so the fp8
    # emulation equals the float64 forward; a dropped or doubled rescale would not
    from oracle import mlp
    rng = np.random.default_rng(4)
    vals = lowp.e4m3_values()
    small = vals[np.abs(vals) <= 8]
    x = rng.choice(small[small >= 0], (16, 8)) * 0.25
    layers = [(rng.choice(small, (12, 8)) * 2.0 ** -5, rng.standard_normal(12) * 0.1),
              (rng.choice(small, (5, 12)) * 2.0 ** -4, rng.standard_normal(5) * 0.1)]
    scales = mlp.fp8_scales(layers, x)
    for (sx, sw) in scales:
        assert np.frexp(sx)[0] == 0.5 and np.frexp(sw)[0] == 0.5
    y64, (hs, _) = mlp.forward(layers, x, "f64")
    # the first layer's operands are representable by construction: its pre-activations match exactly
    z64 = x @ layers[0][0].T.astype(np.float64) + layers[0][1]
    _, (_, z8) = mlp.forward(layers, x, "fp8", scales)
    assert np.array_equal(z8[0], z64)
    # and every scaled layer input stays inside the E4M3 range
    for h, (sx, _) in zip(hs, scales):
        assert np.abs(h / sx).max() <= 448.0
