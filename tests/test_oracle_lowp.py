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
