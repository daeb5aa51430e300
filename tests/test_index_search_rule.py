"""The fused kernel's BC4 nearest-index rule against the definition, on the CPU in float32.

The definition (paper Sec. 3.2, Eq. dist; ties to the smallest weight index) takes the first minimum
of the float32 squared distances e_n = (x - p_n)^2 over the palette in weight order.  The kernel takes
the last index whose distance is strictly below its predecessor's, which is the same index because the
palette is monotone in weight order in both BC4 modes and float32 rounding is monotone, so e_n is
unimodal.  This test evaluates both rules with float32 arithmetic on every pair of 8-bit endpoints and
on colours at, between and one ulp around every palette value, plus random colours."""
import numpy as np


def _palettes():
    e0, e1 = np.meshgrid(np.arange(256), np.arange(256), indexing="ij")
    e0, e1 = e0.ravel().astype(np.int64), e1.ravel().astype(np.int64)
    eight = e0 > e1
    v = np.zeros((e0.size, 8), np.int64)
    j = np.arange(1, 7)
    v8 = np.concatenate([e0[:, None], ((7 - j) * e0[:, None] + j * e1[:, None] + 3) // 7, e1[:, None]], axis=1)
    k = np.arange(1, 5)
    v6 = np.concatenate([np.zeros_like(e0)[:, None], e0[:, None], ((5 - k) * e0[:, None] + k * e1[:, None] + 2) // 5,
                         e1[:, None], np.full_like(e0, 255)[:, None]], axis=1)
    v[eight] = v8[eight]
    v[~eight] = v6[~eight]
    return v


def _rules(pal, x):
    """pal float32 [P, 8] (weight order), x float32 [P, X] -> (definition, kernel rule) indices [P, X]."""
    d = x[:, :, None] - pal[:, None, :]          # float32 subtraction, rounded once
    e = d * d                                     # float32 square, rounded once
    first_min = np.argmin(e, axis=2)              # numpy returns the first minimum
    dec = e[:, :, 1:] < e[:, :, :-1]              # strict decreases
    idx = np.where(dec, np.arange(1, 8)[None, None, :], 0)
    return first_min, idx.max(axis=2)


def test_bc4_last_strict_decrease_equals_first_minimum():
    v = _palettes()
    pal = v.astype(np.float32) / np.float32(255.0)
    assert pal.dtype == np.float32
    # monotone in weight order in both modes (the property the rule rests on)
    steps = np.diff(v, axis=1)
    eight = v[:, 0] > v[:, 7]
    assert (steps[eight] <= 0).all() and (steps[~eight] >= 0).all()
    rng = np.random.default_rng(5)
    for lo in range(0, pal.shape[0], 8192):
        p = pal[lo:lo + 8192]
        mids = (p[:, 1:] + p[:, :-1]) * np.float32(0.5)
        cols = [p, mids, np.nextafter(mids, np.float32(0)), np.nextafter(mids, np.float32(1)),
                np.nextafter(p, np.float32(0)), np.nextafter(p, np.float32(1)),
                rng.random((p.shape[0], 16), dtype=np.float32),
                np.broadcast_to(np.array([0.0, 1.0], np.float32), (p.shape[0], 2))]
        x = np.clip(np.concatenate(cols, axis=1), 0, 1).astype(np.float32)
        a, b = _rules(p, x)
        assert np.array_equal(a, b), lo


def test_rule_detects_a_non_monotone_palette():
    # the rule needs monotonicity: on a palette that is not monotone it can differ from the definition
    pal = np.array([[0.1, 0.9, 0.5, 0.5, 0.5, 0.5, 0.5, 0.12]], np.float32)
    x = np.array([[0.11]], np.float32)
    a, b = _rules(pal, x)
    assert a[0, 0] == 0 and b[0, 0] == 7
