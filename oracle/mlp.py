"""The MLP trunk (oracle; test infrastructure only).

Paper anchor: small MLPs with sigmoid outputs predicting values in [0,1] (Sec. 3.4, model
configuration).  The workloads built here use one trunk with ReLU hidden layers (the paper's networks
use SELU; a ReLU trunk is the reading used for these workloads):

    h_0 = x,  h_{k+1} = ReLU(W_k h_k + b_k)  (hidden layers),   Y = sigmoid(W_out h + b_out).

Weights are [out][in] float32 arrays, biases [out].  Arithmetic is float64 (``precision="f64"``), or
emulates a reduced-precision matrix path with float64 accumulation:

  * ``"bf16"``: every layer input and every weight rounded to bfloat16 (round-to-nearest-even);
  * ``"fp16"``: the same with IEEE half precision (the paper's network precision);
  * ``"fp8"``: the middle hidden layers (every layer but the first and the head) take E4M3 operands
    with per-layer scales (s_x, s_w): the layer input is rounded to E4M3 as x / s_x, the weight as
    W * (1/s_w) evaluated in float32 (the GPU path's precision for this integer decision), and the
    product is rescaled by s_x * s_w before the bias is added.  The first layer (the grid features)
    and the head (whose outputs decide 8-bit endpoints) take bfloat16 operands as in ``"bf16"``.

FP8 scales (the paper has no FP8 path; this is the reading used here): per layer and per tensor, the
smallest power of two s with max|v| / s <= 448 (the largest finite E4M3 value), so that v / s is exact
and never saturates; s_x from the layer inputs of a float64 forward over calibration rows, s_w from
the layer's weight matrix (biases stay float32).
"""
from __future__ import annotations

import math

import numpy as np

from . import lowp


def sigmoid(z):
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(-z))


def fp8_weight(w, s_w):
    w32 = np.asarray(w, dtype=np.float32)
    inv = np.float32(np.float32(1.0) / np.float32(s_w))
    return lowp.round_e4m3((w32 * inv).astype(np.float64))


def forward(layers, x, precision: str = "f64", scales=None):
    """Returns (Y, cache) for inputs x [n, in].  cache = (inputs h_k, pre-activations z_k)."""
    h = np.asarray(x, dtype=np.float64)
    hs, zs = [], []
    n_layers = len(layers)
    for k, (w, b) in enumerate(layers):
        w = np.asarray(w, dtype=np.float64)
        b = np.asarray(b, dtype=np.float64)
        hs.append(h)
        if precision == "f64":
            z = h @ w.T + b
        elif precision == "bf16":
            z = lowp.round_bf16(h) @ lowp.round_bf16(w).T + b
        elif precision == "fp16":
            z = lowp.round_fp16(h) @ lowp.round_fp16(w).T + b
        elif precision == "fp8" and (k == 0 or k == n_layers - 1):
            z = lowp.round_bf16(h) @ lowp.round_bf16(w).T + b
        elif precision == "fp8":
            s_x, s_w = float(scales[k][0]), float(scales[k][1])
            xq = lowp.round_e4m3(h / s_x)
            wq = fp8_weight(w, s_w)
            z = (xq @ wq.T) * (s_x * s_w) + b
        else:
            raise ValueError(precision)
        zs.append(z)
        h = np.maximum(z, 0.0) if k < n_layers - 1 else sigmoid(z)
    return h, (hs, zs)


def backward(layers, cache, d_y, y, precision: str = "f64"):
    """Gradients (dW list, db list, dx) of a scalar loss given dL/dY (float64), by the chain rule through
    the forward of `cache`: dZ_out = dL/dY * Y (1 - Y); dW_k = dZ_k^T h_k, db_k = sum over rows of dZ_k,
    dh_k = dZ_k W_k, dZ_{k-1} = dh_k * [z_{k-1} > 0].

    ``precision="bf16"`` emulates a backward whose products take bfloat16 operands with float64
    accumulation: every product operand -- dZ_k (in the weight, bias and input products), W_k and h_k --
    rounded to bfloat16 (round-to-nearest-even); the bias gradient sums the rounded dZ_k (it is the
    product of dZ_k with a vector of ones).  The cache is then that of ``forward(..., "bf16")``."""
    hs, zs = cache
    if precision not in ("f64", "bf16"):
        raise ValueError(precision)
    rnd = lowp.round_bf16 if precision == "bf16" else (lambda v: v)
    dz = d_y * y * (1.0 - y)
    dws, dbs = [None] * len(layers), [None] * len(layers)
    for k in range(len(layers) - 1, -1, -1):
        w = rnd(np.asarray(layers[k][0], dtype=np.float64))
        dzr = rnd(dz)
        dws[k] = dzr.T @ rnd(hs[k])
        dbs[k] = dzr.sum(axis=0)
        dh = dzr @ w
        if k > 0:
            dz = dh * (zs[k - 1] > 0)
        else:
            dx = dh
    return dws, dbs, dx


def activation_absmax(layers, x):
    """max |input| of every layer over the rows of x (float64 forward); for FP8 scale calibration."""
    _, (hs, _) = forward(layers, x, "f64")
    return [float(np.abs(h).max()) for h in hs]


E4M3_MAX = 448.0


def pow2_scale(m):
    """The smallest power of two s (down to 2^-126) with m / s <= 448; 1 when m is 0 or not finite."""
    m = float(m)
    if not (m > 0.0 and math.isfinite(m)):
        return 1.0
    e = math.frexp(m)[1] - 9
    while m > math.ldexp(E4M3_MAX, e):
        e += 1
    while e > -126 and m <= math.ldexp(E4M3_MAX, e - 1):
        e -= 1
    return math.ldexp(1.0, e)


def fp8_scales(layers, x):
    """[(s_x, s_w)] per layer for the calibration rows x [n, in]."""
    ax = activation_absmax(layers, x)
    return [(pow2_scale(a), pow2_scale(float(np.abs(np.asarray(w, dtype=np.float32)).max())))
            for a, (w, _) in zip(ax, layers)]
