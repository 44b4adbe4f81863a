"""FP64 oracle of the learned radiance cache (test infrastructure only).

A small MLP stands in for the probe query in the target function: the paper
notes that other caches, such as a neural radiance cache, can be targeted by
the same resampling and are interchangeable with DDGI (Sec. 2, Sec. 5).  The
network's shape and training follow the workload definition; everything the
paper leaves open is a reading, stated here:

* input: the surface point y, normalised to [0,1]^3 by the room bounds, and
  its normal n (6 values); encoding per value v: [v, sin(2^j pi v),
  cos(2^j pi v) for j = 0..5] -> 13 values, 78 in total (feature 13*i + e);
* network 78 -> 64 -> 64 -> 64 -> 64 -> 3, ReLU on the hidden layers, linear
  output; the output approximates E(y, n)/pi, a drop-in for the probe query
  Q (clamped at 0 where used);
* parameters flattened as [W1 (64x78, row-major out x in), b1, W2, b2, W3,
  b3, W4, b4, W5 (3x64), b5] -> 17731 values;
* BF16 precision: every GEMM operand (encoded input, weights, hidden
  activations, back-propagated gradients) is rounded to BF16 (nearest even,
  via FP32); accumulation and biases stay FP32/FP64;
* FP8 (inference only): per-layer scales, each the smallest power of two s
  with amax <= 448 s (s_w from amax|W|, s_a from the activation amax
  calibrated on a batch; given activation scales are rounded up to powers
  of two); operands are x / s rounded to OCP E4M3FN (saturated at 448),
  products accumulate exactly and are scaled back by s_w s_a;
* loss: relative L2, mean over samples and channels of
  (y_hat - t)^2 / (sg(y_hat)^2 + 0.01), sg = stop-gradient;
* optimiser: Adam, lr 1e-2, betas (0.9, 0.99), eps 1e-8, FP32/FP64 master
  weights; bias-corrected moments.

Plain numpy; matrix products are library calls, everything else is written
out in the order above.
"""
from __future__ import annotations

import math

import numpy as np

LAYERS = [(78, 64), (64, 64), (64, 64), (64, 64), (64, 3)]     # (in, out)
N_FREQ = 6
N_ENC = 6 * (1 + 2 * N_FREQ)
N_PARAMS = sum(i * o + o for i, o in LAYERS)


# --------------------------------------------------------------------------
# number formats
# --------------------------------------------------------------------------
def to_f32(x):
    return np.asarray(x, np.float64).astype(np.float32)


def round_bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) through float32."""
    f = np.ascontiguousarray(to_f32(x))
    u = f.view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((u >> 16) & 1)
    r = ((u + bias) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def round_fp8_e4m3(x) -> np.ndarray:
    """Round to OCP FP8 E4M3FN (nearest, ties to even), saturating at +-448.
    Normal numbers have 3 mantissa bits and exponents -6..8; below 2^-6 the
    spacing is 2^-9 (subnormals)."""
    x = np.clip(np.asarray(x, np.float64), -448.0, 448.0)
    a = np.abs(x)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, -6.0)
    step = np.exp2(e - 3.0)
    q = a / step
    r = np.floor(q)
    frac = q - r
    up = (frac > 0.5) | ((frac == 0.5) & (np.mod(r, 2.0) == 1.0))
    r = r + up
    return np.sign(x) * np.minimum(r * step, 448.0)


# --------------------------------------------------------------------------
# parameters
# --------------------------------------------------------------------------
def split(params):
    """Views (W_l (out x in), b_l) of a flat parameter vector."""
    out, o = [], 0
    for i, n in LAYERS:
        W = params[o:o + i * n].reshape(n, i)
        o += i * n
        b = params[o:o + n]
        o += n
        out.append((W, b))
    return out


def init_params(seed) -> np.ndarray:
    """He-uniform weights (bound sqrt(6/fan_in)) and zero biases, from a
    seeded generator; an input of the method shared by both implementations."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, n in LAYERS:
        bound = math.sqrt(6.0 / i)
        parts.append(rng.uniform(-bound, bound, n * i))
        parts.append(np.zeros(n))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


def init_params_philox(seed) -> np.ndarray:
    """Initial parameters drawn from Philox: weight p of a layer with fan-in
    F is (2u - 1) * sqrt(6/F) in FP32 arithmetic (each step rounded to FP32),
    u = (x >> 8) 2^-24 from the first word of counter (p, 0, 12, 0); biases
    zero."""
    from . import ref
    out = np.zeros(N_PARAMS, np.float32)
    o = 0
    for i, n in LAYERS:
        bound = np.sqrt(np.float32(6.0) / np.float32(i), dtype=np.float32)
        for q in range(o, o + i * n):
            u = np.float32((int(ref.philox(seed, [q, 0, 12, 0])[0]) >> 8) * 2.0 ** -24)
            out[q] = (np.float32(2.0) * u - np.float32(1.0)) * bound
        o += i * n + n
    return out.astype(np.float64)


# --------------------------------------------------------------------------
# encoding and network
# --------------------------------------------------------------------------
def encode(pos, nrm, lo, hi) -> np.ndarray:
    p = (np.asarray(pos, np.float64) - np.asarray(lo, np.float64)) / \
        (np.asarray(hi, np.float64) - np.asarray(lo, np.float64))
    v = np.concatenate([p, np.asarray(nrm, np.float64)], axis=1)        # (B, 6)
    feats = []
    for i in range(6):
        x = v[:, i]
        feats.append(x)
        for j in range(N_FREQ):
            feats.append(np.sin((2.0 ** j) * math.pi * x))
            feats.append(np.cos((2.0 ** j) * math.pi * x))
    return np.stack(feats, axis=1)                                       # (B, 78)


def pow2_at_least(x) -> float:
    """The smallest power of two >= x (x > 0 finite); 1 otherwise.  Exact:
    the candidate exponent from log2 is corrected by exact comparisons."""
    x = float(x)
    if not (x > 0.0 and math.isfinite(x)):
        return 1.0
    e = math.ceil(math.log2(x))
    while x > math.ldexp(1.0, e):
        e += 1
    while x <= math.ldexp(1.0, e - 1):
        e -= 1
    return math.ldexp(1.0, e)


def fp8_scale(amax) -> float:
    """Per-layer FP8 scale: the smallest power of two s with amax <= 448 s (1
    for an all-zero tensor, which has no range).  Powers of two make the
    ratio of consecutive layers' scales a power of two as well, an exponent
    the matrix instruction applies."""
    amax = float(amax)
    if not (amax > 0.0 and math.isfinite(amax)):
        return 1.0
    e = math.ceil(math.log2(amax / 448.0))
    while amax > 448.0 * math.ldexp(1.0, e):
        e += 1
    while amax <= 448.0 * math.ldexp(1.0, e - 1):
        e -= 1
    return math.ldexp(1.0, e)


def fp8_weight_scales(params):
    """fp8_scale of amax|W| per layer."""
    return [fp8_scale(np.max(np.abs(W))) for W, _ in split(params)]


def forward(params, X, prec="f64", act_scales=None):
    """Returns (output (B, 3), cache).  prec: 'f64', 'bf16' or 'fp8'."""
    layers = split(params)
    h = np.asarray(X, np.float64)
    cache = {"in": [], "pre": []}
    w_scales = fp8_weight_scales(params) if prec == "fp8" else None
    for li, (W, b) in enumerate(layers):
        if prec == "bf16":
            a_in, W_used = round_bf16(h), round_bf16(W)
            z = a_in @ W_used.T + b
        elif prec == "fp8":
            # activation scales as given, rounded up to powers of two
            sa, sw = pow2_at_least(act_scales[li]), w_scales[li]
            a_in = round_fp8_e4m3(h / sa)
            W_used = round_fp8_e4m3(W / sw)
            z = (a_in @ W_used.T) * (sw * sa) + b
        else:
            a_in, W_used = h, W
            z = a_in @ W_used.T + b
        cache["in"].append(a_in)
        cache["pre"].append(z)
        h = z if li == len(layers) - 1 else np.maximum(z, 0.0)
    return h, cache


def act_amax(params, X):
    """Per-layer amax of each layer's input (FP64 forward), for FP8 scales."""
    layers = split(params)
    h = np.asarray(X, np.float64)
    out = []
    for li, (W, b) in enumerate(layers):
        out.append(float(np.max(np.abs(h))))
        z = h @ W.T + b
        h = z if li == len(layers) - 1 else np.maximum(z, 0.0)
    return out


def loss_and_grad_out(out, target, valid=None):
    """Relative L2: mean of (y - t)^2 / (sg(y)^2 + 0.01) over valid samples and
    channels; returns (loss, dloss/dout)."""
    out, target = np.asarray(out, np.float64), np.asarray(target, np.float64)
    w = np.ones(len(out)) if valid is None else np.asarray(valid, np.float64)
    n = max(w.sum(), 1.0) * out.shape[1]
    den = out * out + 0.01
    r = (out - target) ** 2 / den
    loss = float((r * w[:, None]).sum() / n)
    g = 2.0 * (out - target) / den * w[:, None] / n
    return loss, g


def backward(params, cache, g_out, prec="f64"):
    """Gradient of the loss w.r.t. the flat parameters, given dloss/dout.
    With prec='bf16' each back-propagated gradient is rounded to BF16 before it
    enters a product, like the forward operands."""
    layers = split(params)
    grads = [None] * len(layers)
    g = np.asarray(g_out, np.float64)
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        if li < len(layers) - 1:
            g = g * (cache["pre"][li] > 0.0)
        g_used = round_bf16(g) if prec == "bf16" else g
        W_used = round_bf16(W) if prec == "bf16" else W
        dW = g_used.T @ cache["in"][li]
        db = g.sum(axis=0)
        grads[li] = (dW, db)
        g = g_used @ W_used
    return np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])


def adam_step(params, m, v, grad, t, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-8):
    """One bias-corrected Adam step (t counts from 1); returns new arrays."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
