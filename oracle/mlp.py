"""Reference of the learned bucket map: a 1 -> 32 -> 32 -> 1 perceptron read as a
CDF model (double precision forward and backward, Adam, bucket counts).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  The GPU library implements
the same model in its own FP32 kernels; this module is what their gradients,
optimiser steps and bucket ids are checked against.

Model (every weight matrix non-negative, clamp-to-[0,1] activations):
    xn = (x - x0) * xs
    h1 = clamp(w1 * xn + b1)                 (32)
    h2 = clamp(W2 @ h1 + b2)                 (32; W2[j, i] couples h1_i into h2_j)
    y  = clamp(w3 . h2 + b3)
    bucket = min(255, floor(256 * y))
x is the monotone input map of a key: the key rounded to float32, whose bit
pattern read as an unsigned integer is converted to float and scaled by 2^-31.
Each layer is non-decreasing in its input because its weights are non-negative
and clamp is non-decreasing, so the bucket map is non-decreasing in the key.
The clamp's derivative is 1 strictly inside (0, 1) and 0 elsewhere (kinks count
as flat).
"""
from __future__ import annotations

import ctypes

import numpy as np

H = 32
NPARAM = H + H + H * H + H + H + 1      # 1153 trainable values
NBLOCK = NPARAM + 2                      # plus x0, xs
SL = {"w1": slice(0, H), "b1": slice(H, 2 * H), "W2": slice(2 * H, 2 * H + H * H),
      "b2": slice(2 * H + H * H, 3 * H + H * H), "w3": slice(3 * H + H * H, 4 * H + H * H),
      "b3": slice(4 * H + H * H, 4 * H + H * H + 1)}
X0, XS = NPARAM, NPARAM + 1
NONNEG = ("w1", "W2", "w3")


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return (p[SL["w1"]], p[SL["b1"]], p[SL["W2"]].reshape(H, H), p[SL["b2"]], p[SL["w3"]],
            p[SL["b3"]][0], p[X0], p[XS])


def key_to_x(keys: np.ndarray) -> np.ndarray:
    """x(k): float32(k) bits as uint32 -> float32 -> * 2^-31 (all steps float32)."""
    f = np.asarray(keys, dtype=np.uint64).astype(np.float32)
    bits = f.view(np.uint32)
    return (bits.astype(np.float32) * np.float32(2.0 ** -31)).astype(np.float32)


def forward(p, x):
    w1, b1, W2, b2, w3, b3, x0, xs = unpack(p)
    xn = (np.asarray(x, np.float64) - x0) * xs
    a1 = np.outer(xn, w1) + b1
    h1 = np.clip(a1, 0.0, 1.0)
    a2 = h1 @ W2.T + b2
    h2 = np.clip(a2, 0.0, 1.0)
    a3 = h2 @ w3 + b3
    y = np.clip(a3, 0.0, 1.0)
    return y, (xn, a1, h1, a2, h2, a3)


def loss_and_grad(p, x, t):
    """Mean squared error to targets t and its exact gradient (double)."""
    w1, b1, W2, b2, w3, b3, x0, xs = unpack(p)
    y, (xn, a1, h1, a2, h2, a3) = forward(p, x)
    B = len(x)
    r = y - np.asarray(t, np.float64)
    loss = float(np.mean(r * r))
    d3 = (2.0 / B) * r * ((a3 > 0) & (a3 < 1))
    g = np.zeros(NBLOCK)
    g[SL["w3"]] = h2.T @ d3
    g[SL["b3"]] = d3.sum()
    d2 = np.outer(d3, w3) * ((a2 > 0) & (a2 < 1))
    g[SL["W2"]] = (d2.T @ h1).reshape(-1)
    g[SL["b2"]] = d2.sum(axis=0)
    d1 = (d2 @ W2) * ((a1 > 0) & (a1 < 1))
    g[SL["w1"]] = xn @ d1
    g[SL["b1"]] = d1.sum(axis=0)
    return loss, g


def init_params(seed: int, x0: float, xs: float) -> np.ndarray:
    """The untrained model: 32 unit ramps tiling xn in [0, 1] (w1 = 32, b1 = -i),
    second layer close to an average of them, output the mean of the second layer.
    Random parts come from SplitMix64 outputs of the seed, so the GPU reproduces it."""
    p = np.zeros(NBLOCK)
    p[SL["w1"]] = 32.0
    p[SL["b1"]] = -np.arange(H, dtype=np.float64)
    u = splitmix_uniform(seed, H * H + H)
    p[SL["W2"]] = (1.0 + 0.5 * (u[:H * H] - 0.5)) / H
    p[SL["b2"]] = 0.1 * (u[H * H:] - 0.5)
    p[SL["w3"]] = 1.0 / H
    p[SL["b3"]] = 0.0
    p[X0], p[XS] = x0, xs
    return p.astype(np.float32).astype(np.float64)


def splitmix_uniform(seed: int, count: int) -> np.ndarray:
    """count uniforms in [0, 1): top 24 bits of successive SplitMix64 outputs."""
    import oracle
    vals = oracle.splitmix64(seed, count)
    return np.array([(v >> 40) / float(1 << 24) for v in vals])


def lr_groups() -> np.ndarray:
    """Per-parameter step size multiplier: the first layer lives on a 32x larger scale."""
    m = np.ones(NBLOCK)
    m[SL["w1"]] = 32.0
    m[SL["b1"]] = 32.0
    m[X0] = m[XS] = 0.0
    return m


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) with bias correction, then projection of the
    weight matrices onto the non-negative orthant.  step counts from 1."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    p = p - lr * lr_groups() * mh / (np.sqrt(vh) + eps)
    for k in NONNEG:
        p[SL[k]] = np.maximum(p[SL[k]], 0.0)
    return p, m, v


def lr_at(step: int, steps: int, lr: float) -> float:
    """Linear decay from lr to lr/10 over the run."""
    return lr * (1.0 - 0.9 * (step - 1) / max(steps - 1, 1))


def buckets_f32(p, keys: np.ndarray, nb: int = 256) -> np.ndarray:
    """Bucket ids by the scalar FP32 forward of mlp_oracle.c (fused multiply-adds in
    a fixed order): bit-exact with an FP32 implementation of the same steps."""
    import oracle
    L = oracle.lib()
    pf = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.zeros(k.size, dtype=np.int32)
    L.vqo_mlp_bucket_u64(pf.ctypes.data, k.ctypes.data, k.size, nb, out.ctypes.data)
    return out


def forward_f32(p, x: np.ndarray) -> np.ndarray:
    import oracle
    L = oracle.lib()
    pf = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
    xf = np.ascontiguousarray(x, dtype=np.float32)
    y = np.zeros(xf.size, dtype=np.float32)
    L.vqo_mlp_forward_f32(pf.ctypes.data, xf.ctypes.data, xf.size, y.ctypes.data)
    return y


def mid_rank_targets(sorted_keys: np.ndarray) -> np.ndarray:
    """Empirical CDF at each sample: (first + last + 1) / 2 / m over its run of
    equal keys (equal keys share one target)."""
    s = np.asarray(sorted_keys)
    m = s.size
    first = np.searchsorted(s, s, side="left")
    last = np.searchsorted(s, s, side="right") - 1
    return (first + last + 1) / 2.0 / m


def balance(counts: np.ndarray, n: int) -> dict:
    e = n / counts.size
    return {"max_over_expected": float(counts.max() / e),
            "rms_rel_dev": float(np.sqrt(np.mean((counts / e - 1.0) ** 2)))}
