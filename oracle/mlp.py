"""Float64 reference of the learned combiner (TEST INFRASTRUCTURE).

A fully connected network 16 -> 64 -> 64 -> 1 with ReLU after the two hidden
layers, trained on the mean squared error with Adam (Kingma and Ba, 2015:
bias-corrected first and second moments).  Parameters are one flat vector,
layer by layer, each layer as its weight matrix (out x in, row-major) followed
by its bias.  Plain numpy, no fusion: the reference the GPU kernels are
checked against.
"""
from __future__ import annotations

import numpy as np

SIZES = (16, 64, 64, 1)


_M64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, count: int) -> list[int]:
    """The first ``count`` outputs of SplitMix64 (Steele, Lea and Flood, 2014)
    seeded with ``seed``: the state advances by the golden-ratio increment,
    and each output is the state passed through the generator's mix
    (xor-shift 30, multiply, xor-shift 27, multiply, xor-shift 31)."""
    out, state = [], seed & _M64
    for _ in range(count):
        state = (state + _GAMMA) & _M64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        out.append(z ^ (z >> 31))
    return out


def init(seed: int, sizes=SIZES) -> np.ndarray:
    """Seeded initial parameters (float32): weights of layer i are
    (2u - 1) * sqrt(6 / fan_in_i) (He-uniform), biases 0, where for entry p of
    the packed vector u is the top 24 bits of SplitMix64 output p, over 2^24.
    The product is formed in float64 and rounded to float32 once."""
    total = sum(sizes[i] * sizes[i + 1] + sizes[i + 1] for i in range(len(sizes) - 1))
    draws = splitmix64(seed, total)
    p = np.zeros(total, dtype=np.float64)
    o = 0
    for i in range(len(sizes) - 1):
        fi, fo = sizes[i], sizes[i + 1]
        bound = np.sqrt(6.0 / fi)
        for k in range(fo * fi):
            u = (draws[o + k] >> 40) / float(1 << 24)
            p[o + k] = (2.0 * u - 1.0) * bound
        o += fo * fi + fo
    return p.astype(np.float32)


def unpack(p, sizes=SIZES):
    p = np.asarray(p, dtype=np.float64)
    layers, o = [], 0
    for i in range(len(sizes) - 1):
        fi, fo = sizes[i], sizes[i + 1]
        W = p[o:o + fo * fi].reshape(fo, fi)
        o += fo * fi
        b = p[o:o + fo]
        o += fo
        layers.append((W, b))
    assert o == p.shape[0]
    return layers


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def forward(p, x, sizes=SIZES):
    """Returns the prediction (N,) and the per-layer activations."""
    layers = unpack(p, sizes)
    acts = [np.asarray(x, dtype=np.float64)]
    h = acts[0]
    for i, (W, b) in enumerate(layers):
        z = h @ W.T + b
        h = np.maximum(z, 0.0) if i < len(layers) - 1 else z
        acts.append(h)
    return h[:, 0], acts


def loss(p, x, y, sizes=SIZES):
    yhat, _ = forward(p, x, sizes)
    r = yhat - np.asarray(y, dtype=np.float64)
    return float(np.mean(r * r))


def grad(p, x, y, sizes=SIZES):
    """Gradient of the mean squared error by backpropagation."""
    layers = unpack(p, sizes)
    yhat, acts = forward(p, x, sizes)
    N = acts[0].shape[0]
    g = (2.0 / N) * (yhat - np.asarray(y, dtype=np.float64))[:, None]
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        W, b = layers[i]
        h_in = acts[i]
        grads[i] = (g.T @ h_in, g.sum(axis=0))
        if i > 0:
            g = (g @ W) * (acts[i] > 0.0)
    return pack(grads)


def adam_step(p, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at (1-based) ``step``; returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
