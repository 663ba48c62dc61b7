"""CPU FP64 reference of the warm-start MLP (test infrastructure only).

Network: x -> Linear(n_in, h) -> GELU -> Linear(h, h) -> GELU -> Linear(h, n_out), erf-GELU
0.5 z (1 + erf(z / sqrt 2)), mean-squared-error loss, Adam (Kingma & Ba 2015, bias-corrected).

``mirror_bf16=True`` rounds to bfloat16 (round to nearest, ties to even, from float32) at the
points where the device kernels do: the input, the weights, the hidden activations, the output
gradient and the back-propagated pre-activation gradients.  ``mirror_bf16=False`` is the plain
FP64 network, pinned by finite differences in the tests.

Parameter packing (FP32 on the device): [W1 (h x n_in, row-major), b1, W2, b2, W3, b3].
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

__all__ = ["bf16_round", "unpack", "pack", "forward", "loss_and_grads", "adam_step", "init_params"]


def bf16_round(x) -> np.ndarray:
    """float32 -> bfloat16 (RNE), returned as float64 values."""
    x32 = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = x32.view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = np.where(nan, ((u >> 16) | 0x40) << 16, r)
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params, n_in, h, n_out):
    shapes = [(h, n_in), (h,), (h, h), (h,), (n_out, h), (n_out,)]
    out, off = [], 0
    p = np.asarray(params, dtype=np.float64)
    for s in shapes:
        k = int(np.prod(s))
        out.append(p[off:off + k].reshape(s))
        off += k
    assert off == p.size
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(x, dtype=np.float64).ravel() for x in parts])


def _gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def _gelu_d(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(params, x, n_in, h, n_out, mirror_bf16=False):
    r = bf16_round if mirror_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(params, n_in, h, n_out)
    a0 = r(x)
    z1 = a0 @ r(W1).T + b1
    a1 = r(_gelu(z1))
    z2 = a1 @ r(W2).T + b2
    a2 = r(_gelu(z2))
    y = a2 @ r(W3).T + b3
    return dict(a0=a0, z1=z1, a1=a1, z2=z2, a2=a2, y=y)


def loss_and_grads(params, x, t, n_in, h, n_out, mirror_bf16=False):
    r = bf16_round if mirror_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(params, n_in, h, n_out)
    f = forward(params, x, n_in, h, n_out, mirror_bf16)
    d = f["y"] - t
    loss = float(np.mean(d * d))
    dz3 = r(2.0 * d / d.size)
    gW3 = dz3.T @ f["a2"]
    gb3 = dz3.sum(axis=0)
    dz2 = r((dz3 @ r(W3)) * _gelu_d(f["z2"]))
    gW2 = dz2.T @ f["a1"]
    gb2 = dz2.sum(axis=0)
    dz1 = r((dz2 @ r(W2)) * _gelu_d(f["z1"]))
    gW1 = dz1.T @ f["a0"]
    gb1 = dz1.sum(axis=0)
    return loss, pack([gW1, gb1, gW2, gb2, gW3, gb3]), f


def adam_step(params, grads, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grads
    v = b2 * v + (1 - b2) * grads * grads
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(n_in, h, n_out, seed) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases (float32 values)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fan_out, fan_in in ((h, n_in), (h, h), (n_out, h)):
        bound = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-bound, bound, size=(fan_out, fan_in)))
        parts.append(rng.uniform(-bound, bound, size=fan_out))
    return pack(parts).astype(np.float32)
