"""FP64 reference of the coarse-grid correction network (TEST INFRASTRUCTURE ONLY).

A multilayer perceptron with three hidden layers of equal width and SiLU activations,
f(z) = z sigmoid(z), mapping per-bin features of a coarse-grid measurement to the
fine-grid correction (see the training driver in the product package). Everything is
written out from the definitions:

  forward   z_l = h_{l-1} W_l + b_l, h_l = f(z_l) for the hidden layers, y = h_3 W_4 + b_4
  loss      L = (1 / (B D)) sum (y - t)^2 (mean squared error over the batch and outputs)
  backward  dy = 2 (y - t) / (B D); dW_l = h_{l-1}^T dz_l; db_l = sum_rows dz_l;
            dh_{l-1} = dz_l W_l^T; dz_{l-1} = dh_{l-1} f'(z_{l-1}),
            f'(z) = s (1 + z (1 - s)), s = sigmoid(z)
  Adam      (Kingma & Ba 2015) m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
            theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

Weights are stored [in, out] (row-major), as the device kernels store them. forward and
backward take an optional rounding of the operands of every product, so that a device
computing in a narrower format (bfloat16 operands, wider accumulation) can be compared
element by element with the same network evaluated in FP64 from the same rounded operands.
"""
from __future__ import annotations

import numpy as np


def init_params(din, dout, width=128, depth=3, seed=0):
    """Uniform(-1/sqrt(in), 1/sqrt(in)) weights and zero biases, FP64."""
    rng = np.random.default_rng(seed)
    dims = [din] + [width] * depth + [dout]
    params = []
    for i in range(len(dims) - 1):
        lim = 1.0 / np.sqrt(dims[i])
        params.append((rng.uniform(-lim, lim, (dims[i], dims[i + 1])), np.zeros(dims[i + 1])))
    return params


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def bf16_round(a):
    """Round to the nearest bfloat16 value (8 significant bits: the sign, the 8 exponent bits
    and the top 7 fraction bits of an IEEE single), ties to even, returned as float64.
    The value is first rounded to float32 (as the device holds it)."""
    f = np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    keep = (u >> 16) & 1                       # lowest kept bit: ties go to the even neighbour
    r = ((u + 0x7FFF + keep) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _identity(a):
    return a


def forward(params, x, operand_round=None):
    """operand_round (optional) is applied to both operands of every product (the input
    or hidden activations and the weights), as a device that multiplies in a narrower
    format does; biases, pre-activations and the output stay in FP64."""
    rnd = operand_round or _identity
    h = np.asarray(x, np.float64)
    cache = [h]
    zs = []
    for i, (W, b) in enumerate(params):
        z = rnd(h) @ rnd(W) + b
        if i < len(params) - 1:
            zs.append(z)
            h = silu(z)
            cache.append(h)
        else:
            h = z
    return h, (cache, zs)


def mse(y, t):
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(params, state, dy, operand_round=None):
    """operand_round (optional) is applied to both operands of every product, as in
    forward; the bias gradients are column sums of the unrounded dz."""
    rnd = operand_round or _identity
    cache, zs = state
    grads = [None] * len(params)
    dz = dy
    for i in range(len(params) - 1, -1, -1):
        W, _ = params[i]
        grads[i] = (rnd(cache[i]).T @ rnd(dz), dz.sum(axis=0))
        if i > 0:
            dz = (rnd(dz) @ rnd(W).T) * silu_grad(zs[i - 1])
    return grads


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of every tensor; m and v are lists like params (updated in place)."""
    out = []
    for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        new = []
        for j, (p, g) in enumerate(((W, gW), (b, gb))):
            m[i][j] = b1 * m[i][j] + (1 - b1) * g
            v[i][j] = b2 * v[i][j] + (1 - b2) * g * g
            mh = m[i][j] / (1 - b1 ** t)
            vh = v[i][j] / (1 - b2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
        out.append(tuple(new))
    return out


def zeros_like_params(params):
    return [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
