"""FP64 oracle of the warm-start network: 3x3 convolutions with GELU,
masked mean-squared-error loss, backpropagation and Adam.

TEST INFRASTRUCTURE ONLY (imported by tests/ and the smoke check), written
from the definitions: a 3x3 cross-correlation with zero padding,
GELU(z) = z * Phi(z) = z/2 (1 + erf(z / sqrt 2)), the loss
L = sum(mask * (y - t)^2) / (4 * sum(mask)) over the four output fields,
reverse-mode differentiation of that composition, and Adam (Kingma & Ba,
2015) with bias correction.  Layout: activations [B][H][W][C] (channels
last); weights W[o][c][dy][dx] applied to input (y + dy - 1, x + dx - 1).

Pins (tests/test_oracle_convnet.py): the convolution against
scipy.signal.correlate, gradients against central finite differences.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x [B][H][W][C], w [O][C][3][3], b [O] -> [B][H][W][O]."""
    B, H, W, C = x.shape
    xp = np.zeros((B, H + 2, W + 2, C))
    xp[:, 1:-1, 1:-1, :] = x
    out = np.zeros((B, H, W, w.shape[0])) + b
    for dy in range(3):
        for dx in range(3):
            patch = xp[:, dy:dy + H, dx:dx + W, :]
            out += np.tensordot(patch, w[:, :, dy, dx], axes=([3], [1]))
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def init_params(c_in: int, width: int = 32, c_out: int = 4, seed: int = 0):
    """He-uniform initial weights, zero biases; list of (w, b) per layer."""
    rng = np.random.default_rng(seed)
    chans = [c_in, width, width, width, c_out]
    params = []
    for i in range(4):
        fan_in = 9 * chans[i]
        lim = math.sqrt(6.0 / fan_in)
        params.append((rng.uniform(-lim, lim, (chans[i + 1], chans[i], 3, 3)),
                       np.zeros(chans[i + 1])))
    return params


def flatten(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def unflatten(flat, c_in: int, width: int = 32, c_out: int = 4):
    chans = [c_in, width, width, width, c_out]
    out, o = [], 0
    for i in range(4):
        nw = chans[i + 1] * chans[i] * 9
        w = flat[o:o + nw].reshape(chans[i + 1], chans[i], 3, 3)
        o += nw
        b = flat[o:o + chans[i + 1]]
        o += chans[i + 1]
        out.append((w, b))
    return out


def forward(params, x):
    """Returns (y, cache): GELU after layers 1-3, linear output layer."""
    cache = {"a": [x], "z": []}
    a = x
    for i, (w, b) in enumerate(params):
        z = conv3x3(a, w, b)
        cache["z"].append(z)
        a = gelu(z) if i < 3 else z
        cache["a"].append(a)
    return a, cache


def loss(y, t, mask):
    """Masked MSE over the four output fields."""
    d = y - t
    m = mask[..., None]
    return float(np.sum(m * d * d) / (4.0 * np.sum(mask)))


def loss_grad(y, t, mask):
    m = mask[..., None]
    return 2.0 * m * (y - t) / (4.0 * np.sum(mask))


def backward(params, cache, dy):
    """Gradients [(dw, db)] of a scalar whose gradient w.r.t. y is dy."""
    grads = [None] * 4
    dz = dy
    for i in range(3, -1, -1):
        w, _ = params[i]
        a_in = cache["a"][i]
        B, H, W, C = a_in.shape
        ap = np.zeros((B, H + 2, W + 2, C))
        ap[:, 1:-1, 1:-1, :] = a_in
        dw = np.zeros_like(w)
        for dyy in range(3):
            for dxx in range(3):
                patch = ap[:, dyy:dyy + H, dxx:dxx + W, :]
                dw[:, :, dyy, dxx] = np.tensordot(dz, patch, axes=([0, 1, 2], [0, 1, 2]))
        db = dz.sum(axis=(0, 1, 2))
        grads[i] = (dw, db)
        if i > 0:
            # d a_in = transposed convolution of dz with w
            dzp = np.zeros((B, H + 2, W + 2, dz.shape[3]))
            dzp[:, 1:-1, 1:-1, :] = dz
            da = np.zeros_like(a_in)
            for dyy in range(3):
                for dxx in range(3):
                    patch = dzp[:, 2 - dyy:2 - dyy + H, 2 - dxx:2 - dxx + W, :]
                    da += np.tensordot(patch, w[:, :, dyy, dxx], axes=([3], [0]))
            dz = da * gelu_grad(cache["z"][i - 1])
    return grads


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of flat arrays p, m, v with gradient g (in place)."""
    m[:] = b1 * m + (1 - b1) * g
    v[:] = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p[:] = p - lr * mh / (np.sqrt(vh) + eps)
    return p
