"""Plain numpy reference of the surrogate network -- TEST INFRASTRUCTURE ONLY.

An MLP with GELU hidden layers (GELU in its erf form: z * Phi(z), Hendrycks & Gimpel 2016), the
mean-squared-error loss and one Adam step (Kingma & Ba 2015, Algorithm 1), written out with numpy
matrix products and no blocking or fusion.  Two precisions:

* ``emulate=True`` follows the GPU's number formats: matrix operands rounded to bfloat16 (round to
  nearest even), products accumulated exactly (float64) and rounded to float32 where the GPU stores
  float32 (pre-activations, network output, gradients), hidden activations and backpropagated
  gradients rounded to bfloat16 where the GPU stores them;
* ``emulate=False`` is plain float64 throughout (pinned against central finite differences).

Only ``tests/`` may import this module; it shares no code with the HIP library.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

SQRT1_2 = 0.7071067811865476
INV_SQRT_2PI = 0.3989422804014327


def bf16(x):
    """Round float32 values to the nearest bfloat16 (ties to even); returns float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


def bf16_bits(x):
    """bfloat16 bit patterns (uint16) of float32 values, rounded to nearest even."""
    return (bf16(x).view(np.uint32) >> 16).astype(np.uint16)


def from_bits(h):
    return (np.asarray(h, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + erf(z * SQRT1_2))


def gelu_grad(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + erf(z * SQRT1_2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def init_params(widths, seed):
    """Layer list [(W [out][in], b [out])] with W ~ N(0, 1/in) (float32), b = 0."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(len(widths) - 1):
        W = (rng.standard_normal((widths[i + 1], widths[i])) / np.sqrt(widths[i])).astype(np.float32)
        out.append((W, np.zeros(widths[i + 1], dtype=np.float32)))
    return out


def flatten(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params]).astype(np.float32)


def unflatten(vec, widths):
    out, o = [], 0
    for i in range(len(widths) - 1):
        n, k = widths[i + 1], widths[i]
        W = vec[o:o + n * k].reshape(n, k)
        o += n * k
        b = vec[o:o + n]
        o += n
        out.append((W, b))
    return out


def forward(params, x, emulate=True):
    """Returns (y, acts, zs): the output, the input of every layer and every hidden pre-activation."""
    f = (lambda v: v.astype(np.float32)) if emulate else (lambda v: v)
    a = np.asarray(x, dtype=np.float64)
    acts, zs = [a], [None]
    for i, (W, b) in enumerate(params):
        Wm = bf16(W).astype(np.float64) if emulate else np.asarray(W, dtype=np.float64)
        z = f(a @ Wm.T + np.asarray(b, dtype=np.float64))
        if i + 1 < len(params):
            g = gelu(z)
            a = bf16(g.astype(np.float32)).astype(np.float64) if emulate else g
            acts.append(a)
            zs.append(z)
        else:
            return np.asarray(z, dtype=np.float64), acts, zs
    raise ValueError("empty network")


def mse(y, t, n_valid, emulate=True):
    """(loss, dy): loss over the first n_valid outputs and its gradient with respect to y."""
    B = y.shape[0]
    if emulate:
        y32, t32 = np.asarray(y, np.float32), np.asarray(t, np.float32)
        scale = np.float32(1.0 / (B * n_valid))
        d = y32 - t32
        dy = (np.float32(2.0) * d * scale).astype(np.float32)
        dy[:, n_valid:] = 0.0
        dy = bf16(dy).astype(np.float64)
        loss = float((d[:, :n_valid].astype(np.float64) ** 2).sum() / (B * n_valid))
        return loss, dy
    d = np.asarray(y, np.float64) - np.asarray(t, np.float64)
    loss = float((d[:, :n_valid] ** 2).sum() / (B * n_valid))
    dy = 2.0 * d / (B * n_valid)
    dy[:, n_valid:] = 0.0
    return loss, dy


def backward(params, acts, zs, dy, emulate=True):
    """Gradients [(dW, db)] of the loss whose output gradient is dy."""
    grads = [None] * len(params)
    dz = np.asarray(dy, dtype=np.float64)
    for i in range(len(params) - 1, -1, -1):
        W = params[i][0]
        dW = dz.T @ acts[i]
        db = dz.sum(axis=0)
        if emulate:
            dW, db = dW.astype(np.float32), db.astype(np.float32)
        grads[i] = (dW, db)
        if i == 0:
            break
        Wm = bf16(W).astype(np.float64) if emulate else np.asarray(W, dtype=np.float64)
        da = dz @ Wm
        if emulate:
            da = da.astype(np.float32)
            dz = bf16((da * gelu_grad(zs[i])).astype(np.float32)).astype(np.float64)
        else:
            dz = da * gelu_grad(zs[i])
    return grads


def adam(p, g, m, v, t, lr, b1, b2, eps):
    """One Adam step at step count t (1-based), in float32 as stated by the algorithm."""
    p, g, m, v = (np.asarray(a, np.float32).copy() for a in (p, g, m, v))
    f = np.float32
    m = f(b1) * m + (f(1) - f(b1)) * g
    v = f(b2) * v + (f(1) - f(b2)) * g * g
    bc1, bc2 = f(1.0 - b1 ** t), f(1.0 - b2 ** t)
    p = p - f(lr) * (m / bc1) / (np.sqrt(v / bc2) + f(eps))
    return p, m, v
