"""FP64 reference of the surrogate MLP (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark import this module; the GPU surrogate shares no code with it.

Network: widths w_0 -> w_1 -> ... -> w_L, layer l computes
z_l = a_{l-1} W_l^T + b_l with W_l of shape (w_l, w_{l-1}); hidden layers
apply the exact GELU a = z (1 + erf(z / sqrt 2)) / 2, the last layer is
linear.  Loss: mean squared error over all outputs.  Optimiser: Adam with
bias correction.

With ``bf16=True`` the values are rounded to bfloat16 (round to nearest,
ties to even) at the points where the GPU kernels store bfloat16 operands:
the input and every hidden activation before a product, the weights used
in products, and the output-side gradient before the two backward products.
All arithmetic stays FP64, so the emulated reference differs from the GPU
only by FP32 accumulation.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
SQRT2PI = math.sqrt(2.0 * math.pi)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    r = ((u >> 16) & 1) + 0x7FFF
    u2 = ((u + r) & 0xFFFF0000).astype(np.uint32)
    return u2.view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * np.exp(-0.5 * z * z) / SQRT2PI


def init_params(widths, seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases."""
    rng = np.random.default_rng(seed)
    ps = []
    for k, n in zip(widths[:-1], widths[1:]):
        bound = 1.0 / math.sqrt(k)
        ps.append((rng.uniform(-bound, bound, size=(n, k)), rng.uniform(-bound, bound, size=n)))
    return ps


def forward(params, X, bf=False):
    r = bf16 if bf else (lambda v: v)
    a = np.asarray(X, np.float64)
    cache = []
    L = len(params)
    for l, (W, b) in enumerate(params):
        ain = r(a)
        z = ain @ r(W).T + b
        cache.append((ain, z))
        a = gelu(z) if l < L - 1 else z
    return a, cache


def mse(y, t):
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(params, cache, dY, bf=False):
    r = bf16 if bf else (lambda v: v)
    grads = [None] * len(params)
    dz = np.asarray(dY, np.float64)
    for l in range(len(params) - 1, -1, -1):
        W, _b = params[l]
        ain, _z = cache[l]
        g = r(dz)
        grads[l] = (g.T @ ain, dz.sum(axis=0))
        if l > 0:
            da = g @ r(W)
            dz = da * gelu_grad(cache[l - 1][1])
    return grads


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for l, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new = []
            for q, (p, g) in enumerate(((W, gW), (b, gb))):
                m = self.b1 * self.m[l][q] + (1 - self.b1) * g
                v = self.b2 * self.v[l][q] + (1 - self.b2) * g * g
                self.m[l] = (m, self.m[l][1]) if q == 0 else (self.m[l][0], m)
                self.v[l] = (v, self.v[l][1]) if q == 0 else (self.v[l][0], v)
                new.append(p - self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps))
            out.append((new[0], new[1]))
        return out


def flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def unflat(vec, widths):
    ps, o = [], 0
    for k, n in zip(widths[:-1], widths[1:]):
        W = vec[o:o + n * k].reshape(n, k)
        o += n * k
        b = vec[o:o + n]
        o += n
        ps.append((W, b))
    return ps
