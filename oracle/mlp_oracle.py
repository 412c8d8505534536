"""Plain FP64 reference of the learned viscosity closure: a multilayer
perceptron 3 -> 64 -> 64 -> 1 with SiLU activations (x sigma(x)), trained
with mean-squared error and Adam.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` (and the benchmark's CPU
leg).  Shares no code with the HIP library.

Parameter vector of one member (length 4481), in this order:
W1 [64][3], b1 [64], W2 [64][64], b2 [64], W3 [64], b3 [1]; the hidden
layers compute z1 = W1 x + b1, h1 = silu(z1), z2 = W2 h1 + b2,
h2 = silu(z2), y = W3 . h2 + b3.

``bf16=True`` evaluates the same network as the device does: the weights
W1, W2, W3 and the first hidden layer h1 (the operand of the 64 x 64
product) rounded to bfloat16 (round to nearest even), everything else in
FP64.  The backward pass likewise rounds the operands the device rounds
(dz2 and h1 for the W2 gradient, dz2 and W2 for the h1 gradient).
"""
from __future__ import annotations

import numpy as np

H = 64
NIN = 3
SIZES = [("W1", (H, NIN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, k = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = p[k:k + n].reshape(shape)
        k += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(rng, members):
    """He-uniform weights, zero biases (the random numbers are the caller's)."""
    ps = []
    for _ in range(members):
        d = {}
        for name, shape in SIZES:
            if name.startswith("W"):
                fan_in = shape[-1] if len(shape) == 2 else H
                lim = np.sqrt(6.0 / fan_in)
                d[name] = rng.uniform(-lim, lim, size=shape)
            else:
                d[name] = np.zeros(shape)
        ps.append(pack(d))
    return np.array(ps)


def forward(p, x, bf16_ops=False, keep=False):
    """y for inputs x [n][3] (already normalised)."""
    d = unpack(p)
    W1, W2, W3 = d["W1"], d["W2"], d["W3"]
    if bf16_ops:
        W1, W2, W3 = bf16(W1), bf16(W2), bf16(W3)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1.T + d["b1"]
    h1 = silu(z1)
    h1o = bf16(h1) if bf16_ops else h1
    z2 = h1o @ W2.T + d["b2"]
    h2 = silu(z2)
    y = h2 @ W3 + d["b3"][0]
    if keep:
        return y, dict(x=x, z1=z1, h1=h1o, z2=z2, h2=h2, W1=W1, W2=W2, W3=W3)
    return y


def loss_and_grad(p, x, t, bf16_ops=False):
    """Mean squared error over the batch and its gradient (backpropagation)."""
    y, c = forward(p, x, bf16_ops, keep=True)
    n = len(y)
    r = y - np.asarray(t, dtype=np.float64)
    L = float(np.mean(r * r))
    dy = 2.0 * r / n
    g = {}
    g["W3"] = dy @ c["h2"]
    g["b3"] = np.array([dy.sum()])
    dz2 = np.outer(dy, c["W3"]) * dsilu(c["z2"])
    dz2o = bf16(dz2) if bf16_ops else dz2
    g["W2"] = dz2o.T @ c["h1"]
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2o @ c["W2"]
    dz1 = dh1 * dsilu(c["z1"])
    g["W1"] = dz1.T @ c["x"]
    g["b1"] = dz1.sum(axis=0)
    return L, pack(g)


class Adam:
    """Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
    p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""

    def __init__(self, p, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.p = np.array(p, dtype=np.float64)
        self.m = np.zeros_like(self.p)
        self.v = np.zeros_like(self.p)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        self.p = self.p - self.lr * mh / (np.sqrt(vh) + self.eps)
        return self.p
