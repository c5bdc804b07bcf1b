"""Oracle of the surrogate network (FP64, plain NumPy).  Test infrastructure:
only the tests, the smoke check and the benchmark's CPU baseline use it.

A multilayer perceptron n_in -> hidden x n_hidden_layers (GELU) -> n_out
(linear), trained by mean squared error with Adam.  The network, loss and
optimiser are textbook definitions written out directly:
  * GELU(z) = z Phi(z), Phi the standard normal CDF (the exact erf form),
    GELU'(z) = Phi(z) + z phi(z);
  * loss = mean over rows and outputs of (y - t)^2;
  * backward pass by the chain rule, layer by layer;
  * Adam (Kingma and Ba, with bias correction):
      m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
      p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
Parameters are one flat array, layer by layer: W_l as [out][in], then b_l.

`bf16=True` reproduces the rounding points of a bfloat16 product pipeline:
weights, hidden activations and back-propagated gradients are rounded to
bfloat16 (round to nearest even, through float32) where they are stored; the
network input and all accumulation stay in FP64.
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_prime(z):
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def round_bf16(a):
    """Nearest-even rounding of float32(a) to bfloat16, returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def layer_sizes(n_in: int, hidden: int, n_hidden_layers: int, n_out: int) -> List[Tuple[int, int]]:
    """(in, out) of every layer."""
    dims = [n_in] + [hidden] * n_hidden_layers + [n_out]
    return list(zip(dims[:-1], dims[1:]))


def unpack(params, sizes):
    """Views (W_l [out][in], b_l [out]) into the flat parameter array."""
    out, o = [], 0
    for (i, n) in sizes:
        W = params[o:o + n * i].reshape(n, i)
        o += n * i
        b = params[o:o + n]
        o += n
        out.append((W, b))
    assert o == params.size
    return out


def num_params(sizes) -> int:
    return sum(n * (i + 1) for (i, n) in sizes)


def forward(params, sizes, x, bf16=False):
    """Returns the output y [rows][n_out] and the per-layer (input, pre-activation)."""
    x = np.asarray(x, np.float64)
    layers = unpack(np.asarray(params, np.float64), sizes)
    cache = []
    a = x
    for l, (W, b) in enumerate(layers):
        Wq = round_bf16(W) if bf16 else W
        z = a @ Wq.T + b
        cache.append((a, z))
        if l < len(layers) - 1:
            a = gelu(z)
            if bf16:
                a = round_bf16(a)
        else:
            a = z
    return a, cache


def loss_grad(params, sizes, x, t, bf16=False):
    """Mean squared error and its gradient with respect to the flat parameters."""
    y, cache = forward(params, sizes, x, bf16)
    t = np.asarray(t, np.float64)
    count = y.size
    loss = float(((y - t) ** 2).sum() / count)
    dz = 2.0 * (y - t) / count
    if bf16:
        dz = round_bf16(dz)
    layers = unpack(np.asarray(params, np.float64), sizes)
    grads = []
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        a_in, _ = cache[l]
        gW = dz.T @ a_in
        gb = dz.sum(axis=0)
        grads.append((gW, gb))
        if l > 0:
            Wq = round_bf16(W) if bf16 else W
            dz = (dz @ Wq) * gelu_prime(cache[l - 1][1])
            if bf16:
                dz = round_bf16(dz)
    flat = []
    for gW, gb in reversed(grads):
        flat.append(gW.ravel())
        flat.append(gb.ravel())
    return loss, np.concatenate(flat)


class Adam:
    """Adam state over a flat parameter array (FP64)."""

    def __init__(self, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, params, g):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mh = self.m / (1.0 - self.b1 ** self.t)
        vh = self.v / (1.0 - self.b2 ** self.t)
        return params - self.lr * mh / (np.sqrt(vh) + self.eps)


def train(params, sizes, x, t, idx, batch, opt: Adam, bf16=False):
    """Adam steps over the minibatches idx[s*batch:(s+1)*batch]; returns the
    final parameters and the loss of every step."""
    p = np.asarray(params, np.float64).copy()
    idx = np.asarray(idx)
    steps = idx.size // batch
    losses = []
    for s in range(steps):
        rows = idx[s * batch:(s + 1) * batch]
        loss, g = loss_grad(p, sizes, x[rows], t[rows], bf16)
        losses.append(loss)
        p = opt.step(p, g)
    return p, np.array(losses)
