"""Interface-variable MLP, FP64 oracle (test infrastructure only).

Not a part of the paper's method: a small network that maps the source
coefficients of a Poisson problem to the interface variable u_Gamma of the
Schur complement system (Section 3, eq. schur) for a fixed geometry and
hidden layer.  Its prediction is only an initial guess for the interface
solve; the exact Schur solve stays the judge.

Network: x -> GELU(W1 x + b1) -> GELU(W2 h1 + b2) -> W3 h2 + b3, with the
exact GELU z Phi(z) (Phi the standard normal CDF; Hendrycks and Gimpel,
arXiv:1606.08415).  Loss: mean squared error over the batch and the output
entries, L = (1 / (B O)) sum (y - t)^2.  Optimiser: Adam (Kingma and Ba,
ICLR 2015) with bias correction.

Flat parameter layout (shared with the GPU library): for every layer its
weight matrix (fan_out x fan_in) column-major, then its bias.  Batches are
row-major (B, features).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def unflatten(flat, dims):
    """[(W, b)] per layer, W of shape (fan_out, fan_in), from the flat vector."""
    flat = np.asarray(flat, dtype=np.float64)
    out, o = [], 0
    for fi, fo in zip(dims[:-1], dims[1:]):
        W = flat[o:o + fo * fi].reshape(fi, fo).T     # column-major storage
        o += fo * fi
        b = flat[o:o + fo]
        o += fo
        out.append((W, b))
    assert o == flat.size
    return out


def flatten(layers):
    parts = []
    for W, b in layers:
        parts.append(np.asarray(W).T.ravel())
        parts.append(np.asarray(b).ravel())
    return np.concatenate(parts)


def forward(layers, X):
    """Network output Y (B, out) and the pre-activations of the hidden layers."""
    h = np.asarray(X, dtype=np.float64)
    zs, hs = [], [h]
    for i, (W, b) in enumerate(layers):
        z = h @ W.T + b
        if i < len(layers) - 1:
            zs.append(z)
            h = gelu(z)
            hs.append(h)
        else:
            h = z
    return h, (zs, hs)


def loss_and_grad(layers, X, T):
    """Mean squared error and its gradient with respect to every (W, b)."""
    Y, (zs, hs) = forward(layers, X)
    B, O = Y.shape
    diff = Y - T
    loss = float(np.sum(diff * diff) / (B * O))
    d = 2.0 * diff / (B * O)                       # dL/dY
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        grads[i] = (d.T @ hs[i], d.sum(axis=0))
        if i > 0:
            d = (d @ W) * gelu_grad(zs[i - 1])
    return loss, grads


class Adam:
    """Adam state over a flat parameter vector."""

    def __init__(self, size, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(size)
        self.v = np.zeros(size)
        self.t = 0
        self.beta1, self.beta2, self.eps = beta1, beta2, eps

    def step(self, theta, g, lr):
        self.t += 1
        b1, b2 = self.beta1, self.beta2
        self.m = b1 * self.m + (1.0 - b1) * g
        self.v = b2 * self.v + (1.0 - b2) * g * g
        mhat = self.m / (1.0 - b1 ** self.t)
        vhat = self.v / (1.0 - b2 ** self.t)
        return theta - lr * mhat / (np.sqrt(vhat) + self.eps)


def cosine_lr(step, total, base=1e-3):
    """Cosine decay from base to 0 over total steps."""
    return 0.5 * base * (1.0 + math.cos(math.pi * min(step, total) / total))
