"""FP64 oracle of the warm-start network: a small multilayer perceptron.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  The network maps per-node
features to a correction of the extrapolated initial guess of the Krylov
iteration.  Architecture: dense layers y = x W + b (W of shape fan_in x
fan_out), SiLU activations s(z) = z / (1 + exp(-z)) on hidden layers, linear
output of width 1; loss = mean squared error; optimiser Adam with bias
correction (b1 = 0.9, b2 = 0.999, eps = 1e-8).

Flat parameter order (shared contract with the library's binding): for each
layer l in order, W_l row-major, then b_l.

The paper has no learned component; what this oracle fixes is the
arithmetic of forward, backward and update (pinned by finite differences
and closed forms).  Whether the trained network helps is measured, not
pinned ("parity unpinned" for the network's accuracy).
"""
from __future__ import annotations

import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def layer_shapes(d_in: int, width: int, depth: int):
    dims = [d_in] + [width] * depth + [1]
    return [(dims[i], dims[i + 1]) for i in range(len(dims) - 1)]


def n_params(d_in: int, width: int, depth: int) -> int:
    return sum(a * b + b for a, b in layer_shapes(d_in, width, depth))


def unflatten(theta: np.ndarray, d_in: int, width: int, depth: int):
    out = []
    o = 0
    for a, b in layer_shapes(d_in, width, depth):
        W = theta[o:o + a * b].reshape(a, b)
        o += a * b
        bb = theta[o:o + b]
        o += b
        out.append((W, bb))
    return out


def forward(theta, X, d_in, width, depth):
    """Output (n,) and the cache of pre-activations / activations."""
    layers = unflatten(theta, d_in, width, depth)
    acts = [X]
    pre = []
    h = X
    for li, (W, b) in enumerate(layers):
        z = h @ W + b
        pre.append(z)
        h = silu(z) if li + 1 < len(layers) else z
        acts.append(h)
    return h[:, 0], (acts, pre)


def loss_and_grad(theta, X, T, d_in, width, depth):
    """MSE loss mean((y - t)^2) and its gradient (manual backward)."""
    y, (acts, pre) = forward(theta, X, d_in, width, depth)
    n = X.shape[0]
    r = y - T
    loss = float(np.mean(r * r))
    layers = unflatten(theta, d_in, width, depth)
    grads = []
    dz = (2.0 / n) * r[:, None]
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        h_in = acts[li]
        dW = h_in.T @ dz
        db = dz.sum(axis=0)
        grads.append((dW, db))
        if li > 0:
            dh = dz @ W.T
            dz = dh * silu_grad(pre[li - 1])
    grads.reverse()
    return loss, np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])


class Adam:
    def __init__(self, n, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.b1, self.b2, self.eps = b1, b2, eps

    def step(self, theta, g, lr):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return theta - lr * mh / (np.sqrt(vh) + self.eps)


def init_params(d_in, width, depth, seed=0):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in layer_shapes(d_in, width, depth):
        s = 1.0 / np.sqrt(a)
        parts.append(rng.uniform(-s, s, size=a * b))
        parts.append(np.zeros(b))
    return np.concatenate(parts)
