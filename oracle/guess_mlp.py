"""FP64 CPU oracle of the learned-guess network (forward, loss, gradient, Adam).

TEST INFRASTRUCTURE ONLY (see oracle.py).  The network is not part of the
paper's method; it proposes the initial vector of the Z0 solve.  Definition:
  o(x) = relu(relu(x W1 + b1) W2 + b2) . w3 + b3,   g(x) = (o(x) - o(-x)) / 2,
with parameters packed as W1 [116][128], b1 [128], W2 [128][128], b2 [128],
w3 [128], b3; training loss L = (1/n) sum_s (g(x_s) - y_s)^2; Adam with bias
correction.  Written out with plain numpy matrix products, one branch at a
time, so that each line can be read against the definition.
"""
from __future__ import annotations

import numpy as np

NF, NH = 116, 128
NPARAMS = NF * NH + NH + NH * NH + NH + NH + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.size == NPARAMS
    o = 0
    W1 = p[o:o + NF * NH].reshape(NF, NH); o += NF * NH
    b1 = p[o:o + NH]; o += NH
    W2 = p[o:o + NH * NH].reshape(NH, NH); o += NH * NH
    b2 = p[o:o + NH]; o += NH
    w3 = p[o:o + NH]; o += NH
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]])


def relu(a):
    return np.maximum(a, 0.0)


def branch(p, x):
    """o(x) for a batch x [n][116]; returns o and the intermediate values."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    a1 = x @ W1 + b1
    h1 = relu(a1)
    a2 = h1 @ W2 + b2
    h2 = relu(a2)
    return h2 @ w3 + b3, (a1, h1, a2, h2)


def g(p, x):
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * (branch(p, x)[0] - branch(p, -x)[0])


def loss(p, x, y):
    return float(np.mean((g(p, x) - np.asarray(y, dtype=np.float64)) ** 2))


def grad(p, x, y):
    """dL/dp by the chain rule, branch by branch."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    W1, b1, W2, b2, w3, b3 = unpack(p)
    n = x.shape[0]
    dg = 2.0 * (g(p, x) - y) / n
    gW1 = np.zeros_like(W1); gb1 = np.zeros_like(b1)
    gW2 = np.zeros_like(W2); gb2 = np.zeros_like(b2)
    gw3 = np.zeros_like(w3)
    for sign in (1.0, -1.0):
        xs = sign * x
        _, (a1, h1, a2, h2) = branch(p, xs)
        do = 0.5 * sign * dg                 # d g / d o(sigma x) = sigma / 2
        gw3 += h2.T @ do
        da2 = (do[:, None] * w3[None, :]) * (a2 > 0)
        gW2 += h1.T @ da2
        gb2 += da2.sum(axis=0)
        da1 = (da2 @ W2.T) * (a1 > 0)
        gW1 += xs.T @ da1
        gb1 += da1.sum(axis=0)
    return pack(gW1, gb1, gW2, gb2, gw3, 0.0)  # b3 cancels in g


def adam(p, gr, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (returns new p, m, v)."""
    m = b1 * m + (1.0 - b1) * gr
    v = b2 * v + (1.0 - b2) * gr * gr
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
