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


# ------------------------------------------------------------ inference precision
def bf16(a):
    """Round to the nearest bfloat16 value, ties to even (the 16 low bits of the
    float32 value rounded away), returned as FP64.  Inputs are first rounded
    to float32, as the inference kernel holds them."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def g_bf16(p, x):
    """g(x) with the roundings the inference definition states: the features x
    (already bf16 values), W1, W2 and the first hidden layer rounded to bf16;
    everything else, and every sum, in FP64."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    W1b, W2b = bf16(W1), bf16(W2)
    x = np.asarray(x, dtype=np.float64)

    def o(xx):
        h1 = bf16(relu(xx @ W1b + b1))
        return relu(h1 @ W2b + b2) @ w3 + b3
    return 0.5 * (o(x) - o(-x))


def g_bf16_bound(p, x):
    """First-order bound on |g_bf16(x) - g(x)| per sample, from the three bf16
    roundings (relative error at most u = 2^-9 each; relu is 1-Lipschitz):
      |d a1_k| <= u sum_f |x_f W1_fk|,   |d h1_k| <= |d a1_k| + u |h1_k|,
      |d a2_c| <= sum_k |d h1_k| |W2_kc| + u sum_k |h1_k W2_kc|,
      |d o|    <= sum_c |w3_c| |d a2_c|,  and |d g| <= (|d o(x)| + |d o(-x)|) / 2."""
    u = 2.0 ** -9
    W1, b1, W2, b2, w3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)

    def do(xx):
        h1 = relu(xx @ W1 + b1)
        da1 = u * (np.abs(xx) @ np.abs(W1))
        dh1 = da1 + u * np.abs(h1)
        da2 = dh1 @ np.abs(W2) + u * (np.abs(h1) @ np.abs(W2))
        return da2 @ np.abs(w3)
    return 0.5 * (do(x) + do(-x))
