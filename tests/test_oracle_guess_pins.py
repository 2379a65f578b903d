"""Pins of the learned-guess oracle (CPU): the chain-rule gradient against
central finite differences of the loss, the oddness of g, the cancellation of
b3, and Adam's first step (which moves every parameter by lr g / (|g| + eps), that
is lr times the sign of its gradient up to eps)."""
import numpy as np

from oracle import guess_mlp as M


def _params(rng, scale=1.0):
    W1 = rng.standard_normal((M.NF, M.NH)) * np.sqrt(2 / M.NF) * scale
    W2 = rng.standard_normal((M.NH, M.NH)) * np.sqrt(2 / M.NH) * scale
    return M.pack(W1, rng.standard_normal(M.NH) * 0.3, W2, rng.standard_normal(M.NH) * 0.3,
                  rng.standard_normal(M.NH) / np.sqrt(M.NH), 0.7)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = _params(rng)
    x = rng.standard_normal((9, M.NF))
    y = rng.standard_normal(9) * 0.1
    gr = M.grad(p, x, y)
    # every parameter block, several entries each, central differences
    offs = np.cumsum([0, M.NF * M.NH, M.NH, M.NH * M.NH, M.NH, M.NH])
    idx = np.concatenate([o + rng.choice(n, 6, replace=False) for o, n in
                          zip(offs, [M.NF * M.NH, M.NH, M.NH * M.NH, M.NH, M.NH])] + [[M.NPARAMS - 1]])
    h = 1e-6
    for k in idx:
        e = np.zeros(M.NPARAMS); e[k] = h
        fd = (M.loss(p + e, x, y) - M.loss(p - e, x, y)) / (2 * h)
        assert abs(fd - gr[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, gr[k])


def test_network_is_odd_and_b3_cancels():
    rng = np.random.default_rng(2)
    p = _params(rng)
    x = rng.standard_normal((5, M.NF))
    assert np.allclose(M.g(p, -x), -M.g(p, x), rtol=0, atol=1e-15)
    q = p.copy(); q[-1] += 3.0
    assert np.allclose(M.g(q, x), M.g(p, x), rtol=0, atol=1e-14)
    assert M.grad(p, x, np.zeros(5))[-1] == 0.0
    assert np.all(M.g(np.zeros(M.NPARAMS), x) == 0.0)


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(3)
    p = rng.standard_normal(M.NPARAMS)
    gr = rng.standard_normal(M.NPARAMS)
    q, m, v = M.adam(p, gr, np.zeros_like(p), np.zeros_like(p), 1, lr=1e-2)
    # first step: m_hat = g and v_hat = g^2 exactly, so the move is lr g / (|g| + eps)
    assert np.allclose(p - q, 1e-2 * gr / (np.abs(gr) + 1e-8), rtol=1e-12, atol=0)
