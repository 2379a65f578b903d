"""Pins of the guess network's inference-precision oracle (oracle/guess_mlp.py):
the bf16 rounding against values fixed by the format (8 significant bits,
round to nearest, ties to even), exactness of the rounded forward pass when
every rounded quantity is already a bf16 value, and the first-order rounding
bound holding on random networks."""
import numpy as np

from oracle import guess_mlp as GM


def test_bf16_rounding_values():
    one = 1.0
    cases = [(one, one), (one + 2 ** -8, one),                  # tie -> even (1.0)
             (one + 3 * 2 ** -8, one + 2 ** -6),                 # tie -> even (1 + 2^-6)
             (one + 2 ** -8 + 2 ** -12, one + 2 ** -7),          # above the tie
             (-(one + 2 ** -7), -(one + 2 ** -7)), (0.0, 0.0),
             (3.0 * 2 ** 100, 3.0 * 2 ** 100), (2 ** -130, 2 ** -130)]   # subnormal float32 with few bits
    for a, b in cases:
        assert GM.bf16(np.array([a]))[0] == b, (a, GM.bf16(np.array([a]))[0], b)


def test_bf16_forward_exact_on_representable_values():
    """Weights, inputs and hidden values that are small dyadic numbers with at
    most 8 significant bits: every rounding is exact, so g_bf16 == g."""
    rng = np.random.default_rng(1)
    q = lambda shape, s: rng.integers(-4, 5, size=shape) * s
    W1 = q((116, 128), 2.0 ** -6); W2 = q((128, 128), 2.0 ** -9)
    b1 = np.zeros(128); b2 = q(128, 2.0 ** -4); w3 = q(128, 2.0 ** -3)
    p = GM.pack(W1, b1, W2, b2, w3, 0.25)
    x = rng.integers(-1, 2, size=(20, 116)) * 0.5
    h1 = np.maximum(x @ W1, 0.0)                         # multiples of 2^-7 below 2^0: exact in bf16
    assert np.array_equal(GM.bf16(h1), h1)
    assert np.array_equal(GM.g_bf16(p, x), GM.g(p, x))


def test_bf16_forward_within_rounding_bound():
    rng = np.random.default_rng(2)
    for trial in range(5):
        p = GM.pack(rng.standard_normal((116, 128)) * np.sqrt(2 / 116), rng.standard_normal(128) * 0.3,
                    rng.standard_normal((128, 128)) * np.sqrt(2 / 128), rng.standard_normal(128) * 0.3,
                    rng.standard_normal(128) / np.sqrt(128), 0.2)
        x = GM.bf16(rng.uniform(-1, 1, size=(64, 116)))
        d = np.abs(GM.g_bf16(p, x) - GM.g(p, x))
        bnd = GM.g_bf16_bound(p, x)
        assert np.all(d <= bnd * (1 + 1e-6)), (d / bnd).max()
        assert d.max() > 0.0                              # the roundings do act
