"""Independent closed forms and brute-force quadratures used to pin the oracle.

Nothing here is shared with the oracle or the HIP library: these are textbook
results written out for the tests.
"""
import math

import numpy as np


def triangle_frame(P):
    P = np.asarray(P, float)
    n = np.cross(P[1] - P[0], P[2] - P[0])
    A = 0.5 * np.linalg.norm(n)
    return n / (2 * A), A


def static_potentials(x, P):
    """Potential integrals of a uniform flat triangle (Wilton et al., 1984):
    returns (int 1/R dS,  int grad_y(1/R) dS)  with R = |x - y|.

    For each edge with unit direction t, outward in-plane normal m, endpoint
    coordinates s-/s+ along t measured from the projection x0 of x, signed
    distance d = (P - x0).m and height h:
        f = log((R+ + s+)/(R- + s-)),
        beta = atan(d s+/(R0^2 + |h| R+)) - atan(d s-/(R0^2 + |h| R-)),
        int 1/R = sum_e (d f - |h| beta),
        int grad_y(1/R) = sum_e m f + n sign(h) sum_e beta.
    """
    P = np.asarray(P, float)
    x = np.asarray(x, float)
    n, A = triangle_frame(P)
    h = float((x - P[0]) @ n)
    x0 = x - h * n
    c = P.mean(axis=0)
    s_pot = 0.0
    grad = np.zeros(3)
    beta_sum = 0.0
    for e in range(3):
        a, b = P[e], P[(e + 1) % 3]
        t = (b - a) / np.linalg.norm(b - a)
        m = np.cross(t, n)
        if (c - a) @ m > 0:
            m = -m
        d = float((a - x0) @ m)
        sm, sp = float((a - x0) @ t), float((b - x0) @ t)
        R0sq = d * d + h * h
        Rm, Rp = math.sqrt(sm * sm + R0sq), math.sqrt(sp * sp + R0sq)
        if sm >= 0:
            f = math.log((Rp + sp) / (Rm + sm))
        else:
            f = math.log((Rm - sm) / (Rp - sp))
        beta = math.atan(d * sp / (R0sq + abs(h) * Rp)) - math.atan(d * sm / (R0sq + abs(h) * Rm))
        s_pot += d * f - abs(h) * beta
        grad += m * f
        beta_sum += beta
    grad += n * math.copysign(1.0, h) * beta_sum if h != 0 else 0.0
    return s_pot, grad


def monomial_triangle(P, px, py, pz):
    """Exact integral of x^px y^py z^pz over a flat triangle, via the
    simplex moment formula  int l1^a l2^b l3^c dS = 2A a! b! c!/(a+b+c+2)!
    applied to the multinomial expansion of x = sum_k l_k P_k."""
    P = np.asarray(P, float)
    _, A = triangle_frame(P)
    from itertools import product
    tot = 0.0
    deg = (px, py, pz)
    # expand each coordinate power as products of barycentric terms
    terms = {(0, 0, 0): 1.0}
    for axis, p in enumerate(deg):
        for _ in range(p):
            new = {}
            for key, cf in terms.items():
                for k in range(3):
                    kk = list(key); kk[k] += 1
                    kk = tuple(kk)
                    new[kk] = new.get(kk, 0.0) + cf * P[k, axis]
            terms = new
    for (a, b, c), cf in terms.items():
        tot += cf * 2 * A * math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 2)
    return tot


# 7-point degree-5 rule on the reference triangle (Radon / Strang-Fix)
_S15 = math.sqrt(15.0)
_A1, _A2 = (6 - _S15) / 21, (6 + _S15) / 21
_W1, _W2 = (155 - _S15) / 1200, (155 + _S15) / 1200
_RULE7 = [((1 / 3, 1 / 3, 1 / 3), 9 / 40)]
for a, w in ((_A1, _W1), (_A2, _W2)):
    b = 1 - 2 * a
    _RULE7 += [((a, a, b), w), ((a, b, a), w), ((b, a, a), w)]
RULE7_B = np.array([r[0] for r in _RULE7])
RULE7_W = np.array([r[1] for r in _RULE7])


def subdivide(P, levels):
    """Uniform 4^levels subdivision of a triangle (array [n, 3, 3])."""
    T = np.asarray(P, float)[None]
    for _ in range(levels):
        a, b, c = T[:, 0], T[:, 1], T[:, 2]
        ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
        T = np.concatenate([np.stack([a, ab, ca], 1), np.stack([ab, b, bc], 1),
                            np.stack([ca, bc, c], 1), np.stack([ab, bc, ca], 1)])
    return T


def brute_points(P, levels):
    """Quadrature points and weights from the 7-point rule on a subdivision."""
    T = subdivide(P, levels)
    n = np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0])
    A = 0.5 * np.linalg.norm(n, axis=1)
    Y = np.einsum('qk,tkc->tqc', RULE7_B, T).reshape(-1, 3)
    W = (A[:, None] * RULE7_W[None, :]).reshape(-1)
    return Y, W


def static_first_moment(x, P):
    """int_T (y - x)/R dS: in-plane part by the gradient theorem (grad_s R =
    (y - x0)/R, so it equals sum_e m_e int_e R dl, with
    int sqrt(s^2 + R0^2) ds = [s R + R0^2 log(s + R)]/2), normal part -h int 1/R."""
    P = np.asarray(P, float)
    x = np.asarray(x, float)
    n, A = triangle_frame(P)
    h = float((x - P[0]) @ n)
    x0 = x - h * n
    c = P.mean(axis=0)
    v = np.zeros(3)
    for e in range(3):
        a, b = P[e], P[(e + 1) % 3]
        t = (b - a) / np.linalg.norm(b - a)
        m = np.cross(t, n)
        if (c - a) @ m > 0:
            m = -m
        d = float((a - x0) @ m)
        R0sq = d * d + h * h

        def F(s):
            R = math.sqrt(s * s + R0sq)
            if R0sq == 0.0:
                return 0.5 * s * R
            # log(s + R) written stably for s < 0
            lg = math.log(s + R) if s >= 0 else math.log(R0sq / (R - s))
            return 0.5 * (s * R + R0sq * lg)

        v += m * (F(float((b - x0) @ t)) - F(float((a - x0) @ t)))
    s_pot, _ = static_potentials(x, P)
    return v - h * n * s_pot
