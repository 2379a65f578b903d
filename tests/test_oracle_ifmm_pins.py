"""Pins of the plain IFMM oracle (O2).

* Table 1 of Section 4.1: maximum level and steps per interval of the
  space-time hierarchy for the paper's sphere meshes.
* Program 2 / the interaction lists: near pairs and far pairs (through I(C) at
  exactly one level) cover every (target, source) pair exactly once.
* Polynomial-kernel exactness: with kernels of degree <= 3 in every variable the
  Lagrange interpolation of Eq. U_expand is exact, so the whole chain
  P2M -> M2M -> M2L -> L2L -> L2P must equal a direct double quadrature over
  the same far pairs and earlier source intervals (written here from the
  channel definitions of Eqs. ddotA_M, dotphi_fmm, P_fmm and eval).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from oracle.ifmm import IFMM, Hierarchy, W_KAPPA
from paper_2303_05006_amd.inputs import icosphere, C0, EPS0, MU0

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("case", json.load(open(os.path.join(HERE, "golden", "table1_hierarchy.json")))["cases"])
def test_table1_hierarchy(case):
    v, f = icosphere(case["levels"], 0.5)
    assert len(f) == case["n_triangles"]
    m = O.Mesh(v, f)
    H = Hierarchy(m, 0.005, leaf_max=99)
    assert H.lmax == case["lmax"]
    assert H.Mt[H.lmax] == case["Mt"]


def _far_level(H, leaf, i, j):
    """Level at which the ancestors of i and j are in each other's interaction
    list, or None for a near pair."""
    li, ci = leaf[i]
    lj, cj = leaf[j]
    anc_i = {li: ci}
    for l in range(li, 0, -1):
        anc_i[l - 1] = H.levels[l][anc_i[l]].parent
    anc_j = {lj: cj}
    for l in range(lj, 0, -1):
        anc_j[l - 1] = H.levels[l][anc_j[l]].parent
    for l in range(2, min(li, lj) + 1):
        if anc_j[l] in H.ilist[l][anc_i[l]]:
            return l
    return None


def test_near_far_partition_covers_all_pairs_once():
    v, f = icosphere(2)
    m = O.Mesh(v, f)
    H = Hierarchy(m, 0.05, leaf_max=6)
    assert H.lmax >= 3
    leaf = H.leaf_of_edge()
    near = H.near_pairs()
    assert len(near) == len(set(near))
    near = set(near)
    for i in range(m.ne):
        for j in range(m.ne):
            fl = _far_level(H, leaf, i, j)
            assert (fl is None) == ((i, j) in near), (i, j)
    # lists: neighbours symmetric, interaction lists never touch
    for l in range(2, H.lmax + 1):
        for c in range(len(H.levels[l])):
            for s in H.nbr[l][c]:
                assert c in H.nbr[l][s]
            for s in H.ilist[l][c]:
                d = max(abs(a - b) for a, b in zip(H.levels[l][s].idx, H.levels[l][c].idx))
                assert 2 <= d <= 3


# polynomial kernels in (r^2, tau): degree 2 in every coordinate, 2 in time
P0 = (0.3, -0.7, 1.1, 0.45, 0.2)
P1 = (-0.4, 0.25, 0.6, -0.3, 0.5)
P2 = (0.15, 0.35, -0.8, 0.25, -0.6)


def _poly(cf):
    a0, a1, a2, a3, a4 = cf

    def k(r, tau):
        r2 = r * r
        return a0 + a1 * r2 + a2 * tau + a3 * tau * tau + a4 * r2 * tau
    return k


def test_hermite_interpolant_properties():
    """The temporal CHI-FD cardinal functions: cardinality at the nodes,
    reproduction of polynomials of degree <= 2 (values and derivatives, also
    outside [-1, 1] on the end pieces), continuous derivative at the interior
    nodes, and not reproducing cubics (so the test can tell it from Lagrange)."""
    from oracle.ifmm import chi_fd, nodes
    p = 4
    w = nodes(p)
    v, _ = chi_fd(p, w)
    assert np.allclose(v, np.eye(p), atol=1e-15)
    x = np.linspace(-1.2, 1.2, 97)
    v, d = chi_fd(p, x)
    for c in ([1, 0, 0], [0.3, -1.2, 0], [0.5, 0.7, -2.1]):
        f = c[0] + c[1] * w + c[2] * w**2
        assert np.allclose(v @ f, c[0] + c[1] * x + c[2] * x**2, atol=1e-13)
        assert np.allclose(d @ f, c[1] + 2 * c[2] * x, atol=1e-12)
    eps = 1e-9
    for node in w[1:-1]:
        dl = chi_fd(p, np.array([node - eps]))[1]
        dr = chi_fd(p, np.array([node + eps]))[1]
        assert np.allclose(dl, dr, atol=1e-6)
    assert np.abs(chi_fd(p, x)[0] @ w**3 - x**3).max() > 1e-3


@pytest.mark.parametrize("p", [4, 6])
def test_second_derivatives_of_the_temporal_interpolants(p):
    """l_n'': exact for quadratics (both interpolants; CHI-FD reproduces
    quadratics, so its piecewise-linear second derivative is their constant
    second derivative), for polynomials of degree p-1 (Lagrange), and the
    central difference of l_n' away from the CHI-FD nodes."""
    from oracle.ifmm import chi_fd, chi_fd_d2, lagrange, lagrange_d2, nodes
    w = nodes(p)
    x = np.linspace(-1.1, 1.1, 53) + 1e-3
    c = [0.3, -1.2, 0.7]
    f = c[0] + c[1] * w + c[2] * w ** 2
    assert np.allclose(chi_fd_d2(p, x) @ f, 2 * c[2], atol=1e-11)
    assert np.allclose(lagrange_d2(p, x) @ f, 2 * c[2], atol=1e-11)
    fp = w ** (p - 1)
    assert np.allclose(lagrange_d2(p, x) @ fp, (p - 1) * (p - 2) * x ** (p - 3), atol=1e-10)
    h = 1e-6
    for d2, d1 in ((chi_fd_d2, chi_fd), (lagrange_d2, lagrange)):
        num = (d1(p, x + h)[1] - d1(p, x - h)[1]) / (2 * h)
        assert np.allclose(d2(p, x), num, atol=1e-4)
    # CHI-FD: discontinuous at the interior nodes; a node takes the limit from the left
    for node in w[1:]:
        left, right = chi_fd_d2(p, np.array([node - 1e-7]))[0], chi_fd_d2(p, np.array([node + 1e-7]))[0]
        assert np.allclose(chi_fd_d2(p, np.array([node]))[0], left, atol=1e-5)
        if node < 1.0:
            assert np.abs(left - right).max() > 0.1


@pytest.mark.parametrize("interp_t,widen,cfie,dt2", [("lagrange", False, 1, "split"), ("chi", False, 1, "split"),
                                                   ("chi", True, 1, "split"), ("chi", False, 2, "kernel"),
                                                   ("lagrange", False, 3, "interp"), ("chi", False, 3, "interp")])
def test_polynomial_kernel_exactness(interp_t, widen, cfie, dt2):
    """The CFIE variants weight the magnetic channels' target derivative
    (kd, kz) = (1, zeta), (1, 0), (0, zeta); the second time derivative of the
    vector potential sits on kernel and interpolant (split: kernel P1 with
    d/dt of the interpolant), on the kernel (P2 with the interpolant itself)
    or on the interpolant (P0 with its second derivative, 2 a3)."""
    v, f = icosphere(2)
    m = O.Mesh(v, f)
    dt = 0.03 / C0
    theta, zeta = 1.0, C0 / 2
    F = IFMM(m, dt, theta, zeta, EPS0, MU0, leaf_max=6, kernels=(_poly(P1), _poly(P0), _poly(P2)),
             interp_t=interp_t, widen=widen, cfie=cfie, dt2=dt2)
    kd, kz = {1: (1.0, zeta), 2: (1.0, 0.0), 3: (0.0, zeta)}[cfie]
    assert (F.delta > 0) == widen
    H = F.H
    assert H.lmax >= 3 and H.Mt[H.lmax] >= 3
    nb = 4 * H.Mt[2] + 3
    rng = np.random.default_rng(5)
    J = rng.standard_normal((nb, m.ne))
    far = F.far_history(J)
    # direct double quadrature
    Jh = np.zeros_like(J)
    for b in range(nb):
        for k in range(4):
            if b - k >= 0:
                Jh[b] += W_KAPPA[k] * J[b - k]
    leaf = H.leaf_of_edge()
    eta = math.sqrt(MU0 / EPS0)
    sc = (C0 * dt) ** -2
    a0, a1, a2, a3, a4 = P0
    b0, b1, b2, b3, b4 = P1
    c0, c1, c2, c3, c4 = P2
    targets = list(range(0, m.ne, 29))
    ref = np.zeros((nb + 1, len(targets)))
    avec = np.arange(1, nb + 2)
    bvec = np.arange(nb)
    TAU = (avec[:, None] - bvec[None, :]) * dt                  # [a, beta]
    def side_points(e):
        """The 6 quadrature points of edge e's two triangles: points, weights,
        f_e, div f_e and inward normals, as arrays."""
        P_, W_, F_, D_, N_ = [], [], [], [], []
        for rho in (0, 1):
            t_ = m.etri[e, rho]
            X, W = m.quad_points(t_)
            for x, w in zip(X, W):
                f_, d_ = m.rwg(e, rho, x)
                P_.append(x); W_.append(w); F_.append(f_); D_.append(d_); N_.append(-m.n_out[t_])
        return np.array(P_), np.array(W_), np.array(F_), np.array(D_), np.array(N_)

    pts = [side_points(e) for e in range(m.ne)]
    for ti, i in enumerate(targets):
        xi_, wi_, fi_, di_, ni_ = pts[i]
        for j in range(m.ne):
            l = _far_level(H, leaf, i, j)
            if l is None:
                continue
            M = H.Mt[l]
            # quadrature moments of the pair (6 test x 6 source points): the
            # kernels are polynomials in (r^2, tau)
            yj_, wj_, fj_, dj_, _ = pts[j]
            ww = wi_[:, None] * wj_[None, :]
            d = yj_[None, :, :] - xi_[:, None, :]                    # y - x
            r2 = (d * d).sum(-1)
            ff = fi_ @ fj_.T
            dd = di_[:, None] * dj_[None, :]
            Sff = (ww * ff).sum(); Sffr = (ww * ff * r2).sum()
            Sdd = (ww * dd).sum(); Sddr = (ww * dd * r2).sum()
            # theta eta f_i.(n x ((1/4pi) f_j x (y - x))), times the radial factor below
            fxd = np.cross(fj_[None, :, :], d)
            nxf = np.cross(ni_[:, None, :], fxd)
            SP = theta * eta / (4 * math.pi) * (ww * (fi_[:, None, :] * nxf).sum(-1)).sum()
            # vector potential: (mu/4pi) f_i.f_j d/dt[dU-kernel]; scalar: -div_i (-1/4 pi eps) div_j U-kernel;
            # magnetic: grad_y (d/dt + zeta) K0 = (2 a4 + zeta (2 a1 + 2 a4 tau)) (y - x)
            T = TAU
            if dt2 == "split":
                vec = (b2 + 2 * b3 * T) * Sff + b4 * Sffr
            elif dt2 == "kernel":
                vec = (c0 + c2 * T + c3 * T * T) * Sff + (c1 + c4 * T) * Sffr
            else:
                vec = 2 * a3 * Sff + 0.0 * T
            tot = sc * (MU0 / (4 * math.pi) * vec
                        + 1.0 / (4 * math.pi * EPS0) * ((a0 + a2 * T + a3 * T * T) * Sdd + (a1 + a4 * T) * Sddr)
                        + (kd * 2 * a4 + kz * (2 * a1 + 2 * a4 * T)) * SP)
            mask = bvec[None, :] < ((avec[:, None] - 1) // M) * M            # earlier intervals at level l
            ref[:, ti] += (tot * mask) @ Jh[:, j]
    got = far[:, targets]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < 1e-11, err
