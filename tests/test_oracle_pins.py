"""Pins of the CPU oracle against closed forms, invariants and brute force.

Every function of the oracle's coefficient computation is checked against
something other than itself: B-spline identities of Section 2.2, exactness of
the 3-point rule of Section 2.4, the RWG divergence and Gram closed forms,
textbook static potential integrals of a triangle (the B-spline partition of
unity turns the sum over lags of every retarded kernel into a static one),
exact full-disk / full-annulus values, and brute-force quadrature.
"""
import math

import numpy as np
import pytest

from closed_forms import static_potentials, static_first_moment, monomial_triangle, brute_points
from oracle import oracle as O
from paper_2303_05006_amd.inputs import icosphere, cube, C0, EPS0, MU0

ETA0 = math.sqrt(MU0 / EPS0)


# ------------------------------------------------------------ B-spline (Sec. 2.2)
def test_bspline_weights_and_values():
    # w^{kappa,2} = 3/prod_{i != kappa}(i - kappa) = (1/2, -3/2, 3/2, -1/2)
    w = [3.0 / np.prod([i - k for i in range(4) if i != k]) for k in range(4)]
    assert np.allclose(w, [0.5, -1.5, 1.5, -0.5])
    assert O.bspline(0, 1.0) == 0.5 and O.bspline(0, 2.0) == 0.5
    assert O.bspline(0, 1.5) == 0.75
    assert O.bspline(1, 1.0) == 1.0 and O.bspline(1, 2.0) == -1.0
    assert O.bspline(-1, 3.0) == 1.0 and O.bspline(-1, 0.0) == 0.0
    # second derivative is the shell function +1, -2, +1
    assert [O.bspline(2, t) for t in (0.5, 1.5, 2.5, 3.5, -0.5)] == [1.0, -2.0, 1.0, 0.0, 0.0]


@pytest.mark.parametrize("x", [0.0, 0.3, 1.0, 2.71, 5.5])
def test_bspline_partition_of_unity(x):
    s0 = sum(O.bspline(0, g - x) for g in range(0, 12))
    s1 = sum(O.bspline(1, g - x) for g in range(0, 12))
    s2 = sum(O.bspline(2, g - x) for g in range(0, 12))
    assert abs(s0 - 1.0) < 1e-14 and abs(s1) < 1e-14 and abs(s2) < 1e-14


def test_bspline_derivatives_by_differences():
    for t in np.linspace(0.05, 2.95, 37):
        h = 1e-6
        d0 = (O.bspline(0, t + h) - O.bspline(0, t - h)) / (2 * h)
        dm = (O.bspline(-1, t + h) - O.bspline(-1, t - h)) / (2 * h)
        assert abs(d0 - O.bspline(1, t)) < 1e-8
        assert abs(dm - O.bspline(0, t)) < 1e-8


# --------------------------------------------------- quadrature, RWG, Gram
def test_three_point_rule_exact_for_quadratics():
    P = np.array([[0.1, 0.2, 0.3], [1.1, -0.3, 0.2], [0.4, 0.8, -0.5]])
    apex = P.mean(axis=0) + 0.7 * np.cross(P[1] - P[0], P[2] - P[0])
    v = np.vstack([P, apex])
    f = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [2, 0, 3]], dtype=np.int32)
    m = O.Mesh(v, f)
    X, W = m.quad_points(0)
    for deg in [(0, 0, 0), (1, 0, 0), (0, 1, 1), (2, 0, 0), (1, 1, 0), (0, 0, 2)]:
        num = sum(w * x[0] ** deg[0] * x[1] ** deg[1] * x[2] ** deg[2] for x, w in zip(X, W))
        assert abs(num - monomial_triangle(P, *deg)) < 1e-14


def test_rwg_divergence_and_normal_flux():
    m = O.Mesh(*icosphere(1))
    for j in range(0, m.ne, 7):
        for side in (0, 1):
            t = m.etri[j, side]
            c = m.centroid[t]
            _, div = m.rwg(j, side, c)
            assert abs(div - (1 if side == 0 else -1) * m.elen[j] / m.area[t]) < 1e-12
        # normal component of f_j across edge j is continuous: f.(m_hat) l = 1 on both sides
        a, b = m.xyz[m.edges[j, 0]], m.xyz[m.edges[j, 1]]
        mid = 0.5 * (a + b)
        fp, _ = m.rwg(j, 0, mid)
        fm, _ = m.rwg(j, 1, mid)
        # each side measured with its own in-plane edge normal, pointing T+ -> T-
        flux = []
        for side, fv in ((0, fp), (1, fm)):
            tt = m.etri[j, side]
            mh = np.cross(b - a, m.n_out[tt]); mh /= np.linalg.norm(mh)
            if (m.centroid[tt] - mid) @ mh > 0:
                mh = -mh          # outward from triangle tt
            flux.append(fv @ mh if side == 0 else -(fv @ mh))
        assert abs(flux[0] - 1.0) < 1e-12 and abs(flux[1] - 1.0) < 1e-12


def test_gram_against_closed_form():
    m = O.Mesh(*icosphere(1))
    rng = np.random.default_rng(0)
    for _ in range(20):
        t = rng.integers(len(m.tri))
        e = m.tedge[t]
        for a in e:
            for b in e:
                sa = 0 if m.etri[a, 0] == t else 1
                sb = 0 if m.etri[b, 0] == t else 1
                P = m.xyz[m.tri[t]]
                oa, ob = m.xyz[m.efree[a, sa]], m.xyz[m.efree[b, sb]]
                ka = (1 if sa == 0 else -1) * m.elen[a] / (2 * m.area[t])
                kb = (1 if sb == 0 else -1) * m.elen[b] / (2 * m.area[t])
                # int (x-oa).(x-ob) = int |x|^2 - (oa+ob).int x + A oa.ob (exact monomials)
                x2 = sum(monomial_triangle(P, *d) for d in [(2, 0, 0), (0, 2, 0), (0, 0, 2)])
                xm = np.array([monomial_triangle(P, *d) for d in [(1, 0, 0), (0, 1, 0), (0, 0, 1)]])
                exact = ka * kb * (x2 - (oa + ob) @ xm + m.area[t] * (oa @ ob))
                if a == b:
                    g = O.gram(m, [a], [b])[0]
                    # the other side's triangle contributes too; compare on this triangle only
                    other = m.etri[a, 1 - sa]
                    P2 = m.xyz[m.tri[other]]
                    o2 = m.xyz[m.efree[a, 1 - sa]]
                    k2 = (1 if sa == 1 else -1) * m.elen[a] / (2 * m.area[other])
                    x2b = sum(monomial_triangle(P2, *d) for d in [(2, 0, 0), (0, 2, 0), (0, 0, 2)])
                    xmb = np.array([monomial_triangle(P2, *d) for d in [(1, 0, 0), (0, 1, 0), (0, 0, 1)]])
                    exact += k2 * k2 * (x2b - 2 * o2 @ xmb + m.area[other] * (o2 @ o2))
                    assert abs(g - exact) < 1e-12 * abs(exact)
                else:
                    g = O.gram(m, [a], [b])[0]
                    assert abs(g - exact) < 1e-12 * max(abs(exact), 1e-3)


# ------------------------------------------------------------ inner integrals
CDT = 0.15
DT = CDT / C0
ZETA = C0 / 2


def _tri():
    return np.array([[0.0, 0.0, 0.0], [0.9, 0.05, 0.02], [0.25, 0.8, -0.04]])


def _sum_over_lags(x, P, self_term=False):
    rmax = max(np.linalg.norm(P - x, axis=1))
    G = int(rmax / CDT) + 4
    r = O.tri_integrals(x, P, CDT, DT, ZETA, 1, G, self_term)
    return r.sum(axis=0), r


def _bary(l1, l2, l3):
    P = _tri()
    return l1 * P[0] + l2 * P[1] + l3 * P[2]


@pytest.mark.parametrize("x,self_term", [
    (np.array([0.3, 0.3, 0.25]), False),      # above the interior
    (np.array([0.3, 0.3, -0.01]), False),     # just below the interior
    (np.array([1.6, -0.7, 0.3]), False),      # far, outside
    (_bary(-0.5, 1.3, 0.2), False),           # in plane, outside
    (_bary(0.4, 0.3, 0.3), True),             # in plane, inside (principal value)
])
def test_lag_sums_equal_static_integrals(x, self_term):
    """Partition of unity: sum_g B(tau_g) = 1, sum_g B' = sum_g B'' = 0, so
    sum_g int B/r = int 1/r, sum_g int B''/r = 0, sum_g int grad(F/r) = zeta int grad(1/r)."""
    P = _tri()
    tot, _ = _sum_over_lags(x, P, self_term)
    s_pot, g_pot = static_potentials(x, P)
    assert abs(tot[1] - s_pot) < 1e-12 * s_pot
    assert abs(tot[0]) < 1e-12 * s_pot / CDT
    assert np.all(np.abs(tot[3:6]) < 1e-12 * s_pot)
    ref = ZETA * g_pot
    if self_term:
        # principal value: the normal part is zero for a field point in the plane
        nrm = np.cross(P[1] - P[0], P[2] - P[0]); nrm /= np.linalg.norm(nrm)
        ref = ref - (ref @ nrm) * nrm
    assert np.allclose(tot[6:9], ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


def _above(l1, l2, l3, h):
    P = _tri()
    n = np.cross(P[1] - P[0], P[2] - P[0]); n /= np.linalg.norm(n)
    return l1 * P[0] + l2 * P[1] + l3 * P[2] + h * n


@pytest.mark.parametrize("x", [
    _above(0.6, 0.4, 0.0, 0.3),      # projection on an edge (subtended angle pi)
    _above(1.3, -0.3, 0.0, -0.2),    # projection on an edge's extension
    _above(1.0, 0.0, 0.0, 0.25),     # projection on a vertex (corner angle)
    _above(0.5, 0.5, 0.0, 0.02),     # close above the edge midpoint
])
def test_lag_sums_static_projection_on_boundary(x):
    P = _tri()
    tot, _ = _sum_over_lags(x, P, False)
    s_pot, g_pot = static_potentials(x, P)
    assert abs(tot[1] - s_pot) < 1e-12 * s_pot
    assert np.allclose(tot[6:9], ZETA * g_pot, rtol=1e-11, atol=1e-11 * np.abs(ZETA * g_pot).max())


def test_full_disk_and_annulus_closed_forms():
    """Field point above the interior with every light-cone circle inside the
    triangle: each lag integral is 2 pi int_{|h|}^{inf} phi(r) r dr in closed form."""
    P = np.array([[-1.0, -1.0, 0.0], [2.0, -1.0, 0.0], [-1.0, 2.0, 0.0]]) * 3
    x = np.array([0.2, 0.1, 0.03])
    cdt = 0.05
    dt = cdt / C0
    h = 0.03
    ng = 6
    r = O.tri_integrals(x, P, cdt, dt, ZETA, 1, ng)
    for gi in range(ng):
        g = gi + 1
        # int B''(tau)/r dS over the plane = 2pi int_h^inf B''(g - r/cdt) dr = 2pi cdt B'(g - h/cdt)
        a_ex = 2 * math.pi * cdt * O.bspline(1, g - h / cdt)
        # int B(tau)/r = 2pi cdt Bint(g - h/cdt)
        p_ex = 2 * math.pi * cdt * O.bspline(-1, g - h / cdt)
        # normal part of int grad(F/r): -h int psi = -h * 2pi[F/r]_h^inf = 2pi F(tau(h))
        F = O.bspline(1, g - h / cdt) / dt + ZETA * O.bspline(0, g - h / cdt)
        assert abs(r[gi, 0] - a_ex) < 1e-12 * max(1.0, abs(a_ex))
        assert abs(r[gi, 1] - p_ex) < 1e-12 * abs(p_ex) + 1e-16
        nz = r[gi, 8]
        assert abs(nz - 2 * math.pi * F) < 1e-10 * max(abs(2 * math.pi * F), 1.0 / dt)
        # in-plane parts vanish by symmetry of full annuli
        assert np.all(np.abs(r[gi, 3:5]) < 1e-12) and np.all(np.abs(r[gi, 6:8]) < 1e-9 / dt)


def _theta_midpoint_scalars(x, P, g, cdt, dt, zeta, n=40000):
    """Brute force: angular midpoint rule about the projected point (no splitting
    at light-cone crossings) with the closed radial antiderivatives."""
    nrm = np.cross(P[1] - P[0], P[2] - P[0]); nrm /= np.linalg.norm(nrm)
    h = (x - P[0]) @ nrm
    x0 = x - h * nrm
    B1 = np.vectorize(lambda t: O.bspline(1, t))
    Bm = np.vectorize(lambda t: O.bspline(-1, t))

    def Q(R):
        tau = g - R / cdt
        return -cdt * B1(tau), -cdt * Bm(tau)

    tot = np.zeros(2)
    for e in range(3):
        a, b = P[e], P[(e + 1) % 3]
        # parametrise the edge and integrate dtheta numerically via the chord
        s = (np.arange(n) + 0.5) / n
        Y = a[None] + s[:, None] * (b - a)[None]
        V = Y - x0
        # signed angle increments between consecutive points on the edge
        Yb = a[None] + (np.arange(n + 1) / n)[:, None] * (b - a)[None]
        Vb = Yb - x0
        cr = np.cross(Vb[:-1], Vb[1:]) @ nrm
        dt_ = np.arctan2(cr, np.einsum('ij,ij->i', Vb[:-1], Vb[1:]))
        R = np.sqrt(np.einsum('ij,ij->i', V, V) + h * h)
        qa, qp = Q(R)
        tot += np.array([(qa * dt_).sum(), (qp * dt_).sum()])
    # subtract Q(|h|) * total angle (2 pi if the projection is inside)
    ins = all(np.cross(P[(e + 1) % 3] - P[e], x0 - P[e]) @ nrm > 0 for e in range(3))
    if ins:
        qa, qp = Q(np.array([abs(h)]))
        tot -= 2 * math.pi * np.array([qa[0], qp[0]])
    return tot


@pytest.mark.parametrize("x,g,self_term", [(np.array([0.3, 0.2, 0.1]), 3, False),
                                           (np.array([0.5, 0.25, -0.05]), 4, False),
                                           (np.array([1.3, 0.6, 0.2]), 7, False),
                                           (_bary(0.5, 0.2, 0.3), 2, True),
                                           (_bary(0.5, 0.2, 0.3), 4, True)])
def test_per_lag_scalars_against_midpoint_brute_force(x, g, self_term):
    P = _tri()
    r = O.tri_integrals(x, P, CDT, DT, ZETA, g, 1, self_term)
    bf = _theta_midpoint_scalars(x, P, g, CDT, DT, ZETA)
    scale = max(abs(r[0, 0]), 1e-3)
    assert abs(r[0, 0] - bf[0]) < 2e-7 * scale
    assert abs(r[0, 1] - bf[1]) < 2e-7 * max(abs(r[0, 1]), 1e-4)


@pytest.mark.parametrize("x", [np.array([0.3, 0.2, 0.1]), np.array([1.0, 0.9, 0.3])])
def test_per_lag_vectors_against_subdivision_brute_force(x):
    """Brute force over a 4^7 subdivision with a degree-5 rule; kernels with
    jumps (B'') converge only to ~1e-3, the smooth ones far better."""
    P = _tri()
    G = int(max(np.linalg.norm(P - x, axis=1)) / CDT) + 4
    r = O.tri_integrals(x, P, CDT, DT, ZETA, 1, G)
    Y, W = brute_points(P, 7)
    R = np.linalg.norm(Y - x, axis=1)
    bf = []
    for g in range(1, G + 1):
        tau = g - R / CDT
        B0 = np.array([O.bspline(0, t) for t in tau])
        B1 = np.array([O.bspline(1, t) for t in tau])
        B2 = np.array([O.bspline(2, t) for t in tau])
        phis = (W * B0 / R).sum()
        av = (W[:, None] * (Y - x) * (B2 / R)[:, None]).sum(0)
        # grad_y(F/r) = (y-x)/r d/dr(F/r),  dF/dr = -(B''/dt + zeta B')/cdt
        F = B1 / DT + ZETA * B0
        dF = -(B2 / DT + ZETA * B1) / CDT
        pv = (W[:, None] * (Y - x) * ((dF / R - F / R ** 2) / R)[:, None]).sum(0)
        bf.append(np.concatenate([[phis], av, pv]))
    bf = np.array(bf)
    ref = np.concatenate([r[:, 1:2], r[:, 3:9]], axis=1)
    sc_phi = np.abs(bf[:, 0]).max()
    sc_av = np.abs(bf[:, 1:4]).max()
    sc_pv = np.abs(bf[:, 4:7]).max()
    assert np.abs(ref[:, 0] - bf[:, 0]).max() <= 1e-6 * sc_phi
    assert np.abs(ref[:, 1:4] - bf[:, 1:4]).max() <= 3e-3 * sc_av
    assert np.abs(ref[:, 4:7] - bf[:, 4:7]).max() <= 3e-3 * sc_pv


# ------------------------------------------------------------ assembled matrix
@pytest.mark.parametrize("mesh", ["ico1", "cube2"])
def test_lag_sum_of_coefficients_is_static_operator(mesh):
    """sum_g Zt^(g)_ij = phi-part with 1/r + theta eta zeta (static n x grad part
    + 1/2 Gram): each piece written from the static closed forms.  The cube has
    coplanar neighbours and projections landing on edge lines."""
    m = O.Mesh(*(icosphere(1) if mesh == "ico1" else cube(2, 2.0)))
    cdt = 0.12
    theta, zeta = 1.0, C0 / 2
    rows = [0, 17, 55]
    Z = O.zrows(m, rows, cdt, theta, zeta)
    tot = Z.sum(axis=2)
    for ri, i in enumerate(rows):
        for j in range(0, m.ne, 3):
            ref = 0.0
            for rho in (0, 1):
                ti = m.etri[i, rho]
                X, W = m.quad_points(ti)
                n_in = -m.n_out[ti]
                for x, w in zip(X, W):
                    fi, divi = m.rwg(i, rho, x)
                    for sg in (0, 1):
                        tj = m.etri[j, sg]
                        P = m.xyz[m.tri[tj]]
                        s_pot, g_pot = static_potentials(x, P)
                        if ti == tj:
                            nrm = m.n_out[tj]
                            g_pot = g_pot - (g_pot @ nrm) * nrm
                        _, divj = m.rwg(j, sg, x)
                        ksj = divj / 2
                        oj = m.xyz[m.efree[j, sg]]
                        Pv = ksj / (4 * math.pi) * np.cross(x - oj, zeta * g_pot)
                        ref += w * (divi * divj * s_pot / (4 * math.pi * EPS0) + theta * ETA0 * fi @ np.cross(n_in, Pv))
            ref += 0.5 * theta * ETA0 * zeta * O.gram(m, [i], [j])[0]
            assert abs(tot[ri, j] - ref) < 1e-10 * np.abs(tot[ri]).max()


def test_second_lag_moment_of_vector_potential_term():
    """Quadratic splines reproduce quadratics, so sum_g g^2 B''(g - x) = 2 for
    every x >= 0; the vector-potential part then collapses to
    2 (mu/4pi) dt^-2 sum_q w_q f_i(x_q) . int f_j / R  (closed form)."""
    m = O.Mesh(*icosphere(1))
    cdt = 0.12
    dt = cdt / C0
    rows = [0, 31]
    Z = O.zrows(m, rows, cdt, 1.0, C0 / 2, terms=1)
    g = np.arange(Z.shape[2], dtype=float)
    mom = (Z * g[None, None, :] ** 2).sum(axis=2)
    for ri, i in enumerate(rows):
        for j in range(0, m.ne, 5):
            ref = 0.0
            for rho in (0, 1):
                ti = m.etri[i, rho]
                X, W = m.quad_points(ti)
                for x, w in zip(X, W):
                    fi, _ = m.rwg(i, rho, x)
                    for sg in (0, 1):
                        tj = m.etri[j, sg]
                        P = m.xyz[m.tri[tj]]
                        s_pot, _ = static_potentials(x, P)
                        mv = static_first_moment(x, P)
                        if ti == tj:
                            nrm = m.n_out[tj]
                            mv = mv - (mv @ nrm) * nrm
                        _, divj = m.rwg(j, sg, x)
                        oj = m.xyz[m.efree[j, sg]]
                        fint = divj / 2 * ((x - oj) * s_pot + mv)
                        ref += w * 2 * MU0 / (4 * math.pi) / dt ** 2 * (fi @ fint)
            assert abs(mom[ri, j] - ref) < 1e-10 * np.abs(mom[ri]).max()


def test_operator_terms_add_up():
    m = O.Mesh(*icosphere(1))
    full = O.zrows(m, [7], 0.12, 1.0, C0 / 2)
    parts = sum(O.zrows(m, [7], 0.12, 1.0, C0 / 2, terms=t) for t in (1, 2, 4, 8))
    assert np.abs(full - parts).max() <= 1e-14 * np.abs(full).max()


def test_pairs_and_rows_agree():
    m = O.Mesh(*icosphere(1))
    rows = np.array([3, 40])
    zr = O.zrows(m, rows, 0.1, 1.0, C0 / 2)
    ii = np.repeat(rows, m.ne); jj = np.tile(np.arange(m.ne), len(rows))
    zp = O.zpairs(m, ii, jj, 0.1, 1.0, C0 / 2, G=zr.shape[2]).reshape(zr.shape)
    assert np.abs(zr - zp).max() <= 1e-14 * np.abs(zp).max()


def test_incident_uniform_field_limit():
    """A very long, unmodulated pulse is uniform over the body: the tested
    field reduces to sum_rho s A (c_T - o) . field  (exact first moments)."""
    from paper_2303_05006_amd.inputs import Pulse
    m = O.Mesh(*icosphere(1))
    p = Pulse(k=(0, 0, 1.0), p=(1.0, 0, 0), E0=1.0, f0=0.0, sigma=1.0, delay=0.0, kind="gauss_plain")
    t = 0.3  # tau ~ 0.3 s: exp varies by ~1e-9 across the body
    theta, zeta = 1.0, 10.0
    V = O.vinc(m, p, t, theta, zeta)
    s = 1.0 / math.sqrt(2 * math.pi)
    g = s * math.exp(-t * t / 2)
    gd = -t * g
    Ed = np.array([gd, 0, 0])
    H = np.cross([0, 0, 1.0], [1.0, 0, 0]) / ETA0 * (gd + zeta * g)
    for i in range(0, m.ne, 11):
        ref = 0.0
        for rho in (0, 1):
            t_ = m.etri[i, rho]
            o = m.xyz[m.efree[i, rho]]
            k = (1 if rho == 0 else -1) * m.elen[i] / (2 * m.area[t_])
            fint = k * m.area[t_] * (m.centroid[t_] - o)
            ref += fint @ (-Ed) + theta * ETA0 * fint @ np.cross(-m.n_out[t_], H)
        assert abs(V[i] - ref) < 1e-7 * abs(ref) + 1e-15


# ------------------------------------------------------- CFIE variants (Section 4.3.1)
def test_cfie_variants_are_the_weighted_parts():
    """CFIE1 = dt EFIE + dt MFIE + MFIE, CFIE2 drops the MFIE, CFIE3 its time
    derivative: the operators and the incident fields are linear in those two
    weights, so CFIE1 = CFIE2 + CFIE3 - EFIE part (vector + scalar potential)."""
    from paper_2303_05006_amd.inputs import gaussian_pulse
    m = O.Mesh(*icosphere(1))
    z = {c: O.zrows(m, [5, 61], 0.12, 1.0, C0 / 2, cfie=c) for c in (1, 2, 3)}
    efie = O.zrows(m, [5, 61], 0.12, 1.0, C0 / 2, terms=3)
    assert np.abs(z[1] - (z[2] + z[3] - efie)).max() <= 1e-13 * np.abs(z[1]).max()
    assert np.abs(z[2] - z[1]).max() > 1e-3 * np.abs(z[1]).max()
    p = gaussian_pulse(60e6, 40e6)
    v = {c: O.vinc(m, p, 2.5e-8, 1.0, C0 / 2, cfie=c) for c in (1, 2, 3)}
    ve = O.vinc(m, p, 2.5e-8, 0.0, C0 / 2)
    assert np.abs(v[1] - (v[2] + v[3] - ve)).max() <= 1e-13 * np.abs(v[1]).max()


@pytest.mark.parametrize("mesh", ["ico1", "cube2"])
def test_cfie_time_derivative_part_first_lag_moment(mesh):
    """The MFIE's time-derivative part alone (CFIE2's magnetic and identity
    terms: kernel B'(tau_g)/(dt r), identity 1/2 theta eta Gram (+1/dt, -1/dt) at
    g = 1, 2) has zero lag sum and first lag moment -1/dt times the static
    operator, because sum_g g B'(g - x) = -1 (B reproduces linear functions):
    sum_g g Zt^(g) = -(1/dt) [theta eta (n x static Biot-Savart part) + 1/2 theta eta Gram]."""
    m = O.Mesh(*(icosphere(1) if mesh == "ico1" else cube(2, 2.0)))
    cdt = 0.12
    dt = cdt / C0
    theta = 1.0
    rows = [3, 40]
    Z = O.zrows(m, rows, cdt, theta, C0 / 2, terms=12, cfie=2)
    g = np.arange(Z.shape[2], dtype=float)
    assert np.abs(Z.sum(axis=2)).max() <= 1e-10 * np.abs(Z).max()
    mom = (Z * g[None, None, :]).sum(axis=2)
    for ri, i in enumerate(rows):
        for j in range(0, m.ne, 4):
            ref = 0.0
            for rho in (0, 1):
                ti = m.etri[i, rho]
                X, W = m.quad_points(ti)
                n_in = -m.n_out[ti]
                for x, w in zip(X, W):
                    fi, divi = m.rwg(i, rho, x)
                    for sg in (0, 1):
                        tj = m.etri[j, sg]
                        P = m.xyz[m.tri[tj]]
                        _, g_pot = static_potentials(x, P)
                        if ti == tj:
                            nrm = m.n_out[tj]
                            g_pot = g_pot - (g_pot @ nrm) * nrm
                        _, divj = m.rwg(j, sg, x)
                        oj = m.xyz[m.efree[j, sg]]
                        Pv = divj / 2 / (4 * math.pi) * np.cross(x - oj, g_pot)
                        ref += w * theta * ETA0 * fi @ np.cross(n_in, Pv)
            ref += 0.5 * theta * ETA0 * O.gram(m, [i], [j])[0]
            ref *= -1.0 / dt
            assert abs(mom[ri, j] - ref) < 1e-10 * np.abs(mom[ri]).max(), (i, j, mom[ri, j], ref)
