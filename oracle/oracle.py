"""FP64 CPU oracle: conventional marching-on-in-time TDBEM (O1).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product path.  Shares no code
with the HIP library; only the seeded inputs (meshes, pulses) are common.

Follows T. Takahashi, "A fast time-domain boundary element method for
three-dimensional electromagnetic scattering problems":
  * RWG bases (Section 2.2), with the canonical edge order below;
  * J-form coefficients Zt^(g) (Sections 2.3-2.4, Eqs. layer_disc_tmp, testing,
    z_ij, summed over the B-spline weights; the MFIE identity term gives the
    Gram contribution at g = 1, 2);
  * tested incident field (Eq. v_i);
  * the MOT recursion Zt^(1) J^{alpha-1} = V^{alpha-1} - sum_{g>=2} Zt^(g) J^{alpha-g}
    (Eqs. solve and R, rearranged from the Jhat-form by summation by parts).

Canonical RWG edge order (shared interface convention, each side implements
it): edges sorted lexicographically by (lo, hi) vertex index; T+ is the
triangle whose counter-clockwise (outward) vertex order traverses lo -> hi,
T- the one traversing hi -> lo; o+- are the vertices opposite the edge.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def build(force: bool = False) -> str:
    """Compile the C part of the oracle with gcc (-O2, OpenMP)."""
    src = os.path.join(_HERE, "tdbem_oracle.c")
    out = os.path.join(_HERE, "liboracle.so")
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c99",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


def lib():
    global _LIB
    if _LIB is None:
        _LIB = ctypes.CDLL(build())
        d, i, l = ctypes.c_double, ctypes.c_int, ctypes.c_long
        P = ctypes.c_void_p
        _LIB.orc_bspline.restype = d
        _LIB.orc_bspline.argtypes = [i, d]
        _LIB.orc_tri_integrals.argtypes = [P, P, i, d, d, d, d, i, i, P]
        _LIB.orc_zpairs.argtypes = [P, P, P, P, P, d, d, d, d, d, d, l, P, P, i, P, i]
        _LIB.orc_zrows.argtypes = [P, P, i, P, P, P, i, P, d, d, d, d, d, d, i, P, i, P, i, i]
        _LIB.orc_gram.argtypes = [P, P, P, P, P, l, P, P, P]
        _LIB.orc_vinc.argtypes = [P, P, P, P, P, i, P, d, d, d, d, d, d, P]
        _LIB.orc_history.argtypes = [l, P, P, P, P, P, P, i, P, i, i, i, P]
    return _LIB


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# RWG geometry
# --------------------------------------------------------------------------

class Mesh:
    """RWG data of a closed, consistently (outward) oriented triangle mesh."""

    def __init__(self, verts, tris):
        self.xyz = np.ascontiguousarray(verts, dtype=np.float64)
        self.tri = np.ascontiguousarray(tris, dtype=np.int32)
        nt = len(self.tri)
        plus, minus = {}, {}
        for t in range(nt):
            a = self.tri[t]
            for k in range(3):
                u, v = int(a[k]), int(a[(k + 1) % 3])
                w = int(a[(k + 2) % 3])
                if u < v:
                    plus[(u, v)] = (t, w)
                else:
                    minus[(v, u)] = (t, w)
        keys = sorted(plus.keys())
        if set(keys) != set(minus.keys()):
            raise ValueError("mesh is not closed/consistently oriented")
        self.ne = len(keys)
        self.edges = np.array(keys, dtype=np.int32)
        self.etri = np.array([[plus[k][0], minus[k][0]] for k in keys], dtype=np.int32)
        self.efree = np.array([[plus[k][1], minus[k][1]] for k in keys], dtype=np.int32)
        self.elen = np.linalg.norm(self.xyz[self.edges[:, 0]] - self.xyz[self.edges[:, 1]], axis=1)
        P = self.xyz[self.tri]
        n = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
        self.area = 0.5 * np.linalg.norm(n, axis=1)
        self.n_out = n / (2 * self.area[:, None])
        self.centroid = P.mean(axis=1)
        eid = {k: n for n, k in enumerate(keys)}
        self.tedge = np.array([[eid[tuple(sorted((int(a[k]), int(a[(k + 1) % 3]))))] for k in range(3)]
                               for a in self.tri], dtype=np.int32)

    def quad_points(self, t):
        """Interior 3-point rule on triangle t: points and weights (Section 2.4)."""
        P = self.xyz[self.tri[t]]
        B = np.full((3, 3), 1.0 / 6.0) + np.eye(3) * (2.0 / 3.0 - 1.0 / 6.0)
        return B @ P, np.full(3, self.area[t] / 3.0)

    def rwg(self, j, side, x):
        """f_j(x) on T+ (side 0) or T- (side 1) and its surface divergence."""
        t = self.etri[j, side]
        s = (1.0 if side == 0 else -1.0) * self.elen[j] / (2.0 * self.area[t])
        o = self.xyz[self.efree[j, side]]
        return s * (np.asarray(x) - o), 2.0 * s

    def edge_midpoints(self):
        return 0.5 * (self.xyz[self.edges[:, 0]] + self.xyz[self.edges[:, 1]])


# --------------------------------------------------------------------------
# coefficients
# --------------------------------------------------------------------------

def cfie_weights(cfie, zeta):
    """Weights (kd, zeta) of the MFIE's time derivative and of the MFIE in the
    three CFIEs of Section 4.3.1: CFIE1 = dt EFIE + dt MFIE + MFIE (Eq. cfie),
    CFIE2 = dt EFIE + dt MFIE, CFIE3 = dt EFIE + MFIE."""
    if cfie == 1:
        return 1.0, zeta
    if cfie == 2:
        return 1.0, 0.0
    if cfie == 3:
        return 0.0, zeta
    raise ValueError(f"unknown CFIE variant {cfie}")


def material(eps=None, mu=None):
    from oracle.constants import EPS0, MU0
    return (EPS0 if eps is None else eps), (MU0 if mu is None else mu)


def max_lag(mesh: Mesh, cdt: float) -> int:
    ext = np.linalg.norm(mesh.xyz.max(axis=0) - mesh.xyz.min(axis=0))
    return int(math.floor(ext / cdt)) + 4


def zpairs(mesh: Mesh, pi, pj, cdt, theta, zeta, eps=None, mu=None, G=None, nthreads=0, cfie=1):
    """Dense lag strips Zt^(g)_{ij}, g = 0..G-1 (g = 0 unused), for pairs (pi, pj)."""
    eps, mu = material(eps, mu)
    kd, zeta = cfie_weights(cfie, zeta)
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    pj = np.ascontiguousarray(pj, dtype=np.int32)
    if G is None:
        G = max_lag(mesh, cdt) + 1
    out = np.zeros((len(pi), G), dtype=np.float64)
    lib().orc_zpairs(_p(mesh.xyz), _p(mesh.tri), _p(mesh.etri), _p(mesh.efree), _p(mesh.elen),
                     cdt, eps, mu, theta, zeta, kd, len(pi), _p(pi), _p(pj), G, _p(out), nthreads)
    return out


def zrows(mesh: Mesh, rows, cdt, theta, zeta, eps=None, mu=None, G=None, nthreads=0, terms=15, cfie=1):
    """Dense J-form rows out[r, j, g] = Zt^(g)_{rows[r], j}.  ``terms`` selects
    parts of the operator (1 vector, 2 scalar, 4 magnetic potential, 8 MFIE
    identity term) for the pin tests; 15 is the full operator."""
    eps, mu = material(eps, mu)
    kd, zeta = cfie_weights(cfie, zeta)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    if G is None:
        G = max_lag(mesh, cdt) + 1
    out = np.zeros((len(rows), mesh.ne, G))
    lib().orc_zrows(_p(mesh.xyz), _p(mesh.tri), len(mesh.tri), _p(mesh.etri), _p(mesh.efree),
                    _p(mesh.elen), mesh.ne, _p(mesh.tedge), cdt, eps, mu, theta, zeta, kd,
                    len(rows), _p(rows), G, _p(out), nthreads, int(terms))
    return out


def zdense(mesh: Mesh, cdt, theta, zeta, eps=None, mu=None, nthreads=0, chunk=64, cfie=1):
    """All-pairs J-form tensor Z[g, i, j] for the conventional method."""
    ne = mesh.ne
    G = max_lag(mesh, cdt) + 1
    Z = np.zeros((G, ne, ne))
    for r0 in range(0, ne, chunk):
        rows = np.arange(r0, min(ne, r0 + chunk))
        z = zrows(mesh, rows, cdt, theta, zeta, eps, mu, G, nthreads, cfie=cfie)
        Z[:, rows, :] = z.transpose(2, 0, 1)
    return Z


def gram(mesh: Mesh, pi, pj):
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    pj = np.ascontiguousarray(pj, dtype=np.int32)
    out = np.zeros(len(pi))
    lib().orc_gram(_p(mesh.xyz), _p(mesh.tri), _p(mesh.etri), _p(mesh.efree), _p(mesh.elen),
                   len(pi), _p(pi), _p(pj), _p(out))
    return out


def tri_integrals(x, tri3, cdt, dt, zeta, g0, ng, self_term=False, kd=1.0):
    """Kernel integrals over one triangle for one field point, lags g0..g0+ng-1.
    Returns array [ng, 9]: as, phis, ps, av(3), pv(3)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    t = np.ascontiguousarray(tri3, dtype=np.float64).reshape(9)
    out = np.zeros((ng, 9))
    lib().orc_tri_integrals(_p(x), _p(t), int(self_term), cdt, dt, zeta, kd, g0, ng, _p(out))
    return out


def bspline(which, tau):
    return lib().orc_bspline(int(which), float(tau))


def vinc(mesh: Mesh, pulse, t, theta, zeta, eps=None, mu=None, cfie=1):
    """Tested incident field V_i at time t for one pulse (Eq. v_i)."""
    eps, mu = material(eps, mu)
    kd, zeta = cfie_weights(cfie, zeta)
    pa = np.ascontiguousarray(pulse.as_array() if hasattr(pulse, "as_array") else pulse, dtype=np.float64)
    out = np.zeros(mesh.ne)
    lib().orc_vinc(_p(mesh.xyz), _p(mesh.tri), _p(mesh.etri), _p(mesh.efree), _p(mesh.elen),
                   mesh.ne, _p(pa), eps, mu, theta, zeta, kd, float(t), _p(out))
    return out


# --------------------------------------------------------------------------
# conventional MOT march
# --------------------------------------------------------------------------

def march_dense(Z, V, solver="lu"):
    """MOT recursion with a dense J-form tensor Z[g, i, j] and V[alpha-1, i]:
    Zt^(1) J^{alpha-1} = V^{alpha-1} - sum_{g>=2} Zt^(g) J^{alpha-g}.
    Returns J[alpha-1, i] for alpha = 1..len(V)."""
    import scipy.linalg as sla
    G, ne, _ = Z.shape
    nt = V.shape[0]
    lu = sla.lu_factor(Z[1])
    J = np.zeros((nt, ne))
    for a in range(1, nt + 1):
        r = V[a - 1].copy()
        for g in range(2, min(G, a + 1)):
            r -= Z[g] @ J[a - g]
        J[a - 1] = sla.lu_solve(lu, r)
    return J


def history_dense(Z, J, alpha):
    """sum_{g>=2} Zt^(g) J^{alpha-g} for a history J[0..], J^{<0} = 0."""
    G = Z.shape[0]
    out = np.zeros(Z.shape[1])
    for g in range(2, G):
        b = alpha - g
        if 0 <= b < len(J):
            out += Z[g] @ J[b]
    return out


def incident_all(mesh: Mesh, pulse, dt, nt, theta, zeta, eps=None, mu=None, cfie=1):
    """V^{alpha-1} for alpha = 1..nt-1 evaluated at t_alpha = alpha dt."""
    return np.stack([vinc(mesh, pulse, a * dt, theta, zeta, eps, mu, cfie=cfie) for a in range(1, nt)])
