"""Plain CPU IFMM (O2): the fast method's result, step by step, in FP64.

TEST INFRASTRUCTURE ONLY (see oracle.py).  Follows Section 3 of T. Takahashi,
"A fast time-domain boundary element method for three-dimensional
electromagnetic scattering problems":

* space-time hierarchy (Section 3.4.1): a cube around the surface, cells
  subdivided while they hold more than ``leaf_max`` edges (and at least down
  to level 2), empty cells discarded; neighbour lists N(C) and interaction
  lists I(C) (children of the parent's neighbours that do not touch C); steps
  per interval M_t(l_max) = floor(d_s/(c dt)) (the floor reading of Eq. Mt, the
  one Remark 1 and Table 1 need), M_t(l) = 2 M_t(l+1);
* near field (Program 2): exact coefficients for pairs (O, S) at the same level
  with S in N(O) and O or S a leaf;
* far field: the interpolated kernel of Eq. U_expand, MMs by P2M (Eqs. ddotA_M,
  dotphi_fmm, P_fmm) at leaves and re-interpolation (M2M) above, M2L over ALL
  earlier source intervals at the pair's level (the plain definition; the fast
  code uses a finite window), L2L re-interpolation down, tested L2P (Eq. eval,
  with the minus sign of the scalar-potential term of Eq. testing).

Interpolation on p equispaced nodes omega_n = -1 + 2n/(p-1): Lagrange
polynomials in space; in time either Lagrange or the piecewise cubic Hermite
interpolant with finite-difference node slopes (the interpolant the paper takes
from its earlier work; it reproduces quadratics, which the window truncation of
the fast code needs, and is C^1 inside the interval).
Channels: 0-2 vector potential (kernel dU/dt = c d U^{d-1}, d = 2), 3 scalar
potential (U^d), 4-6 magnetic vector potential (U^d, grad_y on the source).

Variants of Section 4.3: the CFIE (CFIE1 of Eq. cfie, CFIE2 = dt EFIE + dt MFIE,
CFIE3 = dt EFIE + MFIE) weights the magnetic channels' target derivative
(kd l_m' + zeta l_m); the second time derivative of the vector potential is
split between kernel and interpolant (dU/dt with l_m', Eq. ddotA_fmm), or put
on the kernel (d^2U/dt^2 = c^2 d (d-1) U^{d-2} with l_m) or on the
interpolant (U with l_m'').
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

W_KAPPA = np.array([0.5, -1.5, 1.5, -0.5])    # w^{kappa,2}, Section 2.2


# ----------------------------------------------------------------- interpolation
def nodes(p):
    return -1.0 + 2.0 * np.arange(p) / (p - 1)


def lagrange(p, xi):
    """Values l_n(xi) and derivatives l_n'(xi) of the p Lagrange cardinal
    polynomials on the equispaced nodes; xi any array, returns [..., p]."""
    w = nodes(p)
    xi = np.asarray(xi, float)[..., None]
    val = np.ones(xi.shape[:-1] + (p,))
    der = np.zeros(xi.shape[:-1] + (p,))
    for n in range(p):
        others = [m for m in range(p) if m != n]
        den = np.prod([w[n] - w[m] for m in others])
        prod = np.ones(xi.shape[:-1])
        for m in others:
            prod = prod * (xi[..., 0] - w[m])
        val[..., n] = prod / den
        d = np.zeros(xi.shape[:-1])
        for k in others:
            t = np.ones(xi.shape[:-1])
            for m in others:
                if m != k:
                    t = t * (xi[..., 0] - w[m])
            d = d + t
        der[..., n] = d / den
    return val, der


def lagrange_d2(p, xi):
    """Second derivatives l_n''(xi) of the Lagrange cardinal polynomials:
    sum over ordered pairs (k, q), k != q, both != n, of prod_{m != n, k, q} (xi - w_m),
    divided by prod_{m != n} (w_n - w_m)."""
    w = nodes(p)
    xi = np.asarray(xi, float)
    out = np.zeros(xi.shape + (p,))
    for n in range(p):
        others = [m for m in range(p) if m != n]
        den = np.prod([w[n] - w[m] for m in others])
        acc = np.zeros(xi.shape)
        for k in others:
            for q in others:
                if q == k:
                    continue
                t = np.ones(xi.shape)
                for m in others:
                    if m != k and m != q:
                        t = t * (xi - w[m])
                acc = acc + t
        out[..., n] = acc / den
    return out


def chi_fd_d2(p, xi):
    """Second derivatives of the CHI-FD cardinal functions: piecewise linear
    and discontinuous at the interior nodes.  At a node (within 1e-9 of a
    segment) the segment on its left is taken, i.e. the limit from the past;
    target steps fall on nodes whenever (p - 1) q / M_t is an integer."""
    w = nodes(p)
    h = w[1] - w[0]
    xi = np.asarray(xi, float)
    seg = np.clip(np.ceil((xi + 1.0) / h - 1e-9).astype(int) - 1, 0, p - 2)
    t = (xi - w[seg]) / h
    ddH = [12 * t - 6, 6 * t - 4, -12 * t + 6, 6 * t - 2]
    out = np.zeros(xi.shape + (p,))
    for n in range(p):
        f = np.zeros(p)
        f[n] = 1.0
        slope = np.zeros(p)
        slope[0] = (-3 * f[0] + 4 * f[1] - f[2]) / (2 * h)
        slope[p - 1] = (3 * f[p - 1] - 4 * f[p - 2] + f[p - 3]) / (2 * h)
        slope[1:p - 1] = (f[2:] - f[:p - 2]) / (2 * h)
        fa, fb, sa, sb = f[seg], f[seg + 1], slope[seg], slope[seg + 1]
        out[..., n] = (ddH[0] * fa + ddH[1] * h * sa + ddH[2] * fb + ddH[3] * h * sb) / (h * h)
    return out


def chi_fd(p, xi):
    """Values and derivatives of the cardinal functions of piecewise cubic
    Hermite interpolation on the p equispaced nodes, with the node slopes taken
    from finite differences of the node values: central at interior nodes,
    second-order one-sided (-3 f0 + 4 f1 - f2) / 2h at the ends.  Points outside
    [-1, 1] use the end pieces.  xi any array, returns [..., p]."""
    w = nodes(p)
    h = w[1] - w[0]
    xi = np.asarray(xi, float)
    seg = np.clip(np.floor((xi + 1.0) / h).astype(int), 0, p - 2)
    t = (xi - w[seg]) / h
    # Hermite basis on the segment and its t-derivative
    H = [2 * t**3 - 3 * t**2 + 1, t**3 - 2 * t**2 + t, -2 * t**3 + 3 * t**2, t**3 - t**2]
    dH = [6 * t**2 - 6 * t, 3 * t**2 - 4 * t + 1, -6 * t**2 + 6 * t, 3 * t**2 - 2 * t]
    val = np.zeros(xi.shape + (p,))
    der = np.zeros(xi.shape + (p,))
    for n in range(p):
        f = np.zeros(p)
        f[n] = 1.0
        slope = np.zeros(p)
        slope[0] = (-3 * f[0] + 4 * f[1] - f[2]) / (2 * h)
        slope[p - 1] = (3 * f[p - 1] - 4 * f[p - 2] + f[p - 3]) / (2 * h)
        slope[1:p - 1] = (f[2:] - f[:p - 2]) / (2 * h)
        fa, fb, sa, sb = f[seg], f[seg + 1], slope[seg], slope[seg + 1]
        val[..., n] = H[0] * fa + H[1] * h * sa + H[2] * fb + H[3] * h * sb
        der[..., n] = (dH[0] * fa + dH[1] * h * sa + dH[2] * fb + dH[3] * h * sb) / h
    return val, der


# ----------------------------------------------------------------- hierarchy
@dataclass
class Cell:
    level: int
    idx: tuple
    edges: list
    parent: int = -1
    children: list = field(default_factory=list)
    leaf: bool = True


class Hierarchy:
    """Octree over edge midpoints and the time intervals of each level."""

    def __init__(self, mesh, cdt, leaf_max, min_level=2, causal_guard=False):
        lo, hi = mesh.xyz.min(axis=0), mesh.xyz.max(axis=0)
        self.side = float((hi - lo).max())
        self.origin = 0.5 * (lo + hi) - 0.5 * self.side
        mid = mesh.edge_midpoints()
        self.rel = (mid - self.origin) / self.side
        self.levels = [[Cell(0, (0, 0, 0), list(range(mesh.ne)))]]
        l = 0
        while True:
            nxt = []
            for ci, c in enumerate(self.levels[l]):
                if len(c.edges) > leaf_max or l < min_level:
                    c.leaf = False
                    groups = {}
                    for e in c.edges:
                        key = tuple(int(v) for v in np.clip(np.floor(self.rel[e] * 2 ** (l + 1)), 0, 2 ** (l + 1) - 1))
                        groups.setdefault(key, []).append(e)
                    for key in sorted(groups):
                        c.children.append(len(nxt))
                        nxt.append(Cell(l + 1, key, groups[key], parent=ci))
            if not nxt:
                break
            self.levels.append(nxt)
            l += 1
        self.lmax = len(self.levels) - 1
        self.index = [{c.idx: i for i, c in enumerate(L)} for L in self.levels]
        # lists
        self.nbr = []
        self.ilist = []
        for l, L in enumerate(self.levels):
            nb, il = [], []
            for c in L:
                nb.append([self.index[l][q] for q in self._around(c.idx, 1) if q in self.index[l]])
                cur = []
                if l >= 2:
                    par = self.levels[l - 1][c.parent]
                    for pn in self.nbr[l - 1][c.parent]:
                        for s in self.levels[l - 1][pn].children:
                            sidx = L[s].idx
                            if max(abs(a - b) for a, b in zip(sidx, c.idx)) > 1:
                                cur.append(s)
                il.append(cur)
            self.nbr.append(nb)
            self.ilist.append(il)
        # time hierarchy
        d_s = self.side / 2 ** self.lmax
        reach = d_s
        if causal_guard:
            # the cell side minus twice the largest distance from an edge midpoint
            # to a point of its basis support (a vertex of its two triangles), so
            # that no far pair can interact within one interval (the paper's
            # Remark 1 takes the cell side alone)
            delta = 0.5 * float(mesh.elen.max())
            for side in (0, 1):
                o = mesh.xyz[mesh.efree[:, side]]
                delta = max(delta, float(np.linalg.norm(o - mid, axis=1).max()))
            reach = d_s - 2.0 * delta
        self.Mt = [0] * (self.lmax + 1)
        self.Mt[self.lmax] = int(math.floor(reach / cdt))
        for l in range(self.lmax - 1, 1, -1):
            self.Mt[l] = 2 * self.Mt[l + 1]

    @staticmethod
    def _around(idx, r):
        for dx in range(-r, r + 1):
            for dy in range(-r, r + 1):
                for dz in range(-r, r + 1):
                    yield (idx[0] + dx, idx[1] + dy, idx[2] + dz)

    def cell_center(self, l, c):
        d = self.side / 2 ** l
        return self.origin + (np.array(self.levels[l][c].idx) + 0.5) * d

    def leaf_of_edge(self):
        out = {}
        for l, L in enumerate(self.levels):
            for ci, c in enumerate(L):
                if c.leaf:
                    for e in c.edges:
                        out[e] = (l, ci)
        return out

    def near_pairs(self):
        """Program 2: (target, source) edge pairs handled by the direct sum."""
        pairs = []
        for l in range(2, self.lmax + 1):
            for oi, O in enumerate(self.levels[l]):
                for si in self.nbr[l][oi]:
                    S = self.levels[l][si]
                    if O.leaf or S.leaf:
                        for i in O.edges:
                            for j in S.edges:
                                pairs.append((i, j))
        return pairs


# ----------------------------------------------------------------- kernels
def kernel_U2(c):
    """d^2 U^d / dt^2 = c^2 d (d - 1) U^{d-2} = 2 c^2 [c(t-s) > r] / r (d = 2)."""
    def k2(r, tau):
        return np.where(c * tau - r > 0.0, 2.0 * c * c / r, 0.0)
    return k2


def kernel_U(c):
    """U^d (d = 2) and dU^d/dt = 2 c (c(t-s) - r)_+ / r (Eq. U)."""
    def k0(r, tau):
        return np.maximum(c * tau - r, 0.0) ** 2 / r

    def k1(r, tau):
        return 2.0 * c * np.maximum(c * tau - r, 0.0) / r
    return k1, k0


# ----------------------------------------------------------------- the method
class IFMM:
    """Far field of the fast TDBEM for a given current history (all-interval M2L)."""

    def __init__(self, mesh, dt, theta, zeta, eps, mu, p_s=4, p_t=4, leaf_max=64, kernels=None,
                 interp_t="lagrange", widen=False, causal_guard=False, cfie=1, dt2="split"):
        self.m = mesh
        # interpolation boxes: the cells, optionally widened by the largest per-axis
        # distance from an edge midpoint to a vertex of the edge's two triangles
        self.delta = 0.0
        if widen:
            mid = 0.5 * (mesh.xyz[mesh.edges[:, 0]] + mesh.xyz[mesh.edges[:, 1]])
            for v in (mesh.edges[:, 0], mesh.edges[:, 1], mesh.efree[:, 0], mesh.efree[:, 1]):
                self.delta = max(self.delta, float(np.abs(mesh.xyz[v] - mid).max()))
        assert interp_t in ("lagrange", "chi")
        self._tcard = (lambda xi: lagrange(self.pt, xi)) if interp_t == "lagrange" else (lambda xi: chi_fd(self.pt, xi))
        self._tcard2 = (lambda xi: lagrange_d2(self.pt, xi)) if interp_t == "lagrange" else (lambda xi: chi_fd_d2(self.pt, xi))
        assert dt2 in ("split", "kernel", "interp")
        self.dt2 = dt2
        # weights of the MFIE's time derivative and of the MFIE (Section 4.3.1)
        self.kd, self.kz = {1: (1.0, zeta), 2: (1.0, 0.0), 3: (0.0, zeta)}[cfie]
        self.c = 1.0 / math.sqrt(eps * mu)
        self.eta = math.sqrt(mu / eps)
        self.dt, self.cdt = dt, self.c * dt
        self.theta, self.zeta, self.eps, self.mu = theta, zeta, eps, mu
        self.ps, self.pt = p_s, p_t
        self.H = Hierarchy(mesh, self.cdt, leaf_max, causal_guard=causal_guard)
        if self.H.Mt[self.H.lmax] < 1:
            raise ValueError("time hierarchy breaks down (M_t = 0, Remark 1)")
        if kernels is None:
            self.k1, self.k0 = kernel_U(self.c)
            self.k2 = kernel_U2(self.c)
        else:
            self.k1, self.k0 = kernels[0], kernels[1]
            self.k2 = kernels[2] if len(kernels) > 2 else None
        self._tables()

    # per-edge P2M and L2P weights at the 3-point rule of both triangles
    def _tables(self):
        m, H, ps = self.m, self.H, self.ps
        leaf = H.leaf_of_edge()
        self.leaf = leaf
        n3 = ps ** 3
        scale = (self.cdt) ** (-2)
        self.Wm = np.zeros((m.ne, 7, n3))    # P2M weights
        self.El = np.zeros((m.ne, 7, n3))    # L2P weights
        for e in range(m.ne):
            l, ci = leaf[e]
            cen = H.cell_center(l, ci)
            hs = H.side / 2 ** l / 2 + self.delta          # node half-width
            for side in (0, 1):
                t = m.etri[e, side]
                X, Wq = m.quad_points(t)
                n_in = -m.n_out[t]
                for x, w in zip(X, Wq):
                    f, div = m.rwg(e, side, x)
                    xi = (x - cen) / hs
                    v, d = lagrange(ps, xi)                 # [3, ps]
                    lb = np.einsum('i,j,k->ijk', v[0], v[1], v[2]).ravel()
                    gb = np.stack([np.einsum('i,j,k->ijk', d[0], v[1], v[2]).ravel(),
                                   np.einsum('i,j,k->ijk', v[0], d[1], v[2]).ravel(),
                                   np.einsum('i,j,k->ijk', v[0], v[1], d[2]).ravel()], axis=1) / hs
                    # P2M (source side): A-dd, phi-dot, P
                    self.Wm[e, 0:3] += w * scale * self.mu / (4 * math.pi) * np.outer(f, lb)
                    self.Wm[e, 3] += w * scale * (-1.0 / (4 * math.pi * self.eps)) * div * lb
                    self.Wm[e, 4:7] += w * scale / (4 * math.pi) * np.cross(f[None, :], gb).T
                    # L2P (test side): f.L, -div L, theta eta f.(n x L) = theta eta L.(f x n)
                    self.El[e, 0:3] += w * np.outer(f, lb)
                    self.El[e, 3] += w * (-div) * lb
                    self.El[e, 4:7] += w * self.theta * self.eta * np.outer(np.cross(f, n_in), lb)

    def _m2m_matrix(self, l, child, parent, h):
        """Parent cardinal functions at the child's nodes (space x time)."""
        H, ps, pt = self.H, self.ps, self.pt
        hs_p = H.side / 2 ** l / 2 + self.delta            # node half-widths
        hs_c = H.side / 2 ** (l + 1) / 2 + self.delta
        cp = H.cell_center(l, parent)
        cc = H.cell_center(l + 1, child)
        w_s, w_t = nodes(ps), nodes(pt)
        S = []
        for ax in range(3):
            v, _ = lagrange(ps, (cc[ax] + hs_c * w_s - cp[ax]) / hs_p)   # [child node, parent node]
            S.append(v)
        Tm, _ = self._tcard(0.5 * w_t + (h - 0.5))                       # [child node, parent node]
        Sp = np.einsum('ia,jb,kc->ijkabc', S[0], S[1], S[2]).reshape(ps ** 3, ps ** 3)
        return np.kron(Sp, Tm)          # [(child b', n'), (parent b, n)]

    # ----------------------------------------------------------------- far field
    def far_history(self, J):
        """Far-field potentials far[alpha-1, i] for alpha = 1..len(J)+1 from the
        history J[beta, i], beta = 0..len(J)-1 (J^{<0} = 0)."""
        m, H = self.m, self.H
        nb = len(J)
        N = nb + 1                                      # target steps 1..N
        Jh = np.zeros((nb, m.ne))
        for b in range(nb):
            for k in range(4):
                if b - k >= 0:
                    Jh[b] += W_KAPPA[k] * J[b - k]
        n3 = self.ps ** 3
        nn = n3 * self.pt
        MM = {}
        # upward: P2M at leaves, M2M above, for every complete interval
        for l in range(H.lmax, 1, -1):
            M = H.Mt[l]
            ht = M * self.dt / 2
            K = nb // M                                  # complete source intervals
            for si, S in enumerate(H.levels[l]):
                mm = np.zeros((K, 7, n3, self.pt))
                if S.leaf:
                    for k in range(K):
                        beta = np.arange(k * M, (k + 1) * M)
                        lt, _ = self._tcard((beta * self.dt - (k + 0.5) * 2 * ht) / ht)   # [beta, n]
                        Tjn = Jh[beta][:, S.edges].T @ lt                                   # [j, n]
                        mm[k] = np.einsum('jcb,jn->cbn', self.Wm[S.edges], Tjn)
                else:
                    for ch in S.children:
                        for h in (0, 1):
                            A = self._m2m_matrix(l, ch, si, h)          # [(b',n'), (b,n)]
                            child = MM[(l + 1, ch)]
                            for k in range(K):
                                kk = 2 * k + h
                                if kk < len(child):
                                    mm[k] += (child[kk].reshape(7, nn) @ A).reshape(7, n3, self.pt)
                MM[(l, si)] = mm
        # downward: all-interval M2L at each level, L2L to children
        far = np.zeros((N, m.ne))
        LCdown = {}
        for l in range(2, H.lmax + 1):
            M = H.Mt[l]
            KT = (N + M - 1) // M                        # target intervals touching steps 1..N
            ncell = len(H.levels[l])
            LC = np.zeros((ncell, KT, 7, nn))
            for oi in range(ncell):
                if (l, oi) in LCdown:
                    LC[oi] += LCdown[(l, oi)][:KT]
            # M2L over every earlier source interval: LC(O, kt) += K(off, kt - ks) MM(S, ks);
            # pairs sharing an offset share the operator, so they are stacked
            groups = {}
            for oi in range(ncell):
                for si in H.ilist[l][oi]:
                    off = tuple(np.array(H.levels[l][si].idx) - np.array(H.levels[l][oi].idx))
                    groups.setdefault(off, []).append((oi, si))
            for off, prs in groups.items():
                O_idx = np.array([p_[0] for p_ in prs])
                S_idx = [p_[1] for p_ in prs]
                # sources interval-major, channel groups apart: [KS, pairs, channels, nn]
                src = np.stack([MM[(l, si)].reshape(-1, 7, nn) for si in S_idx], axis=1)
                KS, np_ = src.shape[0], src.shape[1]
                srcA = np.ascontiguousarray(src[:, :, 0:3])
                srcP = np.ascontiguousarray(src[:, :, 3:7])
                YA = np.zeros((KT, np_, 3, nn))             # this offset's contributions per pair
                YP = np.zeros((KT, np_, 4, nn))
                for lag in range(1, KT):
                    n_k = min(KT - lag, KS)
                    if n_k <= 0:
                        continue
                    K1, K0 = self._m2l_offset(l, np.array(off), lag)
                    # the products of every (interval, pair, channel) as one matrix product each
                    YA[lag:lag + n_k] += (srcA[:n_k].reshape(-1, nn) @ K1.T).reshape(n_k, np_, 3, nn)
                    YP[lag:lag + n_k] += (srcP[:n_k].reshape(-1, nn) @ K0.T).reshape(n_k, np_, 4, nn)
                LC[O_idx, :, 0:3] += YA.transpose(1, 0, 2, 3)
                LC[O_idx, :, 3:7] += YP.transpose(1, 0, 2, 3)
            for oi, O in enumerate(H.levels[l]):
                lc = LC[oi]
                if O.leaf:
                    ht = M * self.dt / 2
                    for kt in range(KT):
                        for a in range(kt * M + 1, (kt + 1) * M + 1):
                            if a > N:
                                continue
                            xi = (a * self.dt - (kt + 0.5) * 2 * ht) / ht
                            v, d = self._tcard(np.array([xi]))
                            v, d = v[0], d[0] / ht
                            dd = self._tcard2(np.array([xi]))[0] / (ht * ht)
                            wa = {"split": d, "kernel": v, "interp": dd}[self.dt2]
                            wp = self.kd * d + self.kz * v
                            L = lc[kt].reshape(7, n3, self.pt)
                            tw = np.stack([wa, wa, wa, v, wp, wp, wp])  # [7, m]
                            Lt = np.einsum('cbm,cm->cb', L, tw)
                            far[a - 1, O.edges] += np.einsum('jcb,cb->j', self.El[O.edges], Lt)
                else:
                    for ch in O.children:
                        acc = LCdown.setdefault((l + 1, ch), np.zeros((2 * KT + 2, 7, nn)))
                        for h in (0, 1):
                            A = self._m2m_matrix(l, ch, oi, h)          # [(a',m'), (a,m)]
                            acc[h:2 * KT + h:2] += lc @ A.T
        return far

    def _m2l_offset(self, l, off, lag):
        """M2L operators (dU/dt and U node values) for a source cell at integer
        offset `off` from the target cell at level l and `lag` intervals back."""
        H, ps, pt = self.H, self.ps, self.pt
        d = H.side / 2 ** l
        hs = d / 2 + self.delta                             # node half-width
        ht = H.Mt[l] * self.dt / 2
        w_s, w_t = nodes(ps), nodes(pt)
        g = np.stack(np.meshgrid(w_s, w_s, w_s, indexing="ij"), -1).reshape(-1, 3) * hs
        xa = g
        yb = off[None, :] * d + g
        r = np.linalg.norm(xa[:, None, :] - yb[None, :, :], axis=2)        # [a, b]
        tau = lag * 2 * ht + ht * (w_t[:, None] - w_t[None, :])            # [m, n]
        R = r[:, None, :, None]
        T = tau[None, :, None, :]
        n_sp = ps ** 3
        K0 = self.k0(R, T).reshape(n_sp * pt, n_sp * pt)
        ka = {"split": self.k1, "kernel": self.k2, "interp": self.k0}[self.dt2]
        KA = ka(R, T).reshape(n_sp * pt, n_sp * pt)     # vector-potential channels
        return KA, K0
