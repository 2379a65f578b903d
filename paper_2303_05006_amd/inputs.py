"""Seeded synthetic inputs shared by the HIP path, the oracle and the tests.

This module holds geometry and parameter generators only: surface meshes
(vertex coordinates and outward counter-clockwise triangles), incident-pulse
descriptors and sets of incidence directions.  It performs none of the
boundary-element arithmetic (no basis functions, no kernels, no integrals), so
that the HIP library and the CPU oracle can both consume its output without
sharing any of the method's code.

Workloads follow the shapes of the paper's test problem (a PEC sphere meshed
by a subdivided icosahedron, Section 4.1 and Table 1) and of the project
configurations (structured cube, ellipsoid, batched incidence directions).
All units are SI.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

C0 = 299792458.0                     # speed of light in vacuum [m/s]
MU0 = 4.0e-7 * math.pi               # vacuum permeability [H/m] (classical value)
EPS0 = 1.0 / (MU0 * C0 * C0)         # vacuum permittivity [F/m]


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------

def icosahedron():
    """Regular icosahedron inscribed in the unit sphere, outward CCW faces."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]],
                 dtype=np.int32)
    return v, f


def _orient_outward(v, f):
    """Flip faces whose normal points towards the centroid of the vertex set."""
    c = v.mean(axis=0)
    a, b, d = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    nrm = np.cross(b - a, d - a)
    cen = (a + b + d) / 3.0
    flip = np.einsum('ij,ij->i', nrm, cen - c) < 0
    f = f.copy()
    f[flip] = f[flip][:, [0, 2, 1]]
    return f


def icosphere(levels: int, radius: float = 1.0, center=(0.0, 0.0, 0.0)):
    """Icosphere by recursive 4:1 midpoint subdivision, projected to the sphere.

    ``levels`` subdivisions give 20*4**levels triangles (frequency n = 2**levels),
    e.g. 2 -> 320, 4 -> 5120, 5 -> 20480.
    """
    v, f = icosahedron()
    verts = [tuple(p) for p in v]
    for _ in range(levels):
        cache = {}
        newf = []

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key in cache:
                return cache[key]
            p = (np.array(verts[a]) + np.array(verts[b])) * 0.5
            p /= np.linalg.norm(p)
            verts.append(tuple(p))
            cache[key] = len(verts) - 1
            return cache[key]

        for (a, b, c) in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            newf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = np.array(newf, dtype=np.int32)
    v = np.array(verts, dtype=np.float64) * radius + np.asarray(center, dtype=np.float64)
    return v, _orient_outward(v, np.asarray(f, dtype=np.int32))


def cube(n: int, side: float = 2.0):
    """Closed cube of the given side, each face an n x n grid split into 2 triangles.

    12*n*n triangles, 18*n*n edges, centred at the origin.
    """
    h = side / 2.0
    g = np.linspace(-h, h, n + 1)
    index = {}
    verts = []

    def vid(p):
        key = tuple(np.round(np.asarray(p) / side * 4 * n).astype(np.int64))
        if key not in index:
            index[key] = len(verts)
            verts.append(p)
        return index[key]

    faces = []
    for axis in range(3):
        for s in (-1.0, 1.0):
            u_ax, w_ax = [a for a in range(3) if a != axis]
            for i in range(n):
                for j in range(n):
                    q = []
                    for (di, dj) in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        p = [0.0, 0.0, 0.0]
                        p[axis] = s * h
                        p[u_ax] = g[i + di]
                        p[w_ax] = g[j + dj]
                        q.append(vid(tuple(p)))
                    if (i + j) % 2 == 0:
                        faces += [(q[0], q[1], q[2]), (q[0], q[2], q[3])]
                    else:
                        faces += [(q[0], q[1], q[3]), (q[1], q[2], q[3])]
    v = np.array(verts, dtype=np.float64)
    return v, _orient_outward_convex(v, np.array(faces, dtype=np.int32))


def _orient_outward_convex(v, f):
    c = v.mean(axis=0)
    a, b, d = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    nrm = np.cross(b - a, d - a)
    cen = (a + b + d) / 3.0
    flip = np.einsum('ij,ij->i', nrm, cen - c) < 0
    f = f.copy()
    f[flip] = f[flip][:, [0, 2, 1]]
    return f


def ellipsoid(levels: int, semi_axes=(1.0, 1.0, 2.0)):
    """Icosphere scaled per axis (convex, so outward orientation is kept)."""
    v, f = icosphere(levels, 1.0)
    v = v * np.asarray(semi_axes, dtype=np.float64)
    return v, _orient_outward_convex(v, f)


def mesh_edge_lengths(v, f):
    """Lengths of the unique mesh edges (for reporting mesh statistics)."""
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    return np.linalg.norm(v[e[:, 0]] - v[e[:, 1]], axis=1)


# ----------------------------------------------------------------------------
# incident pulses and directions
# ----------------------------------------------------------------------------

@dataclass
class Pulse:
    """Modulated-Gaussian plane wave E = E0 p cos(2 pi f0 tau) exp(-tau^2/(2 sigma^2)),
    tau = t - delay - k.x / c, H = k x E / eta.  ``kind`` selects the waveform:
    "gauss" (modulated Gaussian), "sin2" (the paper's Sin^2 pulse of Section 4.1,
    E = A Sin^2(2 pi (c t + x3 - a)/Lambda) for a pulse along -x3; ``f0`` holds
    c/Lambda and ``delay`` holds a/c), or "gauss_plain" (the paper's Gaussian of
    Section 4.3 with ``sigma`` and ``delay`` = 6 sigma)."""
    k: tuple = (0.0, 0.0, 1.0)
    p: tuple = (1.0, 0.0, 0.0)
    E0: float = 1.0
    f0: float = 60e6
    sigma: float = 0.0
    delay: float = 0.0
    kind: str = "gauss"

    def as_array(self):
        kinds = {"gauss": 0.0, "sin2": 1.0, "gauss_plain": 2.0}
        return np.array(list(self.k) + list(self.p) +
                        [self.E0, self.f0, self.sigma, self.delay, kinds[self.kind]],
                        dtype=np.float64)


def gaussian_pulse(f0, fbw, k=(0, 0, 1), p=(1, 0, 0), E0=1.0, r_max=1.0):
    """Modulated Gaussian with sigma = 3/(2 pi fbw), delayed by 5 sigma + r_max/c
    so that the field is negligible (exp(-12.5)) on the body at t = 0."""
    sigma = 3.0 / (2.0 * math.pi * fbw)
    k = np.asarray(k, float); k = k / np.linalg.norm(k)
    p = np.asarray(p, float); p = p - k * (p @ k)
    if np.linalg.norm(p) < 1e-8:
        # polarisation parallel to the direction: take a perpendicular one
        a = np.array([0.0, 0.0, 1.0]) if abs(k[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
        p = a - k * (a @ k)
    p = p / np.linalg.norm(p)
    return Pulse(k=tuple(k), p=tuple(p), E0=E0, f0=f0, sigma=sigma,
                 delay=5.0 * sigma + r_max / C0, kind="gauss")


def random_pulses(n: int, seed: int, f0_range=(50e6, 150e6), r_max=1.0):
    """n modulated Gaussian pulses with seeded random direction (uniform on the
    sphere), polarisation angle psi ~ U[0, 2 pi), centre frequency f0 uniform in
    f0_range and bandwidth 2/3 f0."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        k = rng.standard_normal(3)
        k /= np.linalg.norm(k)
        a = np.array([1.0, 0.0, 0.0]) if abs(k[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        e1 = a - k * (a @ k); e1 /= np.linalg.norm(e1)
        e2 = np.cross(k, e1)
        psi = rng.uniform(0.0, 2.0 * math.pi)
        f0 = rng.uniform(*f0_range)
        out.append(gaussian_pulse(f0, 2.0 * f0 / 3.0, k=k, p=math.cos(psi) * e1 + math.sin(psi) * e2, r_max=r_max))
    return out


def fibonacci_directions(n: int, seed: int = 2303):
    """n incidence directions on a Fibonacci sphere with seeded uniform random
    polarisation angles psi ~ U[0, 2 pi).  Returns (k[n,3], p[n,3])."""
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    z = 1.0 - (2.0 * i + 1.0) / n
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    rr = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    k = np.stack([rr * np.cos(phi), rr * np.sin(phi), z], axis=1)
    psi = rng.uniform(0.0, 2.0 * math.pi, size=n)
    ps = []
    for kk, ang in zip(k, psi):
        a = np.array([1.0, 0.0, 0.0]) if abs(kk[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        e1 = a - kk * (a @ kk); e1 /= np.linalg.norm(e1)
        e2 = np.cross(kk, e1)
        ps.append(math.cos(ang) * e1 + math.sin(ang) * e2)
    return k, np.array(ps)


# ----------------------------------------------------------------------------
# named workloads (sizes of the project configurations)
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    verts: np.ndarray
    tris: np.ndarray
    dt: float
    nt: int
    pulses: list
    theta: float = 1.0
    zeta: float = C0 / 2.0
    p_s: int = 4
    p_t: int = 4
    leaf_max: int = 64
    extra: dict = field(default_factory=dict)


def workload(name: str, nt: int | None = None, n_rhs: int = 1) -> Workload:
    """Named synthetic workloads.

    conv320   : 320-triangle sphere of radius 1 m, dt = 0.5 ns, Nt = 300,
                f0 = 60 MHz / 40 MHz bandwidth x-polarised pulse along +z.
    sphere5120: 5120-triangle sphere, c dt = 0.02 m, Nt = 1000, 300/200 MHz.
    sphere20480: 20480-triangle sphere, c dt = 0.02 m, Nt = 1000, 300/200 MHz,
                p_s = p_t = 4, leaves of at most 64 edges.
    sphere20480x64: as sphere20480 with 64 Fibonacci directions.
    """
    if name == "conv320":
        v, f = icosphere(2, 1.0)
        pul = [gaussian_pulse(60e6, 40e6)]
        w = Workload(name, v, f, 0.5e-9, 300, pul)
    elif name in ("sphere1280", "sphere5120", "sphere20480", "sphere20480x64"):
        lev = {"sphere1280": 3, "sphere5120": 4}.get(name, 5)
        v, f = icosphere(lev, 1.0)
        if name == "sphere20480x64" or n_rhs > 1:
            nr = 64 if name == "sphere20480x64" else n_rhs
            ks, ps = fibonacci_directions(nr)
            pul = [gaussian_pulse(300e6, 200e6, k=tuple(k), p=tuple(p)) for k, p in zip(ks, ps)]
        else:
            pul = [gaussian_pulse(300e6, 200e6)]
        w = Workload(name, v, f, 0.02 / C0, 1000, pul)
    elif name == "cube82668":
        v, f = cube(83, 2.0)
        w = Workload(name, v, f, 0.015 / C0, 2000, [gaussian_pulse(300e6, 200e6, r_max=3 ** 0.5)])
    elif name == "ellipsoid20480":
        v, f = ellipsoid(5)
        w = Workload(name, v, f, 0.02 / C0, 1000, [gaussian_pulse(100e6, 100e6 * 2 / 3, r_max=2.0)])
    else:
        raise KeyError(name)
    if nt is not None:
        w.nt = nt
    return w
