"""Transient surface current on a perfectly conducting sphere (Mie series with
Fourier synthesis), a reference for the marched solution (test code).

Frequency domain, time factor exp(-i w t), incident E = E0 x exp(i k z) (k = w/c,
propagation +z, polarisation +x).  Fields are expanded in vector spherical
harmonics of order m = 1 (the classical plane-wave expansion):
  E_i = sum_n E_n (M1_o1n - i N1_e1n),               E_n = i^n E0 (2n+1)/(n(n+1)),
  H_i = -(k/(w mu)) sum_n E_n (M1_e1n + i N1_o1n),
  E_s = sum_n E_n (i a_n N3_e1n - b_n M3_o1n),
  H_s = (k/(w mu)) sum_n E_n (i b_n N3_o1n + a_n M3_e1n),
with radial functions j_n (superscript 1) and h_n^(1) (superscript 3).  For a
perfect conductor of radius a, with x = k a, psi_n = x j_n(x), xi_n = x h_n(x):
  a_n = psi_n'(x) / xi_n'(x),   b_n = psi_n(x) / xi_n(x),
which make the tangential total E vanish on r = a (checked by the tests, as is
the incident expansion against the plane wave itself).  The surface current is
J = n_out x H_total.  A real pulse E0 x g(t - z/c - delay) is synthesised as
  J(x, t) = (1/pi) Re int_0^inf G(w) exp(-i w (t - delay)) J_w(x) dw,
  G(w) = int g(u) exp(i w u) du.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import spherical_jn, spherical_yn

C0 = 299792458.0
MU0 = 4e-7 * math.pi
EPS0 = 1.0 / (MU0 * C0 * C0)
ETA0 = math.sqrt(MU0 / EPS0)


def _pi_tau(nmax, mu):
    """pi_n = P_n^1(cos t)/sin t and tau_n = d P_n^1 / dt by upward recurrence."""
    mu = np.asarray(mu, float)
    pi = np.zeros((nmax + 1,) + mu.shape)
    tau = np.zeros_like(pi)
    pi[1] = 1.0
    for n in range(2, nmax + 1):
        pi[n] = (2 * n - 1) / (n - 1) * mu * pi[n - 1] - n / (n - 1) * pi[n - 2]
    for n in range(1, nmax + 1):
        tau[n] = n * mu * pi[n] - (n + 1) * pi[n - 1]
    return pi, tau


def _radial(nmax, rho, kind):
    """z_n(rho) and [rho z_n(rho)]'/rho for n = 0..nmax."""
    n = np.arange(nmax + 1)[:, None]
    rho = np.atleast_1d(np.asarray(rho, float))[None, :]
    z = spherical_jn(n, rho) + (1j * spherical_yn(n, rho) if kind == 3 else 0.0)
    dz = spherical_jn(n, rho, derivative=True) + (1j * spherical_yn(n, rho, derivative=True) if kind == 3 else 0.0)
    return z, (z + rho * dz) / rho


def _vsh(nmax, r, theta, phi, k, kind):
    """M_e1n, M_o1n, N_e1n, N_o1n in spherical components [n][point][r, theta, phi]."""
    pi, tau = _pi_tau(nmax, np.cos(theta))
    z, dz = _radial(nmax, k * r, kind)
    rho = k * r
    n = np.arange(nmax + 1)[:, None]
    s, c, st = np.sin(phi)[None], np.cos(phi)[None], np.sin(theta)[None]
    zero = np.zeros_like(z)
    Me = np.stack([zero, -s * pi * z, -c * tau * z], axis=-1)
    Mo = np.stack([zero, c * pi * z, -s * tau * z], axis=-1)
    Ne = np.stack([c * n * (n + 1) * st * pi * z / rho, c * tau * dz, -s * pi * dz], axis=-1)
    No = np.stack([s * n * (n + 1) * st * pi * z / rho, s * tau * dz, c * pi * dz], axis=-1)
    return Me, Mo, Ne, No


def _to_cartesian(v, theta, phi):
    st, ct, sp, cp = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    er = np.stack([st * cp, st * sp, ct], axis=-1)
    et = np.stack([ct * cp, ct * sp, -st], axis=-1)
    ep = np.stack([-sp, cp, np.zeros_like(sp)], axis=-1)
    return v[..., 0:1] * er + v[..., 1:2] * et + v[..., 2:3] * ep


def nmax_for(ka):
    return int(ka + 4.05 * ka ** (1.0 / 3.0) + 10)


def fields(points, k, a, E0=1.0, scattered=True, incident=True):
    """Total (or partial) E and H at points [p][3] (Cartesian), frequency k."""
    P = np.asarray(points, float)
    r = np.linalg.norm(P, axis=1)
    theta = np.arccos(np.clip(P[:, 2] / r, -1, 1))
    phi = np.arctan2(P[:, 1], P[:, 0])
    nmax = nmax_for(k * max(a, r.max()))
    n = np.arange(nmax + 1)
    En = np.zeros(nmax + 1, complex)
    En[1:] = (1j ** n[1:]) * E0 * (2 * n[1:] + 1) / (n[1:] * (n[1:] + 1))
    w = k * C0
    hk = k / (w * MU0)
    E = np.zeros(P.shape, complex)
    H = np.zeros(P.shape, complex)
    if incident:
        Me, Mo, Ne, No = _vsh(nmax, r, theta, phi, k, 1)
        E += _to_cartesian(np.einsum('n,npc->pc', En[1:], (Mo - 1j * Ne)[1:]), theta, phi)
        H += _to_cartesian(-hk * np.einsum('n,npc->pc', En[1:], (Me + 1j * No)[1:]), theta, phi)
    if scattered:
        x = k * a
        j = spherical_jn(n, x); dj = spherical_jn(n, x, derivative=True)
        h = j + 1j * spherical_yn(n, x); dh = dj + 1j * spherical_yn(n, x, derivative=True)
        psi, dpsi = x * j, j + x * dj
        xi, dxi = x * h, h + x * dh
        an = np.zeros(nmax + 1, complex); bn = np.zeros(nmax + 1, complex)
        an[1:] = dpsi[1:] / dxi[1:]
        bn[1:] = psi[1:] / xi[1:]
        Me, Mo, Ne, No = _vsh(nmax, r, theta, phi, k, 3)
        E += _to_cartesian(np.einsum('n,npc->pc', En[1:], (1j * an[1:, None, None] * Ne[1:]
                                                            - bn[1:, None, None] * Mo[1:])), theta, phi)
        H += _to_cartesian(hk * np.einsum('n,npc->pc', En[1:], (1j * bn[1:, None, None] * No[1:]
                                                                 + an[1:, None, None] * Me[1:])), theta, phi)
    return E, H


def surface_current(points, k, a, E0=1.0):
    """J_w = n_out x H_total at points on r = a (frequency k)."""
    P = np.asarray(points, float)
    nrm = P / np.linalg.norm(P, axis=1)[:, None]
    _, H = fields(P, k, a, E0)
    return np.cross(nrm, H)


def transient_current(points, times, a, f0, sigma, delay, E0=1.0, nw=400, wmax_sigmas=8.0):
    """Physical J(x, t) = n_out x H for the pulse E0 x g(t - z/c - delay),
    g(u) = cos(2 pi f0 u) exp(-u^2 / 2 sigma^2), by trapezoidal synthesis over
    [0, w0 + wmax_sigmas / sigma].  Returns [t][point][3]."""
    w0 = 2 * math.pi * f0
    wmax = w0 + wmax_sigmas / sigma
    ws = np.linspace(wmax / nw, wmax, nw)       # G and J_w are smooth; w = 0 carries no weight here
    dw = ws[1] - ws[0]
    Gw = sigma * math.sqrt(2 * math.pi) / 2 * (np.exp(-sigma**2 * (ws - w0)**2 / 2) + np.exp(-sigma**2 * (ws + w0)**2 / 2))
    P = np.asarray(points, float)
    out = np.zeros((len(times), len(P), 3))
    t = np.asarray(times, float)
    for wi, (w, g) in enumerate(zip(ws, Gw)):
        Jw = surface_current(P, w / C0, a, E0)                     # [p][3]
        ph = g * np.exp(-1j * w * (t - delay))                     # [t]
        wt = 0.5 if wi == len(ws) - 1 else 1.0
        out += wt * dw / math.pi * np.real(ph[:, None, None] * Jw[None])
    return out


def sin2_spectrum(A, lam, c=C0):
    """G(w) = int g(u) exp(i w u) du for the paper's Sin^2 pulse of Section 4.1,
    g(u) = A sin^2(2 pi c u / lam) on 0 <= u <= lam / c (two humps), zero
    outside.  With sin^2 = (1 - cos 2 W u) / 2, W = 2 pi c / lam, and
    int_0^T exp(i v u) du = (exp(i v T) - 1) / (i v)."""
    W = 2 * math.pi * c / lam
    T = lam / c

    def seg(v):
        v = np.asarray(v, float)
        out = np.empty(v.shape, complex)
        small = np.abs(v) * T < 1e-8
        out[small] = T
        vs = v[~small]
        out[~small] = (np.exp(1j * vs * T) - 1.0) / (1j * vs)
        return out

    def G(w):
        return A * (0.5 * seg(w) - 0.25 * (seg(w + 2 * W) + seg(w - 2 * W)))
    return G


def _grid(wmax, nw):
    """Trapezoidal grid on [0, wmax]: nodes and weights.  A unipolar pulse has
    a DC component, so the w = 0 end counts (half weight); its current is
    the w -> 0+ limit, evaluated at 1e-6 of the spacing."""
    ws = np.linspace(0.0, wmax, nw + 1)
    wt = np.full(nw + 1, ws[1])
    wt[0] = wt[-1] = 0.5 * ws[1]
    return ws, wt


def transient_current_spectrum(points, times, a, G, wmax, delay, nw=800):
    """J(x, t) = n_out x H for the pulse x g(t - z/c - delay) with spectrum
    G(w) (sin2_spectrum), trapezoidal synthesis over [0, wmax] (periodic in t
    with period 2 pi nw / wmax).  Returns [t][point][3]."""
    ws, wts = _grid(wmax, nw)
    Gw = G(ws)
    P = np.asarray(points, float)
    out = np.zeros((len(times), len(P), 3))
    t = np.asarray(times, float)
    for w, g, wt in zip(ws, Gw, wts):
        Jw = surface_current(P, max(w, 1e-6 * ws[1]) / C0, a)
        ph = g * np.exp(-1j * w * (t - delay))
        out += wt / math.pi * np.real(ph[:, None, None] * Jw[None])
    return out


def synthesise_waveform(times, G, wmax, nw=800):
    """(1/pi) Re int_0^wmax G(w) exp(-i w t) dw on the grid of
    transient_current_spectrum: the waveform itself, as the incident field at
    the origin sees it (for pinning the synthesis)."""
    ws, wts = _grid(wmax, nw)
    t = np.asarray(times, float)
    return (wts[None, :] / math.pi * np.real(G(ws)[None, :] * np.exp(-1j * ws[None, :] * t[:, None]))).sum(1)
