// Retarded inner integrals and J-form coefficients of one (pair, lag).
// Shared by the device setup kernels and a host build used by the tests:
// TD_HD marks functions (device inline in HIP, inline in a host build),
// TD_CONST marks the quadrature tables (__constant__ / static const).
//
// Inner integrals over a flat source triangle, for one field point x and one
// lag g, use polar coordinates about the projection x0 of x on the source
// plane (r dr = rho drho).  The radial integrals of the retarded kernels are
// closed forms in tau = g - r/(c dt):
//   Qa   = -c dt B'(tau)       (d/dr Qa = B'')
//   Qphi = -c dt Bint(tau)     (d/dr Qphi = B)
//   Qp   = F(tau)/r, F = kd B'(tau)/dt + zeta B(tau)   ((1/r) d/dr Qp = psi, grad(F/r) = (y-x) psi)
// The angular integral over each edge's signed sub-triangle is taken in
// v = asinh(s/|d|) (smooth in a strip of half-width pi/2), split where the
// light-cone circles r = (g-k) c dt cross the edge; in-plane vector moments use
// the surface gradient theorem as line integrals in w = asinh(s/rho).
#define GL_N 10
TD_CONST double c_glx[GL_N] = {
    -0.9739065285171717, -0.8650633666889845, -0.6794095682990244, -0.4333953941292472, -0.1488743389816312,
    0.1488743389816312, 0.4333953941292472, 0.6794095682990244, 0.8650633666889845, 0.9739065285171717};
TD_CONST double c_glw[GL_N] = {
    0.0666713443086881, 0.1494513491505806, 0.2190863625159820, 0.2692667193099963, 0.2955242247147529,
    0.2955242247147529, 0.2692667193099963, 0.2190863625159820, 0.1494513491505806, 0.0666713443086881};

// quadratic cardinal B-spline on (0,3) as explicit pieces
TD_HD double bsp(double t) {
    if (t <= 0.0 || t >= 3.0) return 0.0;
    if (t < 1.0) return 0.5 * t * t;
    if (t < 2.0) { double u = t - 1.5; return 0.75 - u * u; }
    double u = 3.0 - t; return 0.5 * u * u;
}
TD_HD double bsp_d(double t) {
    if (t <= 0.0 || t >= 3.0) return 0.0;
    if (t < 1.0) return t;
    if (t < 2.0) return 3.0 - 2.0 * t;
    return t - 3.0;
}
TD_HD double bsp_int(double t) {
    if (t <= 0.0) return 0.0;
    if (t >= 3.0) return 1.0;
    if (t < 1.0) return t * t * t / 6.0;
    if (t < 2.0) { double u = t - 1.5; return 1.0 / 6.0 + 0.75 * (t - 1.0) - (u * u * u + 0.125) / 3.0; }
    double u = 3.0 - t; return 1.0 - u * u * u / 6.0;
}

struct LagK {
    double cdt, dt, zeta, kd;
    int g;
};
struct Q3 { double a, phi, p; };

TD_HD Q3 radial(const LagK &k, double r) {
    double tau = k.g - r / k.cdt;
    Q3 q;
    double b1 = bsp_d(tau);
    q.a = -k.cdt * b1;
    q.phi = -k.cdt * bsp_int(tau);
    q.p = (k.kd * b1 / k.dt + k.zeta * bsp(tau)) / r;
    return q;
}

TD_HD void sub3(const double *a, const double *b, double *c) { c[0] = a[0] - b[0]; c[1] = a[1] - b[1]; c[2] = a[2] - b[2]; }
TD_HD double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
TD_HD void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1]; c[1] = a[2] * b[0] - a[0] * b[2]; c[2] = a[0] * b[1] - a[1] * b[0];
}

struct TriInt { double as, phis, ps, av[3], pv[3]; };

// angular integral over t in [t0, t1] (t >= 0 along the edge from the foot),
// v = asinh(t/|d|): adds sgn * int Q(R(v)) / cosh v dv.
TD_HD void ang_half(const LagK &k, double d, double h, double t0, double t1, double sgn, double &oa, double &ophi, double &op) {
    if (t1 <= t0) return;
    double ad = fabs(d), c2 = d * d + h * h;
    // breakpoints: R = n cdt for n in (g-3 .. g)
    double br[6];
    int nb = 0;
    br[nb++] = t0;
    for (int n = k.g - 3; n <= k.g; ++n) {
        if (n <= 0) continue;
        double rn = n * k.cdt, s2 = rn * rn - c2;
        if (s2 <= 0.0) continue;
        double t = sqrt(s2);
        if (t > t0 && t < t1) br[nb++] = t;
    }
    br[nb++] = t1;
    for (int b = 0; b + 1 < nb; ++b) {
        double va = asinh(br[b] / ad), vb = asinh(br[b + 1] / ad);
        if (!(vb > va)) continue;
        double tm = 0.5 * (br[b] + br[b + 1]);
        double Rm = sqrt(tm * tm + c2);
        double u = Rm / k.cdt;
        if (u >= k.g) continue;                       // beyond the outer light cone: all zero
        if (u <= k.g - 3) {                           // inside: only Qphi, constant -cdt
            ophi += sgn * (-k.cdt) * (atan(sinh(vb)) - atan(sinh(va)));
            continue;
        }
        int nsub = (int)ceil(vb - va);
        if (nsub < 1) nsub = 1;
        double hs = (vb - va) / nsub;
        for (int s = 0; s < nsub; ++s) {
            double c = va + (s + 0.5) * hs, hw = 0.5 * hs;
            for (int j = 0; j < GL_N; ++j) {
                double v = c + hw * c_glx[j];
                double ch = cosh(v);
                double R = sqrt(d * d * ch * ch + h * h);
                Q3 q = radial(k, R);
                double w = sgn * hw * c_glw[j] / ch;
                oa += w * q.a; ophi += w * q.phi; op += w * q.p;
            }
        }
    }
}

// line integral over t in [t0, t1] (t >= 0 from the foot) of G(r), r = sqrt(t^2 + rho^2),
// G = Qa and Qp (both vanish outside the shell band of lag g).
TD_HD void line_half(const LagK &k, double rho, double t0, double t1, double &la, double &lp) {
    if (t1 <= t0) return;
    double r2 = rho * rho;
    double br[6];
    int nb = 0;
    br[nb++] = t0;
    for (int n = k.g - 3; n <= k.g; ++n) {
        if (n <= 0) continue;
        double rn = n * k.cdt, s2 = rn * rn - r2;
        if (s2 <= 0.0) continue;
        double t = sqrt(s2);
        if (t > t0 && t < t1) br[nb++] = t;
    }
    br[nb++] = t1;
    bool sub = rho > 1e-14 * (t1 + rho);
    for (int b = 0; b + 1 < nb; ++b) {
        double tm = 0.5 * (br[b] + br[b + 1]);
        double u = sqrt(tm * tm + r2) / k.cdt;
        if (u >= k.g || u <= k.g - 3) continue;
        double wa = sub ? asinh(br[b] / rho) : br[b], wb = sub ? asinh(br[b + 1] / rho) : br[b + 1];
        if (!(wb > wa)) continue;
        int nsub = sub ? (int)ceil(wb - wa) : 1;
        if (nsub < 1) nsub = 1;
        double hs = (wb - wa) / nsub;
        for (int s = 0; s < nsub; ++s) {
            double c = wa + (s + 0.5) * hs, hw = 0.5 * hs;
            for (int j = 0; j < GL_N; ++j) {
                double w = c + hw * c_glx[j];
                double r, jac;
                if (sub) { r = rho * cosh(w); jac = r; } else { r = w; jac = 1.0; }
                Q3 q = radial(k, r);
                double wt = hw * c_glw[j] * jac;
                la += wt * q.a; lp += wt * q.p;
            }
        }
    }
}

TD_HD void tri_int(const double *x, const double *P, bool self, const LagK &k, TriInt &o) {
    double e1[3], e2[3], nt[3];
    sub3(P + 3, P, e1); sub3(P + 6, P, e2); cross3(e1, e2, nt);
    double nn = sqrt(dot3(nt, nt));
    nt[0] /= nn; nt[1] /= nn; nt[2] /= nn;
    double xp[3]; sub3(x, P, xp);
    double h = dot3(xp, nt);
    double lmax = fmax(sqrt(dot3(e1, e1)), sqrt(dot3(e2, e2)));
    if (self || fabs(h) < 1e-13 * lmax) h = 0.0;
    double x0[3] = {x[0] - h * nt[0], x[1] - h * nt[1], x[2] - h * nt[2]};
    double sa = 0, sphi = 0, sp = 0;
    double la[3] = {0, 0, 0}, lp[3] = {0, 0, 0};
    double theta_tot = 0.0;   // signed angle subtended by the triangle at x0
    for (int e = 0; e < 3; ++e) {
        const double *A = P + 3 * e, *B = P + 3 * ((e + 1) % 3), *C = P + 3 * ((e + 2) % 3);
        double t[3]; sub3(B, A, t);
        double L = sqrt(dot3(t, t));
        t[0] /= L; t[1] /= L; t[2] /= L;
        double m[3]; cross3(t, nt, m);
        double ca[3]; sub3(C, A, ca);
        if (dot3(ca, m) > 0) { m[0] = -m[0]; m[1] = -m[1]; m[2] = -m[2]; }
        double ax[3], bx[3];
        sub3(A, x0, ax); sub3(B, x0, bx);
        double d = dot3(ax, m), sA = dot3(ax, t), sB = dot3(bx, t);
        if (fabs(d) > 1e-14 * L) {
            theta_tot += atan(sB / d) - atan(sA / d);
            double sg = d > 0 ? 1.0 : -1.0;
            if (sA < 0.0 && sB > 0.0) {
                ang_half(k, d, h, 0.0, -sA, sg, sa, sphi, sp);
                ang_half(k, d, h, 0.0, sB, sg, sa, sphi, sp);
            } else if (sB <= 0.0) {
                ang_half(k, d, h, -sB, -sA, sg, sa, sphi, sp);
            } else {
                ang_half(k, d, h, sA, sB, sg, sa, sphi, sp);
            }
        }
        double rho = sqrt(d * d + h * h);
        double le_a = 0, le_p = 0;
        if (sA < 0.0 && sB > 0.0) {
            line_half(k, rho, 0.0, -sA, le_a, le_p);
            line_half(k, rho, 0.0, sB, le_a, le_p);
        } else if (sB <= 0.0) {
            line_half(k, rho, -sB, -sA, le_a, le_p);
        } else {
            line_half(k, rho, sA, sB, le_a, le_p);
        }
        for (int c = 0; c < 3; ++c) { la[c] += le_a * m[c]; lp[c] += le_p * m[c]; }
    }
    // lower radial limit r = |h| over the total angle (2 pi inside, 0 outside,
    // pi with the projection on an edge, the corner angle at a vertex)
    if (h != 0.0) {
        Q3 q = radial(k, fabs(h));
        sa -= theta_tot * q.a; sphi -= theta_tot * q.phi; sp -= theta_tot * q.p;
    } else {
        sa -= theta_tot * (-k.cdt * bsp_d((double)k.g));
        sphi -= theta_tot * (-k.cdt * bsp_int((double)k.g));
        sp = 0.0;
    }
    o.as = sa; o.phis = sphi; o.ps = sp;
    for (int c = 0; c < 3; ++c) {
        o.av[c] = la[c] - h * nt[c] * sa;
        o.pv[c] = lp[c] - (h != 0.0 ? h * nt[c] * sp : 0.0);
    }
}

// Zt^(g)_{ij} for one pair and one lag (3-point testing x exact source integrals),
// plus the MFIE identity (Gram) term at g = 1, 2.
TD_HD double zt_value(const GeoDev &G, int i, int j, int g) {
    const double PI4 = 12.566370614359172;
    LagK k{G.cdt, G.dt, G.zeta, G.kd, g};
    double z = 0.0;
    for (int rho = 0; rho < 2; ++rho) {
        int ti = G.etri[2 * i + rho];
        double Ai = G.area[ti];
        double si = (rho == 0 ? 1.0 : -1.0) * G.elen[i] / (2.0 * Ai);
        double divi = 2.0 * si;
        const double *oi = G.xyz + 3 * G.efree[2 * i + rho];
        double ni[3] = {-G.nrm[3 * ti], -G.nrm[3 * ti + 1], -G.nrm[3 * ti + 2]};
        for (int sg = 0; sg < 2; ++sg) {
            int tj = G.etri[2 * j + sg];
            double P[9];
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) P[3 * a + c] = G.xyz[3 * G.tri[3 * tj + a] + c];
            double Aj = G.area[tj];
            double sj = (sg == 0 ? 1.0 : -1.0) * G.elen[j] / (2.0 * Aj);
            double divj = 2.0 * sj;
            const double *oj = G.xyz + 3 * G.efree[2 * j + sg];
            for (int q = 0; q < 3; ++q) {
                const double *x = G.qpt + 9 * ti + 3 * q;
                TriInt I;
                tri_int(x, P, ti == tj, k, I);
                double fi[3]; sub3(x, oi, fi);
                double xo[3]; sub3(x, oj, xo);
                double Av[3];
                for (int c = 0; c < 3; ++c) Av[c] = (xo[c] * I.as + I.av[c]);
                double fa = si * dot3(fi, Av) * sj * G.mu / (PI4 * G.dt * G.dt);
                double fphi = divi * divj * I.phis / (PI4 * G.eps);
                double t1[3], nxP[3];
                cross3(xo, I.pv, t1);
                cross3(ni, t1, nxP);
                double fp = G.theta * G.eta * si * sj * dot3(fi, nxP) / PI4;
                z += (Ai / 3.0) * (fa + fphi + fp);
            }
        }
    }
    if (g <= 2) {
        double gram = 0.0;
        for (int rho = 0; rho < 2; ++rho)
            for (int sg = 0; sg < 2; ++sg) {
                int ti = G.etri[2 * i + rho];
                if (ti != G.etri[2 * j + sg]) continue;
                double A = G.area[ti];
                double si = (rho == 0 ? 1.0 : -1.0) * G.elen[i] / (2.0 * A);
                double sj = (sg == 0 ? 1.0 : -1.0) * G.elen[j] / (2.0 * A);
                const double *oi = G.xyz + 3 * G.efree[2 * i + rho], *oj = G.xyz + 3 * G.efree[2 * j + sg];
                for (int q = 0; q < 3; ++q) {
                    const double *x = G.qpt + 9 * ti + 3 * q;
                    double a[3], b[3]; sub3(x, oi, a); sub3(x, oj, b);
                    gram += A / 3.0 * si * sj * dot3(a, b);
                }
            }
        z += 0.5 * G.theta * G.eta * gram * (g == 1 ? (G.kd / G.dt + 0.5 * G.zeta) : (-G.kd / G.dt + 0.5 * G.zeta));
    }
    return z;
}

// ---- exact lag range of a pair: Zt^(g) can be non-zero only for
// r_min/cdt < g < r_max/cdt + 3 with r over test points x source triangles.
TD_HD double pt_tri_dist(const double *x, const double *P) {
    double e1[3], e2[3], n[3];
    sub3(P + 3, P, e1); sub3(P + 6, P, e2); cross3(e1, e2, n);
    double nn = sqrt(dot3(n, n));
    n[0] /= nn; n[1] /= nn; n[2] /= nn;
    double xp[3]; sub3(x, P, xp);
    double h = dot3(xp, n);
    double x0[3] = {x[0] - h * n[0], x[1] - h * n[1], x[2] - h * n[2]};
    bool in = true;
    double best = 1e300;
    for (int e = 0; e < 3; ++e) {
        const double *A = P + 3 * e, *B = P + 3 * ((e + 1) % 3);
        double ab[3], ax[3], c[3];
        sub3(B, A, ab); sub3(x0, A, ax); cross3(ab, ax, c);
        if (dot3(c, n) < 0) in = false;
        double t = dot3(ax, ab) / dot3(ab, ab);
        t = fmin(1.0, fmax(0.0, t));
        double p[3] = {A[0] + t * ab[0] - x[0], A[1] + t * ab[1] - x[1], A[2] + t * ab[2] - x[2]};
        best = fmin(best, sqrt(dot3(p, p)));
    }
    return in ? fabs(h) : best;
}


// exact lag range of a pair: Zt^(g) can be non-zero only for
// r_min/cdt < g < r_max/cdt + 3, r over test points x source triangles
TD_HD void pair_lag_range(const GeoDev &G, int i, int j, int &lo_out, int &hi_out) {
    double rmin = 1e300, rmax = 0.0;
    for (int rho = 0; rho < 2; ++rho) {
        int ti = G.etri[2 * i + rho];
        for (int sg = 0; sg < 2; ++sg) {
            int tj = G.etri[2 * j + sg];
            double P[9];
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) P[3 * a + c] = G.xyz[3 * G.tri[3 * tj + a] + c];
            for (int q = 0; q < 3; ++q) {
                const double *x = G.qpt + 9 * ti + 3 * q;
                rmin = fmin(rmin, ti == tj ? 0.0 : pt_tri_dist(x, P));
                for (int a = 0; a < 3; ++a) {
                    double d[3]; sub3(P + 3 * a, x, d);
                    rmax = fmax(rmax, sqrt(dot3(d, d)));
                }
            }
        }
    }
    int lo = (int)floor(rmin / G.cdt * (1.0 - 1e-12)) + 1;
    int hi = (int)ceil(rmax / G.cdt * (1.0 + 1e-12)) + 2;
    bool share = G.etri[2 * i] == G.etri[2 * j] || G.etri[2 * i] == G.etri[2 * j + 1] ||
                 G.etri[2 * i + 1] == G.etri[2 * j] || G.etri[2 * i + 1] == G.etri[2 * j + 1];
    if (share) { lo = 1; hi = hi < 2 ? 2 : hi; }
    if (lo < 1) lo = 1;
    lo_out = lo;
    hi_out = hi;
}

// incident waveform g(tau) and its time derivative (pulse kinds of tdbem.h)
TD_HD void pulse_g(const double *pl, double tau, double &g, double &gd) {
    int kind = (int)pl[10];
    double f0 = pl[7], sig = pl[8];
    const double TWO_PI = 6.283185307179586;
    if (kind == 0) {
        double e = exp(-tau * tau / (2 * sig * sig));
        double cs = cos(TWO_PI * f0 * tau), sn = sin(TWO_PI * f0 * tau);
        g = cs * e;
        gd = (-TWO_PI * f0 * sn - tau / (sig * sig) * cs) * e;
    } else if (kind == 1) {
        double arg = TWO_PI * f0 * tau;
        if (arg < 0.0 || arg > TWO_PI) { g = 0; gd = 0; return; }
        double s = sin(arg);
        g = s * s;
        gd = 2 * s * cos(arg) * TWO_PI * f0;
    } else {
        double e = exp(-tau * tau / (2 * sig * sig)) / sqrt(TWO_PI * sig * sig);
        g = e;
        gd = -tau / (sig * sig) * e;
    }
}

// tested incident field of leaf-order edge p at time t (Eq. v_i):
// sum_rho sum_q w_q A f_p(x_q) . [-dE/dt + theta eta n x (kd dH/dt + zeta H)], n inward
TD_HD double vinc_value(const GeoDev &G, int p, const double *pl, double t) {
    double kk[3] = {pl[0], pl[1], pl[2]}, pp[3] = {pl[3], pl[4], pl[5]};
    double E0 = pl[6], delay = pl[9];
    double kxp[3]; cross3(kk, pp, kxp);
    double c = G.cdt / G.dt;
    double v = 0.0;
    for (int rho = 0; rho < 2; ++rho) {
        int ti = G.etri[2 * p + rho];
        double A = G.area[ti];
        double s = (rho == 0 ? 1.0 : -1.0) * G.elen[p] / (2.0 * A);
        const double *o = G.xyz + 3 * G.efree[2 * p + rho];
        double n[3] = {-G.nrm[3 * ti], -G.nrm[3 * ti + 1], -G.nrm[3 * ti + 2]};
        for (int q = 0; q < 3; ++q) {
            const double *x = G.qpt + 9 * ti + 3 * q;
            double tau = t - delay - dot3(kk, x) / c, g, gd;
            pulse_g(pl, tau, g, gd);
            double Hs[3], nxH[3], f[3];
            for (int cc = 0; cc < 3; ++cc) Hs[cc] = E0 * kxp[cc] / G.eta * (G.kd * gd + G.zeta * g);
            cross3(n, Hs, nxH);
            sub3(x, o, f);
            double val = 0;
            for (int cc = 0; cc < 3; ++cc) val += s * f[cc] * (-E0 * pp[cc] * gd + G.theta * G.eta * nxH[cc]);
            v += A / 3.0 * val;
        }
    }
    return v;
}
