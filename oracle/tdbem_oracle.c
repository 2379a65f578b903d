/*
 * FP64 CPU oracle for the time-domain CFIE boundary element method.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code with the HIP library.
 *
 * What it computes (T. Takahashi, "A fast time-domain boundary element method
 * for three-dimensional electromagnetic scattering problems"):
 *
 *  - the quadratic temporal B-spline as a weighted sum of truncated powers
 *    (Section 2.2, weights w^{kappa,d});
 *  - the J-form coefficient matrices  Zt^(g) = sum_kappa w^kappa Z^(g-kappa),
 *    i.e. the coefficients of J^{alpha-g} in the tested CFIE at t_alpha
 *    (Section 2.3, Eq. layer_disc_tmp, summed over kappa; Section 2.4, Eqs.
 *    testing and z_ij), plus the identity term 1/2 J of the MFIE (exterior
 *    limit of n x P, inward normal) which contributes
 *    1/2 theta eta Gram_ij (1/dt + zeta/2) at g = 1 and
 *    1/2 theta eta Gram_ij (-1/dt + zeta/2) at g = 2;
 *  - the CFIE variants of Section 4.3.1 through the weights (kd, zeta) of
 *    the MFIE's time derivative and of the MFIE itself: CFIE1 = (1, zeta) is
 *    Eq. cfie, CFIE2 (d/dt EFIE + d/dt MFIE) = (1, 0), CFIE3 (d/dt EFIE +
 *    MFIE) = (0, zeta); kd multiplies every term the time derivative of the
 *    MFIE produces (B'/dt in the P kernel, 1/dt in the identity term, dH/dt
 *    in the incident field);
 *  - the tested incident field V_i^{alpha-1} (Eq. v_i);
 *  - the history sum sum_{g>=2} Zt^(g) J^{alpha-g} (Eq. R).
 *
 * Inner (source) integrals over a flat triangle are evaluated semi-analytically:
 * polar coordinates about the projection of the field point onto the source
 * plane turn r dr into rho drho, the radial integrals of the piecewise
 * polynomial retarded kernels are closed forms, and the remaining angular (and
 * boundary line) integrals are done with adaptive Gauss-Legendre quadrature
 * split at every crossing of a light-cone circle r = n c dt.  In-plane vector
 * moments use the surface gradient theorem.  Outer (test) integrals use the
 * interior 3-point rule with barycentric points (2/3,1/6,1/6) and weights 1/3
 * (Section 2.4).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ---------------------------------------------------------------- B-spline */
/* B(tau) = sum_{k=0}^{3} w_k (tau - k)_+^2 with w = (1/2, -3/2, 3/2, -1/2):
 * the quadratic B-spline N^{beta,2}(t) written in tau = (t - t_beta)/dt
 * (Section 2.2).  Supported on (0, 3); identically zero for tau >= 3 by
 * construction, which is returned exactly to avoid cancellation. */
static const double WK[4] = {0.5, -1.5, 1.5, -0.5};

static double bs0(double tau) {           /* B */
    if (tau <= 0.0 || tau >= 3.0) return 0.0;
    double s = 0.0;
    for (int k = 0; k < 4; ++k) if (tau > k) s += WK[k] * (tau - k) * (tau - k);
    return s;
}
static double bs1(double tau) {           /* B' */
    if (tau <= 0.0 || tau >= 3.0) return 0.0;
    double s = 0.0;
    for (int k = 0; k < 4; ++k) if (tau > k) s += 2.0 * WK[k] * (tau - k);
    return s;
}
static double bsm1(double tau) {          /* antiderivative of B, zero for tau <= 0 */
    if (tau <= 0.0) return 0.0;
    if (tau >= 3.0) return 1.0;
    double s = 0.0;
    for (int k = 0; k < 4; ++k) if (tau > k) s += WK[k] * (tau - k) * (tau - k) * (tau - k) / 3.0;
    return s;
}

double orc_bspline(int which, double tau) {
    if (which == 0) return bs0(tau);
    if (which == 1) return bs1(tau);
    if (which == -1) return bsm1(tau);
    /* B'' : piecewise constant, right-continuous */
    if (tau < 0.0 || tau >= 3.0) return 0.0;
    double s = 0.0;
    for (int k = 0; k < 4; ++k) if (tau >= k) s += 2.0 * WK[k];
    return s;
}

/* ------------------------------------------------------------ small vectors */
static void sub3(const double *a, const double *b, double *c) { c[0]=a[0]-b[0]; c[1]=a[1]-b[1]; c[2]=a[2]-b[2]; }
static double dot3(const double *a, const double *b) { return a[0]*b[0]+a[1]*b[1]+a[2]*b[2]; }
static void cross3(const double *a, const double *b, double *c) {
    c[0]=a[1]*b[2]-a[2]*b[1]; c[1]=a[2]*b[0]-a[0]*b[2]; c[2]=a[0]*b[1]-a[1]*b[0]; }
static double norm3(const double *a) { return sqrt(dot3(a,a)); }

/* ------------------------------------------------------- Gauss-Legendre */
/* Nodes and weights on [-1,1] by Newton iteration on the Legendre recurrence. */
#define GLMAX 32
static double GLX[GLMAX+1][GLMAX], GLW[GLMAX+1][GLMAX];
static int gl_ready = 0;
static void gl_init(void) {
    if (gl_ready) return;
    for (int n = 1; n <= GLMAX; ++n) {
        for (int i = 0; i < n; ++i) {
            double x = cos(PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = x;
                for (int k = 2; k <= n; ++k) { double p2 = ((2.0*k-1.0)*x*p1 - (k-1.0)*p0)/k; p0 = p1; p1 = p2; }
                if (n == 1) { p1 = x; p0 = 1.0; }
                dp = n * (x * p1 - p0) / (x * x - 1.0);
                double dx = p1 / dp; x -= dx;
                if (fabs(dx) < 1e-16) break;
            }
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) { double p2 = ((2.0*k-1.0)*x*p1 - (k-1.0)*p0)/k; p0 = p1; p1 = p2; }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            GLX[n][i] = x; GLW[n][i] = 2.0 / ((1.0 - x * x) * dp * dp);
        }
    }
    gl_ready = 1;
}

/* ------------------------------------------------- retarded radial functions */
/* For lag g, tau_g(r) = g - r/(c dt).  The three radial antiderivatives used:
 *   Qa(r)   = int B''(tau_g) dr = -c dt B'(tau_g)          (A-dd kernel, Eq. def_A)
 *   Qphi(r) = int B(tau_g) dr   = -c dt Bint(tau_g)        (phi-dot kernel, Eq. def_phi)
 *   Qp(r)   = F(tau_g)/r,  F = kd B'(tau_g)/dt + zeta B(tau_g) (kd P-dot + zeta P, Eq. def_P)
 * They satisfy d/dr Qa = B'', d/dr Qphi = B, and (1/r) d/dr Qp = psi where
 * grad_y [F/r] = (y - x) psi(r). */
typedef struct {
    double cdt, dt, zeta, kd;
    int g0, ng;            /* lags g0 .. g0+ng-1 */
} kpar_t;

typedef struct {           /* per-lag accumulators for one (point, triangle) pair */
    double as, phis, ps;   /* int B''/r, int B/r, int psi */
    double av[3], pv[3];   /* int (y-x) B''/r, int grad_y(F/r) */
} acc_t;

#define NGMAX 512

/* value of the three radial functions at r for lags k->g0+ia .. k->g0+ib-1 */
static void radial_q(const kpar_t *k, int ia, int ib, double r, double *qa, double *qphi, double *qp) {
    for (int i = ia; i < ib; ++i) {
        double tau = (k->g0 + i) - r / k->cdt;
        qa[i] = -k->cdt * bs1(tau);
        qphi[i] = -k->cdt * bsm1(tau);
        qp[i] = (k->kd * bs1(tau) / k->dt + k->zeta * bs0(tau)) / r;
    }
}

/* Lags whose kernels vary for r in [rlo, rhi]: tau_g in (0,3) somewhere, i.e.
 * rlo/cdt < g < rhi/cdt + 3.  Lags above the range have Qa = Qp = 0 and
 * Qphi = -cdt (B fully integrated); lags below have all three zero. */
static void active_lags(const kpar_t *k, double rlo, double rhi, int *ia, int *ib, int *ic) {
    int a = (int)floor(rlo / k->cdt) + 1 - k->g0;        /* first g > rlo/cdt */
    int b = (int)ceil(rhi / k->cdt + 3.0) - k->g0;       /* first g >= rhi/cdt + 3 */
    if (a < 0) a = 0;
    if (b > k->ng) b = k->ng;
    if (b < a) b = a;
    *ia = a; *ib = b; *ic = b;                            /* lags [ic, ng) are the constant tail */
}

/* integral over v in [va, vb] (0 <= va < vb) of Q(R(v))/cosh(v),
 * R(v) = sqrt(d^2 cosh^2 v + h^2), for the three Q families and all lags; added
 * with factor fac into oa/ophi/op.  The integrand is smooth on the piece;
 * adaptive Gauss-Legendre (12 vs 24 points) over the varying lags, exact
 * integral atan(sinh v) for the constant tail of Qphi. */
static void ang_piece(const kpar_t *k, double d, double h, double va, double vb, double fac,
                      double *oa, double *ophi, double *op, int depth) {
    int ng = k->ng;
    double ca = cosh(va), cb = cosh(vb);
    int ia, ib, ic;
    active_lags(k, sqrt(d * d * ca * ca + h * h), sqrt(d * d * cb * cb + h * h), &ia, &ib, &ic);
    double qa[ng], qphi[ng], qp[ng];
    double sa1[ng], sphi1[ng], sp1[ng];
    double sa2[ng], sphi2[ng], sp2[ng];
    double c = 0.5 * (va + vb), hw = 0.5 * (vb - va);
    for (int pass = 0; pass < 2; ++pass) {
        int n = pass == 0 ? 12 : 24;
        double *A = pass == 0 ? sa1 : sa2, *P = pass == 0 ? sphi1 : sphi2, *Q = pass == 0 ? sp1 : sp2;
        for (int i = ia; i < ib; ++i) { A[i] = 0.0; P[i] = 0.0; Q[i] = 0.0; }
        for (int j = 0; j < n; ++j) {
            double v = c + hw * GLX[n][j];
            double ch = cosh(v);
            double R = sqrt(d * d * ch * ch + h * h);
            double w = hw * GLW[n][j] / ch;
            radial_q(k, ia, ib, R, qa, qphi, qp);
            for (int i = ia; i < ib; ++i) { A[i] += w * qa[i]; P[i] += w * qphi[i]; Q[i] += w * qp[i]; }
        }
    }
    double err = 0.0, scale = 1e-300;
    for (int i = ia; i < ib; ++i) {
        err = fmax(err, fabs(sa1[i] - sa2[i]) + fabs(sphi1[i] - sphi2[i]) / k->cdt + fabs(sp1[i] - sp2[i]) * k->dt);
        scale = fmax(scale, fabs(sa2[i]) + fabs(sphi2[i]) / k->cdt + fabs(sp2[i]) * k->dt);
    }
    if (err > 1e-13 * scale && depth < 12 && hw > 1e-12) {
        ang_piece(k, d, h, va, c, fac, oa, ophi, op, depth + 1);
        ang_piece(k, d, h, c, vb, fac, oa, ophi, op, depth + 1);
        return;
    }
    for (int i = ia; i < ib; ++i) { oa[i] += fac * sa2[i]; ophi[i] += fac * sphi2[i]; op[i] += fac * sp2[i]; }
    double dth = atan(sinh(vb)) - atan(sinh(va));
    for (int i = ic; i < ng; ++i) ophi[i] += fac * (-k->cdt) * dth;
}

/* line integral over w in [wa, wb] of G(rho cosh w) rho cosh w (s = rho sinh w),
 * or, when rho == 0, of G(|s|) over s in [wa, wb]; G = Qa and Qp; all lags
 * (both vanish outside the varying lags). */
static void line_piece(const kpar_t *k, double rho, double wa, double wb,
                       double *oa, double *op, int depth) {
    int ng = k->ng;
    double rlo = rho > 0.0 ? rho * cosh(wa) : fabs(wa), rhi = rho > 0.0 ? rho * cosh(wb) : fabs(wb);
    if (rlo > rhi) { double t = rlo; rlo = rhi; rhi = t; }
    int ia, ib, ic;
    active_lags(k, rlo, rhi, &ia, &ib, &ic);
    if (ib <= ia) return;
    double qa[ng], qphi[ng], qp[ng];
    double a1[ng], p1[ng], a2[ng], p2[ng];
    double c = 0.5 * (wa + wb), hw = 0.5 * (wb - wa);
    for (int pass = 0; pass < 2; ++pass) {
        int n = pass == 0 ? 12 : 24;
        double *A = pass == 0 ? a1 : a2, *P = pass == 0 ? p1 : p2;
        for (int i = ia; i < ib; ++i) { A[i] = 0.0; P[i] = 0.0; }
        for (int j = 0; j < n; ++j) {
            double w = c + hw * GLX[n][j], r, jac;
            if (rho > 0.0) { r = rho * cosh(w); jac = r; } else { r = fabs(w); jac = 1.0; }
            double wt = hw * GLW[n][j] * jac;
            radial_q(k, ia, ib, r, qa, qphi, qp);
            for (int i = ia; i < ib; ++i) { A[i] += wt * qa[i]; P[i] += wt * qp[i]; }
        }
    }
    double err = 0.0, scale = 1e-300;
    for (int i = ia; i < ib; ++i) {
        err = fmax(err, fabs(a1[i] - a2[i]) + fabs(p1[i] - p2[i]) * k->dt);
        scale = fmax(scale, fabs(a2[i]) + fabs(p2[i]) * k->dt);
    }
    if (err > 1e-13 * scale && depth < 12 && hw > 1e-14) {
        line_piece(k, rho, wa, c, oa, op, depth + 1);
        line_piece(k, rho, c, wb, oa, op, depth + 1);
        return;
    }
    for (int i = ia; i < ib; ++i) { oa[i] += a2[i]; op[i] += p2[i]; }
}

static int cmp_dbl(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* sorted breakpoints in (lo, hi) of the map t -> sqrt(t^2 + c2) = n cdt, t>0 side,
 * mapped through f(t); plus both interval ends. */
static int pieces_pos(double lo, double hi, double c2, double cdt, double *br) {
    /* t in [lo, hi] with 0 <= lo < hi: r(t) = sqrt(t^2+c2) increasing */
    int nb = 0;
    br[nb++] = lo;
    double rlo = sqrt(lo * lo + c2), rhi = sqrt(hi * hi + c2);
    long n0 = (long)floor(rlo / cdt) + 1, n1 = (long)ceil(rhi / cdt) - 1;
    for (long n = n0; n <= n1 && nb < 4000; ++n) {
        double rn = n * cdt;
        double t = sqrt(fmax(rn * rn - c2, 0.0));
        if (t > lo && t < hi) br[nb++] = t;
    }
    br[nb++] = hi;
    qsort(br, nb, sizeof(double), cmp_dbl);
    return nb;
}

/* Integrals of the retarded kernels over triangle P[3] for field point x and
 * lags k->g0 .. k->g0+k->ng-1.  `self` forces the field point into the plane. */
static void tri_integrals(const double *x, const double P[3][3], int self, const kpar_t *k, acc_t *acc) {
    double e1[3], e2[3], nt[3];
    sub3(P[1], P[0], e1); sub3(P[2], P[0], e2); cross3(e1, e2, nt);
    double nn = norm3(nt); nt[0] /= nn; nt[1] /= nn; nt[2] /= nn;
    double xp[3]; sub3(x, P[0], xp);
    double h = dot3(xp, nt);
    double lmax = fmax(norm3(e1), norm3(e2));
    if (self || fabs(h) < 1e-13 * lmax) h = 0.0;
    double x0[3] = { x[0] - h * nt[0], x[1] - h * nt[1], x[2] - h * nt[2] };
    double ah = fabs(h);
    int ng = k->ng;
    double sa[ng], sphi[ng], sp[ng];              /* angular sums of Q(R) */
    double la[ng][3], lp[ng][3];                  /* boundary line sums of G m */
    for (int i = 0; i < ng; ++i) { sa[i] = sphi[i] = sp[i] = 0.0; for (int c = 0; c < 3; ++c) la[i][c] = lp[i][c] = 0.0; }
    double theta_tot = 0.0;   /* total signed angle subtended by T at x0 */
    double br[4100];
    for (int e = 0; e < 3; ++e) {
        const double *A = P[e], *B = P[(e + 1) % 3], *Cv = P[(e + 2) % 3];
        double t[3]; sub3(B, A, t); double L = norm3(t); t[0] /= L; t[1] /= L; t[2] /= L;
        double m[3]; cross3(t, nt, m);               /* in-plane normal to the edge */
        double ca[3]; sub3(Cv, A, ca);
        if (dot3(ca, m) > 0) { m[0] = -m[0]; m[1] = -m[1]; m[2] = -m[2]; } /* outward */
        double ax[3]; sub3(A, x0, ax);
        double bx[3]; sub3(B, x0, bx);
        double d = dot3(ax, m);                       /* >0 when x0 on the inner side */
        double sA = dot3(ax, t), sB = dot3(bx, t);
        /* ---- angular integral over the sub-triangle (x0, A, B); a field point
         * projecting onto the edge line gives a degenerate sub-triangle */
        if (fabs(d) > 1e-14 * L) {
            theta_tot += atan(sB / d) - atan(sA / d);
            double ad = fabs(d), sg = d > 0 ? 1.0 : -1.0;
            double c2 = d * d + h * h;
            /* pieces in s split at 0 and at light-cone crossings */
            double segs[2][2]; int nseg = 0;
            if (sA < 0.0 && sB > 0.0) { segs[0][0] = sA; segs[0][1] = 0.0; segs[1][0] = 0.0; segs[1][1] = sB; nseg = 2; }
            else { segs[0][0] = sA; segs[0][1] = sB; nseg = 1; }
            for (int q = 0; q < nseg; ++q) {
                double s0 = segs[q][0], s1 = segs[q][1];
                double sgn = 1.0;
                if (s1 <= 0.0) { double tt = s0; s0 = -s1; s1 = -tt; sgn = -1.0; } /* reflect to t >= 0 */
                /* now integrate over t in [s0, s1] with orientation sgn (s increasing in original) */
                int nb = pieces_pos(s0, s1, c2, k->cdt, br);
                for (int b = 0; b + 1 < nb; ++b) {
                    double va = asinh(br[b] / ad), vb = asinh(br[b + 1] / ad);
                    if (vb <= va) continue;
                    /* split long pieces into unit lengths in v */
                    int nsub = (int)ceil((vb - va) / 1.0);
                    for (int u = 0; u < nsub; ++u) {
                        double v0 = va + (vb - va) * u / nsub, v1 = va + (vb - va) * (u + 1) / nsub;
                        ang_piece(k, d, h, v0, v1, sg, sa, sphi, sp, 0);
                    }
                }
                (void)sgn;
            }
        }
        /* ---- boundary line integral of G along the edge, times m */
        {
            double rho2 = d * d + h * h, rho = sqrt(rho2);
            double la_e[ng], lp_e[ng];
            for (int i = 0; i < ng; ++i) { la_e[i] = 0.0; lp_e[i] = 0.0; }
            double segs[2][2]; int nseg;
            if (sA < 0.0 && sB > 0.0) { segs[0][0] = 0.0; segs[0][1] = -sA; segs[1][0] = 0.0; segs[1][1] = sB; nseg = 2; }
            else if (sB <= 0.0) { segs[0][0] = -sB; segs[0][1] = -sA; nseg = 1; }
            else { segs[0][0] = sA; segs[0][1] = sB; nseg = 1; }
            for (int q = 0; q < nseg; ++q) {
                double t0 = segs[q][0], t1 = segs[q][1];
                if (t1 <= t0) continue;
                int nb = pieces_pos(t0, t1, rho2, k->cdt, br);
                for (int b = 0; b + 1 < nb; ++b) {
                    double wa, wb;
                    if (rho > 1e-14 * L) { wa = asinh(br[b] / rho); wb = asinh(br[b + 1] / rho); }
                    else { wa = br[b]; wb = br[b + 1]; }
                    if (wb <= wa) continue;
                    double len = wb - wa;
                    int nsub = rho > 1e-14 * L ? (int)ceil(len / 1.0) : 1;
                    for (int u = 0; u < nsub; ++u) {
                        double w0 = wa + len * u / nsub, w1 = wa + len * (u + 1) / nsub;
                        line_piece(k, rho > 1e-14 * L ? rho : 0.0, w0, w1, la_e, lp_e, 0);
                    }
                }
            }
            for (int i = 0; i < ng; ++i)
                for (int c = 0; c < 3; ++c) { la[i][c] += la_e[i] * m[c]; lp[i][c] += lp_e[i] * m[c]; }
        }
    }
    /* subtract Q(|h|) times the total subtended angle: 2 pi with the
     * projection inside, 0 outside, pi on an edge, the corner angle at a vertex */
    double qa[ng], qphi[ng], qp[ng];
    for (int i = 0; i < ng; ++i) {
        acc[i].as = sa[i]; acc[i].phis = sphi[i]; acc[i].ps = sp[i];
    }
    if (ah > 0.0) {
        radial_q(k, 0, ng, ah, qa, qphi, qp);
        for (int i = 0; i < ng; ++i) {
            acc[i].as -= theta_tot * qa[i]; acc[i].phis -= theta_tot * qphi[i]; acc[i].ps -= theta_tot * qp[i];
        }
    } else {
        /* h = 0: Qa(0), Qphi(0) finite; the psi integral only ever enters
         * multiplied by h = 0 */
        for (int i = 0; i < ng; ++i) {
            double tau = (double)(k->g0 + i);
            acc[i].as -= theta_tot * (-k->cdt * bs1(tau));
            acc[i].phis -= theta_tot * (-k->cdt * bsm1(tau));
            acc[i].ps = 0.0;
        }
    }
    for (int i = 0; i < ng; ++i) {
        for (int c = 0; c < 3; ++c) {
            acc[i].av[c] = la[i][c] - h * nt[c] * acc[i].as;
            acc[i].pv[c] = lp[i][c] - (h != 0.0 ? h * nt[c] * acc[i].ps : 0.0);
        }
    }
}

/* exported for pin tests: integrals of the kernels for one field point and
 * triangle.  out layout per lag: [as, phis, ps, av0, av1, av2, pv0, pv1, pv2] */
void orc_tri_integrals(const double *x, const double *tri9, int self, double cdt, double dt,
                       double zeta, double kd, int g0, int ng, double *out) {
    gl_init();
    double P[3][3];
    for (int a = 0; a < 3; ++a) for (int c = 0; c < 3; ++c) P[a][c] = tri9[3 * a + c];
    kpar_t k = { cdt, dt, zeta, kd, g0, ng };
    acc_t acc[NGMAX];
    tri_integrals(x, P, self, &k, acc);
    for (int i = 0; i < ng; ++i) {
        double *o = out + 9 * i;
        o[0] = acc[i].as; o[1] = acc[i].phis; o[2] = acc[i].ps;
        for (int c = 0; c < 3; ++c) { o[3 + c] = acc[i].av[c]; o[6 + c] = acc[i].pv[c]; }
    }
}

/* ------------------------------------------------------------ RWG bases */
/* Edge j: triangles etri[2j] (T+) and etri[2j+1] (T-); free vertices efree[2j], efree[2j+1].
 * f_j(x) = +l/(2A+) (x - o+) on T+,  -l/(2A-) (x - o-) on T-;  div f = +-l/A+-. */
typedef struct {
    const double *xyz; const int *tri; const int *etri; const int *efree; const double *elen;
} mesh_t;

static void tri_verts(const mesh_t *M, int t, double P[3][3]) {
    for (int a = 0; a < 3; ++a) for (int c = 0; c < 3; ++c) P[a][c] = M->xyz[3 * M->tri[3 * t + a] + c];
}
static double tri_area(const double P[3][3], double *nout) {
    double e1[3], e2[3], n[3]; sub3(P[1], P[0], e1); sub3(P[2], P[0], e2); cross3(e1, e2, n);
    double a = norm3(n);
    if (nout) { nout[0] = n[0] / a; nout[1] = n[1] / a; nout[2] = n[2] / a; }
    return 0.5 * a;
}
/* interior 3-point rule: barycentric (2/3,1/6,1/6) and permutations, weights 1/3 */
static void quad_points(const double P[3][3], double X[3][3]) {
    for (int q = 0; q < 3; ++q)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a) s += (a == q ? 2.0 / 3.0 : 1.0 / 6.0) * P[a][c];
            X[q][c] = s;
        }
}

/* J-form coefficients for a list of (i, j) pairs; out[p*G + g], g = 0..G-1 (g=0 unused). */
void orc_zpairs(const double *xyz, const int *tri, const int *etri, const int *efree, const double *elen,
                double cdt, double eps, double mu, double theta, double zeta, double kd,
                long npairs, const int *pi, const int *pj, int G, double *out, int nthreads) {
    gl_init();
    mesh_t M = { xyz, tri, etri, efree, elen };
    double c = cdt; (void)c;
    double cl = 1.0 / sqrt(eps * mu), dt = cdt / cl, eta = sqrt(mu / eps);
    memset(out, 0, sizeof(double) * (size_t)npairs * G);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (long p = 0; p < npairs; ++p) {
        int i = pi[p], j = pj[p];
        double *z = out + (size_t)p * G;
        acc_t *acc = (acc_t *)malloc(sizeof(acc_t) * NGMAX);
        for (int rho = 0; rho < 2; ++rho) {
            int ti = etri[2 * i + rho];
            double Pi[3][3], ni_out[3], X[3][3];
            tri_verts(&M, ti, Pi);
            double Ai = tri_area(Pi, ni_out);
            double ni[3] = { -ni_out[0], -ni_out[1], -ni_out[2] };   /* inward normal */
            quad_points(Pi, X);
            const double *oi = xyz + 3 * efree[2 * i + rho];
            double si = (rho == 0 ? 1.0 : -1.0) * elen[i] / (2.0 * Ai);
            double divi = (rho == 0 ? 1.0 : -1.0) * elen[i] / Ai;
            for (int sg = 0; sg < 2; ++sg) {
                int tj = etri[2 * j + sg];
                double Pj[3][3];
                tri_verts(&M, tj, Pj);
                double Aj = tri_area(Pj, NULL);
                const double *oj = xyz + 3 * efree[2 * j + sg];
                double sj = (sg == 0 ? 1.0 : -1.0) * elen[j] / (2.0 * Aj);
                double divj = (sg == 0 ? 1.0 : -1.0) * elen[j] / Aj;
                for (int q = 0; q < 3; ++q) {
                    const double *x = X[q];
                    /* lag range from distance bounds of x to the triangle: B(tau_g(r)) != 0
                     * needs r/cdt < g < r/cdt + 3 for some r in [rmin, rmax] */
                    double rmax = 0.0, cen[3], rad = 0.0;
                    for (int cc = 0; cc < 3; ++cc) cen[cc] = (Pj[0][cc] + Pj[1][cc] + Pj[2][cc]) / 3.0;
                    for (int a = 0; a < 3; ++a) {
                        double dv[3]; sub3(Pj[a], x, dv); rmax = fmax(rmax, norm3(dv));
                        sub3(Pj[a], cen, dv); rad = fmax(rad, norm3(dv));
                    }
                    double xc[3]; sub3(x, cen, xc);
                    double rmin = fmax(0.0, norm3(xc) - rad);
                    int g0 = (int)floor(rmin / cdt) + 1, g1 = (int)floor(rmax / cdt) + 3;
                    if (g0 < 1) g0 = 1;
                    if (g1 > G - 1) g1 = G - 1;
                    if (g1 < g0) continue;
                    kpar_t kp = { cdt, dt, zeta, kd, g0, g1 - g0 + 1 };
                    tri_integrals(x, Pj, ti == tj, &kp, acc);
                    double fi[3]; sub3(x, oi, fi); fi[0] *= si; fi[1] *= si; fi[2] *= si;
                    double xo[3]; sub3(x, oj, xo);
                    double wq = Ai / 3.0;
                    for (int g = g0; g <= g1; ++g) {
                        acc_t *a = &acc[g - g0];
                        /* A-dd: (mu/4pi) dt^-2 int f_j B''/r = (mu/4pi) dt^-2 s_j [(x-o_j) as + av] */
                        double Av[3];
                        for (int cc = 0; cc < 3; ++cc) Av[cc] = mu / (4 * PI) / (dt * dt) * sj * (xo[cc] * a->as + a->av[cc]);
                        /* scalar: (1/4pi eps) div f_j int B/r */
                        double Ph = 1.0 / (4 * PI * eps) * divj * a->phis;
                        /* P-dot + zeta P: (1/4pi) s_j (x - o_j) x int grad(F/r) */
                        double Pv[3], t1[3];
                        cross3(xo, a->pv, t1);
                        for (int cc = 0; cc < 3; ++cc) Pv[cc] = sj / (4 * PI) * t1[cc];
                        double nxP[3]; cross3(ni, Pv, nxP);
                        z[g] += wq * (dot3(fi, Av) + divi * Ph + theta * eta * dot3(fi, nxP));
                    }
                }
            }
        }
        free(acc);
        /* identity part of the MFIE: 1/2 theta eta Gram_ij (kd dN/dt + zeta N)(t_alpha) */
        double gram = 0.0;
        for (int rho = 0; rho < 2; ++rho)
            for (int sg = 0; sg < 2; ++sg) {
                int ti = etri[2 * i + rho], tj = etri[2 * j + sg];
                if (ti != tj) continue;
                double Pt[3][3], X[3][3];
                tri_verts(&M, ti, Pt);
                double A = tri_area(Pt, NULL);
                quad_points(Pt, X);
                const double *oi = xyz + 3 * efree[2 * i + rho], *oj = xyz + 3 * efree[2 * j + sg];
                double si = (rho == 0 ? 1.0 : -1.0) * elen[i] / (2.0 * A);
                double sj = (sg == 0 ? 1.0 : -1.0) * elen[j] / (2.0 * A);
                for (int q = 0; q < 3; ++q) {
                    double a[3], b[3]; sub3(X[q], oi, a); sub3(X[q], oj, b);
                    gram += A / 3.0 * si * sj * dot3(a, b);
                }
            }
        if (gram != 0.0 && G > 2) {
            z[1] += 0.5 * theta * eta * gram * (kd / dt + 0.5 * zeta);
            z[2] += 0.5 * theta * eta * gram * (-kd / dt + 0.5 * zeta);
        }
    }
}

/* Dense J-form rows: out[r][j][g] = Zt^(g)_{rows[r], j} for all edges j and
 * g = 0..G-1.  The same sum as orc_zpairs, organised per (test triangle,
 * source triangle) so that each inner integral is evaluated once per row. */
void orc_zrows(const double *xyz, const int *tri, int ntri, const int *etri, const int *efree,
               const double *elen, int ne, const int *tedge /* [ntri][3] edge ids */,
               double cdt, double eps, double mu, double theta, double zeta, double kd,
               int nrows, const int *rows, int G, double *out, int nthreads, int terms) {
    /* terms: bit 0 vector potential, bit 1 scalar potential, bit 2 magnetic
     * potential, bit 3 MFIE identity (Gram) term; 15 = the full operator */
    gl_init();
    double tA = (terms & 1) ? 1.0 : 0.0, tP = (terms & 2) ? 1.0 : 0.0, tM = (terms & 4) ? 1.0 : 0.0;
    mesh_t M = { xyz, tri, etri, efree, elen };
    double cl = 1.0 / sqrt(eps * mu), dt = cdt / cl, eta = sqrt(mu / eps);
    memset(out, 0, sizeof(double) * (size_t)nrows * ne * G);
    /* buf[(r*ntri + t)*3*G + k*G + g]: contribution of source triangle t through its k-th edge */
    double *buf = (double *)calloc((size_t)nrows * ntri * 3 * G, sizeof(double));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 8)
#endif
    for (long rt = 0; rt < (long)nrows * ntri; ++rt) {
        int r = (int)(rt / ntri), tj = (int)(rt % ntri);
        int i = rows[r];
        double *b = buf + (size_t)rt * 3 * G;
        acc_t acc[NGMAX];
        double Pj[3][3];
        tri_verts(&M, tj, Pj);
        double Aj = tri_area(Pj, NULL);
        double cen[3], rad = 0.0;
        for (int cc = 0; cc < 3; ++cc) cen[cc] = (Pj[0][cc] + Pj[1][cc] + Pj[2][cc]) / 3.0;
        for (int a = 0; a < 3; ++a) { double dv[3]; sub3(Pj[a], cen, dv); rad = fmax(rad, norm3(dv)); }
        for (int rho = 0; rho < 2; ++rho) {
            int ti = etri[2 * i + rho];
            double Pi[3][3], ni_out[3], X[3][3];
            tri_verts(&M, ti, Pi);
            double Ai = tri_area(Pi, ni_out);
            double ni[3] = { -ni_out[0], -ni_out[1], -ni_out[2] };
            quad_points(Pi, X);
            const double *oi = xyz + 3 * efree[2 * i + rho];
            double si = (rho == 0 ? 1.0 : -1.0) * elen[i] / (2.0 * Ai);
            double divi = (rho == 0 ? 1.0 : -1.0) * elen[i] / Ai;
            for (int q = 0; q < 3; ++q) {
                const double *x = X[q];
                double rmax = 0.0;
                for (int a = 0; a < 3; ++a) { double dv[3]; sub3(Pj[a], x, dv); rmax = fmax(rmax, norm3(dv)); }
                double xc[3]; sub3(x, cen, xc);
                double rmin = fmax(0.0, norm3(xc) - rad);
                int g0 = (int)floor(rmin / cdt) + 1, g1 = (int)floor(rmax / cdt) + 3;
                if (g0 < 1) g0 = 1;
                if (g1 > G - 1) g1 = G - 1;
                if (g1 < g0) continue;
                kpar_t kp = { cdt, dt, zeta, kd, g0, g1 - g0 + 1 };
                tri_integrals(x, Pj, ti == tj, &kp, acc);
                double fi[3]; sub3(x, oi, fi); fi[0] *= si; fi[1] *= si; fi[2] *= si;
                double wq = Ai / 3.0;
                for (int kk = 0; kk < 3; ++kk) {
                    int j = tedge[3 * tj + kk];
                    int sg = etri[2 * j] == tj ? 0 : 1;
                    const double *oj = xyz + 3 * efree[2 * j + sg];
                    double sj = (sg == 0 ? 1.0 : -1.0) * elen[j] / (2.0 * Aj);
                    double divj = (sg == 0 ? 1.0 : -1.0) * elen[j] / Aj;
                    double xo[3]; sub3(x, oj, xo);
                    for (int g = g0; g <= g1; ++g) {
                        acc_t *a = &acc[g - g0];
                        double Av[3];
                        for (int cc = 0; cc < 3; ++cc) Av[cc] = mu / (4 * PI) / (dt * dt) * sj * (xo[cc] * a->as + a->av[cc]);
                        double Ph = 1.0 / (4 * PI * eps) * divj * a->phis;
                        double Pv[3], t1[3];
                        cross3(xo, a->pv, t1);
                        for (int cc = 0; cc < 3; ++cc) Pv[cc] = sj / (4 * PI) * t1[cc];
                        double nxP[3]; cross3(ni, Pv, nxP);
                        b[kk * G + g] += wq * (tA * dot3(fi, Av) + tP * divi * Ph + tM * theta * eta * dot3(fi, nxP));
                    }
                }
            }
        }
    }
    for (int r = 0; r < nrows; ++r) {
        int i = rows[r];
        double *o = out + (size_t)r * ne * G;
        for (int tj = 0; tj < ntri; ++tj)
            for (int kk = 0; kk < 3; ++kk) {
                int j = tedge[3 * tj + kk];
                const double *b = buf + ((size_t)r * ntri + tj) * 3 * G + kk * G;
                for (int g = 0; g < G; ++g) o[(size_t)j * G + g] += b[g];
            }
        /* identity part of the MFIE on shared triangles */
        for (int j = 0; j < ne; ++j) {
            double gram = 0.0;
            for (int rho = 0; rho < 2; ++rho)
                for (int sg = 0; sg < 2; ++sg) {
                    int ti = etri[2 * i + rho], tj = etri[2 * j + sg];
                    if (ti != tj) continue;
                    double Pt[3][3], X[3][3];
                    tri_verts(&M, ti, Pt);
                    double A = tri_area(Pt, NULL);
                    quad_points(Pt, X);
                    const double *oi = xyz + 3 * efree[2 * i + rho], *oj = xyz + 3 * efree[2 * j + sg];
                    double si = (rho == 0 ? 1.0 : -1.0) * elen[i] / (2.0 * A);
                    double sj = (sg == 0 ? 1.0 : -1.0) * elen[j] / (2.0 * A);
                    for (int q = 0; q < 3; ++q) {
                        double a[3], bb[3]; sub3(X[q], oi, a); sub3(X[q], oj, bb);
                        gram += A / 3.0 * si * sj * dot3(a, bb);
                    }
                }
            if (gram != 0.0 && G > 2 && (terms & 8)) {
                o[(size_t)j * G + 1] += 0.5 * theta * eta * gram * (kd / dt + 0.5 * zeta);
                o[(size_t)j * G + 2] += 0.5 * theta * eta * gram * (-kd / dt + 0.5 * zeta);
            }
        }
    }
    free(buf);
}

/* Gram matrix entries for pairs (exact with the 3-point rule: degree-2 integrand). */
void orc_gram(const double *xyz, const int *tri, const int *etri, const int *efree, const double *elen,
              long npairs, const int *pi, const int *pj, double *out) {
    mesh_t M = { xyz, tri, etri, efree, elen };
    for (long p = 0; p < npairs; ++p) {
        int i = pi[p], j = pj[p];
        double g = 0.0;
        for (int rho = 0; rho < 2; ++rho)
            for (int sg = 0; sg < 2; ++sg) {
                int ti = etri[2 * i + rho], tj = etri[2 * j + sg];
                if (ti != tj) continue;
                double Pt[3][3], X[3][3];
                tri_verts(&M, ti, Pt);
                double A = tri_area(Pt, NULL);
                quad_points(Pt, X);
                const double *oi = xyz + 3 * efree[2 * i + rho], *oj = xyz + 3 * efree[2 * j + sg];
                double si = (rho == 0 ? 1.0 : -1.0) * elen[i] / (2.0 * A);
                double sj = (sg == 0 ? 1.0 : -1.0) * elen[j] / (2.0 * A);
                for (int q = 0; q < 3; ++q) {
                    double a[3], b[3]; sub3(X[q], oi, a); sub3(X[q], oj, b);
                    g += A / 3.0 * si * sj * dot3(a, b);
                }
            }
        out[p] = g;
    }
}

/* ------------------------------------------------------- incident field */
/* pulse[11] = k(3), p(3), E0, f0, sigma, delay, kind.
 * kind 0: E = E0 p cos(2 pi f0 tau) exp(-tau^2/2sigma^2), tau = t - delay - k.x/c
 * kind 1: E = E0 p Sin^2(2 pi f0 (tau)) on one period (Section 4.1's Sin^2), tau as above
 * kind 2: E = E0 p exp(-tau^2/2sigma^2)/sqrt(2 pi sigma^2) (Section 4.3)
 * returns g(tau) and g'(tau) (time derivative). */
static void pulse_wave(const double *pl, double tau, double *g, double *gd) {
    int kind = (int)pl[10];
    double f0 = pl[7], sig = pl[8];
    if (kind == 0) {
        double e = exp(-tau * tau / (2 * sig * sig));
        double cs = cos(2 * PI * f0 * tau), sn = sin(2 * PI * f0 * tau);
        *g = cs * e;
        *gd = (-2 * PI * f0 * sn - tau / (sig * sig) * cs) * e;
    } else if (kind == 1) {
        double arg = 2 * PI * f0 * tau;
        if (arg < 0.0 || arg > 2 * PI) { *g = 0.0; *gd = 0.0; return; }
        double s = sin(arg);
        *g = s * s; *gd = 2 * s * cos(arg) * 2 * PI * f0;
    } else {
        double e = exp(-tau * tau / (2 * sig * sig)) / sqrt(2 * PI * sig * sig);
        *g = e; *gd = -tau / (sig * sig) * e;
    }
}

/* V_i^{alpha-1}: tested  -dE/dt + theta eta n x (kd dH/dt + zeta H)  at t = t_alpha (Eq. v_i). */
void orc_vinc(const double *xyz, const int *tri, const int *etri, const int *efree, const double *elen,
              int ne, const double *pulse, double eps, double mu, double theta, double zeta, double kd,
              double t, double *out) {
    mesh_t M = { xyz, tri, etri, efree, elen };
    double cl = 1.0 / sqrt(eps * mu), eta = sqrt(mu / eps);
    const double *kk = pulse, *pp = pulse + 3;
    double E0 = pulse[6], delay = pulse[9];
    double kxp[3]; cross3(kk, pp, kxp);
    for (int i = 0; i < ne; ++i) {
        double v = 0.0;
        for (int rho = 0; rho < 2; ++rho) {
            int ti = etri[2 * i + rho];
            double Pt[3][3], X[3][3], nout[3];
            tri_verts(&M, ti, Pt);
            double A = tri_area(Pt, nout);
            double n[3] = { -nout[0], -nout[1], -nout[2] };
            quad_points(Pt, X);
            const double *o = xyz + 3 * efree[2 * i + rho];
            double s = (rho == 0 ? 1.0 : -1.0) * elen[i] / (2.0 * A);
            for (int q = 0; q < 3; ++q) {
                double tau = t - delay - dot3(kk, X[q]) / cl, g, gd;
                pulse_wave(pulse, tau, &g, &gd);
                double Ed[3], Hs[3], nxH[3];
                for (int c = 0; c < 3; ++c) {
                    Ed[c] = E0 * pp[c] * gd;
                    Hs[c] = E0 * kxp[c] / eta * (kd * gd + zeta * g);
                }
                cross3(n, Hs, nxH);
                double f[3]; sub3(X[q], o, f);
                double val = 0.0;
                for (int c = 0; c < 3; ++c) val += s * f[c] * (-Ed[c] + theta * eta * nxH[c]);
                v += A / 3.0 * val;
            }
        }
        out[i] = v;
    }
}

/* ------------------------------------------------------ history sum */
/* Sparse J-form store: pair p = (row[p], col[p]) holds lags g0[p] .. g0[p]+len[p]-1
 * at vals[off[p] ...].  hist[b*ne + j] = J_j^b for b = 0..nb-1.
 * out[i] = sum_p sum_{g>=gmin} Zt^(g)_{ij} J_j^{alpha-g}   (J^{<0} = 0). */
void orc_history(long npairs, const int *row, const int *col, const int *g0, const int *len,
                 const long *off, const double *vals, int ne, const double *hist, int nb,
                 int alpha, int gmin, double *out) {
    memset(out, 0, sizeof(double) * ne);
    for (long p = 0; p < npairs; ++p) {
        double s = 0.0;
        for (int l = 0; l < len[p]; ++l) {
            int g = g0[p] + l;
            int b = alpha - g;
            if (g < gmin || b < 0 || b >= nb) continue;
            s += vals[off[p] + l] * hist[(size_t)b * ne + col[p]];
        }
        out[row[p]] += s;
    }
}
