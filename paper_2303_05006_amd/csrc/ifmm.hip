// Space-time interpolation-based FMM for the far field (Section 3).
//
// Hierarchy (Section 3.4.1): cells per level, interaction lists I(C), steps per
// interval M_t(l_max) = floor(d_s/(c dt)), M_t(l) = 2 M_t(l+1).  Interpolation:
// Lagrange on p equispaced nodes per axis and in time (p_s = p_t = 4, a
// 256-vector per channel, index ((b1 p + b2) p + b3) p + n as in Section 3.6.1).
// Channels: 0-2 vector potential (kernel dU/dt = 2c(c(t-s)-r)_+/r), 3 scalar
// potential and 4-6 magnetic potential (kernel U = (c(t-s)-r)_+^2/r).
//
// Time gating (Programs 3-4): when alpha is a multiple of M_t(l), interval k =
// alpha/M_t - 1 of level l is complete: P2M at leaves, M2M above (upward), then
// M2L for the next interval k+1, L2L to the children's next two intervals and
// L2P into the right-hand sides of the steps of interval k+1 (downward).
//
// Finite M2L window: sources are the W most recent intervals.  Every node pair
// of lag m >= mu + 1 lies inside the light cone (mu rho >= 4 sqrt 3, rho =
// c M_t dt / d_s), where the node values of U and dU/dt are polynomials of
// degree <= 2 in s; the interpolant reproduces them, and since the B-spline
// weights w annihilate quadratics, the whole older history reduces to the
// window's moments built from the current difference truncated at the oldest
// window interval's start beta* (Eq. hat_J with that beta*).  The truncation
// reaches 3 steps: it changes the oldest interval, and with M_t < 3 steps per
// interval also the next ceil(3/M_t) - 1 ones, so each source interval keeps its
// full moments and NTR = ceil(3/M_t) truncated variants (variant v truncated v
// intervals before its start), and W = mu + NTR keeps every interval a
// truncation touches in the polynomial regime.  This reproduces the sum over
// all earlier intervals exactly for any M_t >= 1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "far_internal.h"
#include "ifmm.h"
#include "mfma.h"

namespace tdbem {

// ------------------------------------------------------------ host helpers
// Cardinal functions on p equispaced nodes w_n = -1 + 2n/(p-1) (p <= PMAX).
static void lagr(int p, double xi, double *v, double *d) {
    double w[PMAX];
    for (int n = 0; n < p; ++n) w[n] = -1.0 + 2.0 * n / (p - 1);
    for (int n = 0; n < p; ++n) {
        double den = 1.0, prod = 1.0, der = 0.0;
        for (int m = 0; m < p; ++m) {
            if (m == n) continue;
            den *= w[n] - w[m];
            prod *= xi - w[m];
        }
        for (int k = 0; k < p; ++k) {
            if (k == n) continue;
            double t = 1.0;
            for (int m = 0; m < p; ++m)
                if (m != n && m != k) t *= xi - w[m];
            der += t;
        }
        v[n] = prod / den;
        if (d) d[n] = der / den;
    }
}

// node slopes of the cardinal function m: finite differences of its node values
// (central inside, second-order one-sided at the ends)
static void chi_slopes(int p, int m, double h, double *f, double *sl) {
    for (int n = 0; n < p; ++n) f[n] = n == m ? 1.0 : 0.0;
    sl[0] = (-3 * f[0] + 4 * f[1] - f[2]) / (2 * h);
    sl[p - 1] = (3 * f[p - 1] - 4 * f[p - 2] + f[p - 3]) / (2 * h);
    for (int n = 1; n < p - 1; ++n) sl[n] = (f[n + 1] - f[n - 1]) / (2 * h);
}

// piecewise cubic Hermite interpolation on the equispaced nodes with node slopes
// from finite differences: cardinal functions and their derivatives at xi
// (reproduces quadratics)
static void chi(int p, double xi, double *v, double *d) {
    const double h = 2.0 / (p - 1);
    int i = (int)std::floor((xi + 1.0) / h);
    i = std::min(std::max(i, 0), p - 2);
    const double t = (xi - (-1.0 + h * i)) / h;
    const double h00 = 2 * t * t * t - 3 * t * t + 1, h10 = t * t * t - 2 * t * t + t;
    const double h01 = -2 * t * t * t + 3 * t * t, h11 = t * t * t - t * t;
    const double d00 = 6 * t * t - 6 * t, d10 = 3 * t * t - 4 * t + 1, d01 = -6 * t * t + 6 * t, d11 = 3 * t * t - 2 * t;
    for (int m = 0; m < p; ++m) {
        double f[PMAX], sl[PMAX];
        chi_slopes(p, m, h, f, sl);
        v[m] = h00 * f[i] + h10 * h * sl[i] + h01 * f[i + 1] + h11 * h * sl[i + 1];
        if (d) d[m] = (d00 * f[i] + d10 * h * sl[i] + d01 * f[i + 1] + d11 * h * sl[i + 1]) / h;
    }
}

// second derivatives of the cardinal functions at xi
static void lagr2(int p, double xi, double *dd) {
    double w[PMAX];
    for (int n = 0; n < p; ++n) w[n] = -1.0 + 2.0 * n / (p - 1);
    for (int n = 0; n < p; ++n) {
        double den = 1.0, s = 0.0;
        for (int m = 0; m < p; ++m)
            if (m != n) den *= w[n] - w[m];
        for (int k = 0; k < p; ++k)
            for (int q = 0; q < p; ++q) {
                if (k == n || q == n || q == k) continue;
                double t = 1.0;
                for (int m = 0; m < p; ++m)
                    if (m != n && m != k && m != q) t *= xi - w[m];
                s += t;
            }
        dd[n] = s / den;
    }
}
// (discontinuous at the interior nodes: a point on a node, within 1e-9 of the
// segment length, takes the segment on its left, the limit from the past)
static void chi2(int p, double xi, double *dd) {
    const double h = 2.0 / (p - 1);
    int i = (int)std::ceil((xi + 1.0) / h - 1e-9) - 1;
    i = std::min(std::max(i, 0), p - 2);
    const double t = (xi - (-1.0 + h * i)) / h;
    const double e00 = 12 * t - 6, e10 = 6 * t - 4, e01 = -12 * t + 6, e11 = 6 * t - 2;
    for (int m = 0; m < p; ++m) {
        double f[PMAX], sl[PMAX];
        chi_slopes(p, m, h, f, sl);
        dd[m] = (e00 * f[i] + e10 * h * sl[i] + e01 * f[i + 1] + e11 * h * sl[i + 1]) / (h * h);
    }
}

// temporal cardinal functions of the configured interpolant
static void tcard(int p, int interp, double xi, double *v, double *d) {
    if (interp == TDBEM_INTERP_CHI_TIME) chi(p, xi, v, d); else lagr(p, xi, v, d);
}
static void tcard2(int p, int interp, double xi, double *dd) {
    if (interp == TDBEM_INTERP_CHI_TIME) chi2(p, xi, dd); else lagr2(p, xi, dd);
}

template <typename T>
static T *falloc(tdbem_ctx *C, size_t n) {
    if (n == 0) n = 1;
    void *p = nullptr;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess)
        throw Error{TDBEM_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed (far field)"};
    C->allocs.push_back(p);
    C->dev_bytes += n * sizeof(T);
    return (T *)p;
}
void *far_alloc(tdbem_ctx *C, size_t bytes) { return falloc<char>(C, bytes); }

template <typename T>
static T *fup(tdbem_ctx *C, const std::vector<T> &v) {
    T *p = falloc<T>(C, v.size());
    if (!v.empty()) TD_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
}

void ifmm_setup(tdbem_ctx *C) {
    const Tree &T = C->T;
    const HostMesh &H = C->H;
    const int P = C->cfg.p_s;
    TD_REQUIRE(C->cfg.p_t == P && (P == 4 || P == 6 || P == 8), TDBEM_EINVAL,
               "the far field is built for p_s = p_t = 4, 6 or 8");
    TD_REQUIRE(C->cfg.m2l >= TDBEM_M2L_AUTO && C->cfg.m2l <= TDBEM_M2L_BF16, TDBEM_EINVAL, "unknown M2L kernel");
    TD_REQUIRE(C->cfg.m2l != TDBEM_M2L_BF16 || P == 4, TDBEM_EINVAL, "the bf16 M2L is built for p_s = p_t = 4");
    TD_REQUIRE(C->cfg.m2l != TDBEM_M2L_FFT || C->cfg.precision == TDBEM_FP64, TDBEM_EINVAL,
               "the Fourier-domain M2L computes in FP64 (precision must be TDBEM_FP64)");
    TD_REQUIRE(T.lmax >= 2, TDBEM_EINVAL, "IFMM needs at least two levels below the root");
    FarState *F = new FarState();
    C->far = F;
    F->P = P;
    F->NS = P * P * P;
    F->NN = F->NS * P;
    F->fft_m2l = C->cfg.m2l == TDBEM_M2L_FFT;
    F->bf16_m2l = C->cfg.m2l == TDBEM_M2L_BF16;
    F->generic_m2l = !F->fft_m2l && (P != 4 || C->cfg.m2l == TDBEM_M2L_GENERIC);
    const int NS = F->NS, NN = F->NN;
    const int interp = C->cfg.interp;
    F->lmax = T.lmax;
    F->nrhs = C->nrhs;
    const double ds_max = T.side / std::ldexp(1.0, T.lmax);
    double reach = ds_max;
    if (C->cfg.causal_guard) {
        // shrink the interval so that no far pair (cells one cell apart, supports
        // reaching beyond their cell by up to delta) interacts within one interval
        const HostMesh &Hm = C->H;
        double delta = 0.0;
        for (int e = 0; e < C->ne; ++e) {
            const double *a = &Hm.xyz[3 * Hm.edge_v[2 * e]], *b = &Hm.xyz[3 * Hm.edge_v[2 * e + 1]];
            double m[3] = {0.5 * (a[0] + b[0]), 0.5 * (a[1] + b[1]), 0.5 * (a[2] + b[2])};
            for (int sd = 0; sd < 2; ++sd) {
                const double *o = &Hm.xyz[3 * Hm.efree[2 * e + sd]];
                delta = std::max(delta, std::sqrt((o[0] - m[0]) * (o[0] - m[0]) + (o[1] - m[1]) * (o[1] - m[1]) +
                                                  (o[2] - m[2]) * (o[2] - m[2])));
            }
            delta = std::max(delta, 0.5 * Hm.elen[e]);
        }
        reach = ds_max - 2.0 * delta;
    }
    int Mmax = (int)std::floor(reach / C->cdt);
    TD_REQUIRE(Mmax >= 1, TDBEM_EBREAKDOWN,
               "time hierarchy breaks down: no step per finest interval (floor(d_s/(c dt)) = " + std::to_string(Mmax) +
                   ", Remark 1)");
    double rho = C->cdt * Mmax / ds_max;
    int mu = std::max(C->cfg.mu_window, (int)std::ceil(4.0 * std::sqrt(3.0) / rho - 1e-12));
    C->Mt.assign(T.lmax + 1, 0);
    F->lev.resize(T.lmax + 1);
    for (int l = 2; l <= T.lmax; ++l) C->Mt[l] = Mmax << (T.lmax - l);
    C->windows.assign(T.lmax + 1, 0);
    C->window = 0;
    for (int l = 2; l <= T.lmax; ++l) {
        FarLevel &FL = F->lev[l];
        const int ntr = (3 + C->Mt[l] - 1) / C->Mt[l];     // truncated variants: ceil(3 / M_t)
        FL.NV = 1 + ntr;
        FL.W = mu + ntr;
        FL.WR = FL.W + 1;
        TD_REQUIRE(FL.W <= 20, TDBEM_EBREAKDOWN,
                   "far-field window of more than 20 intervals (c dt too small for the finest cells)");
        C->windows[l] = FL.W;
        C->window = std::max(C->window, FL.W);
    }
    int FR = 8;
    while (FR < 2 * C->Mt[2] + 2) FR <<= 1;
    F->FR = FR;
    C->far_ring_need = C->Mt[2] + 4;
    const int nr = C->nrhs;
    // interpolation boxes: the cell widened by the largest distance (per axis) that
    // a basis support reaches beyond its edge midpoint, so that every quadrature
    // point of a cell's edges lies inside its box (no extrapolation)
    if (C->cfg.box_widen) {
        double d = 0.0;
        for (int e = 0; e < C->ne; ++e) {
            const double *a = &H.xyz[3 * H.edge_v[2 * e]], *b = &H.xyz[3 * H.edge_v[2 * e + 1]];
            const double *o0 = &H.xyz[3 * H.efree[2 * e]], *o1 = &H.xyz[3 * H.efree[2 * e + 1]];
            for (int k = 0; k < 3; ++k) {
                const double m = 0.5 * (a[k] + b[k]);
                d = std::max(d, std::max(std::max(std::fabs(a[k] - m), std::fabs(b[k] - m)),
                                         std::max(std::fabs(o0[k] - m), std::fabs(o1[k] - m))));
            }
        }
        F->delta = d;
    }
    // per-level structure
    for (int l = 2; l <= T.lmax; ++l) {
        const Level &L = T.lev[l];
        FarLevel &FL = F->lev[l];
        FL.n = L.n;
        FL.M = C->Mt[l];
        FL.ds = T.side / std::ldexp(1.0, l);
        FL.hs = 0.5 * FL.ds;
        FL.hn = FL.hs + F->delta;
        FL.ht = 0.5 * FL.M * C->cfg.dt;
        FL.il_off = fup(C, L.il_off);
        FL.il_src = fup(C, L.il_src);
        FL.il_code = fup(C, L.il_code);
        std::vector<int> ix(3 * (size_t)L.n);
        for (int c = 0; c < L.n; ++c) { ix[3 * c] = L.ix[c]; ix[3 * c + 1] = L.iy[c]; ix[3 * c + 2] = L.iz[c]; }
        FL.ix = fup(C, ix);
        FL.ebeg = fup(C, L.ebeg);
        FL.eend = fup(C, L.eend);
        std::vector<int> lc, pc;
        for (int c = 0; c < L.n; ++c) (L.leaf[c] ? lc : pc).push_back(c);
        FL.nleaf = (int)lc.size();
        FL.nparent = (int)pc.size();
        FL.leaf_cells = fup(C, lc);
        FL.parent_cells = fup(C, pc);
        FL.child_beg = fup(C, L.child_beg);
        FL.child_end = fup(C, L.child_end);
        FL.MM = falloc<double>(C, (size_t)L.n * FL.WR * FL.NV * NCH * nr * NN);
        // reduced copies of the moments, written by P2M / M2M: FP32 for the
        // reduced forms' tuned M2L, bf16 for the bf16 M2L
        const bool tuned = !F->generic_m2l && !F->fft_m2l;
        if (tuned && !F->bf16_m2l && C->cfg.precision != TDBEM_FP64)
            FL.MM32 = falloc<float>(C, (size_t)L.n * FL.WR * FL.NV * NCH * nr * NN);
        if (F->bf16_m2l) FL.MM16 = falloc<unsigned short>(C, (size_t)L.n * FL.WR * FL.NV * NCH * nr * NN);
        FL.LC = falloc<double>(C, (size_t)L.n * NCH * nr * NN);
        FL.PEND = falloc<double>(C, (size_t)L.n * 2 * NCH * nr * NN);
        // time tables: targets t = (k+1) d_t + q dt, q = 1..M, in the target interval
        // [(k+1) d_t, (k+2) d_t]: xi = 2q/M - 1; sources beta - kM = 0..M-1: xi = 2(beta-kM)/M - 1.
        // Target weights per channel group: vector potential l_m' (or l_m with
        // the kernel's second derivative, l_m'' with the kernel itself), scalar
        // potential l_m, magnetic potential kd l_m' + zeta l_m (CFIE variant).
        double kd, zeta;
        cfie_weights(C->cfg, kd, zeta);
        std::vector<double> tw((size_t)FL.M * 3 * P), ls((size_t)FL.M * P);
        for (int q = 1; q <= FL.M; ++q) {
            double v[PMAX], d[PMAX], dd[PMAX];
            tcard(P, interp, 2.0 * q / FL.M - 1.0, v, d);
            tcard2(P, interp, 2.0 * q / FL.M - 1.0, dd);
            for (int m = 0; m < P; ++m) {
                const double d1 = d[m] / FL.ht, d2 = dd[m] / (FL.ht * FL.ht);
                const double wa = C->cfg.dt2 == TDBEM_DT2_SPLIT ? d1 : C->cfg.dt2 == TDBEM_DT2_KERNEL ? v[m] : d2;
                tw[((size_t)(q - 1) * 3 + 0) * P + m] = wa;
                tw[((size_t)(q - 1) * 3 + 1) * P + m] = v[m];
                tw[((size_t)(q - 1) * 3 + 2) * P + m] = kd * d1 + zeta * v[m];
            }
        }
        for (int b = 0; b < FL.M; ++b) {
            double v[PMAX];
            tcard(P, interp, 2.0 * b / FL.M - 1.0, v, nullptr);
            for (int n = 0; n < P; ++n) ls[(size_t)b * P + n] = v[n];
        }
        FL.tw = fup(C, tw);
        FL.ls = fup(C, ls);
        if (F->fft_m2l) m2l_fft_setup(C, FL, L.il_code, m2l_kind_a(C->cfg));
        if (nr == 1 && !L.il_src.empty() && !F->fft_m2l) {
            // group interaction-list entries by offset; columns (entry, channel) per kernel kind
            std::vector<std::vector<int>> by(343);
            for (size_t q = 0; q < L.il_src.size(); ++q) by[L.il_code[q]].push_back((int)q);
            std::vector<int> tc, tk, t0, tn, cq, cch;
            for (int code = 0; code < 343; ++code) {
                if (by[code].empty()) continue;
                for (int kind = 0; kind < 2; ++kind) {
                    int c0 = kind == 0 ? 0 : 3, nc = kind == 0 ? 3 : 4;
                    int start = (int)cq.size();
                    for (int q : by[code])
                        for (int c = 0; c < nc; ++c) { cq.push_back(q); cch.push_back(c0 + c); }
                    for (int b = start; b < (int)cq.size(); b += M2L_NT) {
                        tc.push_back(code); tk.push_back(kind); t0.push_back(b);
                        tn.push_back(std::min(M2L_NT, (int)cq.size() - b));
                    }
                }
            }
            FL.ntile = (int)tc.size();
            FL.tile_code = fup(C, tc); FL.tile_kind = fup(C, tk); FL.tile_col0 = fup(C, t0); FL.tile_ncol = fup(C, tn);
            FL.col_q = fup(C, cq); FL.col_ch = fup(C, cch);
            // a level of few tiles splits its lag window over up to W blocks per
            // tile (about 2048 blocks: eight per CU), each group writing its
            // own copy of the per-entry sums
            FL.nil = (int64_t)L.il_src.size();
            FL.yg_max = FL.ntile > 0 && FL.ntile < M2L_SPLIT_BLOCKS
                            ? std::min(FL.W, (M2L_SPLIT_BLOCKS + FL.ntile - 1) / FL.ntile) : 1;
            FL.YB = falloc<double>(C, (size_t)FL.yg_max * L.il_src.size() * NCH * NN);
        }
    }
    // per-edge P2M / L2P weights at the interior 3-point rule of both triangles
    const int ne = C->ne;
    std::vector<double> Wm((size_t)ne * NCH * NS, 0.0), El((size_t)ne * NCH * NS, 0.0);
    const double PI4 = 4.0 * M_PI;
    const double sc = 1.0 / (C->cdt * C->cdt);   // (c dt)^{-d}, d = 2
    for (int p = 0; p < ne; ++p) {
        int e = T.perm[p];
        int l = T.edge_leaf_level[p], cell = T.edge_leaf_cell[p];
        const Level &L = T.lev[l];
        double ds = T.side / std::ldexp(1.0, l), hs = 0.5 * ds + F->delta;   // node half-width
        double cen[3] = {T.origin[0] + (L.ix[cell] + 0.5) * ds, T.origin[1] + (L.iy[cell] + 0.5) * ds,
                         T.origin[2] + (L.iz[cell] + 0.5) * ds};
        for (int sd = 0; sd < 2; ++sd) {
            int t = H.etri[2 * e + sd];
            double A = H.area[t];
            double s = (sd == 0 ? 1.0 : -1.0) * H.elen[e] / (2.0 * A);
            double div = 2.0 * s;
            const double *o = &H.xyz[3 * H.efree[2 * e + sd]];
            double nin[3] = {-H.nrm[3 * t], -H.nrm[3 * t + 1], -H.nrm[3 * t + 2]};
            for (int q = 0; q < 3; ++q) {
                const double *x = &H.qpt[9 * t + 3 * q];
                double w = A / 3.0;
                double f[3] = {s * (x[0] - o[0]), s * (x[1] - o[1]), s * (x[2] - o[2])};
                double fxn[3] = {f[1] * nin[2] - f[2] * nin[1], f[2] * nin[0] - f[0] * nin[2], f[0] * nin[1] - f[1] * nin[0]};
                double v[3][PMAX], d[3][PMAX];
                for (int k = 0; k < 3; ++k) lagr(P, (x[k] - cen[k]) / hs, v[k], d[k]);
                for (int b1 = 0; b1 < P; ++b1)
                    for (int b2 = 0; b2 < P; ++b2)
                        for (int b3 = 0; b3 < P; ++b3) {
                            int b = (b1 * P + b2) * P + b3;
                            double lb = v[0][b1] * v[1][b2] * v[2][b3];
                            double gb[3] = {d[0][b1] * v[1][b2] * v[2][b3] / hs, v[0][b1] * d[1][b2] * v[2][b3] / hs,
                                            v[0][b1] * v[1][b2] * d[2][b3] / hs};
                            double fxg[3] = {f[1] * gb[2] - f[2] * gb[1], f[2] * gb[0] - f[0] * gb[2], f[0] * gb[1] - f[1] * gb[0]};
                            double *wm = &Wm[(size_t)p * NCH * NS];
                            double *el = &El[(size_t)p * NCH * NS];
                            for (int c = 0; c < 3; ++c) {
                                wm[c * NS + b] += w * sc * C->cfg.mu / PI4 * f[c] * lb;
                                wm[(4 + c) * NS + b] += w * sc / PI4 * fxg[c];
                                el[c * NS + b] += w * f[c] * lb;
                                el[(4 + c) * NS + b] += w * C->cfg.theta * C->eta * fxn[c] * lb;
                            }
                            wm[3 * NS + b] += w * sc * (-1.0 / (PI4 * C->cfg.eps)) * div * lb;
                            el[3 * NS + b] += w * (-div) * lb;
                        }
            }
        }
    }
    F->Wm = fup(C, Wm);
    F->El = fup(C, El);
    // re-interpolation factors per parent level l: space [2][P][P] (child node in
    // the parent's box: ((2h - 1) hs_child + hn_child w) / hn_parent), time [2][P][P]
    std::vector<double> S1((size_t)(T.lmax + 1) * 4 * P * P, 0.0);
    for (int l = 2; l < T.lmax; ++l) {
        const double hsc = T.side / std::ldexp(1.0, l + 2), hnc = hsc + F->delta, hnp = 2.0 * hsc + F->delta;
        double *S = &S1[(size_t)l * 4 * P * P];
        for (int h = 0; h < 2; ++h)
            for (int bc = 0; bc < P; ++bc) {
                const double w = -1.0 + 2.0 * bc / (P - 1);
                double v[PMAX];
                lagr(P, ((2 * h - 1) * hsc + hnc * w) / hnp, v, nullptr);
                for (int bp = 0; bp < P; ++bp) S[(h * P + bp) * P + bc] = v[bp];   // [h][parent][child]
                tcard(P, interp, (h - 0.5) + 0.5 * w, v, nullptr);
                for (int bp = 0; bp < P; ++bp) S[2 * P * P + (h * P + bp) * P + bc] = v[bp];   // time factor
            }
    }
    F->S1 = fup(C, S1);
    F->FAR = falloc<double>(C, (size_t)F->FR * ne * nr);
    ifmm_reset(C);
}

void ifmm_reset(tdbem_ctx *C) {
    FarState *F = C->far;
    if (!F) return;
    const int NN = F->NN;
    hipStream_t s = C->stream;
    const int nr = C->nrhs;
    for (int l = 2; l <= F->lmax; ++l) {
        FarLevel &FL = F->lev[l];
        TD_HIP(hipMemsetAsync(FL.MM, 0, sizeof(double) * (size_t)FL.n * FL.WR * FL.NV * NCH * nr * NN, s));
        TD_HIP(hipMemsetAsync(FL.PEND, 0, sizeof(double) * (size_t)FL.n * 2 * NCH * nr * NN, s));
        TD_HIP(hipMemsetAsync(FL.LC, 0, sizeof(double) * (size_t)FL.n * NCH * nr * NN, s));
        if (FL.MH)
            TD_HIP(hipMemsetAsync(FL.MH, 0, sizeof(double2) * (size_t)FL.n * FL.WR * FL.NV * NCH * nr * F->NF, s));
        if (FL.MM32) TD_HIP(hipMemsetAsync(FL.MM32, 0, sizeof(float) * (size_t)FL.n * FL.WR * FL.NV * NCH * nr * NN, s));
        if (FL.MM16)
            TD_HIP(hipMemsetAsync(FL.MM16, 0, sizeof(unsigned short) * (size_t)FL.n * FL.WR * FL.NV * NCH * nr * NN, s));
    }
    TD_HIP(hipMemsetAsync(F->FAR, 0, sizeof(double) * (size_t)F->FR * C->ne * nr, s));
}

void ifmm_destroy(tdbem_ctx *C) {
    delete C->far;
    C->far = nullptr;
}

// ------------------------------------------------------------------ kernels
__constant__ double c_wk[4] = {0.5, -1.5, 1.5, -0.5};

template <int P> struct Dim {
    static constexpr int NS = P * P * P, NN = NS * P;
    static constexpr int NPT = (NN + 255) / 256;   // outputs per thread of a 256-thread block
};

// the reduced forms' copies of moments just written (FP32: rounded to float;
// BF16: rounded to float, then to bf16, nearest even)
template <int CNT>
__device__ __forceinline__ void reduced_copy(const double *o, float *MMf, unsigned short *MMh, size_t oi) {
#pragma unroll
    for (int n = 0; n < CNT; ++n) {
        const float f = (float)o[n];
        if (MMf) MMf[oi + n] = f;
        if (MMh) {
            unsigned u = __float_as_uint(f);
            u += 0x7fffu + ((u >> 16) & 1u);
            MMh[oi + n] = (unsigned short)(u >> 16);
        }
    }
}

// P2M at the leaves of one level: one block per (leaf, rhs).
// T[j][v][n] = sum_beta l_n(xi_beta) Jhat^beta_j for the moment variants v:
// v = 0 the full difference Jhat^beta = sum_{kappa <= 3} w^kappa J^{beta-kappa};
// v >= 1 truncated v - 1 intervals before the start, i.e. without the terms
// with beta - kappa < (k - v + 1) M.  MM[v][c][b][n] = sum_j Wm[j][c][b] T[j][v][n]
// over the leaf's edges, taken 64 at a time (the first chunk writes, later
// chunks add); thread = output (c, b).
template <int P>
__global__ void __launch_bounds__(256) k_p2m(const int *leaf_cells, const int *ebeg, const int *eend, int k, int M,
                                             const double *ls, const double *ring, int R, int nrhs,
                                             const double *Wm, double *MM, int slot, int WR, int NV, float *MMf,
                                             unsigned short *MMh) {
    constexpr int NS = Dim<P>::NS, NN = Dim<P>::NN;
    int cell = leaf_cells[blockIdx.x];
    int r = blockIdx.y;
    int e0 = ebeg[cell], e1 = eend[cell];
    __shared__ double T[64][NV_MAX][P];
    int beta0 = k * M;
    for (int jb = e0; jb < e1; jb += 64) {
        int nj = min(64, e1 - jb);
        __syncthreads();
        for (int q = threadIdx.x; q < nj * NV * P; q += blockDim.x) {
            int j = q / (NV * P), v = (q / P) % NV, n = q % P;
            const double *J = ring + (size_t)(jb + j) * R * nrhs + r;
            double s = 0.0;
            for (int bo = 0; bo < M; ++bo) {
                int beta = beta0 + bo;
                double jh = 0.0;
                int kmax = v == 0 ? 3 : min(3, bo + (v - 1) * M);
                for (int kap = 0; kap <= kmax; ++kap) {
                    int b = beta - kap;
                    if (b >= 0) jh += c_wk[kap] * J[(size_t)(b & (R - 1)) * nrhs];
                }
                s += ls[bo * P + n] * jh;
            }
            T[j][v][n] = s;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < NCH * NS; q += blockDim.x) {
            const int c = q / NS, b = q % NS;
            // every variant from one load of each weight (per (v, n) the sum
            // over j in the same order)
            double a[NV_MAX][P];
#pragma unroll
            for (int v = 0; v < NV_MAX; ++v)
#pragma unroll
                for (int n = 0; n < P; ++n) a[v][n] = 0.0;
            for (int j = 0; j < nj; ++j) {
                const double w = Wm[(size_t)(jb + j) * NCH * NS + q];
#pragma unroll
                for (int v = 0; v < NV_MAX; ++v) {
                    if (v >= NV) break;
#pragma unroll
                    for (int n = 0; n < P; ++n) a[v][n] += w * T[j][v][n];
                }
            }
#pragma unroll
            for (int v = 0; v < NV_MAX; ++v) {
                if (v >= NV) continue;
                const size_t oi = ((((size_t)cell * WR + slot) * NV + v) * NCH + c) * nrhs * NN + (size_t)r * NN + b * P;
                double *o = MM + oi;
#pragma unroll
                for (int n = 0; n < P; ++n) o[n] = jb == e0 ? a[v][n] : o[n] + a[v][n];
                if (jb + 64 >= e1) reduced_copy<P>(o, MMf, MMh, oi);      // the last chunk: final values
            }
        }
    }
}

// One 1-D re-interpolation along axis AX (0..2 space, 3 time) of a P^4-vector
// indexed ((i1 P + i2) P + i3) P + i4: out[.., o, ..] = sum_q A[o][q] in[.., q, ..].
template <int P, int AX>
__device__ __forceinline__ double reinterp_axis(const double *in, const double *A, int v) {
    constexpr int stride = AX == 0 ? P * P * P : AX == 1 ? P * P : AX == 2 ? P : 1;
    const int o = (v / stride) % P, base = v - o * stride;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < P; ++q) s += A[o * P + q] * in[base + q * stride];
    return s;
}

// (Ax (x) Ay (x) Az (x) At) applied to buf[0] as four 1-D passes through LDS
// (buf[0] -> buf[1] -> buf[0] -> buf[1] -> registers); the last pass adds the
// outputs v = threadIdx.x + 256 i into out[i].  All 256 threads take part.
template <int P>
__device__ __forceinline__ void reinterp4(double (*buf)[Dim<P>::NN], const double (*A)[P * P],
                                          double (&out)[Dim<P>::NPT]) {
    constexpr int NN = Dim<P>::NN;
    for (int v = threadIdx.x; v < NN; v += 256) buf[1][v] = reinterp_axis<P, 3>(buf[0], A[3], v);
    __syncthreads();
    for (int v = threadIdx.x; v < NN; v += 256) buf[0][v] = reinterp_axis<P, 2>(buf[1], A[2], v);
    __syncthreads();
    for (int v = threadIdx.x; v < NN; v += 256) buf[1][v] = reinterp_axis<P, 1>(buf[0], A[1], v);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < Dim<P>::NPT; ++i) {
        const int v = threadIdx.x + 256 * i;
        if (v < NN) out[i] += reinterp_axis<P, 0>(buf[1], A[0], v);
    }
}

// M2M for the non-leaf cells of a level: MM(S, k) = sum_{children, h} T_{oct,h} MM(child, 2k+h).
// A parent variant truncated v intervals before its start (index v + 1) takes
// from child h the variant truncated 2v + h child intervals before the
// child's start, which is the full moment once that reaches 3 steps back.
// T is the tensor product of the parent's 1-D cardinal functions at the child's
// nodes, applied axis by axis.  One block per (parent, channel, rhs, variant).
template <int P>
__global__ void __launch_bounds__(256) k_m2m(const int *parent_cells, const int *child_beg, const int *child_end,
                                             const int *cix, const double *S1, const double *MMc, int slot0, int slot1,
                                             int WRc, int NVc, double *MMp, int slot, int WRp, int NVp, int nrhs,
                                             float *MMf, unsigned short *MMh) {
    constexpr int NN = Dim<P>::NN, NPT = Dim<P>::NPT;
    int cell = parent_cells[blockIdx.x];
    int c = blockIdx.y % NCH, tf = blockIdx.y / NCH;
    int r = blockIdx.z;
    __shared__ double buf[2][NN];
    __shared__ double A[4][P * P];
    double acc[NPT];
#pragma unroll
    for (int i = 0; i < NPT; ++i) acc[i] = 0.0;
    for (int ch = child_beg[cell]; ch < child_end[cell]; ++ch) {
        const int hsx[3] = {cix[3 * ch] & 1, cix[3 * ch + 1] & 1, cix[3 * ch + 2] & 1};
        for (int h = 0; h < 2; ++h) {
            int stf = 0;
            if (tf > 0) {
                const int w = 2 * (tf - 1) + h;
                stf = w < NVc - 1 ? w + 1 : 0;
            }
            int sl = h == 0 ? slot0 : slot1;
            __syncthreads();
            const double *src = MMc + ((((size_t)ch * WRc + sl) * NVc + stf) * NCH + c) * nrhs * NN + (size_t)r * NN;
            for (int v = threadIdx.x; v < NN; v += 256) buf[0][v] = src[v];
            if ((int)threadIdx.x < 4 * P * P) {
                const int ax = threadIdx.x / (P * P), e = threadIdx.x % (P * P);   // A[ax][o][q] = S1[h_ax][o][q]
                A[ax][e] = ax < 3 ? S1[hsx[ax] * P * P + e] : S1[2 * P * P + h * P * P + e];
            }
            __syncthreads();
            reinterp4<P>(buf, A, acc);
        }
    }
    const size_t di = ((((size_t)cell * WRp + slot) * NVp + tf) * NCH + c) * nrhs * NN + (size_t)r * NN;
    double *dst = MMp + di;
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
        const int v = threadIdx.x + 256 * i;
        if (v < NN) {
            dst[v] = acc[i];
            reduced_copy<1>(&acc[i], MMf, MMh, di + v);
        }
    }
}

// LC(O) = PEND(O, parity) + sum over O's interaction-list entries of YB, and
// over the lag groups of each entry (target-owned, fixed order)
template <int P>
__global__ void __launch_bounds__(256) k_m2l_reduce(int n, const int *il_off, const double *YB, int ng,
                                                    size_t gstride, const double *PEND, int parity, double *LC) {
    constexpr int NN = Dim<P>::NN;
    constexpr int QU = 8;              // entries whose loads are issued together (one lag group)
    int O = blockIdx.x, c = blockIdx.y;
    const int q0 = il_off[O], q1 = il_off[O + 1];
    for (int v = threadIdx.x; v < NN; v += 256) {
        double s = PEND[(((size_t)O * 2 + parity) * NCH + c) * NN + v];
        const double *y = YB + ((size_t)q0 * NCH + c) * NN + v;
        int q = q0;
        if (ng == 1) {
            // the same additions in the same order, QU loads in flight
            for (; q + QU <= q1; q += QU, y += (size_t)QU * NCH * NN) {
                double t[QU];
#pragma unroll
                for (int u = 0; u < QU; ++u) t[u] = y[(size_t)u * NCH * NN];
#pragma unroll
                for (int u = 0; u < QU; ++u) s += t[u];
            }
        }
        for (; q < q1; ++q, y += (size_t)NCH * NN)
            for (int g = 0; g < ng; ++g) s += y[g * gstride];
        LC[((size_t)O * NCH + c) * NN + v] = s;
    }
}

// ------------------------------------------------------- generic dense M2L
// acc[rows x 64 columns] += K(off, lag) X for any P, on the matrix cores.  The
// operator is never tabulated: node offsets lie on a lattice of spacing
// 2/(P-1) h in space and time, so every entry is the kernel at a lattice
// distance r (tabulated per offset in LDS, (2P-1)^3 values) and a time lattice
// point (P-1) lag + m - n, formed per lane in the product loop.  The source
// dimension (b, n) is staged through LDS in chunks of KC values per column.
// Rows are (a, m); a block covers ROWS of them (4 row wavefronts of RB 16-row
// blocks) and 64 columns (2 column wavefronts of 32).
template <int P> struct Gen {
    static constexpr int NN = Dim<P>::NN, L = 2 * P - 1, L3 = L * L * L;
    static constexpr int RB = P == 6 ? 3 : 4;              // 16-row blocks per wavefront
    static constexpr int ROWS = 64 * RB;                   // rows per block
    static constexpr int NRT = (NN + ROWS - 1) / ROWS;     // row tiles
    static constexpr int KC = P == 6 ? 48 : 64;            // staged source values per chunk (divides NN)
    static_assert(NN % KC == 0 && KC % 4 == 0, "chunks tile the source dimension");
};
template <int P, typename T> struct GenX { static constexpr int XS = Gen<P>::KC + (sizeof(T) == 8 ? 2 : 4); };

// lattice distances for offset (ox, oy, oz) between cells of side ds with node
// spacing gs: rd[idx] = |gs d - ds off|, d = idx's lattice vector - (P - 1)
template <int P, typename T>
__device__ void gen_dist(double *rd, T *ird, int ox, int oy, int oz, double gs, double ds) {
    constexpr int L = Gen<P>::L;
    for (int d = threadIdx.x; d < Gen<P>::L3; d += blockDim.x) {
        const double v1 = gs * (d / (L * L) - (P - 1)) - ds * ox, v2 = gs * ((d / L) % L - (P - 1)) - ds * oy,
                     v3 = gs * (d % L - (P - 1)) - ds * oz;
        const double r = sqrt(v1 * v1 + v2 * v2 + v3 * v3);
        rd[d] = r;
        ird[d] = (T)(r > 0.0 ? 1.0 / r : 0.0);
    }
}

// per lane and row block: lattice base of the row's target node a (plus P - 1
// per axis), its time node m, and whether the row exists
template <int P>
__device__ void gen_rows(int (&abase)[Gen<P>::RB], int (&mrow)[Gen<P>::RB], bool (&rok)[Gen<P>::RB], int rt, int wr,
                         int lane) {
    constexpr int L = Gen<P>::L, RB = Gen<P>::RB;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int row = rt * Gen<P>::ROWS + wr * 16 * RB + 16 * rb + (lane & 15);
        rok[rb] = row < Gen<P>::NN;
        const int a = row / P, m = row % P;
        const int a1 = a / (P * P), a2 = (a / P) % P, a3 = a % P;
        abase[rb] = ((a1 + P - 1) * L + a2 + P - 1) * L + a3 + P - 1;
        mrow[rb] = m;
    }
}

// source index k = b P + n: lattice index of b and n, packed
template <int P>
__device__ void gen_kinfo(int *kinfo) {
    constexpr int L = Gen<P>::L;
    for (int k = threadIdx.x; k < Gen<P>::NN; k += blockDim.x) {
        const int b = k / P, n = k % P;
        kinfo[k] = (((b / (P * P)) * L + (b / P) % P) * L + b % P) | (n << 16);
    }
}

// one (offset, lag): acc += K X with X read per column at MM[cb[col] + mo + k]
// (acc [RB][2] and X [64][XS] passed flat; the function is inlined into the
// kernels, so every index below is a compile-time constant or a lane value)
template <int P, typename T>
__device__ __forceinline__ void gen_lag(typename Mma<T>::acc_t *acc, T *X, const int64_t *cb, const double *MM,
                                        int64_t mo, const double *rd, const T *ird, const int *kinfo, const int *abase,
                                        const int *mrow, const bool *rok, int lag, int kfun, double cgt, double c2,
                                        int wc, int lane) {
    constexpr int NN = Gen<P>::NN, KC = Gen<P>::KC, RB = Gen<P>::RB, XS = GenX<P, T>::XS;
    const int colA = 32 * wc + (lane & 15);
    const int tshift = (P - 1) * lag;
    for (int k0 = 0; k0 < NN; k0 += KC) {
        __syncthreads();                      // the previous chunk's products are done with X
        for (int e = threadIdx.x; e < M2L_NT * KC; e += blockDim.x) {
            const int col = e / KC, kk = e % KC;
            const int64_t b = cb[col];
            X[col * XS + kk] = b >= 0 ? (T)MM[b + mo + k0 + kk] : (T)0;
        }
        __syncthreads();
        for (int ks = 0; ks < KC / 4; ++ks) {
            const int kk = 4 * ks + (lane >> 4);
            const int ki = kinfo[k0 + kk];
            const int bidx = ki & 0xffff, n = ki >> 16;
            const T bv0 = X[colA * XS + kk], bv1 = X[(colA + 16) * XS + kk];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                T kv = (T)0;
                if (rok[rb]) {
                    const int idx = abase[rb] - bidx;
                    const double r = rd[idx];
                    const double u = cgt * (tshift + mrow[rb] - n) - r;
                    if (u > 0.0 && r > 0.0)
                        kv = (T)((kfun == 0 ? c2 * u : kfun == 1 ? u * u : 0.5 * c2 * c2) * (double)ird[idx]);
                }
                acc[2 * rb] = Mma<T>::op(kv, bv0, acc[2 * rb]);
                acc[2 * rb + 1] = Mma<T>::op(kv, bv1, acc[2 * rb + 1]);
            }
        }
    }
}

// offset-major generic M2L for one right-hand side: one block per (column
// tile, row tile); columns = (interaction-list entry, channel) sharing one
// offset; writes the per-entry contributions YB summed over the window's lags
template <int P, typename T>
__global__ void __launch_bounds__(512) k_m2l_gen_off(const int *tile_code, const int *tile_kind, const int *tile_col0,
                                                     const int *tile_ncol, const int *col_q, const int *col_ch,
                                                     const int *il_src, const double *MM, int WR, int NV, int k, int W,
                                                     double hn, double ds, double ht, double cl, double *YB, int kindA) {
    constexpr int NN = Gen<P>::NN, RB = Gen<P>::RB;
    const int tile = blockIdx.x, rt = blockIdx.y;
    const int code = tile_code[tile], kind = tile_kind[tile], col0 = tile_col0[tile], ncol = tile_ncol[tile];
    const int kfun = kind == 0 ? kindA : 1;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, wr = wave & 3, wc = wave >> 2;
    __shared__ double rd[Gen<P>::L3];
    __shared__ T ird[Gen<P>::L3];
    __shared__ int kinfo[NN];
    __shared__ __attribute__((aligned(16))) T X[M2L_NT][GenX<P, T>::XS];
    __shared__ int64_t cb[M2L_NT];
    if (tid < M2L_NT)
        cb[tid] = tid < ncol ? ((int64_t)il_src[col_q[col0 + tid]] * WR * NV * NCH + col_ch[col0 + tid]) * NN : -1;
    gen_kinfo<P>(kinfo);
    gen_dist<P, T>(rd, ird, code / 49 - 3, (code / 7) % 7 - 3, code % 7 - 3, hn * (2.0 / (P - 1)), ds);
    int abase[RB], mrow[RB];
    bool rok[RB];
    gen_rows<P>(abase, mrow, rok, rt, wr, lane);
    typename Mma<T>::acc_t acc[RB][2];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[rb][0] = acc[rb][1] = typename Mma<T>::acc_t{0, 0, 0, 0};
    const double cgt = cl * ht * (2.0 / (P - 1));
    const int nlag = min(W, k + 1);
    for (int lag = 1; lag <= nlag; ++lag) {
        const int var = W - lag < NV - 1 ? W - lag + 1 : 0;     // the window's oldest intervals: truncated
        const int64_t mo = (int64_t)(((k + 1 - lag) % WR) * NV + var) * NCH * NN;
        gen_lag<P, T>(&acc[0][0], &X[0][0], cb, MM, mo, rd, ird, kinfo, abase, mrow, rok, lag, kfun, cgt,
                          2.0 * cl, wc, lane);
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
        for (int cbk = 0; cbk < 2; ++cbk) {
            const int j = 32 * wc + 16 * cbk + (lane & 15);
            if (j >= ncol) continue;
            const int q = col_q[col0 + j], ch = col_ch[col0 + j];
            for (int v = 0; v < 4; ++v) {
                const int row = rt * Gen<P>::ROWS + wr * 16 * RB + 16 * rb + Mma<T>::row(lane, v);
                if (row < NN) YB[((size_t)q * NCH + ch) * NN + row] = (double)acc[rb][cbk][v];
            }
        }
}

// target-major generic M2L for batched right-hand sides: one block per
// (target, kind, (channel, rhs) column tile x row tile); items are
// (interaction-list entry, lag); LC = PEND + the sum
template <int P, typename T>
__global__ void __launch_bounds__(512) k_m2l_gen_tgt(const int *il_off, const int *il_src, const int *il_code,
                                                     const double *MM, int WR, int NV, int k, int W, double hn,
                                                     double ds, double ht, double cl, const double *PEND, double *LC,
                                                     int nrhs, int kindA) {
    constexpr int NN = Gen<P>::NN, RB = Gen<P>::RB;
    const int O = blockIdx.x, kind = blockIdx.y;
    const int ctile = blockIdx.z / Gen<P>::NRT, rt = blockIdx.z % Gen<P>::NRT;
    const int kfun = kind == 0 ? kindA : 1;
    const int c0 = kind == 0 ? 0 : 3, nc = kind == 0 ? 3 : 4;
    const int ncolt = nc * nrhs, col0 = ctile * M2L_NT;
    if (col0 >= ncolt) return;
    const int ncol = min(M2L_NT, ncolt - col0);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, wr = wave & 3, wc = wave >> 2;
    const int parity = (k + 1) & 1;
    __shared__ double rd[Gen<P>::L3];
    __shared__ T ird[Gen<P>::L3];
    __shared__ int kinfo[NN];
    __shared__ __attribute__((aligned(16))) T X[M2L_NT][GenX<P, T>::XS];
    __shared__ int64_t cb[M2L_NT];
    if (tid < M2L_NT) {
        int64_t b = -1;
        if (tid < ncol) {
            const int cc = (col0 + tid) / nrhs, r = (col0 + tid) % nrhs;
            b = ((int64_t)(c0 + cc) * nrhs + r) * NN;
        }
        cb[tid] = b;
    }
    gen_kinfo<P>(kinfo);
    int abase[RB], mrow[RB];
    bool rok[RB];
    gen_rows<P>(abase, mrow, rok, rt, wr, lane);
    typename Mma<T>::acc_t acc[RB][2];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[rb][0] = acc[rb][1] = typename Mma<T>::acc_t{0, 0, 0, 0};
    const double cgt = cl * ht * (2.0 / (P - 1));
    const int nlag = min(W, k + 1);
    const int64_t strideS = (int64_t)WR * NV * NCH * nrhs * NN;
    for (int q = il_off[O]; q < il_off[O + 1]; ++q) {
        const int code = il_code[q];
        __syncthreads();                      // the previous entry's products are done with rd
        gen_dist<P, T>(rd, ird, code / 49 - 3, (code / 7) % 7 - 3, code % 7 - 3, hn * (2.0 / (P - 1)), ds);
        for (int lag = 1; lag <= nlag; ++lag) {
            const int var = W - lag < NV - 1 ? W - lag + 1 : 0;
            const int64_t mo = (int64_t)il_src[q] * strideS + (int64_t)(((k + 1 - lag) % WR) * NV + var) * NCH * nrhs * NN;
            gen_lag<P, T>(&acc[0][0], &X[0][0], cb, MM, mo, rd, ird, kinfo, abase, mrow, rok, lag, kfun, cgt,
                          2.0 * cl, wc, lane);
        }
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
        for (int cbk = 0; cbk < 2; ++cbk) {
            const int j = 32 * wc + 16 * cbk + (lane & 15);
            if (j >= ncol) continue;
            const int cc = (col0 + j) / nrhs, r = (col0 + j) % nrhs;
            for (int v = 0; v < 4; ++v) {
                const int row = rt * Gen<P>::ROWS + wr * 16 * RB + 16 * rb + Mma<T>::row(lane, v);
                if (row >= NN) continue;
                const size_t o = (((size_t)O * NCH + c0 + cc) * nrhs + r) * NN + row;
                const size_t pe = ((((size_t)O * 2 + parity) * NCH + c0 + cc) * nrhs + r) * NN + row;
                LC[o] = (double)acc[rb][cbk][v] + PEND[pe];
            }
        }
}

template <int P, typename T>
static void m2l_gen_launch(tdbem_ctx *C, FarLevel &FL, int k, hipStream_t s) {
    const int nr = C->nrhs;
    const int kindA = m2l_kind_a(C->cfg);
    PhaseScope ps(C->prof, TDBEM_PH_M2L, s);
    if (nr == 1) {
        if (FL.ntile > 0)
            hipLaunchKernelGGL((k_m2l_gen_off<P, T>), dim3(FL.ntile, Gen<P>::NRT), dim3(512), 0, s, FL.tile_code,
                               FL.tile_kind, FL.tile_col0, FL.tile_ncol, FL.col_q, FL.col_ch, FL.il_src, FL.MM, FL.WR,
                               FL.NV, k, FL.W, FL.hn, FL.ds, FL.ht, C->c, FL.YB, kindA);
    } else {
        const unsigned nct = (unsigned)((4 * nr + M2L_NT - 1) / M2L_NT);
        hipLaunchKernelGGL((k_m2l_gen_tgt<P, T>), dim3(FL.n, 2, nct * Gen<P>::NRT), dim3(512), 0, s, FL.il_off,
                           FL.il_src, FL.il_code, FL.MM, FL.WR, FL.NV, k, FL.W, FL.hn, FL.ds, FL.ht, C->c, FL.PEND,
                           FL.LC, nr, kindA);
    }
    TD_HIP(hipGetLastError());
}

// M2L of one level at gate k (the tuned kernel at p = 4 unless the generic one
// is asked for), then for one right-hand side the per-target sum
template <int P>
static void m2l_level(tdbem_ctx *C, FarLevel &FL, int k, hipStream_t s) {
    const bool f64 = C->cfg.precision == TDBEM_FP64;
    if (C->far->fft_m2l) {
        m2l_fft_level(C, FL, k, s);      // writes LC itself
        return;
    }
    FL.yg = 1;                            // the tuned FP64 / FP32 kernel may split the lags
    if (P == 4 && !C->far->generic_m2l) {
        if (C->far->bf16_m2l) m2l_bf16_launch(C, FL, k, s);
        else if (f64) m2l_p4_launch<double>(C, FL, k, s);
        else m2l_p4_launch<float>(C, FL, k, s);
    } else {
        if (f64) m2l_gen_launch<P, double>(C, FL, k, s); else m2l_gen_launch<P, float>(C, FL, k, s);
    }
    if (C->nrhs == 1) {
        PhaseScope ps(C->prof, TDBEM_PH_M2L_SUM, s);
        hipLaunchKernelGGL(k_m2l_reduce<P>, dim3(FL.n, NCH), dim3(256), 0, s, FL.n, FL.il_off, FL.YB, FL.yg,
                           (size_t)FL.nil * NCH * Dim<P>::NN, FL.PEND, (k + 1) & 1, FL.LC);
        TD_HIP(hipGetLastError());
    }
}

// L2L: PEND(child, h) = T_{oct,h}^T LC(parent) for the child's intervals 2(k+1)+h.
// One block per (parent, channel, rhs, h); every child in turn.
template <int P>
__global__ void __launch_bounds__(256) k_l2l(const int *parent_cells, const int *child_beg, const int *child_end,
                                             const int *cix, const double *S1, const double *LCp, double *PENDc, int nrhs) {
    constexpr int NN = Dim<P>::NN, NPT = Dim<P>::NPT;
    int cell = parent_cells[blockIdx.x];
    int c = blockIdx.y % NCH, h = blockIdx.y / NCH;
    int r = blockIdx.z;
    __shared__ double buf[2][NN];
    __shared__ double A[4][P * P];
    const double *lcp = LCp + ((size_t)cell * NCH + c) * nrhs * NN + (size_t)r * NN;
    for (int ch = child_beg[cell]; ch < child_end[cell]; ++ch) {
        const int hsx[3] = {cix[3 * ch] & 1, cix[3 * ch + 1] & 1, cix[3 * ch + 2] & 1};
        __syncthreads();
        for (int v = threadIdx.x; v < NN; v += 256) buf[0][v] = lcp[v];
        if ((int)threadIdx.x < 4 * P * P) {
            // transpose: child output o from parent input q, A[ax][o][q] = S1[h_ax][q][o]
            const int ax = threadIdx.x / (P * P), o = (threadIdx.x % (P * P)) / P, q = threadIdx.x % P;
            const int hh = ax < 3 ? hsx[ax] : h;
            A[ax][o * P + q] = S1[(ax < 3 ? 0 : 2 * P * P) + (hh * P + q) * P + o];
        }
        __syncthreads();
        double out[NPT];
#pragma unroll
        for (int i = 0; i < NPT; ++i) out[i] = 0.0;
        reinterp4<P>(buf, A, out);
        double *dst = PENDc + (((size_t)ch * 2 + h) * NCH + c) * nrhs * NN + (size_t)r * NN;
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int v = threadIdx.x + 256 * i;
            if (v < NN) dst[v] = out[i];
        }
    }
}

// L2P: FAR(slot of step alpha') for the edges of a leaf, alpha' = (k+1)M + q, q = 1..M:
// sum_c sum_a El[i][c][a] Lt[q][c][a], Lt[q][c][a] = sum_m LC[c][a][m] tw_g(c)(m, q) with the
// target weights of the channel's group (vector, scalar, magnetic potential).  One block per (leaf, rhs): the
// leaf's time-contracted expansions Lt are formed once in LDS for a chunk of
// QC target steps and shared by all its edges.
template <int P>
__global__ void __launch_bounds__(256) k_l2p(const int *leaf_cells, const int *ebeg, const int *eend, int k, int M,
                                             const double *tw, const double *El, const double *LC,
                                             double *FAR, int FR, int ne, int nrhs) {
    constexpr int NS = Dim<P>::NS, NN = Dim<P>::NN;
    constexpr int QC = P == 4 ? 8 : P == 6 ? 2 : 1;
    const int cell = leaf_cells[blockIdx.x], r = blockIdx.y;
    const int e0 = ebeg[cell], nloc = eend[cell] - e0;
    __shared__ double Lt[QC][NCH][NS];
    const double *L = LC + (size_t)cell * NCH * nrhs * NN + (size_t)r * NN;
    for (int q0 = 1; q0 <= M; q0 += QC) {
        const int nq = min(QC, M - q0 + 1);
        __syncthreads();
        for (int t = threadIdx.x; t < nq * NCH * NS; t += blockDim.x) {
            const int qi = t / (NCH * NS), c = (t / NS) % NCH, a = t % NS;
            const double *tv = tw + (size_t)(q0 + qi - 1) * 3 * P + (c < 3 ? 0 : c == 3 ? P : 2 * P);
            const double *l = L + (size_t)c * nrhs * NN + a * P;
            double s = 0.0;
            for (int m = 0; m < P; ++m) s += l[m] * tv[m];
            Lt[qi][c][a] = s;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < nloc * nq; t += blockDim.x) {
            const int j = t / nq, qi = t % nq, i = e0 + j;
            const double *e = El + (size_t)i * NCH * NS;
            double s = 0.0;
            for (int ca = 0; ca < NCH * NS; ++ca) s += e[ca] * (&Lt[qi][0][0])[ca];
            const int alpha = (k + 1) * M + q0 + qi;
            FAR[((size_t)((alpha - 1) & (FR - 1)) * ne + i) * nrhs + r] = s;
        }
    }
}

__global__ void k_far_apply(int64_t n, double sign, const double *FAR, double *y) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] += sign * FAR[t];
}

// ------------------------------------------------------------------ driver
// this step's far-field potential (the slot L2P wrote for step alpha)
const double *ifmm_far_slot(const tdbem_ctx *C, int alpha) {
    const FarState *F = C->far;
    return F->FAR + (size_t)((alpha - 1) & (F->FR - 1)) * C->ne * C->nrhs;
}

void ifmm_subtract_far(tdbem_ctx *C, int alpha, double *rhs, hipStream_t s) {
    FarState *F = C->far;
    int64_t n = (int64_t)C->ne * C->nrhs;
    const double *src = F->FAR + (size_t)((alpha - 1) & (F->FR - 1)) * n;
    hipLaunchKernelGGL(k_far_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, -1.0, src, rhs);
    TD_HIP(hipGetLastError());
}

void ifmm_add_far(tdbem_ctx *C, int alpha, double *out, hipStream_t s) {
    FarState *F = C->far;
    int64_t n = (int64_t)C->ne * C->nrhs;
    const double *src = F->FAR + (size_t)((alpha - 1) & (F->FR - 1)) * n;
    hipLaunchKernelGGL(k_far_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, 1.0, src, out);
    TD_HIP(hipGetLastError());
}

template <int P>
static void after_solve(tdbem_ctx *C, int alpha, hipStream_t s) {
    FarState *F = C->far;
    const int nr = C->nrhs;
    // upward pass (Program 3)
    for (int l = F->lmax; l >= 2; --l) {
        FarLevel &FL = F->lev[l];
        if (alpha % FL.M) continue;
        int k = alpha / FL.M - 1;
        int slot = k % FL.WR;
        if (FL.nleaf > 0) {
            PhaseScope ps(C->prof, TDBEM_PH_P2M, s);
            hipLaunchKernelGGL(k_p2m<P>, dim3(FL.nleaf, nr), dim3(256), 0, s, FL.leaf_cells, FL.ebeg, FL.eend, k, FL.M,
                               FL.ls, C->d_Jring, C->ring, nr, F->Wm, FL.MM, slot, FL.WR, FL.NV, FL.MM32, FL.MM16);
        }
        if (FL.nparent > 0) {
            PhaseScope ps(C->prof, TDBEM_PH_M2M, s);
            FarLevel &CL = F->lev[l + 1];
            hipLaunchKernelGGL(k_m2m<P>, dim3(FL.nparent, FL.NV * NCH, nr), dim3(256), 0, s, FL.parent_cells,
                               FL.child_beg, FL.child_end, CL.ix, F->S1 + (size_t)l * 4 * P * P, CL.MM, (2 * k) % CL.WR,
                               (2 * k + 1) % CL.WR, CL.WR, CL.NV, FL.MM, slot, FL.WR, FL.NV, nr, FL.MM32, FL.MM16);
        }
        TD_HIP(hipGetLastError());
    }
    // downward pass (Program 4)
    for (int l = 2; l <= F->lmax; ++l) {
        FarLevel &FL = F->lev[l];
        if (alpha % FL.M) continue;
        int k = alpha / FL.M - 1;
        m2l_level<P>(C, FL, k, s);
        if (FL.nparent > 0) {
            PhaseScope ps(C->prof, TDBEM_PH_L2L, s);
            FarLevel &CL = F->lev[l + 1];
            hipLaunchKernelGGL(k_l2l<P>, dim3(FL.nparent, 2 * NCH, nr), dim3(256), 0, s, FL.parent_cells, FL.child_beg,
                               FL.child_end, CL.ix, F->S1 + (size_t)l * 4 * P * P, FL.LC, CL.PEND, nr);
        }
        if (FL.nleaf > 0) {
            PhaseScope ps(C->prof, TDBEM_PH_L2P, s);
            hipLaunchKernelGGL(k_l2p<P>, dim3(FL.nleaf, nr), dim3(256), 0, s, FL.leaf_cells, FL.ebeg, FL.eend, k, FL.M,
                               FL.tw, F->El, FL.LC, F->FAR, F->FR, C->ne, nr);
        }
        TD_HIP(hipGetLastError());
    }
}

// the levels whose time gate step alpha passes (bit l): they alone decide
// which kernels follow a step's solve
uint32_t ifmm_gate_mask(const tdbem_ctx *C, int alpha) {
    const FarState *F = C->far;
    uint32_t m = 0;
    for (int l = 2; l <= F->lmax; ++l)
        if (alpha % F->lev[l].M == 0) m |= 1u << l;
    return m;
}

void ifmm_after_solve(tdbem_ctx *C, int alpha, hipStream_t s) {
    switch (C->far->P) {
        case 4: after_solve<4>(C, alpha, s); break;
        case 6: after_solve<6>(C, alpha, s); break;
        default: after_solve<8>(C, alpha, s); break;
    }
}

size_t ifmm_state_bytes(const tdbem_ctx *C) {
    const FarState *F = C->far;
    const size_t nr = C->nrhs, NN = F->NN;
    size_t n = (size_t)F->FR * C->ne * nr;
    for (int l = 2; l <= F->lmax; ++l) {
        const FarLevel &FL = F->lev[l];
        n += (size_t)FL.n * FL.WR * FL.NV * NCH * nr * NN + (size_t)FL.n * NCH * nr * NN + (size_t)FL.n * 2 * NCH * nr * NN;
    }
    return n * sizeof(double);
}

void ifmm_state_copy(tdbem_ctx *C, char *host, bool save, hipStream_t s) {
    FarState *F = C->far;
    const size_t nr = C->nrhs, NN = F->NN;
    auto io = [&](double *dev, size_t n) {
        const size_t b = n * sizeof(double);
        if (save) TD_HIP(hipMemcpyAsync(host, dev, b, hipMemcpyDeviceToHost, s));
        else TD_HIP(hipMemcpyAsync(dev, host, b, hipMemcpyHostToDevice, s));
        host += b;
    };
    io(F->FAR, (size_t)F->FR * C->ne * nr);
    for (int l = 2; l <= F->lmax; ++l) {
        FarLevel &FL = F->lev[l];
        io(FL.MM, (size_t)FL.n * FL.WR * FL.NV * NCH * nr * NN);
        io(FL.LC, (size_t)FL.n * NCH * nr * NN);
        io(FL.PEND, (size_t)FL.n * 2 * NCH * nr * NN);
    }
    // the reduced copies and the Fourier-domain M2L's transformed moments
    // follow from the restored moments
    if (!save)
        for (int l = 2; l <= F->lmax; ++l) mm_copies_refresh(C, F->lev[l], s);
    if (!save && F->fft_m2l)
        for (int l = 2; l <= F->lmax; ++l)
            for (int slot = 0; slot < F->lev[l].WR; ++slot) m2l_fft_moments(C, F->lev[l], slot, s);
}

}  // namespace tdbem
