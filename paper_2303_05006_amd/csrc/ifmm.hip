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
// Finite M2L window: sources are the W = mu + 1 most recent intervals.  When
// every node pair of lag W lies inside the light cone (mu rho >= 4 sqrt 3, rho =
// c M_t dt / d_s), the node values of U and dU/dt are polynomials of degree <= 2
// in s there and in every older interval; the interpolant reproduces them, and
// since the B-spline weights w annihilate quadratics, the whole older history
// reduces to the oldest window interval's moments built from the current
// difference truncated at that interval's start (Eq. hat_J with beta* the
// interval start).  This reproduces the sum over all earlier intervals.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "ifmm.h"

namespace tdbem {

static constexpr int P = 4;        // interpolation points per axis and in time
static constexpr int NS = P * P * P;
static constexpr int NN = NS * P;   // 256
static constexpr int NCH = 7;
static constexpr int M2L_NT = 64;  // columns per M2L tile

struct FarLevel {
    int n = 0, M = 0;
    double ds = 0, hs = 0, hn = 0, ht = 0;   // cell side, cell half-width, node half-width, time half-width
    int *il_off = nullptr, *il_src = nullptr, *il_code = nullptr;  // interaction lists
    int *ix = nullptr;                                             // [n][3] integer coords
    int *ebeg = nullptr, *eend = nullptr;
    int nleaf = 0, nparent = 0;
    int *leaf_cells = nullptr, *parent_cells = nullptr;
    int *child_beg = nullptr, *child_end = nullptr;                // children at level+1
    double *MM = nullptr;     // [n][WR][2][NCH][nrhs][NN]
    float *MM32 = nullptr;    // FP32 copy of MM staged by the reduced forms' M2L
    double *LC = nullptr;     // [n][NCH][nrhs][NN]
    double *PEND = nullptr;   // [n][2][NCH][nrhs][NN]
    double *tw = nullptr;     // [M][2][P]: l_m and dl_m/dt at target step q = 1..M
    double *ls = nullptr;     // [M][P]: l_n at source step beta - kM = 0..M-1
    // offset-major M2L tiles (one right-hand side)
    int ntile = 0;
    int *tile_code = nullptr, *tile_kind = nullptr, *tile_col0 = nullptr, *tile_ncol = nullptr;
    int *col_q = nullptr, *col_ch = nullptr;
    double *YB = nullptr;     // [interaction-list entries][NCH][NN]
};

struct FarState {
    int lmax = 0, W = 0, WR = 0, FR = 0, nrhs = 1;
    double delta = 0;         // widening of the interpolation boxes beyond the cells
    std::vector<FarLevel> lev;
    double *Wm = nullptr;     // [ne][NCH][NS] P2M weights
    double *El = nullptr;     // [ne][NCH][NS] L2P weights
    double *FAR = nullptr;    // [FR][ne][nrhs] far-field potential per target slot
    double *S1 = nullptr;     // [parent level][space, time][2][P][P]: parent cardinal at child node, half h
};

// ------------------------------------------------------------ host helpers
static void lagr(double xi, double *v, double *d) {
    double w[P];
    for (int n = 0; n < P; ++n) w[n] = -1.0 + 2.0 * n / (P - 1);
    for (int n = 0; n < P; ++n) {
        double den = 1.0, prod = 1.0, der = 0.0;
        for (int m = 0; m < P; ++m) {
            if (m == n) continue;
            den *= w[n] - w[m];
            prod *= xi - w[m];
        }
        for (int k = 0; k < P; ++k) {
            if (k == n) continue;
            double t = 1.0;
            for (int m = 0; m < P; ++m)
                if (m != n && m != k) t *= xi - w[m];
            der += t;
        }
        v[n] = prod / den;
        if (d) d[n] = der / den;
    }
}

// piecewise cubic Hermite interpolation on the equispaced nodes with node slopes
// from finite differences (central inside, second-order one-sided at the ends):
// cardinal functions and their derivatives at xi (reproduces quadratics)
static void chi(double xi, double *v, double *d) {
    const double h = 2.0 / (P - 1);
    int i = (int)std::floor((xi + 1.0) / h);
    i = std::min(std::max(i, 0), P - 2);
    const double t = (xi - (-1.0 + h * i)) / h;
    const double h00 = 2 * t * t * t - 3 * t * t + 1, h10 = t * t * t - 2 * t * t + t;
    const double h01 = -2 * t * t * t + 3 * t * t, h11 = t * t * t - t * t;
    const double d00 = 6 * t * t - 6 * t, d10 = 3 * t * t - 4 * t + 1, d01 = -6 * t * t + 6 * t, d11 = 3 * t * t - 2 * t;
    for (int m = 0; m < P; ++m) {
        double f[P], sl[P];
        for (int n = 0; n < P; ++n) f[n] = n == m ? 1.0 : 0.0;
        sl[0] = (-3 * f[0] + 4 * f[1] - f[2]) / (2 * h);
        sl[P - 1] = (3 * f[P - 1] - 4 * f[P - 2] + f[P - 3]) / (2 * h);
        for (int n = 1; n < P - 1; ++n) sl[n] = (f[n + 1] - f[n - 1]) / (2 * h);
        v[m] = h00 * f[i] + h10 * h * sl[i] + h01 * f[i + 1] + h11 * h * sl[i + 1];
        if (d) d[m] = (d00 * f[i] + d10 * h * sl[i] + d01 * f[i + 1] + d11 * h * sl[i + 1]) / h;
    }
}

// temporal cardinal functions of the configured interpolant
static void tcard(int interp, double xi, double *v, double *d) {
    if (interp == TDBEM_INTERP_CHI_TIME) chi(xi, v, d); else lagr(xi, v, d);
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
template <typename T>
static T *fup(tdbem_ctx *C, const std::vector<T> &v) {
    T *p = falloc<T>(C, v.size());
    if (!v.empty()) TD_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
}

void ifmm_setup(tdbem_ctx *C) {
    const Tree &T = C->T;
    const HostMesh &H = C->H;
    TD_REQUIRE(C->cfg.p_s == P && C->cfg.p_t == P, TDBEM_EINVAL, "the far field is built for p_s = p_t = 4");
    TD_REQUIRE(T.lmax >= 2, TDBEM_EINVAL, "IFMM needs at least two levels below the root");
    FarState *F = new FarState();
    C->far = F;
    const int interp = C->cfg.interp;
    F->lmax = T.lmax;
    F->nrhs = C->nrhs;
    const double ds_max = T.side / std::ldexp(1.0, T.lmax);
    double reach = ds_max;
    if (const char *g = getenv("TDBEM_CAUSAL_GUARD"); g && atoi(g) == 1) {
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
    TD_REQUIRE(Mmax >= 3, TDBEM_EBREAKDOWN,
               "time hierarchy breaks down: floor(d_s/(c dt)) = " + std::to_string(Mmax) + " < 3 steps per finest interval");
    double rho = C->cdt * Mmax / ds_max;
    int mu = std::max(C->cfg.mu_window, (int)std::ceil(4.0 * std::sqrt(3.0) / rho - 1e-12));
    TD_REQUIRE(mu <= 19, TDBEM_EBREAKDOWN, "far-field window of more than 20 intervals (c dt too small for the finest cells)");
    F->W = mu + 1;
    F->WR = F->W + 1;
    C->window = F->W;
    C->Mt.assign(T.lmax + 1, 0);
    F->lev.resize(T.lmax + 1);
    for (int l = 2; l <= T.lmax; ++l) C->Mt[l] = Mmax << (T.lmax - l);
    int FR = 8;
    while (FR < 2 * C->Mt[2] + 2) FR <<= 1;
    F->FR = FR;
    C->far_ring_need = C->Mt[2] + 4;
    const int nr = C->nrhs;
    // interpolation boxes: the cell widened by the largest distance (per axis) that
    // a basis support reaches beyond its edge midpoint, so that every quadrature
    // point of a cell's edges lies inside its box (no extrapolation)
    if (const char *g = getenv("TDBEM_BOX_WIDEN"); g && atoi(g) == 1) {
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
        FL.MM = falloc<double>(C, (size_t)L.n * F->WR * 2 * NCH * nr * NN);
        if (C->cfg.precision != TDBEM_FP64) FL.MM32 = falloc<float>(C, (size_t)L.n * F->WR * 2 * NCH * nr * NN);
        FL.LC = falloc<double>(C, (size_t)L.n * NCH * nr * NN);
        FL.PEND = falloc<double>(C, (size_t)L.n * 2 * NCH * nr * NN);
        // time tables: targets t = (k+1) d_t + q dt, q = 1..M, in the target interval
        // [(k+1) d_t, (k+2) d_t]: xi = 2q/M - 1; sources beta - kM = 0..M-1: xi = 2(beta-kM)/M - 1
        std::vector<double> tw((size_t)FL.M * 2 * P), ls((size_t)FL.M * P);
        for (int q = 1; q <= FL.M; ++q) {
            double v[P], d[P];
            tcard(interp, 2.0 * q / FL.M - 1.0, v, d);
            for (int m = 0; m < P; ++m) {
                tw[((size_t)(q - 1) * 2 + 0) * P + m] = v[m];
                tw[((size_t)(q - 1) * 2 + 1) * P + m] = d[m] / FL.ht;
            }
        }
        for (int b = 0; b < FL.M; ++b) {
            double v[P];
            tcard(interp, 2.0 * b / FL.M - 1.0, v, nullptr);
            for (int n = 0; n < P; ++n) ls[(size_t)b * P + n] = v[n];
        }
        FL.tw = fup(C, tw);
        FL.ls = fup(C, ls);
        if (nr == 1 && !L.il_src.empty()) {
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
            FL.YB = falloc<double>(C, L.il_src.size() * NCH * NN);
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
                double v[3][P], d[3][P];
                for (int k = 0; k < 3; ++k) lagr((x[k] - cen[k]) / hs, v[k], d[k]);
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
                double v[P];
                lagr(((2 * h - 1) * hsc + hnc * w) / hnp, v, nullptr);
                for (int bp = 0; bp < P; ++bp) S[(h * P + bp) * P + bc] = v[bp];   // [h][parent][child]
                tcard(interp, (h - 0.5) + 0.5 * w, v, nullptr);
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
    hipStream_t s = C->stream;
    const int nr = C->nrhs;
    for (int l = 2; l <= F->lmax; ++l) {
        FarLevel &FL = F->lev[l];
        TD_HIP(hipMemsetAsync(FL.MM, 0, sizeof(double) * (size_t)FL.n * F->WR * 2 * NCH * nr * NN, s));
        TD_HIP(hipMemsetAsync(FL.PEND, 0, sizeof(double) * (size_t)FL.n * 2 * NCH * nr * NN, s));
        TD_HIP(hipMemsetAsync(FL.LC, 0, sizeof(double) * (size_t)FL.n * NCH * nr * NN, s));
    }
    TD_HIP(hipMemsetAsync(F->FAR, 0, sizeof(double) * (size_t)F->FR * C->ne * nr, s));
}

void ifmm_destroy(tdbem_ctx *C) {
    delete C->far;
    C->far = nullptr;
}

// ------------------------------------------------------------------ kernels
__constant__ double c_wk[4] = {0.5, -1.5, 1.5, -0.5};

// P2M at the leaves of one level: one block per (leaf, rhs).
// T[j][tf][n] = sum_beta l_n(xi_beta) Jhat^beta_j (tf 0 full, 1 truncated at kM),
// MM[c][b][n][tf] = sum_j Wm[j][c][b] T[j][tf][n].
__global__ void __launch_bounds__(256) k_p2m(const int *leaf_cells, const int *ebeg, const int *eend, int k, int M,
                                             const double *ls, const double *ring, int R, int nrhs,
                                             const double *Wm, double *MM, int slot, int WR) {
    int cell = leaf_cells[blockIdx.x];
    int r = blockIdx.y;
    int e0 = ebeg[cell], e1 = eend[cell];
    __shared__ double T[64][2][P];
    __shared__ double acc_sh[2 * NCH * NN];
    for (int q = threadIdx.x; q < 2 * NCH * NN; q += blockDim.x) acc_sh[q] = 0.0;
    int beta0 = k * M;
    for (int jb = e0; jb < e1; jb += 64) {
        int nj = min(64, e1 - jb);
        __syncthreads();
        for (int q = threadIdx.x; q < nj * 2 * P; q += blockDim.x) {
            int j = q / (2 * P), tf = (q / P) % 2, n = q % P;
            const double *J = ring + (size_t)(jb + j) * R * nrhs + r;
            double s = 0.0;
            for (int bo = 0; bo < M; ++bo) {
                int beta = beta0 + bo;
                double jh = 0.0;
                int kmax = tf ? min(3, bo) : 3;
                for (int kap = 0; kap <= kmax; ++kap) {
                    int b = beta - kap;
                    if (b >= 0) jh += c_wk[kap] * J[(size_t)(b & (R - 1)) * nrhs];
                }
                s += ls[bo * P + n] * jh;
            }
            T[j][tf][n] = s;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < NCH * NS; q += blockDim.x) {
            int c = q / NS, b = q % NS;
            double a[2][P] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
            for (int j = 0; j < nj; ++j) {
                double w = Wm[((size_t)(jb + j) * NCH + c) * NS + b];
                for (int tf = 0; tf < 2; ++tf)
                    for (int n = 0; n < P; ++n) a[tf][n] += w * T[j][tf][n];
            }
            for (int tf = 0; tf < 2; ++tf)
                for (int n = 0; n < P; ++n) acc_sh[(tf * NCH + c) * NN + b * P + n] += a[tf][n];
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 2 * NCH * NN; q += blockDim.x) {
        int tf = q / (NCH * NN), c = (q / NN) % NCH, v = q % NN;
        MM[((((size_t)cell * WR + slot) * 2 + tf) * NCH + c) * nrhs * NN + (size_t)r * NN + v] = acc_sh[q];
    }
}

// One 1-D re-interpolation along axis AX (0..2 space, 3 time) of a 256-vector
// indexed ((i1 P + i2) P + i3) P + i4: out[.., o, ..] = sum_q A[o][q] in[.., q, ..].
template <int AX>
__device__ __forceinline__ double reinterp_axis(const double *in, const double *A, int v) {
    constexpr int stride = AX == 0 ? P * P * P : AX == 1 ? P * P : AX == 2 ? P : 1;
    const int o = (v / stride) % P, base = v - o * stride;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < P; ++q) s += A[o * P + q] * in[base + q * stride];
    return s;
}

// out = (Ax (x) Ay (x) Az (x) At) in, applied as four 1-D passes through LDS
// (buf holds the input on entry; A[4][P][P] in LDS).  All 256 threads take part.
__device__ __forceinline__ double reinterp4(double (*buf)[NN], const double (*A)[P * P], int v) {
    double t = reinterp_axis<3>(buf[0], A[3], v);
    __syncthreads();
    buf[1][v] = t;
    __syncthreads();
    t = reinterp_axis<2>(buf[1], A[2], v);
    buf[0][v] = t;
    __syncthreads();
    t = reinterp_axis<1>(buf[0], A[1], v);
    buf[1][v] = t;
    __syncthreads();
    return reinterp_axis<0>(buf[1], A[0], v);
}

// M2M for the non-leaf cells of a level: MM(S, k) = sum_{children, h} T_{oct,h} MM(child, 2k+h);
// truncated: h = 0 from the child's truncated MM, h = 1 from its full MM.
// T is the tensor product of the parent's 1-D cardinal functions at the child's
// nodes, applied axis by axis.  One block per (parent, channel, rhs, tf); thread
// = output (b, n).
__global__ void __launch_bounds__(256) k_m2m(const int *parent_cells, const int *child_beg, const int *child_end,
                                             const int *cix, const double *S1, const double *MMc, int slot0, int slot1,
                                             int WRc, double *MMp, int slot, int WRp, int nrhs) {
    int cell = parent_cells[blockIdx.x];
    int c = blockIdx.y % NCH, tf = blockIdx.y / NCH;
    int r = blockIdx.z;
    int v = threadIdx.x;
    __shared__ double buf[2][NN];
    __shared__ double A[4][P * P];
    double acc = 0.0;
    for (int ch = child_beg[cell]; ch < child_end[cell]; ++ch) {
        const int hsx[3] = {cix[3 * ch] & 1, cix[3 * ch + 1] & 1, cix[3 * ch + 2] & 1};
        for (int h = 0; h < 2; ++h) {
            int stf = (tf == 1 && h == 0) ? 1 : 0;
            int sl = h == 0 ? slot0 : slot1;
            __syncthreads();
            buf[0][v] = MMc[((((size_t)ch * WRc + sl) * 2 + stf) * NCH + c) * nrhs * NN + (size_t)r * NN + v];
            if (v < 4 * P * P) {
                const int ax = v / (P * P), e = v % (P * P);     // A[ax][o][q] = S1[h_ax][o][q]
                A[ax][e] = ax < 3 ? S1[hsx[ax] * P * P + e] : S1[2 * P * P + h * P * P + e];
            }
            __syncthreads();
            acc += reinterp4(buf, A, v);
        }
    }
    MMp[((((size_t)cell * WRp + slot) * 2 + tf) * NCH + c) * nrhs * NN + (size_t)r * NN + v] = acc;
}

// ---------------------------------------------------------------- M2L engine
// acc[256 x NT] += K(off, lag) X[256 x NT] on the matrix cores.  Rows are target
// nodes (a, m), columns of X are source moment vectors indexed (b, n); the
// 16x16x4 instruction's k-step of 4 is one source node b and its 4 time nodes.
// Node offsets lie on a lattice of spacing (2/3) h_s in space and (2/3) h_t in
// time: x_a - y_b = (2/3) h_s ((a - b) - 3 off), t_m - s_n = (2/3) h_t (3 lag +
// m - n).  For one (offset, lag) the operator therefore takes only 7^3 * 7
// distinct values, indexed by a - b in [-3, 3]^3 and m - n in [-3, 3]: the block
// tabulates them in LDS once per lag and every lane reads its A operand from the
// table at an address that is its own row base minus a constant of the k-step.
// T is the arithmetic type of the operator and the products (FP64 form: double
// with the f64 instruction; FP32 form: float with the f32 instruction); the
// moments and the accumulated local expansions stay in FP64 in HBM.
//
// X sits in LDS column-major, X[column][k] with M2L_XS(T) values per column:
// a lane's B operands of all 64 k-steps then lie within 2 KB of one address
// (immediate offsets, no address arithmetic between the reads, so the reads can
// run ahead of the products), and the padding (2 doubles or 4 floats) puts the
// 16 columns x 4 k-rows of one read on distinct banks.
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct Mma;
template <> struct Mma<double> {
    typedef v4d acc_t;
    __device__ static acc_t op(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int v) { return 4 * v + (lane >> 4); }      // output layout of the f64 form
};
template <> struct Mma<float> {
    typedef v4f acc_t;
    __device__ static acc_t op(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }      // output layout of the f32 form
};

static constexpr int KTAB = 2401;          // 7^3 spatial differences x 7 time differences
static constexpr int KTAB_MID = 1197;      // table index of a - b = (0, 0, 0), m - n = -3
static constexpr int M2L_THREADS = 512;    // 8 wavefronts: 4 row blocks of 64 x 2 column halves
template <typename T> struct M2lX { static constexpr int XS = NN + (sizeof(T) == 8 ? 2 : 4); };

// operator table of one (offset, lag): tab[((d1 + 3) * 7 + d2 + 3) * 7 + d3 + 3) * 7 + w + 3] =
// kernel at spatial lattice vector d - 3 off and time lattice 3 lag + w.
// kind 0: dU/dt = 2c (c tau - r)_+ / r; kind 1: U = (c tau - r)_+^2 / r.
// The distance r and 1 / r of the 343 spatial differences do not depend on the
// lag: m2l_dist tabulates them once per block, and each lag's table is then a
// multiply-add and a product per entry.  r stays FP64 (c tau - r cancels near
// the light cone); 1 / r is kept in T (the FP32 form rounds the table to float
// anyway, and two of its blocks then still fit one CU's LDS).
template <typename T>
__device__ void m2l_dist(double *rd, T *ird, int ox, int oy, int oz, double gs, double ds) {
    for (int d = threadIdx.x; d < 343; d += blockDim.x) {
        const double v1 = gs * (d / 49 - 3) - ds * ox, v2 = gs * ((d / 7) % 7 - 3) - ds * oy,
                     v3 = gs * (d % 7 - 3) - ds * oz;
        const double r = sqrt(v1 * v1 + v2 * v2 + v3 * v3);
        rd[d] = r;
        ird[d] = (T)(r > 0.0 ? 1.0 / r : 0.0);
    }
}

template <typename T>
__device__ void m2l_table(T *tab, const double *rd, const T *ird, int lag, int kind, double cgt, double c2) {
    for (int e = threadIdx.x; e < KTAB; e += blockDim.x) {
        const int w = e % 7 - 3, d = e / 7;
        const double r = rd[d];
        const double u = cgt * (3 * lag + w) - r;
        double kv = 0.0;
        if (u > 0.0 && r > 0.0) kv = kind == 0 ? c2 * u * (double)ird[d] : u * u * (double)ird[d];
        tab[e] = (T)kv;
    }
}

// per lane: table index of its rows at b = 0, minus KTAB_MID (k-step ks = b reads at
// base + KTAB_MID - 7 * (49 b1 + 7 b2 + b3), always inside [0, KTAB))
__device__ __forceinline__ void m2l_row_base(int (&base)[4], int wr, int lane) {
    const int n = lane >> 4;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        const int row = 64 * wr + 16 * rb + (lane & 15);
        const int a = row >> 2, m = row & 3;
        base[rb] = (((((a >> 4) + 3) * 7 + ((a >> 2) & 3) + 3) * 7 + (a & 3) + 3) * 7 + m - n + 3) - KTAB_MID;
    }
}

// acc (this wave's 64 rows x 32 columns) += K X for the table in LDS.  Per
// k-step a lane reads its 4 A operands from the table and its 2 B operands
// from X, all at immediate offsets, and issues 8 products.  The second wave on
// each SIMD covers the LDS latency (reading a whole k-step ahead measured no
// faster).
template <typename T>
__device__ __forceinline__ void m2l_operands(T (&kv)[4], T &bv0, T &bv1, const T (*X)[M2lX<T>::XS], const T *tab,
                                             const int (&base)[4], int ks, int n, int col) {
    const int b1 = ks >> 4, b2 = (ks >> 2) & 3, b3 = ks & 3;
    const int toff = KTAB_MID - 7 * ((b1 * 7 + b2) * 7 + b3);
    bv0 = X[col][4 * ks + n];
    bv1 = X[col + 16][4 * ks + n];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) kv[rb] = tab[base[rb] + toff];
}

template <typename T>
__device__ __forceinline__ void m2l_apply(typename Mma<T>::acc_t (&acc)[4][2], const T (*X)[M2lX<T>::XS],
                                          const T *tab, const int (&base)[4], int wc, int lane) {
    const int n = lane >> 4, col = 32 * wc + (lane & 15);
#pragma unroll
    for (int ks = 0; ks < 64; ++ks) {
        T kv[4], bv0, bv1;
        m2l_operands<T>(kv, bv0, bv1, X, tab, base, ks, n, col);
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            acc[rb][0] = Mma<T>::op(kv[rb], bv0, acc[rb][0]);
            acc[rb][1] = Mma<T>::op(kv[rb], bv1, acc[rb][1]);
        }
    }
}

// Staging of X: each thread owns the row pair (2 xr, 2 xr + 1) and the columns
// j = xg, xg + 4, ..., so every global load and LDS store moves two adjacent
// rows at once (16-byte moment loads; column bases are multiples of 256
// values and the padded column strides keep the LDS stores aligned).
// m2l_fetch issues the global loads of one lag (all in flight together) into
// registers; m2l_store writes them to LDS.  The kernels fetch the next lag
// before the current lag's products, so the loads overlap the matrix cores.
static constexpr int M2L_PRE = M2L_NT / 4;
template <typename T> struct M2lPair;
template <> struct M2lPair<double> { typedef double2 type; };
template <> struct M2lPair<float> { typedef float2 type; };
template <typename T>
__device__ __forceinline__ void m2l_fetch(typename M2lPair<T>::type (&pre)[M2L_PRE], const int64_t *cbase,
                                          const double *MM, int64_t loff, int xg) {
#pragma unroll
    for (int i = 0; i < M2L_PRE; ++i) {
        const int64_t b = cbase[xg + 4 * i];
        double2 v = make_double2(0.0, 0.0);
        if (b >= 0) v = *reinterpret_cast<const double2 *>(MM + b + loff);
        pre[i].x = (T)v.x;
        pre[i].y = (T)v.y;
    }
}
template <typename T>
__device__ __forceinline__ void m2l_store(T (*X)[M2lX<T>::XS], const typename M2lPair<T>::type (&pre)[M2L_PRE],
                                          int xr, int xg) {
#pragma unroll
    for (int i = 0; i < M2L_PRE; ++i) *reinterpret_cast<typename M2lPair<T>::type *>(&X[xg + 4 * i][2 * xr]) = pre[i];
}

// offset-major M2L for one right-hand side: one block per (offset, kind, column
// tile); columns are (interaction-list entry q, channel).  Writes the per-entry
// contribution YB[q][ch][NN] summed over the window's lags.
template <typename T>
__global__ void __launch_bounds__(M2L_THREADS, sizeof(T) == 4 ? 4 : 2) k_m2l_off(const int *tile_code, const int *tile_kind,
                                                         const int *tile_col0, const int *tile_ncol, const int *col_q,
                                                         const int *col_ch, const int *il_src, const double *MM, int WR,
                                                         int k, int W, double hn, double ds, double ht, double cl,
                                                         double *YB, const float *MMf) {
    const int tile = blockIdx.x;
    const int code = tile_code[tile], kind = tile_kind[tile], col0 = tile_col0[tile], ncol = tile_ncol[tile];
    const int ox = code / 49 - 3, oy = (code / 7) % 7 - 3, oz = code % 7 - 3;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wr = wave & 3, wc = wave >> 2;
    __shared__ __attribute__((aligned(16))) T X[M2L_NT][M2lX<T>::XS];
    __shared__ T tab[KTAB];
    __shared__ double rd[343];
    __shared__ T ird[343];
    __shared__ int64_t cbase[M2L_NT];
    int base[4];
    m2l_row_base(base, wr, lane);
    const double gs = hn * (2.0 / (P - 1)), cgt = cl * ht * (2.0 / (P - 1));
    typename Mma<T>::acc_t acc[4][2];
    for (int rb = 0; rb < 4; ++rb) acc[rb][0] = acc[rb][1] = typename Mma<T>::acc_t{0, 0, 0, 0};
    // MM offset of every column at slot 0 (-1: padding column)
    if (tid < M2L_NT) {
        int64_t b = -1;
        if (tid < ncol) b = ((int64_t)il_src[col_q[col0 + tid]] * WR * 2 * NCH + col_ch[col0 + tid]) * NN;
        cbase[tid] = b;
    }
    const int xr = tid & (NN / 2 - 1), xg = tid >> 7;   // row pair, first column
    const int nlag = min(W, k + 1);               // lags whose source interval exists
    auto loff = [&](int lag) {
        return (int64_t)(((k + 1 - lag) % WR) * 2 + (lag == W ? 1 : 0)) * NCH * NN + 2 * xr;
    };
    m2l_dist<T>(rd, ird, ox, oy, oz, gs, ds);
    if constexpr (sizeof(T) == 4) {
        // FP32 form: X from the FP32 copy of the moments (the same values the
        // conversion at staging gave), four rows per 16-byte load and store;
        // thread = row quad xq and columns xh, xh + 8, ...
        const int xq = tid & 63, xh = tid >> 6;
        auto loff4 = [&](int lag) {
            return (int64_t)(((k + 1 - lag) % WR) * 2 + (lag == W ? 1 : 0)) * NCH * NN + 4 * xq;
        };
        float4 p4[M2L_NT / 8];
        auto fetch4 = [&](int64_t lo) {
#pragma unroll
            for (int i = 0; i < M2L_NT / 8; ++i) {
                const int64_t b = cbase[xh + 8 * i];
                p4[i] = b >= 0 ? *reinterpret_cast<const float4 *>(MMf + b + lo) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        };
        __syncthreads();                          // cbase, rd and ird visible
        fetch4(loff4(1));
        for (int lag = 1; lag <= nlag; ++lag) {
            __syncthreads();                      // the previous products are done with X and tab
#pragma unroll
            for (int i = 0; i < M2L_NT / 8; ++i) *reinterpret_cast<float4 *>(&X[xh + 8 * i][4 * xq]) = p4[i];
            m2l_table<T>(tab, rd, ird, lag, kind, cgt, 2.0 * cl);
            __syncthreads();
            if (lag < nlag) fetch4(loff4(lag + 1));
            m2l_apply<T>(acc, X, tab, base, wc, lane);
        }
    } else {
        typename M2lPair<T>::type pre[M2L_PRE];
        __syncthreads();                          // cbase, rd and ird visible
        m2l_fetch<T>(pre, cbase, MM, loff(1), xg);
        for (int lag = 1; lag <= nlag; ++lag) {
            __syncthreads();                      // the previous products are done with X and tab
            m2l_store<T>(X, pre, xr, xg);
            m2l_table<T>(tab, rd, ird, lag, kind, cgt, 2.0 * cl);
            __syncthreads();
            if (lag < nlag) m2l_fetch<T>(pre, cbase, MM, loff(lag + 1), xg);
            m2l_apply<T>(acc, X, tab, base, wc, lane);
        }
    }
    for (int rb = 0; rb < 4; ++rb)
        for (int cb = 0; cb < 2; ++cb) {
            int j = 32 * wc + 16 * cb + (lane & 15);
            if (j >= ncol) continue;
            int q = col_q[col0 + j], ch = col_ch[col0 + j];
            for (int v = 0; v < 4; ++v) {
                int row = 64 * wr + 16 * rb + Mma<T>::row(lane, v);
                YB[((size_t)q * NCH + ch) * NN + row] = (double)acc[rb][cb][v];
            }
        }
}

// LC(O) = PEND(O, parity) + sum over O's interaction-list entries of YB (target-owned, fixed order)
__global__ void k_m2l_reduce(int n, const int *il_off, const double *YB, const double *PEND, int parity, double *LC) {
    int O = blockIdx.x, c = blockIdx.y, v = threadIdx.x;
    double s = PEND[(((size_t)O * 2 + parity) * NCH + c) * NN + v];
    for (int q = il_off[O]; q < il_off[O + 1]; ++q) s += YB[((size_t)q * NCH + c) * NN + v];
    LC[((size_t)O * NCH + c) * NN + v] = s;
}

// target-major M2L for batched right-hand sides: one block per (target, kind,
// (channel, rhs) tile of 64 columns); items are (interaction-list source, lag).
template <typename T>
__global__ void __launch_bounds__(M2L_THREADS, sizeof(T) == 4 ? 4 : 2) k_m2l_tgt(const int *il_off, const int *il_src, const int *il_code,
                                                         const double *MM, int WR, int k, int W, double hn, double ds,
                                                         double ht, double cl, const double *PEND, double *LC,
                                                         int nrhs, const float *MMf) {
    const int O = blockIdx.x, kind = blockIdx.y;
    const int c0 = kind == 0 ? 0 : 3, nc = kind == 0 ? 3 : 4;
    const int ncolt = nc * nrhs;
    const int col0 = blockIdx.z * M2L_NT;
    if (col0 >= ncolt) return;
    const int ncol = min(M2L_NT, ncolt - col0);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wr = wave & 3, wc = wave >> 2;
    const int parity = (k + 1) & 1;
    __shared__ __attribute__((aligned(16))) T X[M2L_NT][M2lX<T>::XS];
    __shared__ T tab[KTAB];
    __shared__ double rd[343];
    __shared__ T ird[343];
    __shared__ int64_t cbase[M2L_NT];
    int base[4];
    m2l_row_base(base, wr, lane);
    const double gs = hn * (2.0 / (P - 1)), cgt = cl * ht * (2.0 / (P - 1));
    typename Mma<T>::acc_t acc[4][2];
    for (int rb = 0; rb < 4; ++rb) acc[rb][0] = acc[rb][1] = typename Mma<T>::acc_t{0, 0, 0, 0};
    const int xr = tid & (NN / 2 - 1), xg = tid >> 7;   // row pair, first column
    // column offsets within one source cell's moments (the source enters per item)
    if (tid < M2L_NT) {
        int64_t b = -1;
        if (tid < ncol) {
            const int cc = (col0 + tid) / nrhs, r = (col0 + tid) % nrhs;
            b = ((int64_t)(c0 + cc) * nrhs + r) * NN;
        }
        cbase[tid] = b;
    }
    // items (interaction-list entry, lag), entries outer
    const int q0 = il_off[O], nq = il_off[O + 1] - q0;
    const int nlag = min(W, k + 1);
    const int nitem = nq * nlag;
    const int64_t strideS = (int64_t)WR * 2 * NCH * nrhs * NN;
    auto loff = [&](int it) {
        const int q = q0 + it / nlag, lag = it % nlag + 1;
        return (int64_t)il_src[q] * strideS +
               (int64_t)(((k + 1 - lag) % WR) * 2 + (lag == W ? 1 : 0)) * NCH * nrhs * NN + 2 * xr;
    };
    if constexpr (sizeof(T) == 4) {
        // FP32 form: X from the FP32 copy of the moments, four rows per
        // 16-byte load and store (thread = row quad xq, columns xh + 8 i)
        const int xq = tid & 63, xh = tid >> 6;
        auto loff4 = [&](int it) {
            const int q = q0 + it / nlag, lag = it % nlag + 1;
            return (int64_t)il_src[q] * strideS +
                   (int64_t)(((k + 1 - lag) % WR) * 2 + (lag == W ? 1 : 0)) * NCH * nrhs * NN + 4 * xq;
        };
        float4 p4[M2L_NT / 8];
        auto fetch4 = [&](int64_t lo) {
#pragma unroll
            for (int i = 0; i < M2L_NT / 8; ++i) {
                const int64_t b = cbase[xh + 8 * i];
                p4[i] = b >= 0 ? *reinterpret_cast<const float4 *>(MMf + b + lo) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        };
        __syncthreads();                          // cbase visible
        if (nitem > 0) fetch4(loff4(0));
        for (int it = 0; it < nitem; ++it) {
            const int q = q0 + it / nlag, lag = it % nlag + 1;
            const int code = il_code[q];
            const int ox = code / 49 - 3, oy = (code / 7) % 7 - 3, oz = code % 7 - 3;
            __syncthreads();
#pragma unroll
            for (int i = 0; i < M2L_NT / 8; ++i) *reinterpret_cast<float4 *>(&X[xh + 8 * i][4 * xq]) = p4[i];
            if (lag == 1) {                       // a new source entry: its offset's distances
                m2l_dist<T>(rd, ird, ox, oy, oz, gs, ds);
                __syncthreads();
            }
            m2l_table<T>(tab, rd, ird, lag, kind, cgt, 2.0 * cl);
            __syncthreads();
            if (it + 1 < nitem) fetch4(loff4(it + 1));
            m2l_apply<T>(acc, X, tab, base, wc, lane);
        }
    } else {
        typename M2lPair<T>::type pre[M2L_PRE];
        __syncthreads();                          // cbase visible
        if (nitem > 0) m2l_fetch<T>(pre, cbase, MM, loff(0), xg);
        for (int it = 0; it < nitem; ++it) {
            const int q = q0 + it / nlag, lag = it % nlag + 1;
            const int code = il_code[q];
            const int ox = code / 49 - 3, oy = (code / 7) % 7 - 3, oz = code % 7 - 3;
            __syncthreads();
            m2l_store<T>(X, pre, xr, xg);
            if (lag == 1) {                       // a new source entry: its offset's distances
                m2l_dist<T>(rd, ird, ox, oy, oz, gs, ds);
                __syncthreads();
            }
            m2l_table<T>(tab, rd, ird, lag, kind, cgt, 2.0 * cl);
            __syncthreads();
            if (it + 1 < nitem) m2l_fetch<T>(pre, cbase, MM, loff(it + 1), xg);
            m2l_apply<T>(acc, X, tab, base, wc, lane);
        }
    }
    for (int rb = 0; rb < 4; ++rb)
        for (int cb = 0; cb < 2; ++cb) {
            int j = 32 * wc + 16 * cb + (lane & 15);
            if (j >= ncol) continue;
            int cc = (col0 + j) / nrhs, r = (col0 + j) % nrhs;
            for (int v = 0; v < 4; ++v) {
                int row = 64 * wr + 16 * rb + Mma<T>::row(lane, v);
                size_t o = (((size_t)O * NCH + c0 + cc) * nrhs + r) * NN + row;
                size_t pe = ((((size_t)O * 2 + parity) * NCH + c0 + cc) * nrhs + r) * NN + row;
                LC[o] = (double)acc[rb][cb][v] + PEND[pe];
            }
        }
}

// FP32 copy of a level's moments for the reduced forms' M2L (rounded once here
// instead of at every staging of X)
__global__ void k_mm_to_f32(int64_t n, const double *__restrict__ src, float *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

// launch of the M2L of one level at gate k
template <typename T>
static void m2l_launch(tdbem_ctx *C, FarLevel &FL, int k, hipStream_t s) {
    FarState *F = C->far;
    const int nr = C->nrhs;
    if (sizeof(T) == 4 && (nr > 1 || FL.ntile > 0)) {
        // the reduced forms stage X from an FP32 copy of this level's moments
        PhaseScope ps(C->prof, TDBEM_PH_OTHER, s);
        const int64_t nmm = (int64_t)FL.n * F->WR * 2 * NCH * nr * NN;
        hipLaunchKernelGGL(k_mm_to_f32, dim3((unsigned)((nmm + 255) / 256)), dim3(256), 0, s, nmm, FL.MM, FL.MM32);
    }
    if (nr == 1) {
        if (FL.ntile > 0) {
            PhaseScope ps(C->prof, TDBEM_PH_M2L, s);
            hipLaunchKernelGGL(k_m2l_off<T>, dim3(FL.ntile), dim3(M2L_THREADS), 0, s, FL.tile_code, FL.tile_kind,
                               FL.tile_col0, FL.tile_ncol, FL.col_q, FL.col_ch, FL.il_src, FL.MM, F->WR, k, F->W, FL.hn,
                               FL.ds, FL.ht, C->c, FL.YB, (const float *)FL.MM32);
        }
        PhaseScope ps(C->prof, TDBEM_PH_M2L_SUM, s);
        hipLaunchKernelGGL(k_m2l_reduce, dim3(FL.n, NCH), dim3(NN), 0, s, FL.n, FL.il_off, FL.YB, FL.PEND, (k + 1) & 1,
                           FL.LC);
    } else {
        PhaseScope ps(C->prof, TDBEM_PH_M2L, s);
        hipLaunchKernelGGL(k_m2l_tgt<T>, dim3(FL.n, 2, (4 * nr + M2L_NT - 1) / M2L_NT), dim3(M2L_THREADS), 0, s,
                           FL.il_off, FL.il_src, FL.il_code, FL.MM, F->WR, k, F->W, FL.hn, FL.ds, FL.ht, C->c, FL.PEND, FL.LC,
                           nr, (const float *)FL.MM32);
    }
}

// L2L: PEND(child, h) = T_{oct,h}^T LC(parent) for the child's intervals 2(k+1)+h.
// One block per (parent, channel, rhs, h) per child; thread = child output (a', m').
__global__ void __launch_bounds__(256) k_l2l(const int *parent_cells, const int *child_beg, const int *child_end,
                                             const int *cix, const double *S1, const double *LCp, double *PENDc, int nrhs) {
    int cell = parent_cells[blockIdx.x];
    int c = blockIdx.y % NCH, h = blockIdx.y / NCH;
    int r = blockIdx.z;
    int v = threadIdx.x;
    __shared__ double buf[2][NN];
    __shared__ double A[4][P * P];
    const double lc = LCp[((size_t)cell * NCH + c) * nrhs * NN + (size_t)r * NN + v];
    for (int ch = child_beg[cell]; ch < child_end[cell]; ++ch) {
        const int hsx[3] = {cix[3 * ch] & 1, cix[3 * ch + 1] & 1, cix[3 * ch + 2] & 1};
        __syncthreads();
        buf[0][v] = lc;
        if (v < 4 * P * P) {
            // transpose: child output o from parent input q, A[ax][o][q] = S1[h_ax][q][o]
            const int ax = v / (P * P), o = (v % (P * P)) / P, q = v % P;
            const int hh = ax < 3 ? hsx[ax] : h;
            A[ax][o * P + q] = S1[(ax < 3 ? 0 : 2 * P * P) + (hh * P + q) * P + o];
        }
        __syncthreads();
        const double out = reinterp4(buf, A, v);
        PENDc[(((size_t)ch * 2 + h) * NCH + c) * nrhs * NN + (size_t)r * NN + v] = out;
    }
}

// L2P: FAR(slot of step alpha') for the edges of a leaf, alpha' = (k+1)M + q, q = 1..M:
// sum_c sum_a El[i][c][a] Lt[q][c][a], Lt[q][c][a] = sum_m LC[c][a][m] tw_c(m, q); tw: l_m' for
// channels 0-2, l_m for 3, l_m' + zeta l_m for 4-6.  One block per (leaf, rhs): the
// leaf's time-contracted expansions Lt are formed once in LDS for a chunk of
// L2P_QC target steps and shared by all its edges.
static constexpr int L2P_QC = 8;
__global__ void __launch_bounds__(256) k_l2p(const int *leaf_cells, const int *ebeg, const int *eend, int k, int M,
                                             const double *tw, double zeta, const double *El, const double *LC,
                                             double *FAR, int FR, int ne, int nrhs) {
    const int cell = leaf_cells[blockIdx.x], r = blockIdx.y;
    const int e0 = ebeg[cell], nloc = eend[cell] - e0;
    __shared__ double Lt[L2P_QC][NCH][NS];
    const double *L = LC + (size_t)cell * NCH * nrhs * NN + (size_t)r * NN;
    for (int q0 = 1; q0 <= M; q0 += L2P_QC) {
        const int nq = min(L2P_QC, M - q0 + 1);
        __syncthreads();
        for (int t = threadIdx.x; t < nq * NCH * NS; t += blockDim.x) {
            const int qi = t / (NCH * NS), c = (t / NS) % NCH, a = t % NS;
            const double *tv = tw + (size_t)(q0 + qi - 1) * 2 * P;
            const double *l = L + (size_t)c * nrhs * NN + a * P;
            double s = 0.0;
            for (int m = 0; m < P; ++m) {
                const double w = c < 3 ? tv[P + m] : (c == 3 ? tv[m] : tv[P + m] + zeta * tv[m]);
                s += l[m] * w;
            }
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

void ifmm_after_solve(tdbem_ctx *C, int alpha, hipStream_t s) {
    FarState *F = C->far;
    const int nr = C->nrhs;
    // upward pass (Program 3)
    for (int l = F->lmax; l >= 2; --l) {
        FarLevel &FL = F->lev[l];
        if (alpha % FL.M) continue;
        int k = alpha / FL.M - 1;
        int slot = k % F->WR;
        if (FL.nleaf > 0) {
            PhaseScope ps(C->prof, TDBEM_PH_P2M, s);
            hipLaunchKernelGGL(k_p2m, dim3(FL.nleaf, nr), dim3(256), 0, s, FL.leaf_cells, FL.ebeg, FL.eend, k, FL.M,
                               FL.ls, C->d_Jring, C->ring, nr, F->Wm, FL.MM, slot, F->WR);
        }
        if (FL.nparent > 0) {
            PhaseScope ps(C->prof, TDBEM_PH_M2M, s);
            FarLevel &CL = F->lev[l + 1];
            hipLaunchKernelGGL(k_m2m, dim3(FL.nparent, 2 * NCH, nr), dim3(NN), 0, s, FL.parent_cells, FL.child_beg,
                               FL.child_end, CL.ix, F->S1 + (size_t)l * 4 * P * P, CL.MM, (2 * k) % F->WR, (2 * k + 1) % F->WR, F->WR, FL.MM,
                               slot, F->WR, nr);
        }
        TD_HIP(hipGetLastError());
    }
    // downward pass (Program 4)
    for (int l = 2; l <= F->lmax; ++l) {
        FarLevel &FL = F->lev[l];
        if (alpha % FL.M) continue;
        int k = alpha / FL.M - 1;
        if (C->cfg.precision == TDBEM_FP64) m2l_launch<double>(C, FL, k, s); else m2l_launch<float>(C, FL, k, s);
        if (FL.nparent > 0) {
            PhaseScope ps(C->prof, TDBEM_PH_L2L, s);
            FarLevel &CL = F->lev[l + 1];
            hipLaunchKernelGGL(k_l2l, dim3(FL.nparent, 2 * NCH, nr), dim3(NN), 0, s, FL.parent_cells, FL.child_beg,
                               FL.child_end, CL.ix, F->S1 + (size_t)l * 4 * P * P, FL.LC, CL.PEND, nr);
        }
        if (FL.nleaf > 0) {
            PhaseScope ps(C->prof, TDBEM_PH_L2P, s);
            hipLaunchKernelGGL(k_l2p, dim3(FL.nleaf, nr), dim3(256), 0, s, FL.leaf_cells, FL.ebeg, FL.eend, k, FL.M,
                               FL.tw, C->cfg.zeta, F->El, FL.LC, F->FAR, F->FR, C->ne, nr);
        }
        TD_HIP(hipGetLastError());
    }
}

}  // namespace tdbem
