// extern "C" entry points and the marching driver (Program 1).
#include <algorithm>
#include <functional>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "ifmm.h"
#include "tdbem_internal.h"

namespace tdbem {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

hipEvent_t Profiler::get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e;
    TD_HIP(hipEventCreate(&e));
    return e;
}
void Profiler::begin(int, hipStream_t s, hipEvent_t &e0) {
    e0 = get();
    TD_HIP(hipEventRecord(e0, s));
}
void Profiler::end(int ph, hipStream_t s, hipEvent_t e0) {
    hipEvent_t e1 = get();
    if (hipEventRecord(e1, s) != hipSuccess) return;
    pending.push_back({ph, {e0, e1}});
}
void Profiler::fold(hipStream_t s) {
    TD_HIP(hipStreamSynchronize(s));
    for (auto &p : pending) {
        float t = 0.f;
        TD_HIP(hipEventElapsedTime(&t, p.second.first, p.second.second));
        ms[p.first] += t;
        count[p.first] += 1;
        pool.push_back(p.second.first);
        pool.push_back(p.second.second);
    }
    pending.clear();
}
void Profiler::clear() {
    for (auto &p : pending) { pool.push_back(p.second.first); pool.push_back(p.second.second); }
    pending.clear();
    for (int i = 0; i < TDBEM_NPHASE; ++i) { ms[i] = 0; count[i] = 0; }
}
Profiler::~Profiler() {
    for (auto &p : pending) { (void)hipEventDestroy(p.second.first); (void)hipEventDestroy(p.second.second); }
    for (auto e : pool) (void)hipEventDestroy(e);
}

void launch_lag_range(const GeoDev &G, int64_t npairs, const int *pi, const int *pj, int *lo, int *hi, hipStream_t s);
void launch_zfill(const GeoDev &G, int64_t n, int64_t k0, int64_t npairs, const int *pi, const int *pj, const int *g0,
                  const int64_t *off, double *val, hipStream_t s);
void launch_vinc(const GeoDev &G, int ne, int nrhs, const double *pulses, const int *perm, double t, double *V, hipStream_t s);
void launch_near(const tdbem_ctx *C, int alpha, double *out, double scale, hipStream_t s);
void launch_gather_in(const tdbem_ctx *C, const double *src, double *dst, hipStream_t s);
void launch_scatter_out(const tdbem_ctx *C, const double *src, double *dst, hipStream_t s);
void launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s);
void launch_ring_put(const tdbem_ctx *C, int slot, const double *x, hipStream_t s);
void launch_extrap(const tdbem_ctx *C, int alpha, double *x, hipStream_t s);
void launch_rhs_finish(const tdbem_ctx *C, int alpha, const double *far, hipStream_t s);
void launch_ring_out(const tdbem_ctx *C, int slot, double *Jout, hipStream_t s);
void launch_to_f32(const double *src, float *dst, int64_t n, hipStream_t s);
void launch_near_to_jds(const tdbem_ctx *C, const int64_t *src_off, const double *src, hipStream_t s);
void launch_gather_vals(const double *val, const int64_t *idx, int64_t n, double *out, hipStream_t s);
int gmres_solve(tdbem_ctx *C, const double *b, double *x, double rtol, int maxit, bool *ok, hipStream_t s);
size_t gmres_work_doubles(const tdbem_ctx *C, int maxit);
bool gmres_coop_launch(tdbem_ctx *C, const double *b, double *x, double rtol, int maxit, hipStream_t s);
bool gmres_coop_launch_static(tdbem_ctx *C, const double *b, double *x, double rtol, int maxit, hipStream_t s,
                              int **iflag_out);
double *noalloc_scratch(size_t *capacity);
size_t noalloc_need(const tdbem_ctx *C);
size_t gmres_coop_work_doubles(int ne, int nrhs);
void launch_fill(int64_t n, double v, double *p, hipStream_t s);
int near_variants();
constexpr int NEAR_DEFAULT_LEAF = 5;    // the per-leaf kernel, 2 lag steps x 2 pair blocks per round
void near_variant_shape(int v, int *nu, int *nc);

size_t near_leaf_lds_budget(int L);
int near_leaf_rows();
bool near_leaf_sorted();

// The per-leaf form of the one-rhs near field: per leaf cell, its rows (a
// range in leaf order), the sorted source edges of its rows' pairs, each
// pair's index in that list, and per source the lags its strips reach there
// (the source's part of the leaf's current window; the parts are laid end to
// end).  Leaves whose window exceeds the LDS budget keep the row kernel; the
// others are cut into chunks of rows, a block each.  The box window [gmin,
// gmin + gw) of all strips serves the batched matrix-core form.
static void build_near_leaves(tdbem_ctx *C, const std::vector<int> &nrow, const std::vector<int> &nj,
                              const std::vector<int> &ngl) {
    const Tree &T = C->T;
    const size_t jt = C->cfg.precision == TDBEM_FP64 ? sizeof(double) : sizeof(float);
    const size_t budget = std::min<size_t>(near_leaf_lds_budget(C->near_L) / jt, 65535);
    const int crow = near_leaf_rows();
    std::vector<int> r0, r1, soff(1, 0), src, g, loc(nj.size(), 0), pwl(nj.size(), 0), ws, chunk, rest;
    C->h_leaf_w.clear();
    C->h_colmap.clear();
    C->h_pcol.assign(C->nrhs > 1 ? nj.size() : 0, 0);
    size_t maxw = 0;
    for (int l = 0; l <= T.lmax; ++l) {
        const Level &Lv = T.lev[l];
        for (int c = 0; c < Lv.n; ++c) {
            if (!Lv.leaf[c] || Lv.eend[c] <= Lv.ebeg[c]) continue;
            const int a = Lv.ebeg[c], b = Lv.eend[c];
            std::vector<int> list;
            int gmin = 1 << 30, gmax = -1;
            for (int q = nrow[a]; q < nrow[b]; ++q) {
                list.push_back(nj[q]);
                gmin = std::min(gmin, ngl[q] & 0xffff);
                gmax = std::max(gmax, (ngl[q] & 0xffff) + (ngl[q] >> 16) - 1);
            }
            std::sort(list.begin(), list.end());
            list.erase(std::unique(list.begin(), list.end()), list.end());
            const int id = (int)r0.size();
            r0.push_back(a);
            r1.push_back(b);
            const int gw = gmax >= gmin ? gmax - gmin + 1 : 1;
            g.push_back(gmax >= gmin ? gmin : 2);
            g.push_back(gw);
            std::vector<int> lo(list.size(), 1 << 30), hi(list.size(), -1);
            for (int q = nrow[a]; q < nrow[b]; ++q) {
                const int li = (int)(std::lower_bound(list.begin(), list.end(), nj[q]) - list.begin());
                loc[q] = li;
                const int g0 = ngl[q] & 0xffff, len = ngl[q] >> 16;
                if (len > 0) {
                    lo[li] = std::min(lo[li], g0);
                    hi[li] = std::max(hi[li], g0 + len - 1);
                }
            }
            std::vector<int> woff(list.size());
            size_t w = 0;
            const bool mm = C->nrhs > 1;       // the batched matrix-core form's column map
            for (size_t k = 0; k < list.size(); ++k) {
                woff[k] = (int)std::min<size_t>(w, 1 << 30);
                const int n = hi[k] >= lo[k] ? hi[k] - lo[k] + 1 : 0;
                ws.push_back(list[k]);
                ws.push_back(n > 0 ? lo[k] : 0);
                ws.push_back(woff[k]);
                ws.push_back(n);
                if (mm)
                    for (int t = 0; t < n; ++t) {
                        C->h_colmap.push_back(list[k]);
                        C->h_colmap.push_back(lo[k] + t);
                    }
                w += (size_t)n;
            }
            TD_REQUIRE(w < (size_t)1 << 31, TDBEM_EINVAL, "a leaf's near-field window exceeds 2^31 columns");
            C->h_leaf_w.push_back((int)w);
            if (mm)
                for (int q = nrow[a]; q < nrow[b]; ++q)
                    C->h_pcol[q] = woff[loc[q]] + ((ngl[q] & 0xffff) - lo[loc[q]]);
            src.insert(src.end(), list.begin(), list.end());
            soff.push_back((int)src.size());
            if (w <= budget) {
                for (int q = nrow[a]; q < nrow[b]; ++q) {
                    const int li = loc[q], g0 = ngl[q] & 0xffff, len = ngl[q] >> 16;
                    pwl[q] = (len > 0 ? woff[li] + g0 - lo[li] : 0) | (len << 16);
                }
                for (int r = a; r < b; r += crow) {
                    chunk.push_back(id);
                    chunk.push_back(r);
                    chunk.push_back(std::min(b, r + crow));
                }
                maxw = std::max(maxw, w);
            } else {
                for (int r = a; r < b; ++r) rest.push_back(r);
            }
        }
    }
    // the leaves' rows must partition the rows; otherwise every row takes the row kernel
    size_t covered = 0;
    for (size_t i = 0; i < r0.size(); ++i) covered += (size_t)(r1[i] - r0[i]);
    if (covered != (size_t)C->ne) {
        chunk.clear();
        rest.resize(C->ne);
        std::iota(rest.begin(), rest.end(), 0);
    }
    NearLeaves &NL = C->nleaf;
    NL.nleaves = (int)r0.size();
    C->h_leaf_r0 = r0;
    C->h_leaf_r1 = r1;
    C->leaf_cover = covered == (size_t)C->ne;
    if (near_leaf_sorted()) {
        // largest chunks (stored coefficients) first: the last blocks to start
        // are the small ones, so the CUs finish together
        std::vector<int64_t> work(chunk.size() / 3, 0);
        for (size_t c = 0; c < work.size(); ++c)
            for (int r = chunk[3 * c + 1]; r < chunk[3 * c + 2]; ++r)
                for (int q = nrow[r]; q < nrow[r + 1]; ++q) work[c] += ngl[q] >> 16;
        std::vector<int> ord(work.size());
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return work[x] > work[y]; });
        std::vector<int> sorted(chunk.size());
        for (size_t c = 0; c < ord.size(); ++c)
            for (int t = 0; t < 3; ++t) sorted[3 * c + t] = chunk[3 * (size_t)ord[c] + t];
        chunk.swap(sorted);
    }
    NL.nchunk = (int)(chunk.size() / 3);
    NL.nrest = (int)rest.size();
    NL.max_window = std::max<size_t>(maxw, 1);
    if (C->trace)
        std::fprintf(stderr, "[tdbem] per-leaf near field: %zu leaves, %d chunks of <= %d rows, %d rows left to the "
                     "row kernel, largest window %zu values\n", r0.size(), NL.nchunk, crow, NL.nrest, maxw);
    NL.d_chunk = dupload(C, chunk);
    NL.d_r0 = dupload(C, r0);
    NL.d_r1 = dupload(C, r1);
    NL.d_soff = dupload(C, soff);
    NL.d_src = dupload(C, src);
    NL.d_g = dupload(C, g);
    NL.d_loc = dupload(C, loc);
    NL.d_ws = dupload(C, ws);
    NL.d_pwl = dupload(C, pwl);
    NL.d_rest = dupload(C, rest);
}

void launch_leaf_mm_fill(const tdbem_ctx *C, int64_t np, const int *prow, const int *pcol, const int64_t *psrc,
                         const int *row_leaf, const int64_t *aoff, const int *kpad, const double *val, hipStream_t s);

// Batched right-hand sides: the dense per-leaf coefficient blocks of the
// matrix-core near field (rows x the leaf's compressed window, padded to 4 columns),
// filled from the pair-major set-up coefficients.  Skipped when the leaves do
// not partition the rows or the blocks would exceed 32 GB.
static void build_leaf_mm(tdbem_ctx *C, const std::vector<int> &nrow, const int64_t *d_psrc, const double *d_val) {
    if (!C->leaf_cover) return;
    const size_t nl = C->h_leaf_r0.size();
    std::vector<int64_t> aoff(nl), coff(nl);
    std::vector<int> kpad(nl), row_leaf(C->ne, 0), colmap;
    int64_t tot = 0, ctot = 0, csrc = 0;
    // a leaf's columns are its compressed window (per source the lags its
    // strips reach), padded to a multiple of 4 with (edge 0, lag 0) columns
    // whose coefficients stay zero
    colmap.reserve(C->h_colmap.size() + 8 * nl);
    for (size_t i = 0; i < nl; ++i) {
        const int K = C->h_leaf_w[i];
        kpad[i] = std::max(4, (K + 3) / 4 * 4);
        aoff[i] = tot;
        coff[i] = ctot;
        tot += (int64_t)(C->h_leaf_r1[i] - C->h_leaf_r0[i]) * kpad[i];
        colmap.insert(colmap.end(), C->h_colmap.begin() + 2 * csrc, C->h_colmap.begin() + 2 * (csrc + K));
        colmap.resize(colmap.size() + 2 * (size_t)(kpad[i] - K), 0);
        csrc += K;
        ctot += kpad[i];
        for (int r = C->h_leaf_r0[i]; r < C->h_leaf_r1[i]; ++r) row_leaf[r] = (int)i;
    }
    std::vector<int>().swap(C->h_colmap);
    const size_t vb = C->cfg.precision == TDBEM_FP64 ? sizeof(double) : sizeof(float);
    if ((double)tot * vb > 32e9) { std::vector<int>().swap(C->h_pcol); return; }
    std::vector<int> prow(nrow.back());
    for (int i = 0; i < C->ne; ++i)
        for (int q = nrow[i]; q < nrow[i + 1]; ++q) prow[q] = i;
    hipStream_t s = C->stream;
    C->leaf_mm_bytes = tot * (int64_t)vb;
    if (C->cfg.precision == TDBEM_FP64) {
        C->d_leafA64 = dalloc<double>(C, tot);
        TD_HIP(hipMemsetAsync(C->d_leafA64, 0, tot * sizeof(double), s));
    } else {
        C->d_leafA32 = dalloc<float>(C, tot);
        TD_HIP(hipMemsetAsync(C->d_leafA32, 0, tot * sizeof(float), s));
    }
    C->d_leaf_aoff = dupload(C, aoff);
    C->d_leaf_kpad = dupload(C, kpad);
    C->d_leaf_coff = dupload(C, coff);
    C->d_leaf_colmap = dupload(C, colmap);
    int *d_prow = dupload(C, prow);
    int *d_pcol = dupload(C, C->h_pcol);
    C->d_row_leaf = dupload(C, row_leaf);
    launch_leaf_mm_fill(C, (int64_t)prow.size(), d_prow, d_pcol, d_psrc, C->d_row_leaf, C->d_leaf_aoff,
                        C->d_leaf_kpad, d_val, s);
    TD_HIP(hipStreamSynchronize(s));
    dfree(C, d_prow, prow.size());
    dfree(C, d_pcol, C->h_pcol.size());
    std::vector<int>().swap(C->h_pcol);
    // column segments of at most LEAF_KSEG columns, one block each, so that
    // large leaves do not leave the other CUs idle; partial sums per segment
    constexpr int LEAF_KSEG = 2048;
    std::vector<int> seg_leaf, seg_k, leaf_seg(1, 0);
    std::vector<int64_t> seg_poff;
    int64_t poff = 0;
    for (size_t i = 0; i < nl; ++i) {
        const int nr = C->h_leaf_r1[i] - C->h_leaf_r0[i];
        for (int k = 0; k < kpad[i]; k += LEAF_KSEG) {
            seg_leaf.push_back((int)i);
            seg_k.push_back(k);
            seg_k.push_back(std::min(kpad[i], k + LEAF_KSEG));
            seg_poff.push_back(poff);
            poff += (int64_t)nr * C->nrhs;
        }
        leaf_seg.push_back((int)seg_leaf.size());
    }
    C->leaf_nseg = (int)seg_leaf.size();
    std::vector<int> order(seg_leaf.size());
    std::iota(order.begin(), order.end(), 0);
    auto seg_work = [&](int g) {
        const int lf = seg_leaf[g];
        return (int64_t)(C->h_leaf_r1[lf] - C->h_leaf_r0[lf]) * (seg_k[2 * g + 1] - seg_k[2 * g]);
    };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return seg_work(x) > seg_work(y); });
    C->d_seg_order = dupload(C, order);
    C->d_seg_leaf = dupload(C, seg_leaf);
    C->d_seg_k = dupload(C, seg_k);
    C->d_seg_poff = dupload(C, seg_poff);
    C->d_leaf_seg = dupload(C, leaf_seg);
    C->d_leaf_part = dalloc<double>(C, (size_t)std::max<int64_t>(poff, 1));
    C->leaf_mm_ready = true;
}

// Set-up autotuner: times the candidates on the context's own data and keeps
// the fastest.  Near field (one rhs): each round shape, 2 warm-up and 5 timed
// launches of the history sum (the values of the zero ring do not change the
// work).  Device solve (one rhs, gmres_blocks = 0): 16 Krylov iterations of
// an unreachable tolerance on b = 1 for each candidate block count, 3 timed
// solves each.
static float time_launches(hipStream_t s, int warm, int reps, const std::function<void()> &f) {
    hipEvent_t e0, e1;
    TD_HIP(hipEventCreate(&e0));
    TD_HIP(hipEventCreate(&e1));
    for (int i = 0; i < warm; ++i) f();
    TD_HIP(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i) f();
    TD_HIP(hipEventRecord(e1, s));
    TD_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    TD_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms / reps;
}

static void autotune(tdbem_ctx *C) {
    hipStream_t s = C->stream;
    if (C->nrhs == 1 && C->near_nnz > 0) {
        int best = 0;
        float tbest = 1e30f;
        for (int v = 0; v < near_variants(); ++v) {
            C->near_variant = v;
            const float t = time_launches(s, 2, 5, [&] { launch_near(C, C->ring, C->d_tmp, 1.0, s); });
            if (t < tbest) { tbest = t; best = v; }
        }
        C->near_variant = best;
    }
    if (C->nrhs > 1 && C->leaf_mm_ready) {
        // batched: the row kernel against the per-leaf matrix-core form
        C->near_variant = 0;
        const float t_row = time_launches(s, 1, 3, [&] { launch_near(C, C->ring, C->d_tmp, 1.0, s); });
        C->near_variant = near_variants();
        const float t_mm = time_launches(s, 1, 3, [&] { launch_near(C, C->ring, C->d_tmp, 1.0, s); });
        C->near_variant = t_mm < t_row ? near_variants() : 0;
    }
    if (C->nrhs == 1 && C->use_coop && C->cfg.gmres_blocks == 0) {
        const int cand[] = {0, 64, 96, 128, 160, 192, 256};
        int best = 0;
        float tbest = 1e30f;
        launch_fill(C->ne, 1.0, C->d_rhs, s);
        for (int nb : cand) {
            C->gmres_blocks = nb;
            bool launched = true;
            const float t = time_launches(s, 1, 3, [&] {
                launch_fill(C->ne, 0.0, C->d_x, s);
                launched = launched && gmres_coop_launch(C, C->d_rhs, C->d_x, 0.0, 16, s);
            });
            if (launched && t < tbest) { tbest = t; best = nb; }
        }
        C->gmres_blocks = best;
        TD_HIP(hipMemsetAsync(C->d_iflag, 0, 4 * (size_t)C->nrhs * sizeof(int), s));
    }
    C->tuned = true;
}

// weights of the MFIE's time derivative (kd) and of the MFIE (zeta) in the
// CFIE variants of Section 4.3.1
void cfie_weights(const tdbem_config &cfg, double &kd, double &zeta) {
    kd = cfg.cfie == TDBEM_CFIE3 ? 0.0 : 1.0;
    zeta = cfg.cfie == TDBEM_CFIE2 ? 0.0 : cfg.zeta;
}

static GeoDev geo(const tdbem_ctx *C) {
    double kd, zeta;
    cfie_weights(C->cfg, kd, zeta);
    return GeoDev{C->d_xyz, C->d_tri, C->d_area, C->d_nrm, C->d_qpt, C->d_etri, C->d_efree, C->d_elen,
                  C->cdt, C->cfg.dt, C->cfg.eps, C->cfg.mu, C->cfg.theta, zeta, C->eta, kd};
}

static uint64_t fingerprint(const tdbem_ctx *C);

// near pairs (leaf order), row-major; DIRECT mode: all pairs
static void build_near_pairs(tdbem_ctx *C, std::vector<int> &pi, std::vector<int> &pj) {
    const int ne = C->ne;
    pi.clear(); pj.clear();
    if (C->cfg.mode == TDBEM_MODE_DIRECT) {
        TD_REQUIRE((int64_t)ne * ne < (1ll << 31), TDBEM_EINVAL, "direct mode: too many edge pairs");
        pi.reserve((size_t)ne * ne); pj.reserve((size_t)ne * ne);
        for (int i = 0; i < ne; ++i)
            for (int j = 0; j < ne; ++j) { pi.push_back(i); pj.push_back(j); }
        return;
    }
    const Tree &T = C->T;
    // leaves partition the leaf-ordered edges into contiguous ranges; visiting
    // them by first edge emits rows in ascending order (the CSR builders need it)
    std::vector<std::pair<int, std::pair<int, int>>> leaves;
    for (int l = 0; l <= T.lmax; ++l)
        for (int c = 0; c < T.lev[l].n; ++c)
            if (T.lev[l].leaf[c]) leaves.push_back({T.lev[l].ebeg[c], {l, c}});
    std::sort(leaves.begin(), leaves.end());
    std::vector<std::pair<int, int>> cells;
    std::vector<int> src;
    for (auto &lf : leaves) {
        int l = lf.second.first, c = lf.second.second;
        const Level &L = T.lev[l];
        near_source_cells(T, l, c, cells);
        src.clear();
        for (auto &sc : cells) {
            const Level &S = T.lev[sc.first];
            for (int e = S.ebeg[sc.second]; e < S.eend[sc.second]; ++e) src.push_back(e);
        }
        std::sort(src.begin(), src.end());
        for (int i = L.ebeg[c]; i < L.eend[c]; ++i)
            for (int j : src) { pi.push_back(i); pj.push_back(j); }
    }
    for (size_t q = 1; q < pi.size(); ++q)
        TD_REQUIRE(pi[q] >= pi[q - 1], TDBEM_EINVAL, "internal: near pairs not sorted by row");
}

static void setup_impl(const tdbem_mesh *mesh, const tdbem_config *cfg, tdbem_ctx *C) {
    auto t0 = std::chrono::steady_clock::now();
    TD_REQUIRE(cfg, TDBEM_EINVAL, "null config");
    C->cfg = *cfg;
    TD_REQUIRE(cfg->d == 2, TDBEM_EINVAL, "only the quadratic B-spline (d = 2) is implemented");
    TD_REQUIRE(cfg->interp == TDBEM_INTERP_LAGRANGE || cfg->interp == TDBEM_INTERP_CHI_TIME, TDBEM_EINVAL,
               "unknown interpolant");
    TD_REQUIRE(cfg->dt > 0 && cfg->eps > 0 && cfg->mu > 0 && cfg->theta >= 0 && cfg->zeta >= 0, TDBEM_EINVAL,
               "dt, eps, mu must be positive; theta, zeta non-negative");
    TD_REQUIRE(cfg->n_rhs >= 1 && cfg->n_rhs <= 4096, TDBEM_EINVAL, "n_rhs out of range");
    TD_REQUIRE(cfg->mode == TDBEM_MODE_DIRECT || cfg->mode == TDBEM_MODE_IFMM, TDBEM_EINVAL, "unknown mode");
    TD_REQUIRE(cfg->precision >= TDBEM_FP64 && cfg->precision <= TDBEM_BF16, TDBEM_EINVAL, "unknown precision");
    TD_REQUIRE(cfg->cfie == TDBEM_CFIE1 || cfg->cfie == TDBEM_CFIE2 || cfg->cfie == TDBEM_CFIE3, TDBEM_EINVAL,
               "unknown CFIE variant (TDBEM_CFIE1, _CFIE2 or _CFIE3)");
    TD_REQUIRE(cfg->n_quad == 3, TDBEM_EINVAL, "only the interior 3-point triangle rule (n_quad = 3) is implemented");
    TD_REQUIRE(cfg->dt2 >= TDBEM_DT2_SPLIT && cfg->dt2 <= TDBEM_DT2_INTERP, TDBEM_EINVAL,
               "unknown placement of the second time derivative");
    TD_REQUIRE(cfg->box_widen == 0 || cfg->box_widen == 1, TDBEM_EINVAL, "box_widen must be 0 or 1");
    TD_REQUIRE(cfg->causal_guard == 0 || cfg->causal_guard == 1, TDBEM_EINVAL, "causal_guard must be 0 or 1");
    TD_REQUIRE(cfg->gmres_maxit >= 1, TDBEM_EINVAL, "gmres_maxit must be positive");
    TD_REQUIRE(cfg->gmres_restart >= 1 && cfg->gmres_restart <= 32, TDBEM_EINVAL, "gmres_restart must be in 1..32");
    TD_REQUIRE(cfg->gmres_rtol >= 0.0, TDBEM_EINVAL, "gmres_rtol must be non-negative");
    TD_REQUIRE(cfg->solver == TDBEM_SOLVER_DEVICE || cfg->solver == TDBEM_SOLVER_HOST, TDBEM_EINVAL, "unknown solver");
    TD_REQUIRE(cfg->gmres_blocks >= 0 && cfg->gmres_blocks <= 256, TDBEM_EINVAL, "gmres_blocks must be in 0..256");
    TD_REQUIRE(cfg->autotune == 0 || cfg->autotune == 1, TDBEM_EINVAL, "autotune must be 0 or 1");
    TD_REQUIRE(cfg->near_kernel >= 0 && cfg->near_kernel <= near_variants() + 1, TDBEM_EINVAL,
               "near_kernel must be 0 (default or tuned) or 1.." + std::to_string(near_variants() + 1));
    TD_REQUIRE(cfg->n_rhs == 1 ? cfg->near_kernel <= near_variants()
                               : (cfg->near_kernel <= 1 || cfg->near_kernel == near_variants() + 1),
               TDBEM_EINVAL,
               "near_kernel 1.." + std::to_string(near_variants()) + " are one-rhs forms; with several rhs 1 is "
                   "the row kernel and " + std::to_string(near_variants() + 1) + " the matrix-core form");
    TD_REQUIRE(cfg->near_kernel != near_variants() + 1 || cfg->precision != TDBEM_BF16, TDBEM_EINVAL,
               "the batched matrix-core near field is built for the FP64 and FP32 forms");
    TD_REQUIRE(cfg->near_kernel == 0 || cfg->autotune == 0, TDBEM_EINVAL, "near_kernel and autotune exclude each other");
    TD_REQUIRE(cfg->graph == 0 || cfg->graph == 1, TDBEM_EINVAL, "graph must be 0 or 1");
    TD_REQUIRE(cfg->graph == 0 || cfg->solver == TDBEM_SOLVER_DEVICE, TDBEM_EINVAL,
               "graph needs the device solver");
    TD_REQUIRE(cfg->growth_limit >= 0.0, TDBEM_EINVAL, "growth_limit must be non-negative");
    TD_REQUIRE(cfg->guess == TDBEM_GUESS_EXTRAP || cfg->guess == TDBEM_GUESS_LEARNED, TDBEM_EINVAL, "unknown guess");
    C->stream = (hipStream_t)cfg->stream;
    if (const char *dbg = std::getenv("TDBEM_TRACE")) C->trace = dbg[0] == '1';   // trace only
    C->use_coop = cfg->solver == TDBEM_SOLVER_DEVICE;
    C->gmres_blocks = cfg->gmres_blocks;
    C->nrhs = cfg->n_rhs;
    C->c = 1.0 / std::sqrt(cfg->eps * cfg->mu);
    C->eta = std::sqrt(cfg->mu / cfg->eps);
    C->cdt = C->c * cfg->dt;
    build_mesh(mesh, C->H);
    C->ne = C->H.ne;
    build_tree(C->H, cfg->mode == TDBEM_MODE_IFMM ? cfg->leaf_max : std::max(cfg->leaf_max, 1),
               std::max(2, cfg->min_level), C->T);
    const HostMesh &H = C->H;
    const Tree &T = C->T;
    const int ne = C->ne;
    // geometry on device, edges in leaf order
    std::vector<int> etri(2 * (size_t)ne), efree(2 * (size_t)ne);
    std::vector<double> elen(ne);
    for (int p = 0; p < ne; ++p) {
        int e = T.perm[p];
        etri[2 * p] = H.etri[2 * e]; etri[2 * p + 1] = H.etri[2 * e + 1];
        efree[2 * p] = H.efree[2 * e]; efree[2 * p + 1] = H.efree[2 * e + 1];
        elen[p] = H.elen[e];
    }
    C->d_xyz = dupload(C, H.xyz);
    C->d_tri = dupload(C, H.tri);
    C->d_area = dupload(C, H.area);
    C->d_nrm = dupload(C, H.nrm);
    C->d_qpt = dupload(C, H.qpt);
    C->d_etri = dupload(C, etri);
    C->d_efree = dupload(C, efree);
    C->d_elen = dupload(C, elen);
    C->d_perm = dupload(C, T.perm);
    hipStream_t s = C->stream;
    GeoDev G = geo(C);

    // ---- near pairs, exact lag ranges, coefficients
    std::vector<int> pi, pj;
    build_near_pairs(C, pi, pj);
    int64_t np = (int64_t)pi.size();
    if (C->trace) std::fprintf(stderr, "[tdbem] near pairs listed: %lld\n", (long long)np);
    int *d_pi = dalloc<int>(C, np), *d_pj = dalloc<int>(C, np);
    TD_HIP(hipMemcpy(d_pi, pi.data(), np * sizeof(int), hipMemcpyHostToDevice));
    TD_HIP(hipMemcpy(d_pj, pj.data(), np * sizeof(int), hipMemcpyHostToDevice));
    int *d_lo = dalloc<int>(C, np), *d_hi = dalloc<int>(C, np);
    launch_lag_range(G, np, d_pi, d_pj, d_lo, d_hi, s);
    std::vector<int> glo(np), ghi(np);
    TD_HIP(hipMemcpyAsync(glo.data(), d_lo, np * sizeof(int), hipMemcpyDeviceToHost, s));
    TD_HIP(hipMemcpyAsync(ghi.data(), d_hi, np * sizeof(int), hipMemcpyDeviceToHost, s));
    TD_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> off(np);
    int64_t nnz = 0;
    int maxlag = 2;
    for (int64_t p = 0; p < np; ++p) {
        off[p] = nnz;
        nnz += ghi[p] - glo[p] + 1;
        maxlag = std::max(maxlag, ghi[p]);
    }
    int64_t *d_off = dupload(C, off);
    double *d_val = dalloc<double>(C, nnz);
    if (C->trace) std::fprintf(stderr, "[tdbem] %lld pairs, %lld coefficients\n", (long long)np, (long long)nnz);
    {
        // in chunks, so that a trace shows progress on large problems
        constexpr int64_t ZCHUNK = (int64_t)1 << 28;
        for (int64_t c0 = 0; c0 < nnz; c0 += ZCHUNK) {
            launch_zfill(G, std::min(ZCHUNK, nnz - c0), c0, np, d_pi, d_pj, d_lo, d_off, d_val, s);
            if (C->trace && nnz > ZCHUNK) {
                TD_HIP(hipStreamSynchronize(s));
                std::fprintf(stderr, "[tdbem] coefficients %lld / %lld\n", (long long)std::min(nnz, c0 + ZCHUNK),
                             (long long)nnz);
            }
        }
    }
    // ---- Z0 = Zt^(1): pairs whose range starts at g = 1
    std::vector<int64_t> z0idx;
    std::vector<int> z0ptr(ne + 1, 0), z0col;
    for (int64_t p = 0; p < np; ++p)
        if (glo[p] == 1) { z0idx.push_back(off[p]); z0col.push_back(pj[p]); z0ptr[pi[p] + 1]++; }
    for (int i = 0; i < ne; ++i) z0ptr[i + 1] += z0ptr[i];
    C->z0_nnz = (int64_t)z0idx.size();
    int64_t *d_z0idx = dupload(C, z0idx);
    C->d_z0_val = dalloc<double>(C, C->z0_nnz);
    launch_gather_vals(d_val, d_z0idx, C->z0_nnz, C->d_z0_val, s);
    std::vector<double> z0v(C->z0_nnz);
    TD_HIP(hipMemcpyAsync(z0v.data(), C->d_z0_val, C->z0_nnz * sizeof(double), hipMemcpyDeviceToHost, s));
    TD_HIP(hipStreamSynchronize(s));
    std::vector<double> dinv(ne, 1.0);
    for (int i = 0; i < ne; ++i)
        for (int q = z0ptr[i]; q < z0ptr[i + 1]; ++q)
            if (z0col[q] == i) dinv[i] = z0v[q] != 0.0 ? 1.0 / z0v[q] : 1.0;
    C->d_z0_ptr = dupload(C, z0ptr);
    C->d_z0_col = dupload(C, z0col);
    C->d_z0_dinv = dupload(C, dinv);
    {
        std::vector<double> vald(C->z0_nnz);
        for (int64_t q = 0; q < C->z0_nnz; ++q) vald[q] = z0v[q] * dinv[z0col[q]];
        C->d_z0_vald = dupload(C, vald);
    }
    // ---- near store (g >= 2) in the jagged-diagonal layout
    std::vector<int> nrow(ne + 1, 0), nj, ngl;
    std::vector<int64_t> nsrc, vbase(ne, 0);
    nj.reserve(np); ngl.reserve(np); nsrc.reserve(np);
    int L = 0;
    int64_t nnz2 = 0;
    {
        std::vector<int64_t> order;
        int64_t p = 0;
        for (int i = 0; i < ne; ++i) {
            order.clear();
            int64_t pe = p;
            while (pe < np && pi[pe] == i) ++pe;
            for (int64_t q = p; q < pe; ++q)
                if (ghi[q] >= std::max(glo[q], 2)) order.push_back(q);
            auto len_of = [&](int64_t q) { return ghi[q] - std::max(glo[q], 2) + 1; };
            std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return len_of(a) > len_of(b); });
            vbase[i] = nnz2;
            for (int64_t q : order) {
                int g0 = std::max(glo[q], 2), len = len_of(q);
                TD_REQUIRE(g0 < 65536 && len < 32768, TDBEM_EINVAL, "lag range too long for the near-field store");
                nj.push_back(pj[q]);
                ngl.push_back(g0 | (len << 16));
                nsrc.push_back(off[q] + (g0 - glo[q]));
                nnz2 += len;
                L = std::max(L, len);
            }
            nrow[i + 1] = nrow[i] + (int)order.size();
            p = pe;
        }
    }
    if (C->trace) std::fprintf(stderr, "[tdbem] near-field store: %lld pairs, %lld values\n", (long long)nj.size(),
                               (long long)nnz2);
    TD_REQUIRE(L <= 512, TDBEM_EINVAL, "near-field lag strips longer than 512 steps");
    std::vector<int> nl((size_t)ne * std::max(L, 1), 0);
    for (int i = 0; i < ne; ++i)
        for (int q = nrow[i]; q < nrow[i + 1]; ++q) {
            int len = ngl[q] >> 16;
            for (int l = 0; l < len; ++l) nl[(size_t)i * L + l]++;
        }
    C->near_L = std::max(L, 1);
    build_near_leaves(C, nrow, nj, ngl);
    C->near_pairs = (int64_t)nj.size();
    C->near_nnz = nnz2;
    C->d_nrow_ptr = dupload(C, nrow);
    C->d_nrow_vbase = dupload(C, vbase);
    C->d_nl = dupload(C, nl);
    C->d_npair_j = dupload(C, nj);
    C->d_npair_gl = dupload(C, ngl);
    C->d_nval = dalloc<double>(C, nnz2);
    if (cfg->precision == TDBEM_FP32) C->d_nval32 = dalloc<float>(C, nnz2);
    if (cfg->precision == TDBEM_BF16) C->d_nval16 = dalloc<unsigned short>(C, nnz2);
    {
        int64_t *d_src = dupload(C, nsrc);
        launch_near_to_jds(C, d_src, d_val, s);
        if (C->nrhs > 1 && cfg->precision != TDBEM_BF16) build_leaf_mm(C, nrow, d_src, d_val);
        std::vector<int>().swap(C->h_colmap);     // set-up only
        std::vector<int>().swap(C->h_pcol);
        TD_HIP(hipStreamSynchronize(s));
        dfree(C, d_src, nsrc.size());
    }
    // the pair-major coefficients leave the device: a host copy serves
    // tdbem_near_rows; the other set-up arrays are released
    C->h_coef.resize(nnz);
    TD_HIP(hipMemcpy(C->h_coef.data(), d_val, nnz * sizeof(double), hipMemcpyDeviceToHost));
    dfree(C, d_val, nnz);
    dfree(C, d_z0idx, z0idx.size());
    dfree(C, d_off, off.size());
    dfree(C, d_pi, np);
    dfree(C, d_pj, np);
    dfree(C, d_lo, np);
    dfree(C, d_hi, np);
    C->max_lag = maxlag;
    // keep host copies of the pair structure for inspection
    C->hp_i.swap(pi); C->hp_j.swap(pj); C->hp_lo.swap(glo); C->hp_hi.swap(ghi); C->hp_off.swap(off);
    C->hp_nnz = nnz;
    // ---- far field
    if (cfg->mode == TDBEM_MODE_IFMM) ifmm_setup(C);
    guess_setup(C);
    // ---- march state
    int R = 8;
    int need = std::max(maxlag + 2, C->far_ring_need);
    while (R < need) R <<= 1;
    C->ring = R;
    const size_t nv = (size_t)ne * C->nrhs;
    C->d_Jring = dalloc<double>(C, (size_t)ne * R * C->nrhs);
    if (cfg->precision != TDBEM_FP64) C->d_Jring32 = dalloc<float>(C, (size_t)ne * R * C->nrhs);
    C->d_rhs = dalloc<double>(C, nv);
    C->d_x = dalloc<double>(C, nv);
    C->d_tmp = dalloc<double>(C, nv);
    C->d_work = dalloc<double>(C, std::max(gmres_work_doubles(C, cfg->gmres_restart),
                                           gmres_coop_work_doubles(ne, C->nrhs)));
    C->d_iflag = dalloc<int>(C, 4 * (size_t)C->nrhs);
    TD_HIP(hipMemset(C->d_iflag, 0, 4 * (size_t)C->nrhs * sizeof(int)));
    C->d_gbar = dalloc<unsigned>(C, (size_t)GMRES_BAR_WORDS * C->nrhs);
    TD_HIP(hipMemset(C->d_gbar, 0, (size_t)GMRES_BAR_WORDS * C->nrhs * sizeof(unsigned)));
    TD_HIP(hipHostMalloc((void **)&C->h_iflag, 4 * (size_t)C->nrhs * sizeof(int), hipHostMallocDefault));
    C->d_stat = dalloc<double>(C, 2 * (size_t)C->nrhs);
    TD_HIP(hipHostMalloc((void **)&C->h_stat, 2 * (size_t)C->nrhs * sizeof(double), hipHostMallocDefault));
    C->mon_vmax.assign(C->nrhs, 0.0);
    C->mon_jdrive.assign(C->nrhs, 0.0);
    C->mon_trip.assign(C->nrhs, 0);
    C->d_scal = dalloc<double>(C, 64 * (size_t)C->nrhs);
    C->d_pulse = dalloc<double>(C, 11 * (size_t)C->nrhs);
    TD_HIP(hipMemsetAsync(C->d_Jring, 0, (size_t)ne * R * C->nrhs * sizeof(double), s));
    if (C->d_Jring32) TD_HIP(hipMemsetAsync(C->d_Jring32, 0, (size_t)ne * R * C->nrhs * sizeof(float), s));
    TD_HIP(hipStreamSynchronize(s));
    // defaults: one rhs the per-leaf kernel where leaves are staged, several
    // the per-leaf matrix-core form where it was built; otherwise the row kernel
    if (cfg->near_kernel > 0)
        C->near_variant = cfg->near_kernel - 1;
    else if (C->nrhs == 1)
        C->near_variant = C->nleaf.nchunk > 0 ? NEAR_DEFAULT_LEAF : 0;
    else
        C->near_variant = C->leaf_mm_ready ? near_variants() : 0;
    TD_REQUIRE(C->near_variant != near_variants() || C->leaf_mm_ready, TDBEM_EINVAL,
               "the batched matrix-core near field could not be built (leaves or memory)");
    if (cfg->autotune) {
        autotune(C);
        TD_HIP(hipStreamSynchronize(s));
    }
    C->alpha = 1;
    C->fingerprint = fingerprint(C);
    noalloc_scratch(nullptr);       // the allocation-free step's workspace address on this device
    C->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

static void reset_impl(tdbem_ctx *C) {
    hipStream_t s = C->stream;
    std::fill(C->mon_vmax.begin(), C->mon_vmax.end(), 0.0);
    std::fill(C->mon_jdrive.begin(), C->mon_jdrive.end(), 0.0);
    std::fill(C->mon_trip.begin(), C->mon_trip.end(), 0);
    TD_HIP(hipMemsetAsync(C->d_Jring, 0, (size_t)C->ne * C->ring * C->nrhs * sizeof(double), s));
    if (C->d_Jring32) TD_HIP(hipMemsetAsync(C->d_Jring32, 0, (size_t)C->ne * C->ring * C->nrhs * sizeof(float), s));
    if (C->cfg.mode == TDBEM_MODE_IFMM) ifmm_reset(C);
    C->alpha = 1;
}

// Late-time stability monitor (Section 4.3 observes growth after the
// excitation for some variants): per right-hand side, once the tested incident
// field has fallen below 1e-6 of its largest norm so far, the current's norm
// must stay within growth_limit times its largest norm during the excitation.
static bool monitor_update(tdbem_ctx *C) {
    bool trip = false;
    for (int r = 0; r < C->nrhs; ++r) {
        const double v = std::sqrt(C->h_stat[2 * r]), j = std::sqrt(C->h_stat[2 * r + 1]);
        C->mon_vmax[r] = std::max(C->mon_vmax[r], v);
        const bool driven = C->mon_vmax[r] > 0.0 && v > 1e-6 * C->mon_vmax[r];
        if (driven) C->mon_jdrive[r] = std::max(C->mon_jdrive[r], j);
        else if (j > C->cfg.growth_limit * C->mon_jdrive[r] || !std::isfinite(j)) C->mon_trip[r] = 1;
        trip = trip || C->mon_trip[r];
    }
    return trip;
}

// Deferred step status (tdbem_march): the device solve's status words and the
// monitor's norms of step k are copied on the device into record slot k and
// read by the host once, after the last step.
struct MarchRec {
    int *flags = nullptr;       // [steps][n_rhs][4]
    double *stat = nullptr;     // [steps][n_rhs][2]
    int k = 0;
};

// the kernels of a step before the solve: tested field in, monitor norm,
// near-field history sum, right-hand side, far field, initial guess
static void step_pre(tdbem_ctx *C, const double *V, int a, bool monitor, hipStream_t s) {
    {
        PhaseScope ps(C->prof, TDBEM_PH_OTHER, s);
        launch_gather_in(C, V, C->d_rhs, s);
        if (monitor) launch_colnorm2(C, C->d_rhs, C->d_stat, 0, s);
    }
    { PhaseScope ps(C->prof, TDBEM_PH_NEAR, s); launch_near(C, a, C->d_tmp, 1.0, s); }
    {
        PhaseScope ps(C->prof, TDBEM_PH_OTHER, s);
        launch_rhs_finish(C, a, C->cfg.mode == TDBEM_MODE_IFMM ? ifmm_far_slot(C, a) : nullptr, s);
        if (guess_active(C)) launch_guess(C, a, s);
    }
}

// deferred record of a step's solver status (and monitor norms) on the device
static void step_rec(tdbem_ctx *C, const int *dflag, MarchRec *rec, bool monitor, hipStream_t s) {
    const size_t nf = 4 * (size_t)C->nrhs;
    if (monitor) {
        launch_colnorm2(C, C->d_x, C->d_stat, 1, s);
        launch_copy_words(C->d_stat, rec->stat + (size_t)rec->k * 2 * C->nrhs, 4 * (size_t)C->nrhs, s);
    }
    launch_copy_words(dflag, rec->flags + (size_t)rec->k * nf, nf, s);
}

// the kernels of a step after the solve: ring, far field, current out
static void step_post(tdbem_ctx *C, double *Jout, int a, hipStream_t s) {
    { PhaseScope ps(C->prof, TDBEM_PH_OTHER, s); launch_ring_out(C, (a - 1) & (C->ring - 1), Jout, s); }
    if (C->cfg.mode == TDBEM_MODE_IFMM) ifmm_after_solve(C, a, s);
}

static int step_impl(tdbem_ctx *C, const double *V, double *Jout, bool solve, const double *Jgiven,
                     bool noalloc = false, MarchRec *rec = nullptr) {
    hipStream_t s = C->stream;
    int a = C->alpha;
    int rc = TDBEM_OK;
    const bool monitor = solve && C->cfg.growth_limit > 0.0;
    if (solve) {
        step_pre(C, V, a, monitor, s);
        bool ok = true;
        {
            PhaseScope ps(C->prof, TDBEM_PH_GMRES, s);
            const int maxit = std::max(1, C->cfg.gmres_maxit);
            int *dflag = C->d_iflag;
            const bool launched = noalloc
                ? gmres_coop_launch_static(C, C->d_rhs, C->d_x, C->cfg.gmres_rtol, maxit, s, &dflag)
                : C->use_coop && gmres_coop_launch(C, C->d_rhs, C->d_x, C->cfg.gmres_rtol, maxit, s);
            TD_REQUIRE(launched || (!noalloc && !rec), TDBEM_EHIP, "the device cannot run the cooperative solve");
            if (launched && rec) {
                // deferred: keep this step's status on the device, no host wait
                step_rec(C, dflag, rec, monitor, s);
            } else if (launched) {
                const size_t nf = 4 * (size_t)C->nrhs;
                if (monitor) {
                    launch_colnorm2(C, C->d_x, C->d_stat, 1, s);
                    TD_HIP(hipMemcpyAsync(C->h_stat, C->d_stat, 2 * C->nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
                }
                TD_HIP(hipMemcpyAsync(C->h_iflag, dflag, nf * sizeof(int), hipMemcpyDeviceToHost, s));
                TD_HIP(hipStreamSynchronize(s));
                int its = 0;
                bool timeout = false;
                for (int r = 0; r < C->nrhs; ++r) {
                    its = std::max(its, C->h_iflag[4 * r]);
                    ok = ok && C->h_iflag[4 * r + 1] != 0;
                    timeout = timeout || C->h_iflag[4 * r + 2] != 0;
                }
                C->last_iters = its;
                if (timeout) {
                    if (!noalloc) TD_HIP(hipMemset(C->d_gbar, 0, (size_t)GMRES_BAR_WORDS * C->nrhs * sizeof(unsigned)));
                    throw Error{TDBEM_EHIP, "device solve: a grid barrier wait timed out"};
                }
            } else {
                C->last_iters = gmres_solve(C, C->d_rhs, C->d_x, C->cfg.gmres_rtol, maxit, &ok, s);
                if (monitor) {
                    launch_colnorm2(C, C->d_x, C->d_stat, 1, s);
                    TD_HIP(hipMemcpyAsync(C->h_stat, C->d_stat, 2 * C->nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
                    TD_HIP(hipStreamSynchronize(s));
                }
            }
        }
        if (!ok) rc = TDBEM_ENOCONV;
        if (monitor && !(rec && C->use_coop) && monitor_update(C)) rc = TDBEM_EUNSTABLE;
    } else {
        launch_gather_in(C, Jgiven, C->d_x, s);
    }
    step_post(C, Jout, a, s);
    C->alpha = a + 1;
    return rc;
}

// Capture fn's launches on the context's capture-only stream into a graph,
// refresh the executable graph ex with it (its arguments; a new executable
// when the launches differ), and launch ex on the context's stream.
static void run_graph(tdbem_ctx *C, hipGraphExec_t &ex, const std::function<void(hipStream_t)> &fn) {
    hipStream_t cs = C->cap_stream;
    TD_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipGraph_t g = nullptr;
    try {
        fn(cs);
    } catch (...) {
        if (hipStreamEndCapture(cs, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
        throw;
    }
    TD_HIP(hipStreamEndCapture(cs, &g));
    struct GFree { hipGraph_t g; ~GFree() { if (g) (void)hipGraphDestroy(g); } } gfree{g};
    if (ex) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult r = hipGraphExecUpdateError;
        if (hipGraphExecUpdate(ex, g, &bad, &r) == hipSuccess && r == hipGraphExecUpdateSuccess) {
            ++C->graph_updates;
        } else {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(ex);
            ex = nullptr;
        }
    }
    if (!ex) {
        TD_HIP(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
        ++C->graph_builds;
    }
    TD_HIP(hipGraphLaunch(ex, C->stream));
}

// one step of tdbem_march from graphs: the kernels before the solve, the
// cooperative solve (a plain launch), the status record and the kernels
// after it (one executable per pattern of far-field levels at their gate)
static void step_graph(tdbem_ctx *C, const double *V, double *Jout, MarchRec *rec) {
    const int a = C->alpha;
    const bool monitor = C->cfg.growth_limit > 0.0;
    if (!C->cap_stream) TD_HIP(hipStreamCreateWithFlags(&C->cap_stream, hipStreamNonBlocking));
    run_graph(C, C->g_pre, [&](hipStream_t cs) { step_pre(C, V, a, monitor, cs); });
    const bool launched = gmres_coop_launch(C, C->d_rhs, C->d_x, C->cfg.gmres_rtol, std::max(1, C->cfg.gmres_maxit),
                                            C->stream);
    TD_REQUIRE(launched, TDBEM_EHIP, "the device cannot run the cooperative solve");
    const uint32_t key = C->cfg.mode == TDBEM_MODE_IFMM ? ifmm_gate_mask(C, a) : 0u;
    run_graph(C, C->g_post[key], [&](hipStream_t cs) {
        step_rec(C, C->d_iflag, rec, monitor, cs);
        step_post(C, Jout, a, cs);
    });
    C->alpha = a + 1;
}

void launch_count_d0(const GeoDev &G, int ne, unsigned long long *count, hipStream_t s);

int64_t count_d0_nnz(const tdbem_ctx *C) {
    unsigned long long *d = nullptr, h = 0;
    TD_HIP(hipMalloc(&d, sizeof(unsigned long long)));
    struct Free { void *p; ~Free() { (void)hipFree(p); } } guard{d};
    TD_HIP(hipMemsetAsync(d, 0, sizeof(unsigned long long), C->stream));
    launch_count_d0(geo(C), C->ne, d, C->stream);
    TD_HIP(hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, C->stream));
    TD_HIP(hipStreamSynchronize(C->stream));
    return (int64_t)h;
}

// FNV-1a over the mesh and every configuration field that shapes the state
static uint64_t fnv(uint64_t h, const void *p, size_t n) {
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
    return h;
}
static uint64_t fingerprint(const tdbem_ctx *C) {
    uint64_t h = 14695981039346656037ull;
    h = fnv(h, C->H.xyz.data(), C->H.xyz.size() * sizeof(double));
    h = fnv(h, C->H.tri.data(), C->H.tri.size() * sizeof(int));
    const tdbem_config &c = C->cfg;
    const double dv[] = {c.dt, c.eps, c.mu, c.theta, c.zeta, c.gmres_rtol, c.growth_limit};
    const int32_t iv[] = {c.nt, c.d, c.cfie, c.n_quad, c.p_s, c.p_t, c.interp, c.dt2, c.m2l, c.leaf_max, c.min_level,
                          c.mu_window, c.box_widen, c.causal_guard, c.mode, c.precision, c.n_rhs, c.gmres_maxit,
                          c.gmres_restart, c.guess, c.solver, c.gmres_blocks, c.autotune, c.near_kernel};
    h = fnv(h, dv, sizeof(dv));
    return fnv(h, iv, sizeof(iv));
}

// checkpoint layout: header, per-rhs monitor state, current ring, FP32 ring
// copy (reduced forms), far-field state
struct CkptHeader {
    char magic[8];
    uint64_t fingerprint;
    int64_t ne, nrhs, ring, far_bytes;
    int32_t alpha, last_iters;
};
static size_t ring_bytes(const tdbem_ctx *C) { return (size_t)C->ne * C->ring * C->nrhs * sizeof(double); }
static size_t ring32_bytes(const tdbem_ctx *C) {
    return C->d_Jring32 ? (size_t)C->ne * C->ring * C->nrhs * sizeof(float) : 0;
}
static size_t far_bytes(const tdbem_ctx *C) { return C->far ? ifmm_state_bytes(C) : 0; }
static size_t ckpt_bytes(const tdbem_ctx *C) {
    return sizeof(CkptHeader) + (size_t)C->nrhs * (2 * sizeof(double) + sizeof(int32_t)) + ring_bytes(C) +
           ring32_bytes(C) + far_bytes(C);
}

static void checkpoint_impl(tdbem_ctx *C, char *buf) {
    CkptHeader hd;
    std::memcpy(hd.magic, "TDBEMCK1", 8);
    hd.fingerprint = C->fingerprint;
    hd.ne = C->ne; hd.nrhs = C->nrhs; hd.ring = C->ring; hd.far_bytes = (int64_t)far_bytes(C);
    hd.alpha = C->alpha; hd.last_iters = C->last_iters;
    char *p = buf;
    std::memcpy(p, &hd, sizeof(hd)); p += sizeof(hd);
    std::memcpy(p, C->mon_vmax.data(), C->nrhs * sizeof(double)); p += C->nrhs * sizeof(double);
    std::memcpy(p, C->mon_jdrive.data(), C->nrhs * sizeof(double)); p += C->nrhs * sizeof(double);
    for (int r = 0; r < C->nrhs; ++r) { int32_t t = C->mon_trip[r]; std::memcpy(p, &t, 4); p += 4; }
    hipStream_t s = C->stream;
    TD_HIP(hipMemcpyAsync(p, C->d_Jring, ring_bytes(C), hipMemcpyDeviceToHost, s)); p += ring_bytes(C);
    if (C->d_Jring32) { TD_HIP(hipMemcpyAsync(p, C->d_Jring32, ring32_bytes(C), hipMemcpyDeviceToHost, s)); p += ring32_bytes(C); }
    if (C->far) ifmm_state_copy(C, p, true, s);
    TD_HIP(hipStreamSynchronize(s));
}

static void restore_impl(tdbem_ctx *C, const char *buf, size_t len) {
    TD_REQUIRE(len >= sizeof(CkptHeader), TDBEM_EINVAL, "checkpoint too short");
    CkptHeader hd;
    std::memcpy(&hd, buf, sizeof(hd));
    TD_REQUIRE(std::memcmp(hd.magic, "TDBEMCK1", 8) == 0, TDBEM_EINVAL, "not a checkpoint of this library");
    TD_REQUIRE(hd.fingerprint == C->fingerprint && hd.ne == C->ne && hd.nrhs == C->nrhs && hd.ring == C->ring &&
                   hd.far_bytes == (int64_t)far_bytes(C),
               TDBEM_EINVAL, "checkpoint of another mesh or configuration");
    TD_REQUIRE(len == ckpt_bytes(C), TDBEM_EINVAL, "checkpoint size does not match the context");
    TD_REQUIRE(hd.alpha >= 1, TDBEM_EINVAL, "malformed checkpoint");
    const char *p = buf + sizeof(hd);
    std::memcpy(C->mon_vmax.data(), p, C->nrhs * sizeof(double)); p += C->nrhs * sizeof(double);
    std::memcpy(C->mon_jdrive.data(), p, C->nrhs * sizeof(double)); p += C->nrhs * sizeof(double);
    for (int r = 0; r < C->nrhs; ++r) { int32_t t; std::memcpy(&t, p, 4); C->mon_trip[r] = t; p += 4; }
    hipStream_t s = C->stream;
    TD_HIP(hipMemcpyAsync(C->d_Jring, p, ring_bytes(C), hipMemcpyHostToDevice, s)); p += ring_bytes(C);
    if (C->d_Jring32) { TD_HIP(hipMemcpyAsync(C->d_Jring32, p, ring32_bytes(C), hipMemcpyHostToDevice, s)); p += ring32_bytes(C); }
    if (C->far) ifmm_state_copy(C, const_cast<char *>(p), false, s);
    TD_HIP(hipStreamSynchronize(s));
    C->alpha = hd.alpha;
    C->last_iters = hd.last_iters;
}

}  // namespace tdbem

using namespace tdbem;

#define TD_GUARD(body)                                                  \
    try {                                                               \
        body;                                                           \
    } catch (const tdbem::Error &e) {                                   \
        set_error(e.msg);                                               \
        return e.code;                                                  \
    } catch (const std::bad_alloc &) {                                  \
        set_error("host allocation failed");                            \
        return TDBEM_ENOMEM;                                            \
    } catch (const std::exception &e) {                                 \
        set_error(e.what());                                            \
        return TDBEM_EINVAL;                                            \
    }

extern "C" {

int tdbem_setup(const tdbem_mesh *mesh, const tdbem_config *cfg, tdbem_ctx **out) {
    if (!out) { set_error("null output pointer"); return TDBEM_EINVAL; }
    *out = nullptr;
    tdbem_ctx *C = new (std::nothrow) tdbem_ctx();
    if (!C) { set_error("host allocation failed"); return TDBEM_ENOMEM; }
    try {
        setup_impl(mesh, cfg, C);
    } catch (const tdbem::Error &e) {
        set_error(e.msg);
        tdbem_destroy(C);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        tdbem_destroy(C);
        return TDBEM_ENOMEM;
    } catch (const std::exception &e) {
        set_error(std::string("setup failed: ") + e.what());
        tdbem_destroy(C);
        return TDBEM_EINVAL;
    }
    *out = C;
    return TDBEM_OK;
}

int tdbem_incident_planewave(tdbem_ctx *C, const double *pulses, int32_t step, double *V_dev) {
    if (!C || !pulses || !V_dev) { set_error("null argument"); return TDBEM_EINVAL; }
    TD_GUARD({
        TD_HIP(hipMemcpyAsync(C->d_pulse, pulses, sizeof(double) * 11 * C->nrhs, hipMemcpyHostToDevice, C->stream));
        launch_vinc(geo(C), C->ne, C->nrhs, C->d_pulse, C->d_perm, step * C->cfg.dt, V_dev, C->stream);
        TD_HIP(hipStreamSynchronize(C->stream));
    });
    return TDBEM_OK;
}

int tdbem_potentials(tdbem_ctx *C, const double *hist, int32_t n_hist, double *out) {
    if (!C || !out || (n_hist > 0 && !hist) || n_hist < 0) { set_error("bad argument"); return TDBEM_EINVAL; }
    TD_GUARD({
        reset_impl(C);
        const size_t nv = (size_t)C->ne * C->nrhs;
        for (int b = 0; b < n_hist; ++b) step_impl(C, nullptr, nullptr, false, hist + (size_t)b * nv);
        // history part of the right-hand side of step alpha = n_hist + 1
        launch_near(C, C->alpha, C->d_tmp, 1.0, C->stream);
        if (C->cfg.mode == TDBEM_MODE_IFMM) ifmm_add_far(C, C->alpha, C->d_tmp, C->stream);
        launch_scatter_out(C, C->d_tmp, out, C->stream);
        TD_HIP(hipStreamSynchronize(C->stream));
    });
    return TDBEM_OK;
}

int tdbem_step(tdbem_ctx *C, const double *V, double *J) {
    if (!C || !V || !J) { set_error("null argument"); return TDBEM_EINVAL; }
    int rc = TDBEM_OK;
    TD_GUARD({ rc = step_impl(C, V, J, true, nullptr); });
    if (rc == TDBEM_ENOCONV) set_error("GMRES did not reach the tolerance");
    if (rc == TDBEM_EUNSTABLE) set_error("late-time growth: the current exceeds growth_limit times its norm during the excitation");
    return rc;
}

int tdbem_checkpoint(const tdbem_ctx *Cc, void *buf, size_t *len) {
    if (!Cc || !len) { set_error("null argument"); return TDBEM_EINVAL; }
    tdbem_ctx *C = const_cast<tdbem_ctx *>(Cc);
    TD_GUARD({
        const size_t need = ckpt_bytes(C);
        if (!buf) { *len = need; return TDBEM_OK; }
        TD_REQUIRE(*len >= need, TDBEM_EINVAL, "checkpoint buffer too small");
        checkpoint_impl(C, (char *)buf);
        *len = need;
    });
    return TDBEM_OK;
}

int tdbem_restore(tdbem_ctx *C, const void *buf, size_t len) {
    if (!C || !buf) { set_error("null argument"); return TDBEM_EINVAL; }
    TD_GUARD({ restore_impl(C, (const char *)buf, len); });
    return TDBEM_OK;
}

int tdbem_step_noalloc(tdbem_ctx *C, const double *V, double *J) {
    if (!C || !V || !J) { set_error("null argument"); return TDBEM_EINVAL; }
    if (!C->use_coop) { set_error("the allocation-free step needs the device solver"); return TDBEM_EINVAL; }
    int rc = TDBEM_OK;
    TD_GUARD({
        size_t cap = 0;
        noalloc_scratch(&cap);
        const size_t need = noalloc_need(C);
        TD_REQUIRE(need <= cap, TDBEM_EINVAL,
                   "the allocation-free step needs " + std::to_string(need * 8) + " bytes of workspace; the static "
                   "array holds " + std::to_string(cap * 8) + " (N_e x n_rhs too large)");
        rc = step_impl(C, V, J, true, nullptr, true);
    });
    if (rc == TDBEM_ENOCONV) set_error("GMRES did not reach the tolerance");
    if (rc == TDBEM_EUNSTABLE) set_error("late-time growth: the current exceeds growth_limit times its norm during the excitation");
    return rc;
}

static int march_impl(tdbem_ctx *C, const double *V, double *J, int32_t n_steps, int32_t *status,
                      int32_t *iters) {
    int first = TDBEM_OK;
    const size_t nv = (size_t)C->ne * C->nrhs, nr = C->nrhs;
    if (!C->use_coop) {
        // the host-driven solver waits on the host anyway: one step at a time
        for (int k = 0; k < n_steps; ++k) {
            const int rc = step_impl(C, V + k * nv, J + k * nv, true, nullptr);
            if (status) status[k] = rc;
            if (iters) iters[k] = C->last_iters;
            if (first == TDBEM_OK) first = rc;
        }
    } else {
        if ((size_t)n_steps > C->march_cap) {
            if (C->d_march) TD_HIP(hipFree(C->d_march));
            C->d_march = nullptr;
            C->march_cap = 0;
            TD_HIP(hipMalloc(&C->d_march, (size_t)n_steps * nr * (4 * sizeof(int) + 2 * sizeof(double))));
            C->march_cap = (size_t)n_steps;
        }
        MarchRec rec;
        rec.stat = (double *)C->d_march;
        rec.flags = (int *)(rec.stat + (size_t)n_steps * 2 * nr);
        const bool graphs = C->cfg.graph && !C->prof.on;
        for (int k = 0; k < n_steps; ++k) {
            rec.k = k;
            if (graphs)
                step_graph(C, V + k * nv, J + k * nv, &rec);
            else
                step_impl(C, V + k * nv, J + k * nv, true, nullptr, false, &rec);
        }
        std::vector<int> fl((size_t)n_steps * 4 * nr);
        std::vector<double> st((size_t)n_steps * 2 * nr);
        if (n_steps > 0) {
            TD_HIP(hipMemcpyAsync(fl.data(), rec.flags, fl.size() * sizeof(int), hipMemcpyDeviceToHost, C->stream));
            if (C->cfg.growth_limit > 0.0)
                TD_HIP(hipMemcpyAsync(st.data(), rec.stat, st.size() * sizeof(double), hipMemcpyDeviceToHost,
                                      C->stream));
        }
        TD_HIP(hipStreamSynchronize(C->stream));
        bool timeout = false;
        for (int k = 0; k < n_steps; ++k) {
            bool ok = true;
            int its = 0;
            for (size_t r = 0; r < nr; ++r) {
                const int *f = &fl[((size_t)k * nr + r) * 4];
                its = std::max(its, f[0]);
                ok = ok && f[1] != 0;
                timeout = timeout || f[2] != 0;
            }
            C->last_iters = its;
            if (iters) iters[k] = its;
            int rc = ok ? TDBEM_OK : TDBEM_ENOCONV;
            if (C->cfg.growth_limit > 0.0) {
                std::copy(st.begin() + (size_t)k * 2 * nr, st.begin() + (size_t)(k + 1) * 2 * nr, C->h_stat);
                if (monitor_update(C)) rc = TDBEM_EUNSTABLE;
            }
            if (status) status[k] = rc;
            if (first == TDBEM_OK) first = rc;
        }
        if (timeout) {
            TD_HIP(hipMemset(C->d_gbar, 0, (size_t)GMRES_BAR_WORDS * C->nrhs * sizeof(unsigned)));
            throw Error{TDBEM_EHIP, "device solve: a grid barrier wait timed out"};
        }
    }
    return first;
}

int tdbem_march(tdbem_ctx *C, const double *V, double *J, int32_t n_steps, int32_t *status, int32_t *iters) {
    if (!C || !V || !J) { set_error("null argument"); return TDBEM_EINVAL; }
    if (n_steps < 0) { set_error("n_steps < 0"); return TDBEM_EINVAL; }
    int first = TDBEM_OK;
    TD_GUARD({ first = march_impl(C, V, J, n_steps, status, iters); });
    if (first == TDBEM_ENOCONV) set_error("GMRES did not reach the tolerance in at least one step");
    if (first == TDBEM_EUNSTABLE) set_error("late-time growth: the current exceeds growth_limit times its norm during the excitation");
    return first;
}

int tdbem_reset(tdbem_ctx *C) {
    if (!C) { set_error("null context"); return TDBEM_EINVAL; }
    TD_GUARD({ reset_impl(C); TD_HIP(hipStreamSynchronize(C->stream)); });
    return TDBEM_OK;
}

int tdbem_query(const tdbem_ctx *C, int32_t key, void *out) {
    if (!C || !out) { set_error("null argument"); return TDBEM_EINVAL; }
    const Tree &T = C->T;
    switch (key) {
        case TDBEM_Q_NE: *(int64_t *)out = C->ne; break;
        case TDBEM_Q_EDGES: std::memcpy(out, C->H.edge_v.data(), sizeof(int) * 2 * (size_t)C->ne); break;
        case TDBEM_Q_LMAX: *(int32_t *)out = T.lmax; break;
        case TDBEM_Q_MT:
            for (int l = 0; l <= T.lmax; ++l) ((int32_t *)out)[l] = l < (int)C->Mt.size() ? C->Mt[l] : 0;
            break;
        case TDBEM_Q_NEAR_NNZ: *(int64_t *)out = C->near_nnz; break;
        case TDBEM_Q_NEAR_PAIRS: *(int64_t *)out = C->near_pairs; break;
        case TDBEM_Q_Z0_NNZ: *(int64_t *)out = C->z0_nnz; break;
        case TDBEM_Q_NCELLS: for (int l = 0; l <= T.lmax; ++l) ((int32_t *)out)[l] = T.lev[l].n; break;
        case TDBEM_Q_NILIST: for (int l = 0; l <= T.lmax; ++l) ((int64_t *)out)[l] = (int64_t)T.lev[l].il_src.size(); break;
        case TDBEM_Q_WINDOW: *(int32_t *)out = C->window; break;
        case TDBEM_Q_GMRES_ITERS: *(int32_t *)out = C->last_iters; break;
        case TDBEM_Q_DEVICE_BYTES: *(int64_t *)out = (int64_t)C->dev_bytes; break;
        case TDBEM_Q_STEP: *(int32_t *)out = C->alpha; break;
        case TDBEM_Q_EDGE_LEAF: std::memcpy(out, T.iperm.data(), sizeof(int) * (size_t)C->ne); break;
        case TDBEM_Q_SETUP_MS: *(double *)out = C->setup_ms; break;
        case TDBEM_Q_CONFIG: std::memcpy(out, &C->cfg, sizeof(tdbem_config)); break;
        case TDBEM_Q_WINDOWS:
            for (int l = 0; l <= T.lmax; ++l) ((int32_t *)out)[l] = l < (int)C->windows.size() ? C->windows[l] : 0;
            break;
        case TDBEM_Q_TUNED: {
            int nu = 0, nc = 0;
            near_variant_shape(C->near_variant, &nu, &nc);
            int32_t *o = (int32_t *)out;
            o[0] = nu; o[1] = nc; o[2] = C->gmres_blocks; o[3] = C->tuned ? 1 : 0;
            break;
        }
        case TDBEM_Q_NEAR_LEAF_BYTES: *(int64_t *)out = C->leaf_mm_bytes; break;
        case TDBEM_Q_GRAPHS: ((int64_t *)out)[0] = C->graph_builds; ((int64_t *)out)[1] = C->graph_updates; break;
        case TDBEM_Q_UNSTABLE:
            for (int r = 0; r < C->nrhs; ++r) ((int32_t *)out)[r] = C->mon_trip[r];
            break;
        case TDBEM_Q_D0_NNZ:
            try {
                if (C->d0_nnz < 0) const_cast<tdbem_ctx *>(C)->d0_nnz = count_d0_nnz(C);
                *(int64_t *)out = C->d0_nnz;
            } catch (const Error &e) {
                set_error(e.msg);
                return e.code;
            }
            break;
        case TDBEM_Q_GUESS_USED:
            try {
                *(int64_t *)out = guess_used(const_cast<tdbem_ctx *>(C));
            } catch (const Error &e) {
                set_error(e.msg);
                return e.code;
            }
            break;
        case TDBEM_Q_PHASE_MS:
        case TDBEM_Q_PHASE_COUNT:
            try {
                const_cast<tdbem_ctx *>(C)->prof.fold(C->stream);
            } catch (const Error &e) {
                set_error(e.msg);
                return e.code;
            }
            if (key == TDBEM_Q_PHASE_MS) std::memcpy(out, C->prof.ms, sizeof(C->prof.ms));
            else std::memcpy(out, C->prof.count, sizeof(C->prof.count));
            break;
        default: set_error("unknown query key"); return TDBEM_EINVAL;
    }
    return TDBEM_OK;
}

int tdbem_near_rows(tdbem_ctx *C, const int32_t *rows, int32_t n, int32_t G, double *out) {
    if (!C || !rows || !out || n < 0 || G < 1) { set_error("bad argument"); return TDBEM_EINVAL; }
    TD_GUARD({
        const int ne = C->ne;
        std::memset(out, 0, sizeof(double) * (size_t)n * ne * G);
        const std::vector<double> &val = C->h_coef;
        // row ranges in the (sorted by i) pair list
        for (int r = 0; r < n; ++r) {
            TD_REQUIRE(rows[r] >= 0 && rows[r] < ne, TDBEM_EINVAL, "row out of range");
            int i = C->T.iperm[rows[r]];
            auto lo = std::lower_bound(C->hp_i.begin(), C->hp_i.end(), i);
            auto hi = std::upper_bound(C->hp_i.begin(), C->hp_i.end(), i);
            for (auto it = lo; it != hi; ++it) {
                size_t p = it - C->hp_i.begin();
                int j = C->T.perm[C->hp_j[p]];
                for (int g = C->hp_lo[p]; g <= C->hp_hi[p]; ++g)
                    if (g < G) out[((size_t)r * ne + j) * G + g] = val[C->hp_off[p] + (g - C->hp_lo[p])];
            }
        }
    });
    return TDBEM_OK;
}

int tdbem_profile(tdbem_ctx *C, int32_t enable) {
    if (!C) { set_error("null context"); return TDBEM_EINVAL; }
    TD_GUARD({
        C->prof.fold(C->stream);
        C->prof.clear();
        C->prof.on = enable != 0;
    });
    return TDBEM_OK;
}

int tdbem_guess_weights(tdbem_ctx *C, const float *params, int64_t n) {
    if (!C || !params) { set_error("null argument"); return TDBEM_EINVAL; }
    TD_GUARD({ guess_load(C, params, n); });
    return TDBEM_OK;
}

int tdbem_guess_capture(tdbem_ctx *C, float *feat, double *aux) {
    if (!C) { set_error("null argument"); return TDBEM_EINVAL; }
    TD_GUARD({ guess_capture(C, feat, aux); });
    return TDBEM_OK;
}

int tdbem_guess_grad(const float *P, const float *X, const float *Y, int64_t n, float *G, float *loss, void *stream) {
    TD_GUARD({ guess_grad(P, X, Y, n, G, loss, (hipStream_t)stream); });
    return TDBEM_OK;
}

int tdbem_guess_adam(float *P, const float *G, float *M, float *V, int32_t t, float lr, float b1, float b2, float eps,
                     void *stream) {
    TD_GUARD({ guess_adam(P, G, M, V, t, lr, b1, b2, eps, (hipStream_t)stream); });
    return TDBEM_OK;
}

void tdbem_destroy(tdbem_ctx *C) {
    if (!C) return;
    if (C->g_pre) (void)hipGraphExecDestroy(C->g_pre);
    for (auto &kv : C->g_post)
        if (kv.second) (void)hipGraphExecDestroy(kv.second);
    if (C->cap_stream) (void)hipStreamDestroy(C->cap_stream);
    ifmm_destroy(C);
    guess_destroy(C);
    for (void *p : C->allocs) (void)hipFree(p);
    if (C->d_march) (void)hipFree(C->d_march);
    if (C->h_scal) (void)hipHostFree(C->h_scal);
    if (C->h_iflag) (void)hipHostFree(C->h_iflag);
    if (C->h_stat) (void)hipHostFree(C->h_stat);
    delete C;
}

const char *tdbem_last_error(void) { return g_err.c_str(); }

}  // extern "C"
