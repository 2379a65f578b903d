// extern "C" entry points and the marching driver (Program 1).
#include <algorithm>
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
void launch_zfill(const GeoDev &G, int64_t nnz, int64_t npairs, const int *pi, const int *pj, const int *g0,
                  const int64_t *off, double *val, hipStream_t s);
void launch_vinc(const GeoDev &G, int ne, int nrhs, const double *pulses, const int *perm, double t, double *V, hipStream_t s);
void launch_near(const tdbem_ctx *C, int alpha, double *out, double scale, hipStream_t s);
void launch_gather_in(const tdbem_ctx *C, const double *src, double *dst, hipStream_t s);
void launch_scatter_out(const tdbem_ctx *C, const double *src, double *dst, hipStream_t s);
void launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s);
void launch_ring_put(const tdbem_ctx *C, int slot, const double *x, hipStream_t s);
void launch_extrap(const tdbem_ctx *C, int alpha, double *x, hipStream_t s);
void launch_to_f32(const double *src, float *dst, int64_t n, hipStream_t s);
void launch_near_to_jds(const tdbem_ctx *C, const int64_t *src_off, const double *src, hipStream_t s);
void launch_gather_vals(const double *val, const int64_t *idx, int64_t n, double *out, hipStream_t s);
int gmres_solve(tdbem_ctx *C, const double *b, double *x, double rtol, int maxit, bool *ok, hipStream_t s);
size_t gmres_work_doubles(const tdbem_ctx *C, int maxit);
bool gmres_coop_launch(tdbem_ctx *C, const double *b, double *x, double rtol, int maxit, hipStream_t s);
size_t gmres_coop_work_doubles(int ne, int nrhs);

static GeoDev geo(const tdbem_ctx *C) {
    return GeoDev{C->d_xyz, C->d_tri, C->d_area, C->d_nrm, C->d_qpt, C->d_etri, C->d_efree, C->d_elen,
                  C->cdt, C->cfg.dt, C->cfg.eps, C->cfg.mu, C->cfg.theta, C->cfg.zeta, C->eta};
}

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
    C->stream = (hipStream_t)cfg->stream;
    if (const char *dbg = std::getenv("TDBEM_DEBUG_GMRES")) C->debug_gmres = dbg[0] == '1';
    if (const char *hs = std::getenv("TDBEM_HOST_GMRES")) C->use_coop = hs[0] != '1';
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
    launch_zfill(G, nnz, np, d_pi, d_pj, d_lo, d_off, d_val, s);
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
    TD_REQUIRE(L <= 512, TDBEM_EINVAL, "near-field lag strips longer than 512 steps");
    std::vector<int> nl((size_t)ne * std::max(L, 1), 0);
    for (int i = 0; i < ne; ++i)
        for (int q = nrow[i]; q < nrow[i + 1]; ++q) {
            int len = ngl[q] >> 16;
            for (int l = 0; l < len; ++l) nl[(size_t)i * L + l]++;
        }
    C->near_L = std::max(L, 1);
    C->near_pairs = (int64_t)nj.size();
    C->near_nnz = nnz2;
    C->d_nrow_ptr = dupload(C, nrow);
    C->d_nrow_vbase = dupload(C, vbase);
    C->d_nl = dupload(C, nl);
    C->d_npair_j = dupload(C, nj);
    C->d_npair_gl = dupload(C, ngl);
    C->d_coef = d_val;
    C->d_nval = dalloc<double>(C, nnz2);
    if (cfg->precision == TDBEM_FP32) C->d_nval32 = dalloc<float>(C, nnz2);
    if (cfg->precision == TDBEM_BF16) C->d_nval16 = dalloc<unsigned short>(C, nnz2);
    {
        int64_t *d_src = dupload(C, nsrc);
        launch_near_to_jds(C, d_src, d_val, s);
        TD_HIP(hipStreamSynchronize(s));
    }
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
    C->d_work = dalloc<double>(C, std::max(gmres_work_doubles(C, std::max(1, cfg->gmres_maxit)),
                                           gmres_coop_work_doubles(ne, C->nrhs)));
    C->d_iflag = dalloc<int>(C, 4 * (size_t)C->nrhs);
    TD_HIP(hipMemset(C->d_iflag, 0, 4 * (size_t)C->nrhs * sizeof(int)));
    C->d_gbar = dalloc<unsigned>(C, (size_t)GMRES_BAR_WORDS * C->nrhs);
    TD_HIP(hipMemset(C->d_gbar, 0, (size_t)GMRES_BAR_WORDS * C->nrhs * sizeof(unsigned)));
    TD_HIP(hipHostMalloc((void **)&C->h_iflag, 4 * (size_t)C->nrhs * sizeof(int), hipHostMallocDefault));
    if (const char *gb = std::getenv("TDBEM_GMRES_BLOCKS")) C->gmres_blocks = std::max(1, std::atoi(gb));
    C->d_scal = dalloc<double>(C, 64 * (size_t)C->nrhs);
    C->d_pulse = dalloc<double>(C, 11 * (size_t)C->nrhs);
    TD_HIP(hipMemsetAsync(C->d_Jring, 0, (size_t)ne * R * C->nrhs * sizeof(double), s));
    if (C->d_Jring32) TD_HIP(hipMemsetAsync(C->d_Jring32, 0, (size_t)ne * R * C->nrhs * sizeof(float), s));
    TD_HIP(hipStreamSynchronize(s));
    C->alpha = 1;
    C->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

static void reset_impl(tdbem_ctx *C) {
    hipStream_t s = C->stream;
    TD_HIP(hipMemsetAsync(C->d_Jring, 0, (size_t)C->ne * C->ring * C->nrhs * sizeof(double), s));
    if (C->d_Jring32) TD_HIP(hipMemsetAsync(C->d_Jring32, 0, (size_t)C->ne * C->ring * C->nrhs * sizeof(float), s));
    if (C->cfg.mode == TDBEM_MODE_IFMM) ifmm_reset(C);
    C->alpha = 1;
}

static int step_impl(tdbem_ctx *C, const double *V, double *Jout, bool solve, const double *Jgiven) {
    hipStream_t s = C->stream;
    const int64_t nv = (int64_t)C->ne * C->nrhs;
    int a = C->alpha;
    int rc = TDBEM_OK;
    if (solve) {
        { PhaseScope ps(C->prof, TDBEM_PH_OTHER, s); launch_gather_in(C, V, C->d_rhs, s); }
        { PhaseScope ps(C->prof, TDBEM_PH_NEAR, s); launch_near(C, a, C->d_tmp, 1.0, s); }
        {
            PhaseScope ps(C->prof, TDBEM_PH_OTHER, s);
            launch_axpby(nv, -1.0, C->d_tmp, 1.0, C->d_rhs, s);
            if (C->cfg.mode == TDBEM_MODE_IFMM) ifmm_subtract_far(C, a, C->d_rhs, s);
            launch_extrap(C, a, C->d_x, s);
            if (guess_active(C)) launch_guess(C, a, s);
        }
        bool ok = true;
        {
            PhaseScope ps(C->prof, TDBEM_PH_GMRES, s);
            const int maxit = std::max(1, C->cfg.gmres_maxit);
            if (C->use_coop && gmres_coop_launch(C, C->d_rhs, C->d_x, C->cfg.gmres_rtol, maxit, s)) {
                const size_t nf = 4 * (size_t)C->nrhs;
                TD_HIP(hipMemcpyAsync(C->h_iflag, C->d_iflag, nf * sizeof(int), hipMemcpyDeviceToHost, s));
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
                    TD_HIP(hipMemset(C->d_gbar, 0, (size_t)GMRES_BAR_WORDS * C->nrhs * sizeof(unsigned)));
                    throw Error{TDBEM_EHIP, "device solve: a grid barrier wait timed out"};
                }
            } else {
                C->last_iters = gmres_solve(C, C->d_rhs, C->d_x, C->cfg.gmres_rtol, maxit, &ok, s);
            }
        }
        if (!ok) rc = TDBEM_ENOCONV;
    } else {
        launch_gather_in(C, Jgiven, C->d_x, s);
    }
    { PhaseScope ps(C->prof, TDBEM_PH_OTHER, s); launch_ring_put(C, (a - 1) & (C->ring - 1), C->d_x, s); }
    if (C->cfg.mode == TDBEM_MODE_IFMM) ifmm_after_solve(C, a, s);
    if (Jout) { PhaseScope ps(C->prof, TDBEM_PH_OTHER, s); launch_scatter_out(C, C->d_x, Jout, s); }
    C->alpha = a + 1;
    return rc;
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
    return rc;
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
        std::vector<double> val(C->hp_nnz);
        TD_HIP(hipMemcpy(val.data(), C->d_coef, C->hp_nnz * sizeof(double), hipMemcpyDeviceToHost));
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
    ifmm_destroy(C);
    guess_destroy(C);
    for (void *p : C->allocs) (void)hipFree(p);
    if (C->h_scal) (void)hipHostFree(C->h_scal);
    if (C->h_iflag) (void)hipHostFree(C->h_iflag);
    delete C;
}

const char *tdbem_last_error(void) { return g_err.c_str(); }

}  // extern "C"
