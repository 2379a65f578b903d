// Internal declarations of the MI355X TDBEM library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <map>
#include <vector>

#include "../../include/tdbem.h"

namespace tdbem {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
struct Error {
    int code;
    std::string msg;
};
#define TD_HIP(call)                                                                     \
    do {                                                                                 \
        hipError_t _e = (call);                                                          \
        if (_e != hipSuccess)                                                            \
            throw ::tdbem::Error{TDBEM_EHIP, std::string(#call) + ": " + hipGetErrorString(_e)}; \
    } while (0)
#define TD_REQUIRE(cond, code, msg)                                                      \
    do {                                                                                 \
        if (!(cond)) throw ::tdbem::Error{code, msg};                                    \
    } while (0)

// ------------------------------------------------------------ host geometry
struct HostMesh {
    int nv = 0, nt = 0, ne = 0;
    std::vector<double> xyz;        // [nv][3]
    std::vector<int> tri;           // [nt][3]
    // canonical edge order
    std::vector<int> edge_v;        // [ne][2] (lo, hi)
    std::vector<int> etri;          // [ne][2] T+, T-
    std::vector<int> efree;         // [ne][2] o+, o-
    std::vector<double> elen;       // [ne]
    std::vector<int> tedge;         // [nt][3]
    std::vector<double> area;       // [nt]
    std::vector<double> nrm;        // [nt][3] outward unit normal
    std::vector<double> qpt;        // [nt][3][3] interior 3-point rule points
};

// octree level data (cells of one level, in Morton order)
struct Level {
    int n = 0;
    std::vector<int> ix, iy, iz;    // integer cell coordinates at this level
    std::vector<int> parent;        // index at level-1 (-1 at level 0)
    std::vector<int> child_beg, child_end;  // children index range at level+1
    std::vector<int> ebeg, eend;    // edge range in leaf order
    std::vector<char> leaf;
    std::vector<int> nbr_off, nbr;  // neighbour list (Chebyshev distance <= 1, incl. self)
    std::vector<int> il_off, il_src, il_code;  // interaction list: source cell, offset code
};

struct Tree {
    double origin[3] = {0, 0, 0};
    double side = 0;
    int lmax = 0;
    std::vector<Level> lev;         // 0..lmax
    std::vector<int> perm;          // leaf position -> canonical edge id
    std::vector<int> iperm;         // canonical edge id -> leaf position
    std::vector<int> edge_leaf_level, edge_leaf_cell;  // per leaf-order edge
};

void build_mesh(const tdbem_mesh *m, HostMesh &H);
void build_tree(const HostMesh &H, int leaf_max, int min_level, Tree &T);
// near source cell lists per leaf cell (as (level, cell) pairs), Program 2
void near_source_cells(const Tree &T, int level, int cell, std::vector<std::pair<int, int>> &out);

// geometry view passed to device kernels (edges in leaf order)
struct GeoDev {
    const double *xyz; const int *tri; const double *area; const double *nrm; const double *qpt;
    const int *etri; const int *efree; const double *elen;
    double cdt, dt, eps, mu, theta, zeta, eta;
    double kd;   // weight of the MFIE's time derivative (CFIE1, CFIE2: 1; CFIE3: 0); zeta is 0 for CFIE2
};

struct FarState;
struct GuessState;  // learned-guess device state (guess.hip)

// per-phase timing with HIP event pairs recorded on the work stream
struct Profiler {
    bool on = false;
    double ms[TDBEM_NPHASE] = {0};
    int64_t count[TDBEM_NPHASE] = {0};
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> pool;
    hipEvent_t get();
    void begin(int phase, hipStream_t s, hipEvent_t &e0);
    void end(int phase, hipStream_t s, hipEvent_t e0);
    void fold(hipStream_t s);
    void clear();
    ~Profiler();
};
struct PhaseScope {
    Profiler &P; int ph; hipStream_t s; hipEvent_t e0 = nullptr;
    PhaseScope(Profiler &P_, int ph_, hipStream_t s_) : P(P_), ph(ph_), s(s_) { if (P.on) P.begin(ph, s, e0); }
    ~PhaseScope() { if (P.on && e0) P.end(ph, s, e0); }
};

// words of grid-barrier state per system of the device solve (two 4 KB pages)
constexpr int GMRES_BAR_WORDS = 2 * 1024;

}  // namespace tdbem

namespace tdbem {
// the per-leaf form of the one-rhs near field: per leaf, its sources and the
// lags of theirs its pairs reach (a compressed current window), the chunks of
// rows of the leaves whose window fits the LDS budget, and the rows of the
// other leaves
struct NearLeaves {
    int nchunk = 0, nrest = 0;
    size_t max_window = 0;          // largest staged window (values)
    int *d_chunk = nullptr;         // [nchunk][3] leaf, first row, end row
    int *d_r0 = nullptr, *d_r1 = nullptr;   // [leaves] row range
    int *d_soff = nullptr, *d_src = nullptr;  // [leaves+1] offsets, source edges (leaf order)
    int *d_g = nullptr;             // [leaves][2] first lag and length of the box window (matrix-core form)
    int *d_loc = nullptr;           // [pairs] source index in the pair's leaf list
    int *d_ws = nullptr;            // [sources][4] edge, first lag, offset in the leaf's window, lags
    int *d_pwl = nullptr;           // [pairs] window offset of the strip's first lag | strip length << 16
    int *d_rest = nullptr;          // [nrest] rows left to the row kernel
    int nleaves = 0;                // leaves (all of them, for the batched matrix-core form)
};
}  // namespace tdbem

struct tdbem_ctx {
    tdbem_config cfg;
    hipStream_t stream = nullptr;
    tdbem::HostMesh H;
    tdbem::Tree T;
    int ne = 0, nrhs = 1;
    double c = 0, eta = 0, cdt = 0;
    int alpha = 1;                  // next step
    int ring = 64;                  // history ring length (power of two)
    int last_iters = 0;
    bool trace = false;             // TDBEM_TRACE=1: set-up layout notes and host-solver residuals on stderr
    double setup_ms = 0;
    size_t dev_bytes = 0;
    std::vector<void *> allocs;

    // geometry on device (leaf order for edges)
    double *d_xyz = nullptr;        // [nv][3]
    int *d_tri = nullptr;           // [nt][3]
    double *d_area = nullptr, *d_nrm = nullptr, *d_qpt = nullptr;
    int *d_etri = nullptr, *d_efree = nullptr;   // [ne][2] leaf order
    double *d_elen = nullptr;
    int *d_perm = nullptr;          // leaf -> canonical

    // near-field store (g >= 2): jagged-diagonal layout per target row (leaf order)
    int64_t near_pairs = 0, near_nnz = 0;
    int *d_nrow_ptr = nullptr;      // [ne+1] pair ranges per row (pairs sorted by strip length)
    int64_t *d_nrow_vbase = nullptr;// [ne] first value of each row
    int *d_nl = nullptr;            // [ne][near_L] pairs with a strip longer than l
    int near_L = 0;                 // longest strip
    int *d_npair_j = nullptr;       // [pairs] source edge (leaf order)
    int *d_npair_gl = nullptr;      // [pairs] first stored lag | strip length << 16
    double *d_nval = nullptr;       // [nnz] FP64 values
    float *d_nval32 = nullptr;      // [nnz] FP32 copy (FP32 form)
    void *d_nval16 = nullptr;       // [nnz] bf16 copy (BF16 form)
    std::vector<double> h_coef;     // pair-major coefficients of every pair (all lags), host copy for inspection
    int max_lag = 0;

    // Z0 = Zt^(1) CSR (leaf order)
    int64_t z0_nnz = 0;
    int *d_z0_ptr = nullptr, *d_z0_col = nullptr;
    double *d_z0_val = nullptr, *d_z0_dinv = nullptr;
    double *d_z0_vald = nullptr;    // Z0 with columns scaled by the Jacobi inverse

    // march state
    double *d_Jring = nullptr;      // [ne][ring][nrhs]
    float *d_Jring32 = nullptr;     // FP32 copy for the near field of the reduced-precision forms
    double *d_rhs = nullptr;        // [ne][nrhs] right-hand side of the step
    double *d_x = nullptr;          // [ne][nrhs] current solution (leaf order)
    double *d_work = nullptr;       // GMRES workspace
    double *d_scal = nullptr;       // small device scalars
    double *h_scal = nullptr;       // pinned host mirror
    double *d_pulse = nullptr;      // [nrhs][11]
    double *d_tmp = nullptr;        // [ne][nrhs] scratch (canonical order io)
    int *d_iflag = nullptr;         // device solver status per rhs: iterations, converged, barrier timeout
    hipStream_t cap_stream = nullptr;                   // capture-only stream of the graph march
    hipGraphExec_t g_pre = nullptr;                     // the kernels before the solve
    std::map<uint32_t, hipGraphExec_t> g_post;          // after the solve, per pattern of gated levels
    int64_t graph_builds = 0, graph_updates = 0;        // executables instantiated, argument refreshes
    void *d_march = nullptr;        // deferred step records of tdbem_march (grown on demand)
    size_t march_cap = 0;           // steps the records hold
    int *h_iflag = nullptr;         // pinned host mirror
    unsigned *d_gbar = nullptr;     // grid-barrier words of the cooperative solve, GMRES_BAR_WORDS per rhs
    int gmres_blocks = 0;           // blocks per system of the cooperative solve (0: automatic)
    int near_variant = 0;           // round shape of the one-rhs near-field kernel (set-up autotuner)
    tdbem::NearLeaves nleaf;        // per-leaf near-field structure (sources, windows)
    // batched rhs: dense per-leaf coefficient blocks for the matrix cores
    bool leaf_mm_ready = false;
    bool leaf_cover = false;        // the leaves' row ranges partition the rows
    std::vector<int> h_leaf_r0, h_leaf_r1, h_leaf_w;   // per leaf: rows, compressed window (columns)
    std::vector<int> h_pcol;        // set-up only: per pair the window column of its strip's first lag
    std::vector<int> h_colmap;      // set-up only: per leaf window column (source edge, lag), leaves in turn
    int64_t *d_leaf_aoff = nullptr; // [leaves] first value of each leaf's block
    int *d_leaf_kpad = nullptr;     // [leaves] block row length (sources x window, padded to 4)
    double *d_leafA64 = nullptr;    // FP64 blocks (FP64 form)
    float *d_leafA32 = nullptr;     // FP32 blocks (FP32 form)
    int64_t leaf_mm_bytes = 0;      // bytes of the dense leaf blocks
    int leaf_nseg = 0;              // column segments (a block each) over all leaves
    int *d_seg_order = nullptr;     // [segments] launch order: largest (rows x columns) first
    int64_t *d_leaf_coff = nullptr; // [leaves] offset of the leaf's columns in the column map
    int *d_leaf_colmap = nullptr;   // [columns][2] source edge and lag of every padded leaf column
    int *d_seg_leaf = nullptr;      // [segments] leaf
    int *d_seg_k = nullptr;         // [segments][2] column range
    int64_t *d_seg_poff = nullptr;  // [segments] offset of the segment's partial sums [rows][n_rhs]
    int *d_leaf_seg = nullptr;      // [leaves+1] segment range per leaf
    int *d_row_leaf = nullptr;      // [ne] leaf of each row
    double *d_leaf_part = nullptr;  // partial sums of the segments
    bool tuned = false;             // the set-up autotuner chose near_variant / gmres_blocks
    bool use_coop = true;           // device-resident solve
    // late-time stability monitor: per rhs, squared norms of V and J of the
    // step ([rhs][2], device and pinned host), largest |V| so far, largest |J|
    // while the excitation lasted, tripped flag
    double *d_stat = nullptr, *h_stat = nullptr;
    std::vector<double> mon_vmax, mon_jdrive;
    std::vector<int> mon_trip;
    uint64_t fingerprint = 0;       // mesh and configuration, recorded in checkpoints
    int64_t d0_nnz = -1;            // all-pairs coefficient count (computed at the first query)

    // host copies of the coefficient pair structure (leaf order, sorted by row)
    std::vector<int> hp_i, hp_j, hp_lo, hp_hi;
    std::vector<int64_t> hp_off;
    int64_t hp_nnz = 0;

    // space-time hierarchy (IFMM)
    std::vector<int> Mt;            // steps per interval per level (0 for levels < 2)
    int window = 0;                 // largest number of source intervals per M2L over the levels
    std::vector<int> windows;       // source intervals per M2L per level (mu + ceil(3 / M_t))
    int far_ring_need = 0;          // history ring length the far field needs
    tdbem::FarState *far = nullptr;
    tdbem::GuessState *guess = nullptr;   // learned initial guess (features, network)
    tdbem::Profiler prof;
};

namespace tdbem {

// device allocations owned by the context (freed in tdbem_destroy)
template <typename T>
inline T *dalloc(tdbem_ctx *C, size_t n) {
    if (n == 0) n = 1;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) throw Error{TDBEM_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed"};
    C->allocs.push_back(p);
    C->dev_bytes += n * sizeof(T);
    return (T *)p;
}
// release a set-up temporary allocated with dalloc before the context ends
template <typename T>
inline void dfree(tdbem_ctx *C, T *&p, size_t n) {
    if (!p) return;
    for (size_t i = 0; i < C->allocs.size(); ++i)
        if (C->allocs[i] == (void *)p) {
            C->allocs.erase(C->allocs.begin() + i);
            break;
        }
    TD_HIP(hipFree(p));
    C->dev_bytes -= std::max<size_t>(n, 1) * sizeof(T);
    p = nullptr;
}
template <typename T>
inline T *dupload(tdbem_ctx *C, const std::vector<T> &v) {
    T *p = dalloc<T>(C, v.size());
    if (!v.empty()) TD_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
}

void guess_setup(tdbem_ctx *C);
void guess_destroy(tdbem_ctx *C);
void guess_load(tdbem_ctx *C, const float *params, int64_t n);
void guess_capture(tdbem_ctx *C, float *feat, double *aux);
bool guess_active(const tdbem_ctx *C);
void launch_guess(tdbem_ctx *C, int alpha, hipStream_t s);
int64_t guess_used(tdbem_ctx *C);
void launch_spmv(const tdbem_ctx *C, const double *x, double *y, hipStream_t s);
void launch_colnorm2(const tdbem_ctx *C, const double *x, double *out, int slot, hipStream_t s);
void launch_copy_words(const void *src, void *dst, size_t words, hipStream_t s);
uint32_t ifmm_gate_mask(const tdbem_ctx *C, int alpha);
int64_t count_d0_nnz(const tdbem_ctx *C);
void cfie_weights(const tdbem_config &cfg, double &kd, double &zeta);
void guess_grad(const float *P, const float *X, const float *Y, int64_t n, float *G, float *loss, hipStream_t s);
void guess_adam(float *P, const float *G, float *M, float *V, int t, float lr, float b1, float b2, float eps,
                hipStream_t s);

}  // namespace tdbem
