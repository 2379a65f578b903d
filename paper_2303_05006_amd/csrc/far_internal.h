// Far-field (IFMM) state shared by the far-field sources (not part of the ABI).
#pragma once

#include <vector>

#include "tdbem_internal.h"

namespace tdbem {

static constexpr int NCH = 7;        // channels: 0-2 vector, 3 scalar, 4-6 magnetic potential
static constexpr int M2L_NT = 64;    // columns per M2L tile
static constexpr int NV_MAX = 4;     // moment variants per interval: full + up to 3 truncated (M_t >= 1)
static constexpr int PMAX = 8;       // largest interpolation order
static constexpr int M2L_SPLIT_BLOCKS = 2048;   // fewer offset-major M2L tiles than this: split the lags

struct FarLevel {
    int n = 0, M = 0;
    int W = 0, WR = 0, NV = 0;   // window, ring slots (W + 1), moment variants per slot (full + truncated)
    double ds = 0, hs = 0, hn = 0, ht = 0;   // cell side, cell half-width, node half-width, time half-width
    int *il_off = nullptr, *il_src = nullptr, *il_code = nullptr;  // interaction lists
    int64_t nil = 0;                                               // interaction-list entries
    int *ix = nullptr;                                             // [n][3] integer coords
    int *ebeg = nullptr, *eend = nullptr;
    int nleaf = 0, nparent = 0;
    int *leaf_cells = nullptr, *parent_cells = nullptr;
    int *child_beg = nullptr, *child_end = nullptr;                // children at level+1
    double *MM = nullptr;     // [n][WR][NV][NCH][nrhs][NN]: variant 0 full, v + 1 truncated v intervals back
    float *MM32 = nullptr;    // FP32 copy of MM for the FP32 form's tuned M2L (p = 4), written by P2M / M2M
    unsigned short *MM16 = nullptr;   // bf16 copy of MM for the BF16 form's tuned M2L (p = 4)
    double *LC = nullptr;     // [n][NCH][nrhs][NN]
    double *PEND = nullptr;   // [n][2][NCH][nrhs][NN]
    double *tw = nullptr;     // [M][3][P]: target weights of the channel groups (A, phi, P) at step q = 1..M
    double *ls = nullptr;     // [M][P]: l_n at source step beta - kM = 0..M-1
    // offset-major M2L tiles (one right-hand side)
    int ntile = 0;
    int *tile_code = nullptr, *tile_kind = nullptr, *tile_col0 = nullptr, *tile_ncol = nullptr;
    int *col_q = nullptr, *col_ch = nullptr;
    double *YB = nullptr;     // [lag groups][interaction-list entries][NCH][NN]
    int yg_max = 1;           // lag groups YB holds (coarse levels split their window over blocks)
    int yg = 1;               // lag groups of the last launch (summed by the reduce)
    // Fourier-domain M2L: transformed kernels, moments (ring) and local sums
    int *fft_code_slot = nullptr;   // [343]: offset code -> row of KH (-1: absent)
    double2 *KH = nullptr;          // [used offset][W][2][NF]
    double2 *MH = nullptr;          // [n][WR][NV][NCH][nrhs][NF]
    double2 *LH = nullptr;          // [n][NCH][nrhs][NF]
};

struct FarState {
    int P = 4, NS = 64, NN = 256;   // interpolation points per axis and in time, P^3, P^4
    bool generic_m2l = false;       // dense M2L with operators formed per lane (any P)
    bool fft_m2l = false;           // M2L through the 4-D Fourier transform
    bool bf16_m2l = false;          // the tuned p = 4 M2L with bf16 operands
    int64_t NF = 0;                 // transformed values per vector: (2P)^3 (P + 1)
    double2 *fft_s1 = nullptr, *fft_s2 = nullptr;   // transform scratch
    int lmax = 0, FR = 0, nrhs = 1;
    double delta = 0;         // widening of the interpolation boxes beyond the cells
    std::vector<FarLevel> lev;
    double *Wm = nullptr;     // [ne][NCH][NS] P2M weights
    double *El = nullptr;     // [ne][NCH][NS] L2P weights
    double *FAR = nullptr;    // [FR][ne][nrhs] far-field potential per target slot
    double *S1 = nullptr;     // [parent level][space, time][2][P][P]: parent cardinal at child node, half h
};

// kernel of the vector-potential channels per placement of the second time
// derivative: 0 dU/dt (split), 2 d^2U/dt^2 (on the kernel), 1 U (on the interpolant)
inline int m2l_kind_a(const tdbem_config &cfg) {
    return cfg.dt2 == TDBEM_DT2_SPLIT ? 0 : cfg.dt2 == TDBEM_DT2_KERNEL ? 2 : 1;
}

// device allocation owned by the context (freed at destroy)
void *far_alloc(tdbem_ctx *C, size_t bytes);

// Fourier-domain M2L: tables of one level, the transform of one ring slot of
// moments, and the M2L of one level at gate k (writes LC)
void m2l_fft_setup(tdbem_ctx *C, FarLevel &FL, const std::vector<int> &il_code, int kindA);
void m2l_fft_moments(tdbem_ctx *C, FarLevel &FL, int slot, hipStream_t s);
void m2l_fft_level(tdbem_ctx *C, FarLevel &FL, int k, hipStream_t s);

// the tuned p = 4 M2L (operator tables in LDS) of one level at gate k; T is the
// product type (double or float)
template <typename T>
void m2l_p4_launch(tdbem_ctx *C, FarLevel &FL, int k, hipStream_t s);
// the BF16 form of the tuned p = 4 M2L (bf16 operands, FP32 accumulation)
void m2l_bf16_launch(tdbem_ctx *C, FarLevel &FL, int k, hipStream_t s);
// the reduced copies of a whole level's moments (after a restore)
void mm_copies_refresh(tdbem_ctx *C, FarLevel &FL, hipStream_t s);

}  // namespace tdbem
