// Learned initial guess for the Z0 solve (an addition to the paper's method,
// which starts the solve of Eq. solve from a given vector; the extrapolation of
// the current history is the baseline guess).
//
// For every edge i and right-hand side, 116 features are formed from quantities
// the step already holds:
//   f = 8 e + (s - 1), e = 0..12, s = 1..8 : sigma_ie J_e^{alpha-1-s}
//   f = 104 + e,       e = 0..11          : sigma_ie (R_e^{alpha-1} - (Z0 x)_e) / Z0_ee
// where e = 0 is the edge itself and e = 1..12 its 12 nearest edges by midpoint
// distance (ties by canonical index), sigma_ie = +-1 aligns the neighbour's
// current direction with edge i's (sign of the dot product of the directions
// from the T+ centroid to the T- centroid), R is the step's right-hand side and
// x the extrapolation, so that the last group is the Jacobi-scaled residual the
// correction has to remove.
// The features are divided by their largest magnitude s_i (1 if all vanish),
// rounded to bf16, and a 116 -> 128 -> 128 -> 1 ReLU network o(x) gives the odd
// correction g(x) = (o(x) - o(-x)) / 2 to the quadratic extrapolation:
//   J_guess = extrap + s_i g(x).
// The solve starts from whichever of the two guesses has the smaller residual
// norm ||R - Z0 x|| (per right-hand side), so the extrapolation is the fallback.
// The matrix products run on the bf16 matrix cores with FP32 accumulation; the
// biases and the last layer are FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "tdbem_internal.h"

namespace tdbem {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

static constexpr int GNF = 116;      // features
static constexpr int GNK = 128;      // padded input width
static constexpr int GNH = 128;      // hidden width
static constexpr int GNN = 12;       // neighbours

struct GuessState {
    int *nn = nullptr;          // [ne][12] leaf-order neighbours
    float *sg = nullptr;        // [ne][12] direction signs
    unsigned short *w1 = nullptr, *w2 = nullptr;   // bf16 B fragments [4 ks][8 ct][64 lanes][8]
    float *b1 = nullptr, *b2 = nullptr, *w3 = nullptr;
    bool ready = false;
    float *cap_feat = nullptr;  // capture: [rhs][ne][116] (canonical order)
    double *cap_aux = nullptr;  // capture: [rhs][ne][2] (scale, extrapolation)
    double *xl = nullptr;       // [ne][rhs] learned guess
    double *zxl = nullptr;      // [ne][rhs] Z0 times the learned guess
    double *part = nullptr;     // [JB][rhs][2] partial residual norms
    int *use = nullptr;         // [rhs] 1 where the learned guess has the smaller residual
    int64_t *used = nullptr;    // device count of (step, rhs) where the learned guess was taken
};
static constexpr int JB = 256;  // blocks of the residual comparison

// round-to-nearest-even FP32 -> bf16 bits
__host__ __device__ inline unsigned short bf16_bits(float f) {
    unsigned int u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40);   // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf16_float(unsigned short b) {
    unsigned int u = (unsigned int)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// ------------------------------------------------------------------ host setup
void guess_setup(tdbem_ctx *C) {
    const HostMesh &H = C->H;
    const int ne = C->ne;
    GuessState *G = new GuessState();
    C->guess = G;
    std::vector<double> mid(3 * (size_t)ne), dir(3 * (size_t)ne);
    double hmax = 0.0;
    for (int e = 0; e < ne; ++e) {
        const double *a = &H.xyz[3 * H.edge_v[2 * e]], *b = &H.xyz[3 * H.edge_v[2 * e + 1]];
        for (int k = 0; k < 3; ++k) mid[3 * e + k] = 0.5 * (a[k] + b[k]);
        hmax = std::max(hmax, H.elen[e]);
        double cp[3] = {0, 0, 0}, cm[3] = {0, 0, 0};
        for (int v = 0; v < 3; ++v)
            for (int k = 0; k < 3; ++k) {
                cp[k] += H.xyz[3 * H.tri[3 * H.etri[2 * e] + v] + k] / 3.0;
                cm[k] += H.xyz[3 * H.tri[3 * H.etri[2 * e + 1] + v] + k] / 3.0;
            }
        for (int k = 0; k < 3; ++k) dir[3 * e + k] = cm[k] - cp[k];
    }
    TD_REQUIRE(ne > GNN, TDBEM_EINVAL, "the learned guess needs more than 12 edges");
    // uniform grid of cell size hmax over the midpoints
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], mid[3 * e + k]); hi[k] = std::max(hi[k], mid[3 * e + k]); }
    int dim[3];
    for (int k = 0; k < 3; ++k) dim[k] = std::max(1, (int)std::floor((hi[k] - lo[k]) / hmax) + 1);
    auto cell_of = [&](int e, int k) { return std::min(dim[k] - 1, (int)std::floor((mid[3 * e + k] - lo[k]) / hmax)); };
    std::vector<int> cstart((size_t)dim[0] * dim[1] * dim[2] + 1, 0), cl(ne);
    for (int e = 0; e < ne; ++e) cstart[((size_t)cell_of(e, 0) * dim[1] + cell_of(e, 1)) * dim[2] + cell_of(e, 2) + 1]++;
    for (size_t c = 1; c < cstart.size(); ++c) cstart[c] += cstart[c - 1];
    {
        std::vector<int> fill(cstart.begin(), cstart.end() - 1);
        for (int e = 0; e < ne; ++e) cl[fill[((size_t)cell_of(e, 0) * dim[1] + cell_of(e, 1)) * dim[2] + cell_of(e, 2)]++] = e;
    }
    std::vector<int> nn((size_t)ne * GNN);
    std::vector<float> sg((size_t)ne * GNN);
    std::vector<std::pair<double, int>> cand;
    for (int e = 0; e < ne; ++e) {
        int c0[3] = {cell_of(e, 0), cell_of(e, 1), cell_of(e, 2)};
        for (int rad = 1;; ++rad) {
            cand.clear();
            for (int x = std::max(0, c0[0] - rad); x <= std::min(dim[0] - 1, c0[0] + rad); ++x)
                for (int y = std::max(0, c0[1] - rad); y <= std::min(dim[1] - 1, c0[1] + rad); ++y)
                    for (int z = std::max(0, c0[2] - rad); z <= std::min(dim[2] - 1, c0[2] + rad); ++z) {
                        size_t c = ((size_t)x * dim[1] + y) * dim[2] + z;
                        for (int q = cstart[c]; q < cstart[c + 1]; ++q) {
                            int f = cl[q];
                            if (f == e) continue;
                            double dx = mid[3 * f] - mid[3 * e], dy = mid[3 * f + 1] - mid[3 * e + 1],
                                   dz = mid[3 * f + 2] - mid[3 * e + 2];
                            cand.push_back({(dx * dx + dy * dy) + dz * dz, f});
                        }
                    }
            bool whole = rad >= std::max(dim[0], std::max(dim[1], dim[2]));
            if ((int)cand.size() >= GNN) {
                std::partial_sort(cand.begin(), cand.begin() + GNN, cand.end());
                double reach = rad * hmax;
                if (cand[GNN - 1].first <= reach * reach || whole) break;
            }
            TD_REQUIRE(!whole || (int)cand.size() >= GNN, TDBEM_EINVAL, "fewer than 13 edges");
        }
        const int p = C->T.iperm[e];
        for (int k = 0; k < GNN; ++k) {
            int f = cand[k].second;
            double d = dir[3 * e] * dir[3 * f] + dir[3 * e + 1] * dir[3 * f + 1] + dir[3 * e + 2] * dir[3 * f + 2];
            nn[(size_t)p * GNN + k] = C->T.iperm[f];
            sg[(size_t)p * GNN + k] = d < 0.0 ? -1.0f : 1.0f;
        }
    }
    G->nn = dupload(C, nn);
    G->sg = dupload(C, sg);
    G->w1 = dalloc<unsigned short>(C, 4 * 8 * 64 * 8);
    G->w2 = dalloc<unsigned short>(C, 4 * 8 * 64 * 8);
    G->b1 = dalloc<float>(C, GNH);
    G->b2 = dalloc<float>(C, GNH);
    G->w3 = dalloc<float>(C, GNH + 1);
    const size_t nv = (size_t)ne * C->nrhs;
    G->xl = dalloc<double>(C, nv);
    G->zxl = dalloc<double>(C, nv);
    G->part = dalloc<double>(C, (size_t)JB * C->nrhs * 2);
    G->use = dalloc<int>(C, C->nrhs);
    G->used = dalloc<int64_t>(C, 1);
    TD_HIP(hipMemset(G->used, 0, sizeof(int64_t)));
}

void guess_destroy(tdbem_ctx *C) {
    delete C->guess;
    C->guess = nullptr;
}

// parameters: W1 [116][128] (input, hidden), b1 [128], W2 [128][128], b2 [128], w3 [128], b3
void guess_load(tdbem_ctx *C, const float *p, int64_t n) {
    GuessState *G = C->guess;
    TD_REQUIRE(G, TDBEM_EINVAL, "the learned guess is not set up");
    TD_REQUIRE(n == TDBEM_GUESS_NPARAMS, TDBEM_EINVAL,
               "expected " + std::to_string(TDBEM_GUESS_NPARAMS) + " parameters, got " + std::to_string(n));
    for (int64_t q = 0; q < n; ++q) TD_REQUIRE(std::isfinite(p[q]), TDBEM_EINVAL, "non-finite guess parameter");
    const float *W1 = p, *b1 = W1 + GNF * GNH, *W2 = b1 + GNH, *b2 = W2 + GNH * GNH, *w3 = b2 + GNH;
    // B-operand fragments of the 16x16x32 bf16 instruction: lane l holds
    // B[32 ks + 8 (l / 16) + e][16 ct + l % 16], e = 0..7
    std::vector<unsigned short> f1(4 * 8 * 64 * 8), f2(4 * 8 * 64 * 8);
    for (int ks = 0; ks < 4; ++ks)
        for (int ct = 0; ct < 8; ++ct)
            for (int l = 0; l < 64; ++l)
                for (int e = 0; e < 8; ++e) {
                    int k = 32 * ks + 8 * (l / 16) + e, c = 16 * ct + l % 16;
                    size_t o = (((size_t)ks * 8 + ct) * 64 + l) * 8 + e;
                    f1[o] = bf16_bits(k < GNF ? W1[(size_t)k * GNH + c] : 0.0f);
                    f2[o] = bf16_bits(W2[(size_t)k * GNH + c]);
                }
    hipStream_t s = C->stream;
    TD_HIP(hipMemcpyAsync(G->w1, f1.data(), f1.size() * 2, hipMemcpyHostToDevice, s));
    TD_HIP(hipMemcpyAsync(G->w2, f2.data(), f2.size() * 2, hipMemcpyHostToDevice, s));
    TD_HIP(hipMemcpyAsync(G->b1, b1, GNH * 4, hipMemcpyHostToDevice, s));
    TD_HIP(hipMemcpyAsync(G->b2, b2, GNH * 4, hipMemcpyHostToDevice, s));
    TD_HIP(hipMemcpyAsync(G->w3, w3, (GNH + 1) * 4, hipMemcpyHostToDevice, s));
    TD_HIP(hipStreamSynchronize(s));
    G->ready = true;
}

void guess_capture(tdbem_ctx *C, float *feat, double *aux) {
    GuessState *G = C->guess;
    TD_REQUIRE(G, TDBEM_EINVAL, "the learned guess is not set up");
    TD_REQUIRE((feat == nullptr) == (aux == nullptr), TDBEM_EINVAL, "give both capture buffers or neither");
    G->cap_feat = feat;
    G->cap_aux = aux;
}

bool guess_active(const tdbem_ctx *C) {
    const GuessState *G = C->guess;
    return G && ((C->cfg.guess == TDBEM_GUESS_LEARNED) || G->cap_feat);
}

// ------------------------------------------------------------------ kernel
struct GuessArgs {
    int ne, nrhs, R, alpha;
    const double *ring, *rhs, *zx, *dinv;   // zx = Z0 x (x the extrapolation)
    const int *nn, *perm;
    const float *sg;
    const unsigned short *w1, *w2;
    const float *b1, *b2, *w3;
    const double *x;            // extrapolation
    double *xl;                 // out: learned guess
    float *cap_feat;
    double *cap_aux;
};

__device__ inline v8bf load_frag(const unsigned short *w, int ks, int ct, int lane) {
    const uint4 q = *(const uint4 *)(w + ((((size_t)ks * 8 + ct) * 64 + lane) * 8));
    return __builtin_bit_cast(v8bf, q);
}

// one wavefront per 16 (edge, rhs) items; lane l owns item l % 16 and the
// features 32 ks + 8 (l / 16) + e, e = 0..7, of each k-step ks
template <bool MLP>
__global__ void __launch_bounds__(256) k_guess(GuessArgs a) {
    __shared__ __align__(16) unsigned short hs[4][2][16][GNK + 8];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = lane & 15, qd = lane >> 4;
    const int64_t nitem = (int64_t)a.ne * a.nrhs;
    const int64_t item = ((int64_t)blockIdx.x * 4 + wave) * 16 + row;
    const bool valid = item < nitem;
    const int i = valid ? (int)(item / a.nrhs) : 0, r = valid ? (int)(item % a.nrhs) : 0;
    // features
    float f[4][8];
    float mx = 0.0f;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        const int en = 4 * ks + qd;           // feature group of 8
#pragma unroll
        for (int e = 0; e < 8; ++e) f[ks][e] = 0.0f;
        if (!valid) continue;
        if (en < 13) {                        // history of edge en
            const int edge = en == 0 ? i : a.nn[(size_t)i * GNN + en - 1];
            const float sgn = en == 0 ? 1.0f : a.sg[(size_t)i * GNN + en - 1];
            const double *J = a.ring + (size_t)edge * a.R * a.nrhs + r;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int b = a.alpha - 2 - e;   // J^{alpha-1-s}, s = e + 1
                f[ks][e] = b < 0 ? 0.0f : sgn * (float)J[(size_t)(b & (a.R - 1)) * a.nrhs];
            }
        } else if (en < 15) {                 // scaled residuals of the extrapolation, e = 8 (en - 13) + k
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 8 * (en - 13) + e;
                if (k >= GNN) break;
                const int edge = k == 0 ? i : a.nn[(size_t)i * GNN + k - 1];
                const float sgn = k == 0 ? 1.0f : a.sg[(size_t)i * GNN + k - 1];
                const size_t q = (size_t)edge * a.nrhs + r;
                f[ks][e] = sgn * (float)(a.dinv[edge] * (a.rhs[q] - a.zx[q]));
            }
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) mx = fmaxf(mx, fabsf(f[ks][e]));
    }
    mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
    mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
    const float scale = mx > 0.0f ? mx : 1.0f;
    const float inv = 1.0f / scale;
    v8bf xa[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const unsigned short b = bf16_bits(f[ks][e] * inv);
            f[ks][e] = bf16_float(b);
            xa[ks][e] = __builtin_bit_cast(__bf16, b);
        }
    if (a.cap_feat && valid) {
        const int ce = a.perm[i];
        float *o = a.cap_feat + ((size_t)r * a.ne + ce) * GNF;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int fi = 32 * ks + 8 * qd + e;
                if (fi < GNF) o[fi] = f[ks][e];
            }
        if (qd == 0) {
            a.cap_aux[((size_t)r * a.ne + ce) * 2] = scale;
            a.cap_aux[((size_t)r * a.ne + ce) * 2 + 1] = a.x[item];
        }
    }
    if (!MLP) return;
    // layer 1: acc = x W1 (bias and sign applied per branch)
    v4f acc[8];
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) acc[ct] = v4f{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int ct = 0; ct < 8; ++ct)
            acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[ks], load_frag(a.w1, ks, ct, lane), acc[ct], 0, 0, 0);
    // h1 for both branches (+x, -x) into LDS in the A-operand order of layer 2
#pragma unroll
    for (int br = 0; br < 2; ++br)
#pragma unroll
        for (int ct = 0; ct < 8; ++ct) {
            const int col = 16 * ct + row;
            const float bb = a.b1[col];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float h = (br == 0 ? acc[ct][v] : -acc[ct][v]) + bb;
                hs[wave][br][4 * qd + v][col] = bf16_bits(h > 0.0f ? h : 0.0f);
            }
        }
    __syncthreads();
    float out[2][4];
#pragma unroll
    for (int br = 0; br < 2; ++br) {
        v4f acc2[8];
#pragma unroll
        for (int ct = 0; ct < 8; ++ct) acc2[ct] = v4f{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const uint4 q = *(const uint4 *)&hs[wave][br][row][32 * ks + 8 * qd];
            const v8bf ha = __builtin_bit_cast(v8bf, q);
#pragma unroll
            for (int ct = 0; ct < 8; ++ct)
                acc2[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ha, load_frag(a.w2, ks, ct, lane), acc2[ct], 0, 0, 0);
        }
        // layer 3: rows 4 qd + v, columns 16 ct + row of this lane
#pragma unroll
        for (int v = 0; v < 4; ++v) out[br][v] = 0.0f;
#pragma unroll
        for (int ct = 0; ct < 8; ++ct) {
            const int col = 16 * ct + row;
            const float bb = a.b2[col], w = a.w3[col];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float h = acc2[ct][v] + bb;
                out[br][v] += (h > 0.0f ? h : 0.0f) * w;
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) out[br][v] += __shfl_xor(out[br][v], o, 64);
    }
    // lane (qd, row < 4) writes the item 4 qd + row; its scale lives in lane 4 qd + row
    float g = 0.0f;
#pragma unroll
    for (int v = 0; v < 4; ++v)
        if (row == v) g = 0.5f * (out[0][v] - out[1][v]);
    const int src = 4 * qd + row;             // lane holding that item's scale (any quarter)
    const float sc = __shfl(scale, src & 15, 64);
    const int64_t it2 = ((int64_t)blockIdx.x * 4 + wave) * 16 + src;
    if (row < 4 && it2 < nitem) a.xl[it2] = a.x[it2] + (double)sc * (double)g;
}

// residual comparison: part[b][r] = sum over block b's rows of (b - Z0 x)^2 for the
// extrapolation and for the learned guess
__global__ void k_judge_part(int ne, int nrhs, const double *rhs, const double *zx, const double *zxl, double *part) {
    __shared__ double red[2][256];
    for (int r = 0; r < nrhs; ++r) {
        double se = 0.0, sl = 0.0;
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += gridDim.x * blockDim.x) {
            const size_t q = (size_t)i * nrhs + r;
            const double de = rhs[q] - zx[q], dl = rhs[q] - zxl[q];
            se += de * de;
            sl += dl * dl;
        }
        red[0][threadIdx.x] = se;
        red[1][threadIdx.x] = sl;
        __syncthreads();
        for (int o = blockDim.x / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) {
                red[0][threadIdx.x] += red[0][threadIdx.x + o];
                red[1][threadIdx.x] += red[1][threadIdx.x + o];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            part[((size_t)blockIdx.x * nrhs + r) * 2] = red[0][0];
            part[((size_t)blockIdx.x * nrhs + r) * 2 + 1] = red[1][0];
        }
        __syncthreads();
    }
}
// one block per rhs: sum the partials by a fixed-order tree and decide
__global__ void __launch_bounds__(JB) k_judge_decide(int nrhs, const double *part, int *use, int64_t *used) {
    __shared__ double red[2][JB];
    const int r = blockIdx.x, t = threadIdx.x;
    red[0][t] = part[((size_t)t * nrhs + r) * 2];
    red[1][t] = part[((size_t)t * nrhs + r) * 2 + 1];
    __syncthreads();
    for (int o = JB / 2; o > 0; o >>= 1) {
        if (t < o) {
            red[0][t] += red[0][t + o];
            red[1][t] += red[1][t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        const bool l = red[1][0] < red[0][0];
        use[r] = l ? 1 : 0;
        if (l) atomicAdd((unsigned long long *)used, 1ull);
    }
}
__global__ void k_judge_apply(int64_t n, int nrhs, const int *use, const double *xl, double *x) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n && use[k % nrhs]) x[k] = xl[k];
}

void launch_guess(tdbem_ctx *C, int alpha, hipStream_t s) {
    GuessState *G = C->guess;
    const bool mlp = C->cfg.guess == TDBEM_GUESS_LEARNED;
    TD_REQUIRE(!mlp || G->ready, TDBEM_EINVAL, "learned guess selected but no parameters were loaded");
    GuessArgs a;
    a.ne = C->ne; a.nrhs = C->nrhs; a.R = C->ring; a.alpha = alpha;
    // Z0 x of the extrapolation into the step's scratch vector
    launch_spmv(C, C->d_x, C->d_tmp, s);
    a.ring = C->d_Jring; a.rhs = C->d_rhs; a.zx = C->d_tmp; a.dinv = C->d_z0_dinv;
    a.nn = G->nn; a.perm = C->d_perm; a.sg = G->sg;
    a.w1 = G->w1; a.w2 = G->w2; a.b1 = G->b1; a.b2 = G->b2; a.w3 = G->w3;
    a.x = C->d_x; a.xl = G->xl; a.cap_feat = G->cap_feat; a.cap_aux = G->cap_aux;
    const int64_t nitem = (int64_t)C->ne * C->nrhs;
    const unsigned nb = (unsigned)((nitem + 63) / 64);
    if (!mlp) {
        hipLaunchKernelGGL(k_guess<false>, dim3(nb), dim3(256), 0, s, a);
        TD_HIP(hipGetLastError());
        return;
    }
    hipLaunchKernelGGL(k_guess<true>, dim3(nb), dim3(256), 0, s, a);
    // the residual judges the learned guess; the extrapolation is the fallback
    launch_spmv(C, G->xl, G->zxl, s);
    hipLaunchKernelGGL(k_judge_part, dim3(JB), dim3(256), 0, s, C->ne, C->nrhs, C->d_rhs, C->d_tmp, G->zxl, G->part);
    hipLaunchKernelGGL(k_judge_decide, dim3(C->nrhs), dim3(JB), 0, s, C->nrhs, G->part, G->use, G->used);
    hipLaunchKernelGGL(k_judge_apply, dim3((unsigned)((nitem + 255) / 256)), dim3(256), 0, s, nitem, C->nrhs, G->use,
                       G->xl, C->d_x);
    TD_HIP(hipGetLastError());
}

int64_t guess_used(tdbem_ctx *C) {
    if (!C->guess) return 0;
    int64_t v = 0;
    TD_HIP(hipMemcpyAsync(&v, C->guess->used, sizeof(int64_t), hipMemcpyDeviceToHost, C->stream));
    TD_HIP(hipStreamSynchronize(C->stream));
    return v;
}

}  // namespace tdbem
