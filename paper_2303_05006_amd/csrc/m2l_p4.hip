// The tuned M2L for p_s = p_t = 4 (Section 3.6.1): operators tabulated in LDS
// per (offset, lag) from the node lattice, products on the matrix cores.
// Offset-major for one right-hand side (columns = interaction-list entries and
// channels sharing an offset), target-major for batched right-hand sides.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "far_internal.h"
#include "mfma.h"

namespace tdbem {

static constexpr int P = 4;         // interpolation points per axis and in time
static constexpr int NS = P * P * P;
static constexpr int NN = NS * P;   // 256

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
static constexpr int KTAB = 2401;          // 7^3 spatial differences x 7 time differences
static constexpr int KTAB_MID = 1197;      // table index of a - b = (0, 0, 0), m - n = -3
static constexpr int M2L_THREADS = 512;    // 8 wavefronts: 4 row blocks of 64 x 2 column halves
template <typename T> struct M2lX { static constexpr int XS = NN + (sizeof(T) == 8 ? 2 : 4); };

// operator table of one (offset, lag): tab[((d1 + 3) * 7 + d2 + 3) * 7 + d3 + 3) * 7 + w + 3] =
// kernel at spatial lattice vector d - 3 off and time lattice 3 lag + w.
// kfun 0: dU/dt = 2c (c tau - r)_+ / r; 1: U = (c tau - r)_+^2 / r;
// 2: d^2U/dt^2 = 2c^2 [c tau > r] / r.
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
__device__ void m2l_table(T *tab, const double *rd, const T *ird, int lag, int kfun, double cgt, double c2) {
    for (int e = threadIdx.x; e < KTAB; e += blockDim.x) {
        const int w = e % 7 - 3, d = e / 7;
        const double r = rd[d];
        const double u = cgt * (3 * lag + w) - r;
        double kv = 0.0;
        if (u > 0.0 && r > 0.0)
            kv = (kfun == 0 ? c2 * u : kfun == 1 ? u * u : 0.5 * c2 * c2) * (double)ird[d];
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
                                                         int NV, int k, int W, double hn, double ds, double ht, double cl,
                                                         double *YB, const float *MMf, int kindA, int lag_per,
                                                         size_t gstride) {
    // blockIdx.y: the group of lags 1 + y lag_per .. (y + 1) lag_per of the
    // window, written to its own copy of YB (coarse levels: more blocks)
    const int tile = blockIdx.x;
    const int code = tile_code[tile], kind = tile_kind[tile], col0 = tile_col0[tile], ncol = tile_ncol[tile];
    const int kfun = kind == 0 ? kindA : 1;     // vector-potential channels: the placement's kernel
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
        if (tid < ncol) b = ((int64_t)il_src[col_q[col0 + tid]] * WR * NV * NCH + col_ch[col0 + tid]) * NN;
        cbase[tid] = b;
    }
    const int xr = tid & (NN / 2 - 1), xg = tid >> 7;   // row pair, first column
    const int lag0 = 1 + (int)blockIdx.y * lag_per;
    const int nlag = min(min(W, k + 1), lag0 + lag_per - 1);   // lags whose source interval exists, in the group
    YB += blockIdx.y * gstride;
    // source interval k + 1 - lag; the window's oldest intervals take the
    // variant truncated at the oldest interval's start
    auto var = [&](int lag) { return W - lag < NV - 1 ? W - lag + 1 : 0; };
    auto loff = [&](int lag) {
        return (int64_t)(((k + 1 - lag) % WR) * NV + var(lag)) * NCH * NN + 2 * xr;
    };
    m2l_dist<T>(rd, ird, ox, oy, oz, gs, ds);
    if constexpr (sizeof(T) == 4) {
        // FP32 form: X from the FP32 copy of the moments (the same values the
        // conversion at staging gave), four rows per 16-byte load and store;
        // thread = row quad xq and columns xh, xh + 8, ...
        const int xq = tid & 63, xh = tid >> 6;
        auto loff4 = [&](int lag) {
            return (int64_t)(((k + 1 - lag) % WR) * NV + var(lag)) * NCH * NN + 4 * xq;
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
        fetch4(loff4(lag0));
        for (int lag = lag0; lag <= nlag; ++lag) {
            __syncthreads();                      // the previous products are done with X and tab
#pragma unroll
            for (int i = 0; i < M2L_NT / 8; ++i) *reinterpret_cast<float4 *>(&X[xh + 8 * i][4 * xq]) = p4[i];
            m2l_table<T>(tab, rd, ird, lag, kfun, cgt, 2.0 * cl);
            __syncthreads();
            if (lag < nlag) fetch4(loff4(lag + 1));
            m2l_apply<T>(acc, X, tab, base, wc, lane);
        }
    } else {
        typename M2lPair<T>::type pre[M2L_PRE];
        __syncthreads();                          // cbase, rd and ird visible
        m2l_fetch<T>(pre, cbase, MM, loff(lag0), xg);
        for (int lag = lag0; lag <= nlag; ++lag) {
            __syncthreads();                      // the previous products are done with X and tab
            m2l_store<T>(X, pre, xr, xg);
            m2l_table<T>(tab, rd, ird, lag, kfun, cgt, 2.0 * cl);
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

// target-major M2L for batched right-hand sides: one block per (target, kind,
// (channel, rhs) tile of 64 columns); items are (interaction-list source, lag).
template <typename T>
__global__ void __launch_bounds__(M2L_THREADS, sizeof(T) == 4 ? 4 : 2) k_m2l_tgt(const int *il_off, const int *il_src, const int *il_code,
                                                         const double *MM, int WR, int NV, int k, int W, double hn,
                                                         double ds, double ht, double cl, const double *PEND, double *LC,
                                                         int nrhs, const float *MMf, int kindA) {
    const int O = blockIdx.x, kind = blockIdx.y;
    const int kfun = kind == 0 ? kindA : 1;
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
    const int64_t strideS = (int64_t)WR * NV * NCH * nrhs * NN;
    auto var = [&](int lag) { return W - lag < NV - 1 ? W - lag + 1 : 0; };
    auto loff = [&](int it) {
        const int q = q0 + it / nlag, lag = it % nlag + 1;
        return (int64_t)il_src[q] * strideS +
               (int64_t)(((k + 1 - lag) % WR) * NV + var(lag)) * NCH * nrhs * NN + 2 * xr;
    };
    if constexpr (sizeof(T) == 4) {
        // FP32 form: X from the FP32 copy of the moments, four rows per
        // 16-byte load and store (thread = row quad xq, columns xh + 8 i)
        const int xq = tid & 63, xh = tid >> 6;
        auto loff4 = [&](int it) {
            const int q = q0 + it / nlag, lag = it % nlag + 1;
            return (int64_t)il_src[q] * strideS +
                   (int64_t)(((k + 1 - lag) % WR) * NV + var(lag)) * NCH * nrhs * NN + 4 * xq;
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
            m2l_table<T>(tab, rd, ird, lag, kfun, cgt, 2.0 * cl);
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
            m2l_table<T>(tab, rd, ird, lag, kfun, cgt, 2.0 * cl);
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


// reduced copies of a whole level's moments (P2M and M2M write them as they
// go; this serves a restore, which brings back the FP64 moments only)
__global__ void k_mm_copies(int64_t n, const double *__restrict__ src, float *__restrict__ f32,
                            unsigned short *__restrict__ b16) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float f = (float)src[i];
    if (f32) f32[i] = f;
    if (b16) {
        unsigned u = __float_as_uint(f);
        u += 0x7fffu + ((u >> 16) & 1u);
        b16[i] = (unsigned short)(u >> 16);
    }
}

void mm_copies_refresh(tdbem_ctx *C, FarLevel &FL, hipStream_t s) {
    if (!FL.MM32 && !FL.MM16) return;
    const int64_t nmm = (int64_t)FL.n * FL.WR * FL.NV * NCH * C->nrhs * NN;
    hipLaunchKernelGGL(k_mm_copies, dim3((unsigned)((nmm + 255) / 256)), dim3(256), 0, s, nmm, FL.MM, FL.MM32, FL.MM16);
    TD_HIP(hipGetLastError());
}

template <typename T>
void m2l_p4_launch(tdbem_ctx *C, FarLevel &FL, int k, hipStream_t s) {
    const int nr = C->nrhs;
    const int kindA = m2l_kind_a(C->cfg);
    if (nr == 1) {
        if (FL.ntile > 0) {
            // lag groups: as many as YB holds and the window's lags allow, none empty
            const int nlag = std::min(FL.W, k + 1);
            const int per = (nlag + std::min(FL.yg_max, nlag) - 1) / std::min(FL.yg_max, nlag);
            FL.yg = (nlag + per - 1) / per;
            PhaseScope ps(C->prof, TDBEM_PH_M2L, s);
            hipLaunchKernelGGL(k_m2l_off<T>, dim3(FL.ntile, FL.yg), dim3(M2L_THREADS), 0, s, FL.tile_code,
                               FL.tile_kind, FL.tile_col0, FL.tile_ncol, FL.col_q, FL.col_ch, FL.il_src, FL.MM, FL.WR,
                               FL.NV, k, FL.W, FL.hn, FL.ds, FL.ht, C->c, FL.YB, (const float *)FL.MM32, kindA, per,
                               (size_t)FL.nil * NCH * NN);
        }
    } else {
        PhaseScope ps(C->prof, TDBEM_PH_M2L, s);
        hipLaunchKernelGGL(k_m2l_tgt<T>, dim3(FL.n, 2, (4 * nr + M2L_NT - 1) / M2L_NT), dim3(M2L_THREADS), 0, s,
                           FL.il_off, FL.il_src, FL.il_code, FL.MM, FL.WR, FL.NV, k, FL.W, FL.hn, FL.ds, FL.ht, C->c,
                           FL.PEND, FL.LC, nr, (const float *)FL.MM32, kindA);
    }
    TD_HIP(hipGetLastError());
}
template void m2l_p4_launch<double>(tdbem_ctx *, FarLevel &, int, hipStream_t);
template void m2l_p4_launch<float>(tdbem_ctx *, FarLevel &, int, hipStream_t);

}  // namespace tdbem
