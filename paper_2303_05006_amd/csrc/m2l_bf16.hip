// The BF16 form of the tuned p = 4 M2L (Section 3.6.1): operator and moments
// rounded to bf16, products on the 16x16x32 bf16 matrix-core instruction with
// FP32 accumulation.  Same decomposition as the FP64 / FP32 kernels
// (offset-major for one right-hand side, target-major for batches; 8 waves =
// 4 row blocks of 64 x 2 column halves of 32) with operands laid out for the
// instruction's 8 values per lane:
//   k = 4 b + n (source node b, time node n); lane group g = lane / 16 of a
//   32-wide k chunk holds source nodes 8 kc + 2 g and 8 kc + 2 g + 1.
//   A (operator): the block's table of one (offset, lag) is stored as
//   tb[d][m][n] = K(d, m - n) for the 343 spatial differences d and the 4 x 4
//   time nodes, so a lane's 4 values of one source node are one 8-byte read.
//   B (moments): X[column][k] with k contiguous, one 16-byte read per lane.
// The moments come from a bf16 copy written by P2M / M2M; the local
// expansions accumulate in FP32 per launch and are stored in FP64.
#include <hip/hip_runtime.h>

#include "far_internal.h"
#include "mfma.h"

namespace tdbem {

namespace {
constexpr int P = 4, NN = 256;
constexpr int XSB = NN + 8;                 // bf16 per X column: 16-byte aligned, columns staggered over banks
constexpr int TB = 343 * 16;                // table entries per (offset, lag)
constexpr int THREADS = 512;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
}  // namespace

// FP32 -> bf16 bits, round to nearest even (the operands are finite)
__device__ __forceinline__ unsigned short bf16_bits(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ void bf_dist(double *rd, float *ird, int ox, int oy, int oz, double gs, double ds) {
    for (int d = threadIdx.x; d < 343; d += blockDim.x) {
        const double v1 = gs * (d / 49 - 3) - ds * ox, v2 = gs * ((d / 7) % 7 - 3) - ds * oy,
                     v3 = gs * (d % 7 - 3) - ds * oz;
        const double r = sqrt(v1 * v1 + v2 * v2 + v3 * v3);
        rd[d] = r;
        ird[d] = (float)(r > 0.0 ? 1.0 / r : 0.0);
    }
}

// tb[(d * 4 + m) * 4 + n] = kernel at spatial lattice difference d (index of
// a - b + 3 per axis) and time lattice 3 lag + m - n; kfun as in the FP64 form
__device__ void bf_table(unsigned short *tb, const double *rd, const float *ird, int lag, int kfun, double cgt,
                         double c2) {
    for (int e = threadIdx.x; e < TB; e += blockDim.x) {
        const int d = e >> 4, m = (e >> 2) & 3, n = e & 3;
        const double r = rd[d];
        const double u = cgt * (3 * lag + m - n) - r;
        double kv = 0.0;
        if (u > 0.0 && r > 0.0) kv = (kfun == 0 ? c2 * u : kfun == 1 ? u * u : 0.5 * c2 * c2) * (double)ird[d];
        tb[e] = bf16_bits((float)kv);
    }
}

// spatial lattice index part of source node b: d = abase(a) - bpart(b)
__device__ __forceinline__ int bpart(int b) { return ((b >> 4) * 7 + ((b >> 2) & 3)) * 7 + (b & 3); }

// per lane and row block: table offset of its row (a, m) at b = 0
__device__ __forceinline__ void bf_rows(int (&aoff)[4], int wr, int lane) {
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        const int row = 64 * wr + 16 * rb + (lane & 15);
        const int a = row >> 2, m = row & 3;
        const int abase = (((a >> 4) + 3) * 7 + ((a >> 2) & 3) + 3) * 7 + (a & 3) + 3;
        aoff[rb] = (abase * 4 + m) * 4;
    }
}

// acc (this wave's 64 rows x 32 columns) += K X over the 8 k chunks of 32
__device__ __forceinline__ void bf_apply(v4f (&acc)[4][2], const unsigned short (*X)[XSB], const unsigned short *tb,
                                         const int (&aoff)[4], int wc, int lane) {
    const int g = lane >> 4, col = 32 * wc + (lane & 15);
#pragma unroll
    for (int kc = 0; kc < 8; ++kc) {
        const int b0 = 8 * kc + 2 * g;
        const int o0 = 16 * bpart(b0), o1 = 16 * bpart(b0 + 1);
        const u16x8 x0 = *reinterpret_cast<const u16x8 *>(&X[col][32 * kc + 8 * g]);
        const u16x8 x1 = *reinterpret_cast<const u16x8 *>(&X[col + 16][32 * kc + 8 * g]);
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            const u16x4 lo = *reinterpret_cast<const u16x4 *>(&tb[aoff[rb] - o0]);
            const u16x4 hi = *reinterpret_cast<const u16x4 *>(&tb[aoff[rb] - o1]);
            const u16x8 av = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
            acc[rb][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                                 __builtin_bit_cast(bf16x8, x0), acc[rb][0], 0, 0, 0);
            acc[rb][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                                 __builtin_bit_cast(bf16x8, x1), acc[rb][1], 0, 0, 0);
        }
    }
}

// staging of X: thread t moves 8-value pieces idx = t + 512 i (i < 4) of
// column idx / 32 at offset 8 (idx % 32); coalesced 16-byte loads
__device__ __forceinline__ void bf_fetch(uint4 (&pre)[4], const int64_t *cbase, const unsigned short *MMh, int64_t lo,
                                         int tid) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int idx = tid + THREADS * i, col = idx >> 5, c8 = idx & 31;
        const int64_t b = cbase[col];
        pre[i] = b >= 0 ? *reinterpret_cast<const uint4 *>(MMh + b + lo + 8 * c8) : make_uint4(0, 0, 0, 0);
    }
}
__device__ __forceinline__ void bf_store(unsigned short (*X)[XSB], const uint4 (&pre)[4], int tid) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int idx = tid + THREADS * i;
        *reinterpret_cast<uint4 *>(&X[idx >> 5][8 * (idx & 31)]) = pre[i];
    }
}

// offset-major, one right-hand side: one block per (offset, kind, column tile);
// columns (interaction-list entry q, channel); YB[q][ch][NN] summed over the lags
__global__ void __launch_bounds__(THREADS, 2) k_m2l_off_bf16(const int *tile_code, const int *tile_kind,
                                                             const int *tile_col0, const int *tile_ncol,
                                                             const int *col_q, const int *col_ch, const int *il_src,
                                                             const unsigned short *MMh, int WR, int NV, int k, int W,
                                                             double hn, double ds, double ht, double cl, double *YB,
                                                             int kindA) {
    const int tile = blockIdx.x;
    const int code = tile_code[tile], kind = tile_kind[tile], col0 = tile_col0[tile], ncol = tile_ncol[tile];
    const int kfun = kind == 0 ? kindA : 1;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, wr = wave & 3, wc = wave >> 2;
    __shared__ __attribute__((aligned(16))) unsigned short X[M2L_NT][XSB];
    __shared__ __attribute__((aligned(16))) unsigned short tb[TB];
    __shared__ double rd[343];
    __shared__ float ird[343];
    __shared__ int64_t cbase[M2L_NT];
    int aoff[4];
    bf_rows(aoff, wr, lane);
    v4f acc[4][2];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[rb][0] = acc[rb][1] = v4f{0.f, 0.f, 0.f, 0.f};
    if (tid < M2L_NT)
        cbase[tid] = tid < ncol ? ((int64_t)il_src[col_q[col0 + tid]] * WR * NV * NCH + col_ch[col0 + tid]) * NN : -1;
    const double gs = hn * (2.0 / (P - 1)), cgt = cl * ht * (2.0 / (P - 1));
    bf_dist(rd, ird, code / 49 - 3, (code / 7) % 7 - 3, code % 7 - 3, gs, ds);
    const int nlag = min(W, k + 1);
    auto loff = [&](int lag) {
        const int var = W - lag < NV - 1 ? W - lag + 1 : 0;       // the window's oldest intervals: truncated
        return (int64_t)(((k + 1 - lag) % WR) * NV + var) * NCH * NN;
    };
    uint4 pre[4];
    __syncthreads();                              // cbase, rd and ird visible
    bf_fetch(pre, cbase, MMh, loff(1), tid);
    for (int lag = 1; lag <= nlag; ++lag) {
        __syncthreads();                          // the previous products are done with X and tb
        bf_store(X, pre, tid);
        bf_table(tb, rd, ird, lag, kfun, cgt, 2.0 * cl);
        __syncthreads();
        if (lag < nlag) bf_fetch(pre, cbase, MMh, loff(lag + 1), tid);
        bf_apply(acc, X, tb, aoff, wc, lane);
    }
    for (int rb = 0; rb < 4; ++rb)
        for (int cb = 0; cb < 2; ++cb) {
            const int j = 32 * wc + 16 * cb + (lane & 15);
            if (j >= ncol) continue;
            const int q = col_q[col0 + j], ch = col_ch[col0 + j];
            for (int v = 0; v < 4; ++v) {
                const int row = 64 * wr + 16 * rb + Mma<float>::row(lane, v);
                YB[((size_t)q * NCH + ch) * NN + row] = (double)acc[rb][cb][v];
            }
        }
}

// target-major, batched right-hand sides: one block per (target, kind, tile of
// 64 (channel, rhs) columns); items (interaction-list entry, lag); LC = PEND + sum
__global__ void __launch_bounds__(THREADS, 2) k_m2l_tgt_bf16(const int *il_off, const int *il_src, const int *il_code,
                                                             const unsigned short *MMh, int WR, int NV, int k, int W,
                                                             double hn, double ds, double ht, double cl,
                                                             const double *PEND, double *LC, int nrhs, int kindA) {
    const int O = blockIdx.x, kind = blockIdx.y;
    const int kfun = kind == 0 ? kindA : 1;
    const int c0 = kind == 0 ? 0 : 3, nc = kind == 0 ? 3 : 4;
    const int ncolt = nc * nrhs, col0 = blockIdx.z * M2L_NT;
    if (col0 >= ncolt) return;
    const int ncol = min(M2L_NT, ncolt - col0);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, wr = wave & 3, wc = wave >> 2;
    const int parity = (k + 1) & 1;
    __shared__ __attribute__((aligned(16))) unsigned short X[M2L_NT][XSB];
    __shared__ __attribute__((aligned(16))) unsigned short tb[TB];
    __shared__ double rd[343];
    __shared__ float ird[343];
    __shared__ int64_t cbase[M2L_NT];
    int aoff[4];
    bf_rows(aoff, wr, lane);
    v4f acc[4][2];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[rb][0] = acc[rb][1] = v4f{0.f, 0.f, 0.f, 0.f};
    if (tid < M2L_NT) {
        int64_t b = -1;
        if (tid < ncol) {
            const int cc = (col0 + tid) / nrhs, r = (col0 + tid) % nrhs;
            b = ((int64_t)(c0 + cc) * nrhs + r) * NN;
        }
        cbase[tid] = b;
    }
    const double gs = hn * (2.0 / (P - 1)), cgt = cl * ht * (2.0 / (P - 1));
    const int q0 = il_off[O], nq = il_off[O + 1] - q0;
    const int nlag = min(W, k + 1), nitem = nq * nlag;
    const int64_t strideS = (int64_t)WR * NV * NCH * nrhs * NN;
    auto loff = [&](int it) {
        const int q = q0 + it / nlag, lag = it % nlag + 1;
        const int var = W - lag < NV - 1 ? W - lag + 1 : 0;
        return (int64_t)il_src[q] * strideS + (int64_t)(((k + 1 - lag) % WR) * NV + var) * NCH * nrhs * NN;
    };
    uint4 pre[4];
    __syncthreads();                              // cbase visible
    if (nitem > 0) bf_fetch(pre, cbase, MMh, loff(0), tid);
    for (int it = 0; it < nitem; ++it) {
        const int q = q0 + it / nlag, lag = it % nlag + 1;
        const int code = il_code[q];
        __syncthreads();
        bf_store(X, pre, tid);
        if (lag == 1) {                           // a new source entry: its offset's distances
            bf_dist(rd, ird, code / 49 - 3, (code / 7) % 7 - 3, code % 7 - 3, gs, ds);
            __syncthreads();
        }
        bf_table(tb, rd, ird, lag, kfun, cgt, 2.0 * cl);
        __syncthreads();
        if (it + 1 < nitem) bf_fetch(pre, cbase, MMh, loff(it + 1), tid);
        bf_apply(acc, X, tb, aoff, wc, lane);
    }
    for (int rb = 0; rb < 4; ++rb)
        for (int cb = 0; cb < 2; ++cb) {
            const int j = 32 * wc + 16 * cb + (lane & 15);
            if (j >= ncol) continue;
            const int cc = (col0 + j) / nrhs, r = (col0 + j) % nrhs;
            for (int v = 0; v < 4; ++v) {
                const int row = 64 * wr + 16 * rb + Mma<float>::row(lane, v);
                const size_t o = (((size_t)O * NCH + c0 + cc) * nrhs + r) * NN + row;
                const size_t pe = ((((size_t)O * 2 + parity) * NCH + c0 + cc) * nrhs + r) * NN + row;
                LC[o] = (double)acc[rb][cb][v] + PEND[pe];
            }
        }
}

void m2l_bf16_launch(tdbem_ctx *C, FarLevel &FL, int k, hipStream_t s) {
    const int nr = C->nrhs;
    const int kindA = m2l_kind_a(C->cfg);
    PhaseScope ps(C->prof, TDBEM_PH_M2L, s);
    if (nr == 1) {
        if (FL.ntile > 0)
            hipLaunchKernelGGL(k_m2l_off_bf16, dim3(FL.ntile), dim3(THREADS), 0, s, FL.tile_code, FL.tile_kind,
                               FL.tile_col0, FL.tile_ncol, FL.col_q, FL.col_ch, FL.il_src, FL.MM16, FL.WR, FL.NV, k,
                               FL.W, FL.hn, FL.ds, FL.ht, C->c, FL.YB, kindA);
    } else {
        hipLaunchKernelGGL(k_m2l_tgt_bf16, dim3(FL.n, 2, (4 * nr + M2L_NT - 1) / M2L_NT), dim3(THREADS), 0, s,
                           FL.il_off, FL.il_src, FL.il_code, FL.MM16, FL.WR, FL.NV, k, FL.W, FL.hn, FL.ds, FL.ht, C->c,
                           FL.PEND, FL.LC, nr, kindA);
    }
    TD_HIP(hipGetLastError());
}

}  // namespace tdbem
