// Per-step kernels of the marching-on-in-time loop (Program 1): the near-field
// history sum sum_{g>=2} Zt^(g) J^{alpha-g} (Program 2, Eq. R), the Z0 GMRES
// building blocks (Section 2.5), ring-buffer and boundary permutation helpers.
//
// Layouts: every per-edge state vector is [edge][rhs] (rhs fastest, leaf edge
// order); the current history ring is [edge][slot][rhs] with slot = beta mod R,
// so one pair's lag strip reads consecutive slots of one edge.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>

#include "mfma.h"
#include "tdbem_internal.h"

namespace tdbem {

// ---------------------------------------------------------------- near field
// Jagged-diagonal layout per target row: the row's pairs are sorted by the
// length of their lag strip (longest first) and the l-th coefficient of every
// pair with a strip longer than l is stored contiguously at off_l + p, so the
// lanes of a wavefront read consecutive values at every lag.  nl[row][l] is the
// number of pairs with a strip longer than l; off_l is its prefix sum.
static constexpr int NEAR_LMAX = 512;
static constexpr int NEAR_NU = 2;      // lag steps of 4 lags loaded together per chunk
static constexpr int NEAR_NC = 1;      // 64-pair blocks per chunk

// bf16 storage of near-field coefficients (BF16 form): round to nearest even on
// the way in, exact widening on the way out; the sums stay FP64
struct bf16s {
    unsigned short b;
    bf16s() = default;
    __device__ explicit bf16s(double v) {
        unsigned int u = __float_as_uint((float)v);
        u += 0x7fffu + ((u >> 16) & 1u);
        b = (unsigned short)(u >> 16);
    }
    __device__ explicit operator double() const { return (double)__uint_as_float((unsigned int)b << 16); }
};

__device__ __forceinline__ int near_offsets(const int *nl_row, int L, int lane, int *off) {
    // exclusive prefix sums of nl_row[0..L) into off[], 64 lags per pass
    int carry = 0;
    for (int l0 = 0; l0 < L; l0 += 64) {
        int l = l0 + lane;
        int v = l < L ? nl_row[l] : 0;
        int x = v;
        for (int o = 1; o < 64; o <<= 1) {
            int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (l < L) off[l] = carry + x - v;
        carry += __shfl(x, 63, 64);
    }
    return carry;
}

// Workgroups are dispatched to the 8 XCDs round-robin and each XCD has its own
// L2: map the launch's blocks so that every XCD works on one contiguous range of
// rows (neighbouring rows share their source edges).  The grid is a multiple of
// 8 blocks; returns the virtual block index (>= the real count: no work).
__device__ __forceinline__ unsigned xcd_block() {
    const unsigned per = gridDim.x / 8;
    return (blockIdx.x % 8) * per + blockIdx.x / 8;
}
static unsigned grid8(uint64_t nb) { return (unsigned)((nb + 7) / 8 * 8); }

// One target row of the one-rhs history sum by a wavefront, the currents
// gathered from the ring (off: the wavefront's L lag offsets in LDS).
template <typename VT, typename JT, int NU, int NC>
__device__ __forceinline__ void near_row_gather(int row, int lane, int *off, const int *__restrict__ row_ptr,
                                                const int64_t *__restrict__ row_vbase, const int *__restrict__ nl,
                                                int L, const int *__restrict__ pj, const int *__restrict__ pgl,
                                                const VT *__restrict__ val, const JT *__restrict__ ring,
                                                int ring_mask, int alpha, double *__restrict__ out) {
    // One wavefront per target row.  The row's pairs are taken 64 NC at a time
    // (a chunk): lane l loads the metadata of pairs l, l + 64, ... of the
    // chunk, and the next chunk's metadata is loaded while this one is summed,
    // so no round waits for it.  Within a chunk the lanes are 16 pairs x 4
    // consecutive lags (a current gather touches a short stretch of 16 ring
    // rows, a coefficient load 16 consecutive values of one lag); the 4 NC
    // groups of 16 pairs and NU lag steps of 4 lags are loaded together,
    // 8 NC NU values per lane in flight, before any product is formed.  Longer
    // strips take further rounds of 4 NU lags (the chunk's first pair is its
    // longest: pairs are sorted by strip length).
    constexpr int CH = 64 * NC, NG = 4 * NC;
    near_offsets(nl + (size_t)row * L, L, lane, off);
    const int pb = row_ptr[row], np = row_ptr[row + 1] - pb;
    const VT *v = val + row_vbase[row];
    const int R = ring_mask + 1;
    const int sub = lane & 3, pg = lane >> 2;
    double acc = 0.0;
    int mj[NC], mgl[NC];
#pragma unroll
    for (int h = 0; h < NC; ++h) {
        const int p = 64 * h + lane;
        mj[h] = p < np ? pj[pb + p] : 0;
        mgl[h] = p < np ? pgl[pb + p] : 0;
    }
    for (int c0 = 0; c0 < np; c0 += CH) {
        int nj[NC], ngl[NC];
#pragma unroll
        for (int h = 0; h < NC; ++h) {
            const int p = c0 + CH + 64 * h + lane;
            nj[h] = p < np ? pj[pb + p] : 0;
            ngl[h] = p < np ? pgl[pb + p] : 0;
        }
        const int cnt = min(CH, np - c0);
        const int lmax = __shfl(mgl[0], 0, 64) >> 16;
        const JT *J[NG];
        int bq[NG], len[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const int q = 16 * g + pg;                    // pair of the chunk
            const int j = __shfl(mj[g / 4], q & 63, 64), gl = __shfl(mgl[g / 4], q & 63, 64);
            J[g] = ring + (size_t)j * R;
            bq[g] = alpha - (gl & 0xffff);
            len[g] = q < cnt ? gl >> 16 : 0;
        }
        for (int lb = 0; lb < lmax; lb += 4 * NU) {
            double a[NG][NU], x[NG][NU];
#pragma unroll
            for (int t = 0; t < NU; ++t) {
                const int l = lb + 4 * t + sub;
                const int ol = l < L ? off[l] : 0;
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const bool ok = l < len[g];
                    a[g][t] = ok ? (double)v[ol + c0 + 16 * g + pg] : 0.0;
                    x[g][t] = ok ? (double)J[g][(bq[g] - l) & ring_mask] : 0.0;
                }
            }
#pragma unroll
            for (int t = 0; t < NU; ++t)
#pragma unroll
                for (int g = 0; g < NG; ++g) acc += a[g][t] * x[g][t];
        }
#pragma unroll
        for (int h = 0; h < NC; ++h) {
            mj[h] = nj[h];
            mgl[h] = ngl[h];
        }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) out[row] = acc;
}

template <typename VT, typename JT, int NU, int NC>
__global__ void __launch_bounds__(256, NC == 1 ? 6 : 4) k_near_jds1(int ne, const int *__restrict__ rows,
                                                   const int *__restrict__ row_ptr, const int64_t *__restrict__ row_vbase,
                                                   const int *__restrict__ nl, int L, const int *__restrict__ pj,
                                                   const int *__restrict__ pgl, const VT *__restrict__ val,
                                                   const JT *__restrict__ ring, int ring_mask, int alpha,
                                                   double *__restrict__ out) {
    __shared__ int offs[4][NEAR_LMAX];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int idx = (int)xcd_block() * 4 + wv;
    if (idx >= ne) return;
    const int row = rows ? rows[idx] : idx;      // rows: the listed rows only (ne of them)
    near_row_gather<VT, JT, NU, NC>(row, lane, offs[wv], row_ptr, row_vbase, nl, L, pj, pgl, val, ring, ring_mask,
                                    alpha, out);
}

// Per-leaf form of the one-rhs history sum: every row of a leaf pairs with the
// same source edges (the edges of the leaf's near cells), so a block per
// chunk of a leaf's rows first stages the currents those sources contribute
// (per source the lags its strips reach in this leaf, laid end to end) in LDS
// with coalesced ring-row loads, then sums its rows with the currents read
// from LDS: only the coefficients and one word of metadata per pair stream
// from HBM.  With no current gather left on the vector memory path, the lanes
// are 16 pairs x 4 lags with the pairs fastest, so that each quarter of a
// coefficient load reads 16 consecutive values of one lag (jagged-diagonal
// layout): whole cache lines.  Pair q's strip starts at window offset
// pwl & 0xffff and has pwl >> 16 lags.  Leaves whose window does not fit the
// LDS budget take the row kernel's gathers, in the first blocks of the same
// launch (their rows are listed separately).
#ifndef TDBEM_NEAR_LEAF_THREADS
#define TDBEM_NEAR_LEAF_THREADS 1024
#endif
#ifndef TDBEM_NEAR_LEAF_ROWS
#define TDBEM_NEAR_LEAF_ROWS 64
#endif
#ifndef TDBEM_NEAR_LEAF_KB
#define TDBEM_NEAR_LEAF_KB 144
#endif
#ifndef TDBEM_NEAR_LEAF_SORT
#define TDBEM_NEAR_LEAF_SORT 1
#endif
static constexpr int NEAR_LEAF_THREADS = TDBEM_NEAR_LEAF_THREADS;        // wavefronts sharing one window x 64
static constexpr int NEAR_LEAF_ROWS = TDBEM_NEAR_LEAF_ROWS;              // rows per chunk (a block)
static constexpr size_t NEAR_LEAF_LDS = TDBEM_NEAR_LEAF_KB * 1024;       // window budget in bytes

template <typename VT, typename JT, int NU, int NC>
__global__ void __launch_bounds__(NEAR_LEAF_THREADS) __attribute__((amdgpu_waves_per_eu(4))) k_near_leaf(const int *__restrict__ chunk,
                                                                 const int *__restrict__ leaf_soff,
                                                                 const int4 *__restrict__ ws, int wbytes,
                                                                 const int *__restrict__ row_ptr,
                                                                 const int64_t *__restrict__ row_vbase,
                                                                 const int *__restrict__ nl, int L,
                                                                 const int *__restrict__ pwl, int nrest,
                                                                 const int *__restrict__ rest,
                                                                 const int *__restrict__ pj,
                                                                 const int *__restrict__ pgl,
                                                                 const VT *__restrict__ val, const JT *__restrict__ ring,
                                                                 int ring_mask, int alpha, double *__restrict__ out) {
    // dynamic LDS: the window (wbytes), then each wavefront's L lag offsets.
    // A round takes NC chunks of 64 pairs and NU lag steps of 4 lags: 4 NC NU
    // coefficient loads per lane in flight; the next chunks' words are loaded
    // during this one.
    constexpr int CH = 64 * NC, NG = 4 * NC;
    extern __shared__ __attribute__((aligned(16))) unsigned char near_lds[];
    JT *W = reinterpret_cast<JT *>(near_lds);
    constexpr int WPB = NEAR_LEAF_THREADS / 64;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int *off = reinterpret_cast<int *>(near_lds + wbytes) + wv * L;
    // the first blocks take the rows of the leaves whose window does not fit,
    // a wavefront per row with the currents gathered from the ring (started
    // first: their gathers take longest)
    const int nrb = (nrest + WPB - 1) / WPB;
    if ((int)blockIdx.x < nrb) {
        const int idx = blockIdx.x * WPB + wv;
        if (idx < nrest)
            near_row_gather<VT, JT, NEAR_NU, NEAR_NC>(rest[idx], lane, off, row_ptr, row_vbase, nl, L, pj, pgl, val,
                                                      ring, ring_mask, alpha, out);
        return;
    }
    const int ck = blockIdx.x - nrb;
    const int lf = chunk[3 * ck], ra = chunk[3 * ck + 1], rb = chunk[3 * ck + 2];
    const int s0 = leaf_soff[lf], ns = leaf_soff[lf + 1] - s0;
    const int R = ring_mask + 1;
    {
        // stage: W[o_s + w] = J at slot alpha - a_s - w of source s (ws[s] = edge,
        // a_s, o_s, n_s); 16 lanes per source, SU sources per lane group with
        // all their loads in flight together
        constexpr int SU = 16, NGRP = NEAR_LEAF_THREADS / 16;
        const int grp = threadIdx.x >> 4, k = threadIdx.x & 15;
        for (int sb = grp; sb < ns; sb += NGRP * SU) {
            int4 m[SU];
#pragma unroll
            for (int u = 0; u < SU; ++u) m[u] = sb + NGRP * u < ns ? ws[s0 + sb + NGRP * u] : make_int4(0, 0, 0, 0);
            JT x[SU];
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const JT *q = ring + (size_t)m[u].x * R + ((alpha - m[u].y - k) & ring_mask);
                if constexpr (sizeof(JT) == 8)
                    x[u] = k < m[u].w ? *q : (JT)0;
                else                             // unconditional (in-bounds: edge 0 for an absent source)
                    x[u] = *q;
            }
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                if (k < m[u].w) W[m[u].z + k] = x[u];
                for (int w = k + 16; w < m[u].w; w += 16)        // sources reaching over 16 lags
                    W[m[u].z + w] = ring[(size_t)m[u].x * R + ((alpha - m[u].y - w) & ring_mask)];
            }
        }
    }
    __syncthreads();
    const int pg = lane & 15, sub = lane >> 4;
    for (int row = ra + wv; row < rb; row += WPB) {
        near_offsets(nl + (size_t)row * L, L, lane, off);
        const int pb = row_ptr[row], np = row_ptr[row + 1] - pb;
        const VT *v = val + row_vbase[row];
        double acc = 0.0;
        int mw[NC];
#pragma unroll
        for (int h = 0; h < NC; ++h) mw[h] = 64 * h + lane < np ? pwl[pb + 64 * h + lane] : 0;
        for (int c0 = 0; c0 < np; c0 += CH) {
            int nw[NC];
#pragma unroll
            for (int h = 0; h < NC; ++h) {
                const int p = c0 + CH + 64 * h + lane;
                nw[h] = p < np ? pwl[pb + p] : 0;
            }
            const int cnt = min(CH, np - c0);
            const int lmax = __shfl(mw[0], 0, 64) >> 16;
            int jb[NG], len[NG];
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int q = 16 * g + pg;
                const int w = __shfl(mw[g / 4], q & 63, 64);
                jb[g] = w & 0xffff;
                len[g] = q < cnt ? w >> 16 : 0;
            }
            for (int lb = 0; lb < lmax; lb += 4 * NU) {
                // all loads of the round first, in the stored types, then the products
                VT a[NG][NU];
                JT x[NG][NU];
                if constexpr (sizeof(VT) == 8) {
                    // loads under the lane mask: rounds past every strip of a
                    // group issue none
#pragma unroll
                    for (int t = 0; t < NU; ++t) {
                        const int l = lb + 4 * t + sub;
                        const int ol = l < L ? off[l] : 0;
#pragma unroll
                        for (int g = 0; g < NG; ++g) {
                            const bool ok = l < len[g];
                            a[g][t] = ok ? v[ol + c0 + 16 * g + pg] : VT(0.0);
                            x[g][t] = ok ? W[jb[g] + l] : JT(0.0);
                        }
                    }
#pragma unroll
                    for (int t = 0; t < NU; ++t)
#pragma unroll
                        for (int g = 0; g < NG; ++g) acc += (double)a[g][t] * (double)x[g][t];
                } else {
                    // values widened after the load: under a lane mask the
                    // compiler waits for each load before the next, so these
                    // load unconditionally (in-bounds indexes either way) and
                    // the terms beyond a strip are zeroed in the products
#pragma unroll
                    for (int t = 0; t < NU; ++t) {
                        const int l = lb + 4 * t + sub;
                        const int ol = l < L ? off[l] : 0;
#pragma unroll
                        for (int g = 0; g < NG; ++g) {
                            const bool ok = l < len[g];
                            a[g][t] = v[ok ? ol + c0 + 16 * g + pg : 0];
                            x[g][t] = W[ok ? jb[g] + l : 0];
                        }
                    }
#pragma unroll
                    for (int t = 0; t < NU; ++t)
#pragma unroll
                        for (int g = 0; g < NG; ++g) {
                            const bool ok = lb + 4 * t + sub < len[g];
                            acc = __builtin_fma(ok ? (double)a[g][t] : 0.0, ok ? (double)x[g][t] : 0.0, acc);
                        }
                }
            }
#pragma unroll
            for (int h = 0; h < NC; ++h) mw[h] = nw[h];
        }
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane == 0) out[row] = acc;
    }
}

// Batched right-hand sides on the matrix cores, per leaf: the leaf's rows
// pair with the same sources, so its coefficients form a dense block
// A_L [rows][K_L], column k = (source s, lag gmin + w) with k = s gw + w (zero
// where a pair's strip does not reach), and the history sum is the product
// A_L J_L, J_L [K_L][rhs] the sources' currents at those lags, read from the
// ring ([edge][slot][rhs]: 16 consecutive rhs of one (source, lag) per k).
// One block of 4 wavefronts per (leaf, 64 rhs); wavefront w owns rhs
// 16 w .. 16 w + 15 and the rows in groups of 64 (4 row blocks of 16).
template <typename T>
__global__ void __launch_bounds__(256) k_near_leaf_mm(const int *__restrict__ seg_order,
                                                      const int *__restrict__ seg_leaf, const int *__restrict__ seg_k,
                                                      const int64_t *__restrict__ seg_poff,
                                                      const int *__restrict__ leaf_r0, const int *__restrict__ leaf_r1,
                                                      const int64_t *__restrict__ coff, const int2 *__restrict__ colmap,
                                                      const int64_t *__restrict__ aoff,
                                                      const int *__restrict__ kpad, const T *__restrict__ A,
                                                      const T *__restrict__ ring, int ring_mask, int nrhs, int alpha,
                                                      double *__restrict__ part) {
    // one block per (segment of a leaf's columns, 64 rhs): chunks of KC
    // columns of A (64 rows) and KC rows of J (64 rhs) staged in LDS with
    // coalesced loads, the next chunk's loads in flight during this chunk's
    // products; the segment's partial sums go to part (summed per leaf in a
    // fixed order by k_near_leaf_sum).  Blocks take the segments largest
    // first (seg_order), and skip the products of 16-row blocks past the
    // leaf's rows.
    constexpr int KC = 32, AS = KC + (sizeof(T) == 8 ? 1 : 2), BS = 64 + (sizeof(T) == 8 ? 1 : 2);
    __shared__ T As[64][AS];
    __shared__ T Bs[KC][BS];
    const int sg = seg_order[blockIdx.x], lf = seg_leaf[sg];
    const int kb = seg_k[2 * sg], ke = seg_k[2 * sg + 1];
    const int nr = leaf_r1[lf] - leaf_r0[lf];
    const int KP = kpad[lf];
    const int2 *cm = colmap + coff[lf];    // column k: (source edge, lag) of the leaf's window
    const T *Al = A + aoff[lf];
    double *P = part + seg_poff[sg];
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int c0 = blockIdx.y * 64;
    const int R = ring_mask + 1;
    // staging map: A (64 x KC): thread -> row tid / 4, columns 8 (tid % 4) .. + 7;
    // J (KC x 64): thread -> k tid / 8, rhs 8 (tid % 8) .. + 7
    const int ar = tid >> 2, ac = 8 * (tid & 3);
    const int bk = tid >> 3, bc = 8 * (tid & 7);
    for (int rg = 0; rg < nr; rg += 64) {
        typename Mma<T>::acc_t acc[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) acc[rb] = typename Mma<T>::acc_t{0, 0, 0, 0};
        T pa[8], pb[8];
        auto fetch = [&](int k0) {
            const int row = rg + ar;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + ac + e;
                pa[e] = (row < nr && k < ke) ? Al[(size_t)row * KP + k] : (T)0;
            }
            const int k = k0 + bk;
            const T *jr = nullptr;
            if (k < ke) {
                const int2 c = cm[k];
                jr = ring + ((size_t)c.x * R + ((alpha - c.y) & ring_mask)) * nrhs;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int c = c0 + bc + e;
                pb[e] = (jr && c < nrhs) ? jr[c] : (T)0;
            }
        };
        fetch(kb);
        for (int k0 = kb; k0 < ke; k0 += KC) {
            __syncthreads();                      // the previous chunk's products are done with As, Bs
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                As[ar][ac + e] = pa[e];
                Bs[bk][bc + e] = pb[e];
            }
            __syncthreads();
            if (k0 + KC < ke) fetch(k0 + KC);
#pragma unroll
            for (int ks = 0; ks < KC / 4; ++ks) {
                const int kk = 4 * ks + (lane >> 4);
                const T bv = Bs[kk][16 * wv + (lane & 15)];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
                    if (rg + 16 * rb < nr)       // uniform: row blocks past the leaf's rows add nothing
                        acc[rb] = Mma<T>::op(As[16 * rb + (lane & 15)][kk], bv, acc[rb]);
            }
        }
        const int col = c0 + 16 * wv + (lane & 15);
        if (col < nrhs) {
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = rg + 16 * rb + Mma<T>::row(lane, v);
                    if (row < nr) P[(size_t)row * nrhs + col] = (double)acc[rb][v];
                }
        }
    }
}

// out[row][rhs] = sum over the leaf's column segments, in segment order
__global__ void k_near_leaf_sum(int ne, int nrhs, const int *__restrict__ row_leaf, const int *__restrict__ leaf_r0,
                                const int *__restrict__ leaf_seg, const int64_t *__restrict__ seg_poff,
                                const double *__restrict__ part, double *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)ne * nrhs) return;
    const int row = (int)(t / nrhs), col = (int)(t % nrhs);
    const int lf = row_leaf[row], lr = row - leaf_r0[lf];
    double s = 0.0;
    for (int sg = leaf_seg[lf]; sg < leaf_seg[lf + 1]; ++sg) s += part[seg_poff[sg] + (size_t)lr * nrhs + col];
    out[t] = s;
}

// the dense leaf blocks from the pair-major coefficients: one thread per
// pair, its strip written at (row, source index gw + lag - gmin)
template <typename T>
__global__ void k_leaf_mm_fill(int64_t np, const int *__restrict__ prow, const int *__restrict__ pcol,
                               const int *__restrict__ pgl, const int64_t *__restrict__ psrc,
                               const int *__restrict__ row_leaf, const int *__restrict__ leaf_r0,
                               const int64_t *__restrict__ aoff, const int *__restrict__ kpad,
                               const double *__restrict__ val, T *__restrict__ A) {
    // pair q's strip: columns pcol[q] .. + len - 1 of its row in the leaf's block
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= np) return;
    const int row = prow[q], lf = row_leaf[row];
    const int len = pgl[q] >> 16;
    T *a = A + aoff[lf] + (size_t)(row - leaf_r0[lf]) * kpad[lf] + pcol[q];
    for (int l = 0; l < len; ++l) a[l] = (T)val[psrc[q] + l];
}

void launch_leaf_mm_fill(const tdbem_ctx *C, int64_t np, const int *prow, const int *pcol, const int64_t *psrc,
                         const int *row_leaf, const int64_t *aoff, const int *kpad, const double *val, hipStream_t s) {
    const NearLeaves &NL = C->nleaf;
    const unsigned nb = (unsigned)((np + 255) / 256);
    if (C->d_leafA64)
        hipLaunchKernelGGL(k_leaf_mm_fill<double>, dim3(nb), dim3(256), 0, s, np, prow, pcol, C->d_npair_gl, psrc,
                           row_leaf, NL.d_r0, aoff, kpad, val, C->d_leafA64);
    if (C->d_leafA32)
        hipLaunchKernelGGL(k_leaf_mm_fill<float>, dim3(nb), dim3(256), 0, s, np, prow, pcol, C->d_npair_gl, psrc,
                           row_leaf, NL.d_r0, aoff, kpad, val, C->d_leafA32);
    TD_HIP(hipGetLastError());
}

// batched right-hand sides: one wavefront per (row, group of 64 rhs); lanes are rhs
template <typename VT, typename JT>
__global__ void __launch_bounds__(256) k_near_jdsN(int ne, int nrhs, const int *__restrict__ row_ptr,
                                                   const int64_t *__restrict__ row_vbase, const int *__restrict__ nl, int L,
                                                   const int *__restrict__ pj, const int *__restrict__ pgl,
                                                   const VT *__restrict__ val, const JT *__restrict__ ring, int ring_mask,
                                                   int alpha, double *__restrict__ out) {
    __shared__ int offs[4][NEAR_LMAX];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ngrp = (nrhs + 63) >> 6;
    const int wave = (int)xcd_block() * 4 + wv;
    if (wave >= ne * ngrp) return;
    const int row = wave / ngrp, r = (wave % ngrp) * 64 + lane;
    int *off = offs[wv];
    near_offsets(nl + (size_t)row * L, L, lane, off);
    const bool act = r < nrhs;
    const int pb = row_ptr[row], np = row_ptr[row + 1] - pb;
    const VT *v = val + row_vbase[row];
    const int R = ring_mask + 1;
    double acc = 0.0;
    for (int p = 0; p < np; ++p) {
        const int j = pj[pb + p], gl = pgl[pb + p];
        const int g0 = gl & 0xffff, len = gl >> 16;
        const JT *J = ring + (size_t)j * R * nrhs + (act ? r : 0);
        const int b = alpha - g0;
        for (int l = 0; l < len; ++l) acc += (double)v[off[l] + p] * (double)J[(size_t)((b - l) & ring_mask) * nrhs];
    }
    if (act) out[(size_t)row * nrhs + r] = acc;
}

// scatter the pair-major coefficient strips into the jagged-diagonal layout
template <typename VT>
__global__ void k_near_to_jds(int ne, const int *row_ptr, const int64_t *row_vbase, const int *nl, int L,
                              const int *pgl, const int64_t *src_off, const double *src, VT *dst) {
    __shared__ int offs[4][NEAR_LMAX];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + wv;
    if (row >= ne) return;
    int *off = offs[wv];
    near_offsets(nl + (size_t)row * L, L, lane, off);
    const int pb = row_ptr[row], np = row_ptr[row + 1] - pb;
    VT *d = dst + row_vbase[row];
    for (int p = lane; p < np; p += 64) {
        const int len = pgl[pb + p] >> 16;
        const double *s = src + src_off[pb + p];
        for (int l = 0; l < len; ++l) d[off[l] + p] = (VT)s[l];
    }
}

void launch_near_to_jds(const tdbem_ctx *C, const int64_t *src_off, const double *src, hipStream_t s) {
    unsigned nb = (unsigned)((C->ne + 3) / 4);
    hipLaunchKernelGGL(k_near_to_jds<double>, dim3(nb), dim3(256), 0, s, C->ne, C->d_nrow_ptr, C->d_nrow_vbase,
                       C->d_nl, C->near_L, C->d_npair_gl, src_off, src, C->d_nval);
    if (C->d_nval32)
        hipLaunchKernelGGL(k_near_to_jds<float>, dim3(nb), dim3(256), 0, s, C->ne, C->d_nrow_ptr, C->d_nrow_vbase,
                           C->d_nl, C->near_L, C->d_npair_gl, src_off, src, C->d_nval32);
    if (C->d_nval16)
        hipLaunchKernelGGL(k_near_to_jds<bf16s>, dim3(nb), dim3(256), 0, s, C->ne, C->d_nrow_ptr, C->d_nrow_vbase,
                           C->d_nl, C->near_L, C->d_npair_gl, src_off, src, (bf16s *)C->d_nval16);
    TD_HIP(hipGetLastError());
}

// round shapes of the one-rhs kernel: (lag steps of 4 lags, 64-pair blocks)
// per round; variant 0 is the default (NEAR_NU, NEAR_NC); variants 5 and 6
// are the per-leaf form with 2 and 1 lag steps (pair blocks reported as 0)
static constexpr int NEAR_NVAR = 7;
static constexpr int NEAR_LEAF_MM = 7;    // batched rhs: the per-leaf matrix-core form (near_kernel 8)
static const int near_var_nu[NEAR_NVAR] = {NEAR_NU, 1, 3, 2, 1, 2, 1};
static const int near_var_nc[NEAR_NVAR] = {NEAR_NC, 1, 1, 2, 2, 0, 0};
int near_variants() { return NEAR_NVAR; }
// window budget of a context whose strips reach L lags: the block's LDS
// (160 KB on gfx950) holds the window and each wavefront's L lag offsets
size_t near_leaf_lds_budget(int L) {
    const size_t offs = sizeof(int) * (NEAR_LEAF_THREADS / 64) * (size_t)L + 16;
    return std::min(NEAR_LEAF_LDS, (size_t)160 * 1024 - offs);
}
int near_leaf_rows() { return NEAR_LEAF_ROWS; }
bool near_leaf_sorted() { return TDBEM_NEAR_LEAF_SORT != 0; }
void near_variant_shape(int v, int *nu, int *nc) {
    if (v == NEAR_LEAF_MM) { *nu = 0; *nc = 0; return; }     // the batched matrix-core form
    *nu = near_var_nu[v];
    *nc = near_var_nc[v];
}

template <typename VT, typename JT, int NU, int NC>
static void launch_jds1(const tdbem_ctx *C, const VT *val, const JT *ring, int alpha, double *out, hipStream_t s,
                        int nrows = -1, const int *rows = nullptr) {
    const int n = rows ? nrows : C->ne;
    unsigned nb = grid8((n + 3) / 4);
    hipLaunchKernelGGL((k_near_jds1<VT, JT, NU, NC>), dim3(nb), dim3(256), 0, s, n, rows, C->d_nrow_ptr,
                       C->d_nrow_vbase, C->d_nl, C->near_L, C->d_npair_j, C->d_npair_gl, val, ring, C->ring - 1, alpha,
                       out);
}

template <typename VT, typename JT, int NU, int NC>
static void launch_leaf(const tdbem_ctx *C, const VT *val, const JT *ring, int alpha, double *out, hipStream_t s) {
    const NearLeaves &NL = C->nleaf;
    const int wbytes = (int)((NL.max_window * sizeof(JT) + 15) / 16 * 16);
    const size_t lds = (size_t)wbytes + sizeof(int) * (NEAR_LEAF_THREADS / 64) * (size_t)C->near_L;
    // dynamic LDS above 64 KB needs the kernel's limit raised, per device
    static size_t lds_set[64] = {};
    int dev = 0;
    TD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64 || lds > lds_set[dev]) {
        TD_HIP(hipFuncSetAttribute((const void *)k_near_leaf<VT, JT, NU, NC>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        if (dev >= 0 && dev < 64) lds_set[dev] = lds;
    }
    const int nb = (NL.nrest + NEAR_LEAF_THREADS / 64 - 1) / (NEAR_LEAF_THREADS / 64) + NL.nchunk;
    if (nb > 0)
        hipLaunchKernelGGL((k_near_leaf<VT, JT, NU, NC>), dim3(nb), dim3(NEAR_LEAF_THREADS), lds, s, NL.d_chunk,
                           NL.d_soff, (const int4 *)NL.d_ws, wbytes, C->d_nrow_ptr, C->d_nrow_vbase, C->d_nl,
                           C->near_L, NL.d_pwl, NL.nrest, NL.d_rest, C->d_npair_j, C->d_npair_gl, val, ring,
                           C->ring - 1, alpha, out);
}

template <typename VT, typename JT>
static void launch_near_t(const tdbem_ctx *C, const VT *val, const JT *ring, int alpha, double *out, hipStream_t s) {
    if (C->nrhs == 1) {
        switch (C->near_variant) {
            case 5: launch_leaf<VT, JT, 2, 2>(C, val, ring, alpha, out, s); break;
            case 6: launch_leaf<VT, JT, 1, 2>(C, val, ring, alpha, out, s); break;
            case 1: launch_jds1<VT, JT, 1, 1>(C, val, ring, alpha, out, s); break;
            case 2: launch_jds1<VT, JT, 3, 1>(C, val, ring, alpha, out, s); break;
            case 3: launch_jds1<VT, JT, 2, 2>(C, val, ring, alpha, out, s); break;
            case 4: launch_jds1<VT, JT, 1, 2>(C, val, ring, alpha, out, s); break;
            default: launch_jds1<VT, JT, NEAR_NU, NEAR_NC>(C, val, ring, alpha, out, s); break;
        }
    } else if (C->near_variant == NEAR_LEAF_MM && C->leaf_mm_ready) {
        const NearLeaves &NL = C->nleaf;
        const dim3 grid((unsigned)C->leaf_nseg, (unsigned)((C->nrhs + 63) / 64));
        if constexpr (sizeof(JT) == 8)
            hipLaunchKernelGGL(k_near_leaf_mm<double>, grid, dim3(256), 0, s, C->d_seg_order, C->d_seg_leaf, C->d_seg_k,
                               C->d_seg_poff, NL.d_r0, NL.d_r1, C->d_leaf_coff, (const int2 *)C->d_leaf_colmap, C->d_leaf_aoff,
                               C->d_leaf_kpad, C->d_leafA64, (const double *)ring, C->ring - 1, C->nrhs, alpha,
                               C->d_leaf_part);
        else
            hipLaunchKernelGGL(k_near_leaf_mm<float>, grid, dim3(256), 0, s, C->d_seg_order, C->d_seg_leaf, C->d_seg_k,
                               C->d_seg_poff, NL.d_r0, NL.d_r1, C->d_leaf_coff, (const int2 *)C->d_leaf_colmap, C->d_leaf_aoff,
                               C->d_leaf_kpad, C->d_leafA32, (const float *)ring, C->ring - 1, C->nrhs, alpha,
                               C->d_leaf_part);
        const int64_t n = (int64_t)C->ne * C->nrhs;
        hipLaunchKernelGGL(k_near_leaf_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C->ne, C->nrhs,
                           C->d_row_leaf, NL.d_r0, C->d_leaf_seg, C->d_seg_poff, C->d_leaf_part, out);
    } else {
        int ngrp = (C->nrhs + 63) / 64;
        unsigned nb = grid8(((int64_t)C->ne * ngrp + 3) / 4);
        hipLaunchKernelGGL((k_near_jdsN<VT, JT>), dim3(nb), dim3(256), 0, s, C->ne, C->nrhs, C->d_nrow_ptr,
                           C->d_nrow_vbase, C->d_nl, C->near_L, C->d_npair_j, C->d_npair_gl, val, ring, C->ring - 1,
                           alpha, out);
    }
    TD_HIP(hipGetLastError());
}

void launch_near(const tdbem_ctx *C, int alpha, double *out, double scale, hipStream_t s) {
    (void)scale;
    // the reduced forms read an FP32 copy of the current ring (half the gather traffic)
    if (C->cfg.precision == TDBEM_FP64)
        launch_near_t<double, double>(C, C->d_nval, C->d_Jring, alpha, out, s);
    else if (C->cfg.precision == TDBEM_FP32)
        launch_near_t<float, float>(C, C->d_nval32, C->d_Jring32, alpha, out, s);
    else
        launch_near_t<bf16s, float>(C, (const bf16s *)C->d_nval16, C->d_Jring32, alpha, out, s);
}

// --------------------------------------------------------------- helpers
// canonical [rhs][ne] -> leaf [ne][rhs]
__global__ void k_gather_in(int ne, int nrhs, const int *perm, const double *src, double *dst) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ne) return;
    int e = perm[p];
    for (int r = 0; r < nrhs; ++r) dst[(size_t)p * nrhs + r] = src[(size_t)r * ne + e];
}
// leaf [ne][rhs] -> canonical [rhs][ne]
__global__ void k_scatter_out(int ne, int nrhs, const int *perm, const double *src, double *dst) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ne) return;
    int e = perm[p];
    for (int r = 0; r < nrhs; ++r) dst[(size_t)r * ne + e] = src[(size_t)p * nrhs + r];
}
// word copy (a kernel rather than a copy command, so that it can sit in a
// captured graph like the step's other work)
__global__ void k_copy_words(size_t n, const uint32_t *__restrict__ src, uint32_t *__restrict__ dst) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

void launch_copy_words(const void *src, void *dst, size_t words, hipStream_t s) {
    if (words == 0) return;
    hipLaunchKernelGGL(k_copy_words, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, words,
                       (const uint32_t *)src, (uint32_t *)dst);
    TD_HIP(hipGetLastError());
}

__global__ void k_fill(int64_t n, double v, double *p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// y = a*x + b*y over n values
__global__ void k_axpby(int64_t n, double a, const double *x, double b, double *y) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) y[k] = a * x[k] + b * y[k];
}
// ring slot write: ring[e][slot][r] = x[e][r]
__global__ void k_ring_put(int ne, int nrhs, int R, int slot, const double *x, double *ring, float *ring32) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)ne * nrhs) return;
    int e = (int)(k / nrhs), r = (int)(k % nrhs);
    const size_t q = ((size_t)e * R + slot) * nrhs + r;
    ring[q] = x[k];
    if (ring32) ring32[q] = (float)x[k];
}
// quadratic extrapolation x = 3 J^{a-2} - 3 J^{a-3} + J^{a-4} (zero history before 0)
__global__ void k_extrap(int ne, int nrhs, int R, int alpha, const double *ring, double *x) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)ne * nrhs) return;
    int e = (int)(k / nrhs), r = (int)(k % nrhs);
    const double *J = ring + (size_t)e * R * nrhs + r;
    auto at = [&](int b) { return b < 0 ? 0.0 : J[(size_t)(b & (R - 1)) * nrhs]; };
    x[k] = 3.0 * at(alpha - 2) - 3.0 * at(alpha - 3) + at(alpha - 4);
}

// The step's right-hand side once the near-field sum is in: rhs -= near,
// rhs -= far (this step's far-field potential, IFMM), and the extrapolated
// initial guess x (as k_extrap); one pass for the three
__global__ void k_rhs_finish(int ne, int nrhs, int R, int alpha, const double *__restrict__ near,
                             const double *__restrict__ far, double *__restrict__ rhs, const double *__restrict__ ring,
                             double *__restrict__ x) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)ne * nrhs) return;
    double v = rhs[k] - near[k];
    if (far) v -= far[k];
    rhs[k] = v;
    int e = (int)(k / nrhs), r = (int)(k % nrhs);
    const double *J = ring + (size_t)e * R * nrhs + r;
    auto at = [&](int b) { return b < 0 ? 0.0 : J[(size_t)(b & (R - 1)) * nrhs]; };
    x[k] = 3.0 * at(alpha - 2) - 3.0 * at(alpha - 3) + at(alpha - 4);
}

// After the solve: the ring slot (and its FP32 copy) and, if asked, the
// current in the caller's order (as k_ring_put and k_scatter_out)
__global__ void k_ring_out(int ne, int nrhs, int R, int slot, const double *__restrict__ x, double *__restrict__ ring,
                           float *__restrict__ ring32, const int *__restrict__ perm, double *__restrict__ Jout) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)ne * nrhs) return;
    int e = (int)(k / nrhs), r = (int)(k % nrhs);
    const size_t q = ((size_t)e * R + slot) * nrhs + r;
    const double v = x[k];
    ring[q] = v;
    if (ring32) ring32[q] = (float)v;
    if (Jout) Jout[(size_t)r * ne + perm[e]] = v;
}

void launch_rhs_finish(const tdbem_ctx *C, int alpha, const double *far, hipStream_t s) {
    const int64_t n = (int64_t)C->ne * C->nrhs;
    hipLaunchKernelGGL(k_rhs_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C->ne, C->nrhs, C->ring, alpha, C->d_tmp,
                       far, C->d_rhs, C->d_Jring, C->d_x);
    TD_HIP(hipGetLastError());
}

void launch_ring_out(const tdbem_ctx *C, int slot, double *Jout, hipStream_t s) {
    const int64_t n = (int64_t)C->ne * C->nrhs;
    hipLaunchKernelGGL(k_ring_out, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C->ne, C->nrhs, C->ring, slot, C->d_x,
                       C->d_Jring, C->d_Jring32, C->d_perm, Jout);
    TD_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ GMRES
// y = A x for a CSR matrix, [ne][rhs] vectors; one thread per (row, rhs)
__global__ void k_spmv(int ne, int nrhs, const int *ptr, const int *col, const double *val, const double *x, double *y) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)ne * nrhs) return;
    int i = (int)(k / nrhs), r = (int)(k % nrhs);
    double s = 0.0;
    for (int q = ptr[i]; q < ptr[i + 1]; ++q) s += val[q] * x[(size_t)col[q] * nrhs + r];
    y[k] = s;
}
// y = b - A x
__global__ void k_resid(int ne, int nrhs, const int *ptr, const int *col, const double *val, const double *x,
                        const double *b, double *y) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)ne * nrhs) return;
    int i = (int)(k / nrhs), r = (int)(k % nrhs);
    double s = 0.0;
    for (int q = ptr[i]; q < ptr[i + 1]; ++q) s += val[q] * x[(size_t)col[q] * nrhs + r];
    y[k] = b[k] - s;
}
// y = Dinv .* x (Jacobi)
__global__ void k_scale_rows(int ne, int nrhs, const double *dinv, const double *x, double *y) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)ne * nrhs) return;
    y[k] = dinv[k / nrhs] * x[k];
}
// partial dots: part[blk][m][r] = sum over this block's rows of V_m[e][r] * w[e][r]
// V is nv vectors of size ne*nrhs, contiguous. Deterministic two-stage reduction.
#define DOT_ROWS 256
__global__ void k_mdot_part(int ne, int nrhs, int nv, const double *V, size_t vstride, const double *w, double *part) {
    int blk = blockIdx.x, m = blockIdx.y;
    int e0 = blk * DOT_ROWS;
    __shared__ double sh[256];
    for (int r = 0; r < nrhs; ++r) {
        double s = 0.0;
        for (int e = e0 + threadIdx.x; e < min(ne, e0 + DOT_ROWS); e += blockDim.x)
            s += V[m * vstride + (size_t)e * nrhs + r] * w[(size_t)e * nrhs + r];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int o = blockDim.x / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[((size_t)blk * nv + m) * nrhs + r] = sh[0];
        __syncthreads();
    }
}
__global__ void k_mdot_final(int nblk, int nv, int nrhs, const double *part, double *out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nv * nrhs) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * nv * nrhs + k];
    out[k] = s;
}
// w[e][r] -= sum_m h[m][r] V_m[e][r]
__global__ void k_mupdate(int ne, int nrhs, int nv, const double *V, size_t vstride, const double *h, double *w) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)ne * nrhs) return;
    int r = (int)(k % nrhs);
    double s = w[k];
    for (int m = 0; m < nv; ++m) s -= h[m * nrhs + r] * V[m * vstride + k];
    w[k] = s;
}
// V_out[e][r] = w[e][r] * s[r]
__global__ void k_scale_rhs(int ne, int nrhs, const double *s, const double *w, double *v) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)ne * nrhs) return;
    v[k] = w[k] * s[k % nrhs];
}
// x += Dinv .* (sum_m y[m][r] V_m)
__global__ void k_xupdate(int ne, int nrhs, int nv, const double *V, size_t vstride, const double *y,
                          const double *dinv, double *x) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)ne * nrhs) return;
    int r = (int)(k % nrhs);
    double s = 0.0;
    for (int m = 0; m < nv; ++m) s += y[m * nrhs + r] * V[m * vstride + k];
    x[k] += dinv[k / nrhs] * s;
}

static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_gather_in(const tdbem_ctx *C, const double *src, double *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_in, dim3(nblk(C->ne, 256)), dim3(256), 0, s, C->ne, C->nrhs, C->d_perm, src, dst);
    TD_HIP(hipGetLastError());
}
void launch_scatter_out(const tdbem_ctx *C, const double *src, double *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_out, dim3(nblk(C->ne, 256)), dim3(256), 0, s, C->ne, C->nrhs, C->d_perm, src, dst);
    TD_HIP(hipGetLastError());
}
void launch_fill(int64_t n, double v, double *p, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(nblk(n, 256)), dim3(256), 0, s, n, v, p);
    TD_HIP(hipGetLastError());
}

void launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby, dim3(nblk(n, 256)), dim3(256), 0, s, n, a, x, b, y);
    TD_HIP(hipGetLastError());
}
void launch_ring_put(const tdbem_ctx *C, int slot, const double *x, hipStream_t s) {
    hipLaunchKernelGGL(k_ring_put, dim3(nblk((int64_t)C->ne * C->nrhs, 256)), dim3(256), 0, s, C->ne, C->nrhs, C->ring, slot, x,
                       C->d_Jring, C->d_Jring32);
    TD_HIP(hipGetLastError());
}
// y = Z0 x with 8 lanes per (row, rhs): coalesced reads of each row's entries
__global__ void k_spmv8(int ne, int nrhs, const int *ptr, const int *col, const double *val, const double *x, double *y) {
    const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
    const int sub = threadIdx.x & 7;
    const bool act = g < (int64_t)ne * nrhs;
    double s = 0.0;
    if (act) {
        const int i = (int)(g / nrhs), r = (int)(g % nrhs);
        for (int q = ptr[i] + sub; q < ptr[i + 1]; q += 8) s += val[q] * x[(size_t)col[q] * nrhs + r];
    }
    for (int o = 4; o > 0; o >>= 1) s += __shfl_xor(s, o, 8);
    if (act && sub == 0) y[g] = s;
}
void launch_spmv(const tdbem_ctx *C, const double *x, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_spmv8, dim3(nblk((int64_t)C->ne * C->nrhs * 8, 256)), dim3(256), 0, s, C->ne, C->nrhs,
                       C->d_z0_ptr, C->d_z0_col, C->d_z0_val, x, y);
    TD_HIP(hipGetLastError());
}
void launch_extrap(const tdbem_ctx *C, int alpha, double *x, hipStream_t s) {
    hipLaunchKernelGGL(k_extrap, dim3(nblk((int64_t)C->ne * C->nrhs, 256)), dim3(256), 0, s, C->ne, C->nrhs, C->ring, alpha, C->d_Jring, x);
    TD_HIP(hipGetLastError());
}

// Right-preconditioned (Jacobi) restarted GMRES on Z0 for every rhs in
// lockstep; Arnoldi with classical Gram-Schmidt applied twice; Givens
// rotations on the host.  Returns iterations used; sets *ok if every rhs
// reached rtol relative to its right-hand-side norm.
int gmres_solve(tdbem_ctx *C, const double *b, double *x, double rtol, int maxit, bool *ok, hipStream_t s) {
    const int ne = C->ne, nr = C->nrhs;
    const int64_t n = (int64_t)ne * nr;
    const int m = std::max(1, std::min(maxit, C->cfg.gmres_restart));
    double *V = C->d_work;                       // (m+1) vectors
    size_t vs = (size_t)n;
    double *w = V + (size_t)(m + 1) * vs;
    double *z = w + vs;
    double *part = z + vs;                       // [nblk][m+1][nr]
    double *dots = C->d_scal;                    // [(m+1) nr]
    int nb = (ne + DOT_ROWS - 1) / DOT_ROWS;
    unsigned g = nblk(n, 256);
    std::vector<double> hd((size_t)(m + 1) * nr), bn(nr), beta(nr);
    std::vector<double> H((size_t)(m + 1) * m * nr), cs((size_t)m * nr), sn((size_t)m * nr), gv((size_t)(m + 1) * nr);
    auto mdot = [&](int nv, const double *Vb, const double *ww, double *host) {
        hipLaunchKernelGGL(k_mdot_part, dim3(nb, nv), dim3(256), 0, s, ne, nr, nv, Vb, vs, ww, part);
        hipLaunchKernelGGL(k_mdot_final, dim3(nblk(nv * nr, 256)), dim3(256), 0, s, nb, nv, nr, part, dots);
        TD_HIP(hipMemcpyAsync(host, dots, sizeof(double) * nv * nr, hipMemcpyDeviceToHost, s));
        TD_HIP(hipStreamSynchronize(s));
    };
    mdot(1, b, b, bn.data());
    for (int r = 0; r < nr; ++r) bn[r] = std::sqrt(bn[r]);
    int total = 0;
    bool conv = false;
    while (total < maxit) {
        hipLaunchKernelGGL(k_resid, dim3(g), dim3(256), 0, s, ne, nr, C->d_z0_ptr, C->d_z0_col, C->d_z0_val, x, b, V);
        mdot(1, V, V, beta.data());
        bool all = true;
        for (int r = 0; r < nr; ++r) {
            beta[r] = std::sqrt(beta[r]);
            if (!(beta[r] <= rtol * bn[r] || bn[r] == 0.0)) all = false;
        }
        if (C->trace) {
            fprintf(stderr, "gmres alpha=%d total=%d:", C->alpha, total);
            for (int r = 0; r < nr; ++r) fprintf(stderr, " %.3e/%.3e", beta[r], bn[r]);
            fprintf(stderr, "\n");
        }
        if (all) { conv = true; break; }
        // per-rhs Arnoldi length: a right-hand side stops contributing columns
        // once its residual estimate meets the tolerance (or is already met)
        std::vector<int> kr(nr, -1);
        std::vector<double> inv(nr);
        for (int r = 0; r < nr; ++r) {
            bool done = beta[r] <= rtol * bn[r] || bn[r] == 0.0;
            inv[r] = (!done && beta[r] > 0) ? 1.0 / beta[r] : 0.0;
            if (done) kr[r] = 0;
        }
        TD_HIP(hipMemcpyAsync(dots, inv.data(), sizeof(double) * nr, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_scale_rhs, dim3(g), dim3(256), 0, s, ne, nr, dots, V, V);
        std::fill(gv.begin(), gv.end(), 0.0);
        for (int r = 0; r < nr; ++r) gv[r] = kr[r] == 0 ? 0.0 : beta[r];
        int k = 0;
        for (; k < m && total < maxit; ++k, ++total) {
            hipLaunchKernelGGL(k_scale_rows, dim3(g), dim3(256), 0, s, ne, nr, C->d_z0_dinv, V + k * vs, z);
            hipLaunchKernelGGL(k_spmv, dim3(g), dim3(256), 0, s, ne, nr, C->d_z0_ptr, C->d_z0_col, C->d_z0_val, z, w);
            std::vector<double> hsum((size_t)(k + 1) * nr, 0.0);
            std::vector<double> wn0(nr);
            mdot(1, w, w, wn0.data());
            for (int pass = 0; pass < 2; ++pass) {
                mdot(k + 1, V, w, hd.data());
                TD_HIP(hipMemcpyAsync(dots, hd.data(), sizeof(double) * (k + 1) * nr, hipMemcpyHostToDevice, s));
                hipLaunchKernelGGL(k_mupdate, dim3(g), dim3(256), 0, s, ne, nr, k + 1, V, vs, dots, w);
                for (size_t q = 0; q < (size_t)(k + 1) * nr; ++q) hsum[q] += hd[q];
            }
            std::vector<double> hn(nr);
            mdot(1, w, w, hn.data());
            std::vector<double> inv2(nr);
            for (int r = 0; r < nr; ++r) {
                hn[r] = std::sqrt(hn[r]);
                // frozen rhs, or an exact (happy) breakdown: no further direction
                bool stop = kr[r] >= 0 || hn[r] <= 1e-15 * std::sqrt(wn0[r]);
                inv2[r] = (!stop && hn[r] > 0) ? 1.0 / hn[r] : 0.0;
                if (stop && kr[r] < 0) hn[r] = 0.0;
            }
            TD_HIP(hipMemcpyAsync(dots, inv2.data(), sizeof(double) * nr, hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_scale_rhs, dim3(g), dim3(256), 0, s, ne, nr, dots, w, V + (k + 1) * vs);
            bool all2 = true;
            for (int r = 0; r < nr; ++r) {
                if (kr[r] >= 0) continue;
                double *Hc = &H[((size_t)r * (m + 1)) * m];   // column-major (m+1) x m per rhs
                for (int q = 0; q <= k; ++q) Hc[q + (size_t)k * (m + 1)] = hsum[(size_t)q * nr + r];
                Hc[k + 1 + (size_t)k * (m + 1)] = hn[r];
                for (int q = 0; q < k; ++q) {
                    double a = Hc[q + (size_t)k * (m + 1)], bb = Hc[q + 1 + (size_t)k * (m + 1)];
                    double c = cs[(size_t)r * m + q], sgn = sn[(size_t)r * m + q];
                    Hc[q + (size_t)k * (m + 1)] = c * a + sgn * bb;
                    Hc[q + 1 + (size_t)k * (m + 1)] = -sgn * a + c * bb;
                }
                double a = Hc[k + (size_t)k * (m + 1)], bb = Hc[k + 1 + (size_t)k * (m + 1)];
                double rr = std::hypot(a, bb);
                double c = rr > 0 ? a / rr : 1.0, sgn = rr > 0 ? bb / rr : 0.0;
                cs[(size_t)r * m + k] = c; sn[(size_t)r * m + k] = sgn;
                Hc[k + (size_t)k * (m + 1)] = rr;
                Hc[k + 1 + (size_t)k * (m + 1)] = 0.0;
                double gk = gv[(size_t)k * nr + r];
                gv[(size_t)k * nr + r] = c * gk;
                gv[(size_t)(k + 1) * nr + r] = -sgn * gk;
                if (std::fabs(gv[(size_t)(k + 1) * nr + r]) <= rtol * bn[r] || hn[r] == 0.0) kr[r] = k + 1;
                else all2 = false;
            }
            if (all2) { ++k; ++total; break; }
        }
        // y = H^{-1} g (upper triangular kr x kr per rhs), x += Dinv V y
        std::vector<double> y((size_t)k * nr, 0.0);
        for (int r = 0; r < nr; ++r) {
            int kk = kr[r] >= 0 ? kr[r] : k;
            double *Hc = &H[((size_t)r * (m + 1)) * m];
            for (int q = kk - 1; q >= 0; --q) {
                double sacc = gv[(size_t)q * nr + r];
                for (int t = q + 1; t < kk; ++t) sacc -= Hc[q + (size_t)t * (m + 1)] * y[(size_t)t * nr + r];
                double dgn = Hc[q + (size_t)q * (m + 1)];
                y[(size_t)q * nr + r] = dgn != 0.0 ? sacc / dgn : 0.0;
            }
        }
        TD_HIP(hipMemcpyAsync(dots, y.data(), sizeof(double) * k * nr, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_xupdate, dim3(g), dim3(256), 0, s, ne, nr, k, V, vs, dots, C->d_z0_dinv, x);
        TD_HIP(hipGetLastError());
    }
    if (!conv) {
        // final residual check after the last restart cycle
        hipLaunchKernelGGL(k_resid, dim3(g), dim3(256), 0, s, ne, nr, C->d_z0_ptr, C->d_z0_col, C->d_z0_val, x, b, V);
        mdot(1, V, V, beta.data());
        conv = true;
        for (int r = 0; r < nr; ++r)
            if (!(std::sqrt(beta[r]) <= rtol * bn[r] * 1.0000001 || bn[r] == 0.0)) conv = false;
    }
    *ok = conv;
    return total;
}

size_t gmres_work_doubles(const tdbem_ctx *C, int restart) {
    const int m = std::max(1, std::min(restart, 32));
    size_t n = (size_t)C->ne * C->nrhs;
    int nb = (C->ne + DOT_ROWS - 1) / DOT_ROWS;
    return (size_t)(m + 3) * n + (size_t)nb * (m + 1) * C->nrhs + 64;
}

}  // namespace tdbem

namespace tdbem {

// out[2 r + slot] = sum_e x[e][r]^2: one block per right-hand side, fixed
// reduction order (the stability monitor's norms)
__global__ void __launch_bounds__(256) k_colnorm2(int ne, int nrhs, const double *__restrict__ x, double *out, int slot) {
    const int r = blockIdx.x;
    __shared__ double part[4];
    double s = 0.0;
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        const double v = x[(size_t)e * nrhs + r];
        s += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[2 * r + slot] = (part[0] + part[1]) + (part[2] + part[3]);
}

void launch_colnorm2(const tdbem_ctx *C, const double *x, double *out, int slot, hipStream_t s) {
    hipLaunchKernelGGL(k_colnorm2, dim3(C->nrhs), dim3(256), 0, s, C->ne, C->nrhs, x, out, slot);
    TD_HIP(hipGetLastError());
}

}  // namespace tdbem
