// Device-resident restarted GMRES for Z0 x = b, Section 2.5.
//
// One cooperative launch runs whole solves: right Jacobi preconditioning,
// Arnoldi with classical Gram-Schmidt and the DGKS second pass, Givens
// rotations and the restart logic.  blockIdx.y selects an independent system (one right-hand
// side, its vectors contiguous); the gridDim.x blocks of a system split its
// rows.  Grid-wide barriers among a system's blocks separate the phases that
// read other blocks' rows (SpMV) or other blocks' partial sums (dot products).
// Partial sums are written per block and every block reduces them in the same
// fixed order, so all blocks of a system hold bitwise-identical scalars and
// take identical branches: every barrier is reached by every block, and the
// loop trip counts are bounded by the iteration cap.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "tdbem_internal.h"


namespace tdbem {

static constexpr int GM_MAXV = 33;      // Krylov vectors per restart cycle (m + 1) plus one self product
static constexpr int GM_THREADS = 1024;
static constexpr int GM_MAXBLK = 256;   // blocks of the cooperative solve at most

struct GmresArgs {
    int ne, m, maxit;
    double rtol;
    const int *ptr, *col;
    const double *val, *dinv;
    const double *vald;   // Z0 with columns scaled by dinv (right Jacobi preconditioner folded in)
    const double *b;
    double *x;
    double *V;        // [(m+1)][ne]
    double *w0, *w1;  // ping-pong work vectors [ne]
    double *part;     // [2][nblk][GM_MAXV]
    int *out;         // [0] iterations, [1] converged, [2] a barrier wait timed out
    unsigned *bar;    // barrier words (device memory, counters zero between launches)
    // per-system strides for blockIdx.y: b and x advance by ne, V (and the
    // w0, w1, part behind it) by sys_ws doubles, out by 4, bar by GMRES_BAR_WORDS
    size_t sys_ws;
};

// Grid barrier of the cooperative launch (every block is resident): one
// arrival counter and a generation word at device scope, each in a 4 KB page of
// its own (bar[0] and bar[GM_BAR_SLOT]), so that the arrivals do not queue
// behind the polling of the generation (measured: a tenth of the solve time
// against both words in one cache line; a two-level arrival tree or one
// generation copy per XCD group were slower).  The last block to arrive resets
// the counter and advances the generation; the others wait for the generation
// to change.  The wait is bounded: after about a second it gives up and flags
// out[2], so the kernel always completes (the host then reports the failure).
// Only thread 0 of a block touches the words.
static constexpr int GM_BAR_SLOT = 1024;
static_assert(2 * GM_BAR_SLOT <= GMRES_BAR_WORDS, "barrier words per system");

__device__ __forceinline__ void grid_barrier(const GmresArgs &A) {
    __syncthreads();
    if (gridDim.x == 1) return;       // a one-block system: the block barrier suffices
    if (threadIdx.x == 0) {
        __threadfence();
        unsigned *cnt = A.bar, *gen = A.bar + GM_BAR_SLOT;
        const unsigned g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__hip_atomic_fetch_add(cnt, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1) {
            __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > (1u << 24)) {
                    A.out[2] = 1;
                    break;
                }
            }
        }
        __threadfence();
    }
    __syncthreads();
}

// per-thread partial sums of <V_j, w> for j < nv over this block's rows,
// reduced over the block into part[round parity][blk][j].  The two buffers
// alternate by round: a block reaches round r+2 only after every block has
// passed the barrier of round r+1, i.e. finished reading round r.
__device__ void block_dots(const GmresArgs &A, int rnd, int nv, const double *Vb, size_t vs, const double *w, int r0,
                           int r1, double *red, bool self = false) {
    double *part = A.part + (size_t)(rnd & 1) * gridDim.x * GM_MAXV;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ntot = nv + (self ? 1 : 0);
    for (int j = 0; j < ntot; ++j) {
        double v = 0.0;
        const double *Vj = j < nv ? Vb + (size_t)j * vs : w;
        for (int i = r0 + (int)threadIdx.x; i < r1; i += GM_THREADS) v += Vj[i] * w[i];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[wave * GM_MAXV + j] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < ntot) {
        double s = 0.0;
        for (int wv = 0; wv < GM_THREADS / 64; ++wv) s += red[wv * GM_MAXV + threadIdx.x];
        part[(size_t)blockIdx.x * GM_MAXV + threadIdx.x] = s;
    }
    __syncthreads();
}

// sum of the per-block partials with a fixed tree (identical in every block):
// thread (j, b) loads part[b][j], then 64-lane groups reduce over b
__device__ void grid_reduce(const GmresArgs &A, int rnd, int nv, double *dst) {
    const double *part = A.part + (size_t)(rnd & 1) * gridDim.x * GM_MAXV;
    const int nb = gridDim.x;                       // <= GM_MAXBLK (launch-checked)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = wave; j < nv; j += GM_THREADS / 64) {
        double v = 0.0;
        for (int b = lane; b < nb; b += 64) v += part[(size_t)b * GM_MAXV + j];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) dst[j] = v;
    }
    __syncthreads();
}

// y_i = sum_q a_q v[col_q] for the block's rows, 32 lanes per row (lane l takes
// entries l, l + 32, ... of the row), shuffle reduction within the half-wave.
// The first 32 entries of GM_GU rows per half-wave are loaded without a loop, so
// that all their loads are in flight together; longer rows finish in a loop.
// mode: y = b - A v if b is given, else y = vscale * A v
static constexpr int GM_GU = 4;
__device__ void block_spmv(const int *ptr, const int *col, const double *a, const double *v, double vscale,
                           const double *b, double *y, int r0, int r1) {
    const int hl = threadIdx.x & 31, hw = threadIdx.x >> 5;
    const int NH = GM_THREADS / 32;
    for (int i0 = r0; i0 < r1; i0 += GM_GU * NH) {
        int ii[GM_GU], q0[GM_GU], q1[GM_GU], cq[GM_GU];
        double aq[GM_GU], s[GM_GU];
#pragma unroll
        for (int u = 0; u < GM_GU; ++u) {
            ii[u] = i0 + u * NH + hw;
            const bool ok = ii[u] < r1;
            q0[u] = ok ? ptr[ii[u]] : 0;
            q1[u] = ok ? ptr[ii[u] + 1] : 0;
        }
#pragma unroll
        for (int u = 0; u < GM_GU; ++u) {
            const int q = q0[u] + hl;
            const bool ok = q < q1[u];
            cq[u] = ok ? col[q] : -1;
            aq[u] = ok ? a[q] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < GM_GU; ++u) s[u] = cq[u] >= 0 ? aq[u] * v[cq[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < GM_GU; ++u)
            for (int q = q0[u] + 32 + hl; q < q1[u]; q += 32) s[u] += a[q] * v[col[q]];
#pragma unroll
        for (int u = 0; u < GM_GU; ++u) {
            for (int o = 16; o > 0; o >>= 1) s[u] += __shfl_xor(s[u], o, 32);
            if (hl == 0 && ii[u] < r1) y[ii[u]] = b ? b[ii[u]] - s[u] : s[u] * vscale;
        }
    }
}

// The preconditioned operator's rows of a block kept in LDS for the whole
// solve: half-wave hw owns rows r0 + hw + 32 u (u < nu <= GM_RU), lane l the
// row's entry l, column at rc[u][thread] (-1: none) and value at ra[u][thread].
// Rows with more than 32 entries have bit u set in the lane's `tail` mask and
// read the rest from memory.  Used when the block has at most 32 GM_RU rows.
static constexpr int GM_RU = 12;
static constexpr int GM_RC = 4;     // slots per chunk: gathers of a chunk in flight together
static_assert(GM_RU % GM_RC == 0, "chunks tile the slots");

__device__ __forceinline__ unsigned load_lds_rows(int *rc, double *ra, const int *ptr, const int *col, const double *a,
                                                  int r0, int r1) {
    const int hl = threadIdx.x & 31, hw = threadIdx.x >> 5;
    unsigned tail = 0;
    for (int u = 0; u < GM_RU; ++u) {
        const int i = r0 + hw + 32 * u;
        int q0 = 0, q1 = 0;
        if (i < r1) { q0 = ptr[i]; q1 = ptr[i + 1]; }
        const int q = q0 + hl;
        rc[u * GM_THREADS + threadIdx.x] = q < q1 ? col[q] : -1;
        ra[u * GM_THREADS + threadIdx.x] = q < q1 ? a[q] : 0.0;
        if (q1 - q0 > 32) tail |= 1u << u;
    }
    return tail;
}

// y_i = vscale * sum_q a_q v[col_q] with the rows in LDS (nu slots in use)
__device__ __forceinline__ void block_spmv_lds(const int *rc, const double *ra, unsigned tail, int nu,
                                               const int *ptr, const int *col, const double *a, const double *v,
                                               double vscale, double *y, int r0, int r1) {
    const int hl = threadIdx.x & 31, hw = threadIdx.x >> 5;
    for (int u0 = 0; u0 < nu; u0 += GM_RC) {
        int c[GM_RC];
        double s[GM_RC];
#pragma unroll
        for (int u = 0; u < GM_RC; ++u) c[u] = rc[(u0 + u) * GM_THREADS + threadIdx.x];
#pragma unroll
        for (int u = 0; u < GM_RC; ++u) s[u] = c[u] >= 0 ? v[c[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < GM_RC; ++u) s[u] *= ra[(u0 + u) * GM_THREADS + threadIdx.x];
        if ((tail >> u0) & ((1u << GM_RC) - 1u)) {
#pragma unroll
            for (int u = 0; u < GM_RC; ++u) {
                if (!((tail >> (u0 + u)) & 1u)) continue;
                const int i = r0 + hw + 32 * (u0 + u);
                const int q1 = ptr[i + 1];
                double t = 0.0;
                for (int q = ptr[i] + 32 + hl; q < q1; q += 32) t += a[q] * v[col[q]];
                s[u] += t;
            }
        }
#pragma unroll
        for (int u = 0; u < GM_RC; ++u) {
            for (int o = 16; o > 0; o >>= 1) s[u] += __shfl_xor(s[u], o, 32);
            const int i = r0 + hw + 32 * (u0 + u);
            if (hl == 0 && i < r1) y[i] = s[u] * vscale;
        }
    }
}

__global__ void __launch_bounds__(GM_THREADS) k_gmres_coop(GmresArgs Ain) {
    GmresArgs A = Ain;
    {
        const size_t sys = blockIdx.y;
        A.b += sys * (size_t)A.ne;
        A.x += sys * (size_t)A.ne;
        A.V += sys * A.sys_ws;
        A.w0 += sys * A.sys_ws;
        A.w1 += sys * A.sys_ws;
        A.part += sys * A.sys_ws;
        A.out += 4 * sys;
        A.bar += (size_t)GMRES_BAR_WORDS * sys;
    }
    __shared__ double red[(GM_THREADS / 64) * GM_MAXV];
    __shared__ double h1[GM_MAXV], h2[GM_MAXV], sc[4];
    __shared__ double H[GM_MAXV * GM_MAXV], cs[GM_MAXV], sn[GM_MAXV], gv[GM_MAXV + 1], y[GM_MAXV];
    const int ne = A.ne, m = A.m;
    const int nb = gridDim.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) A.out[2] = 0;
    const int r0 = (int)((int64_t)ne * blockIdx.x / nb), r1 = (int)((int64_t)ne * (blockIdx.x + 1) / nb);
    const size_t vs = (size_t)ne;
    const bool on_chip = r1 - r0 <= 32 * GM_RU;   // block-uniform: rows held in LDS
    const int nu = (r1 - r0 + 31) / 32;
    __shared__ int rc[GM_RU * GM_THREADS];
    __shared__ double ra[GM_RU * GM_THREADS];
    const unsigned tail = on_chip ? load_lds_rows(rc, ra, A.ptr, A.col, A.vald, r0, r1) : 0u;
    int rnd = 0;
    // ||b||
    block_dots(A, rnd, 1, A.b, vs, A.b, r0, r1, red);
    grid_barrier(A);
    grid_reduce(A, rnd++, 1, sc);
    const double bn = sqrt(sc[0]);
    int total = 0;
    bool conv = false;
    while (true) {
        // r0 = b - A x  -> V_0 (own rows), its norm
        block_spmv(A.ptr, A.col, A.val, A.x, 1.0, A.b, A.V, r0, r1);
        __syncthreads();
        block_dots(A, rnd, 1, A.V, vs, A.V, r0, r1, red);
        grid_barrier(A);
        grid_reduce(A, rnd++, 1, sc);
        const double beta = sqrt(sc[0]);
        if (beta <= A.rtol * bn || bn == 0.0) { conv = true; break; }
        if (total >= A.maxit) break;
        const double ib = 1.0 / beta;
        for (int i = r0 + (int)threadIdx.x; i < r1; i += GM_THREADS) A.V[i] *= ib;
        if (threadIdx.x == 0) {
            for (int q = 0; q <= m; ++q) gv[q] = 0.0;
            gv[0] = beta;
        }
        grid_barrier(A);   // V_0 complete before any block's SpMV
        int k = 0, kused = 0;
        double hscale = 1.0;            // 1/h_{k,k-1}: V_k = w_prev * hscale
        double *wprev = nullptr;
        for (; k < m && total < A.maxit; ++k) {
            ++total;
            // every block's rows of the previous w are final (the Gram-Schmidt
            // update of iteration k-1 follows that iteration's last barrier)
            if (k > 0) grid_barrier(A);
            double *w = (k & 1) ? A.w1 : A.w0;
            // w = A Dinv V_k, with V_k = wprev * hscale for k >= 1 (rows of other blocks)
            if (k == 0) {
                if (on_chip) block_spmv_lds(rc, ra, tail, nu, A.ptr, A.col, A.vald, A.V, 1.0, w, r0, r1);
                else block_spmv(A.ptr, A.col, A.vald, A.V, 1.0, nullptr, w, r0, r1);
            } else {
                if (on_chip) block_spmv_lds(rc, ra, tail, nu, A.ptr, A.col, A.vald, wprev, hscale, w, r0, r1);
                else block_spmv(A.ptr, A.col, A.vald, wprev, hscale, nullptr, w, r0, r1);
            }
            __syncthreads();
            // The scaled operator has a unit diagonal, A Dinv = I + E: Arnoldi runs
            // on E (w = E V_k, the same Krylov space) and the identity returns as
            // the 1 on the Hessenberg diagonal below.  E V_k has no large part
            // along V_k, so the Gram-Schmidt pass seldom cancels and the second
            // (DGKS) pass and its barrier are rarely needed.
            for (int i = r0 + (int)threadIdx.x; i < r1; i += GM_THREADS) {
                const double vk = k == 0 ? A.V[i] : wprev[i] * hscale;
                if (k > 0) A.V[(size_t)k * vs + i] = vk;
                w[i] -= vk;
            }
            __syncthreads();
            // Gram-Schmidt with the norm in the same reduction: h = V^T w and |w|^2;
            // |w - V h|^2 = |w|^2 - |h|^2 unless cancellation (DGKS criterion
            // |w - V h|^2 < |w|^2 / 2), in which case a second pass is made.
            // (A looser threshold, a second pass only below 1e-4 |w|^2, let the
            // least-squares residual estimate drift from the true residual at
            // rtol 1e-12: 30 to 100 iterations per step where 11 to 13 suffice.)
            block_dots(A, rnd, k + 1, A.V, vs, w, r0, r1, red, true);
            grid_barrier(A);
            grid_reduce(A, rnd++, k + 2, h1);
            for (int i = r0 + (int)threadIdx.x; i < r1; i += GM_THREADS) {
                double s = w[i];
                for (int j = 0; j <= k; ++j) s -= h1[j] * A.V[(size_t)j * vs + i];
                w[i] = s;
            }
            if (threadIdx.x == 0) {
                double hh = 0.0;
                for (int j = 0; j <= k; ++j) hh += h1[j] * h1[j];
                double ww = h1[k + 1];
                sc[0] = ww - hh;
                sc[3] = (ww - hh < 0.5 * ww) ? 1.0 : 0.0;
                for (int j = 0; j <= k; ++j) h2[j] = 0.0;
            }
            __syncthreads();
            if (sc[3] != 0.0) {
                block_dots(A, rnd, k + 1, A.V, vs, w, r0, r1, red, true);
                grid_barrier(A);
                grid_reduce(A, rnd++, k + 2, h2);
                for (int i = r0 + (int)threadIdx.x; i < r1; i += GM_THREADS) {
                    double s = w[i];
                    for (int j = 0; j <= k; ++j) s -= h2[j] * A.V[(size_t)j * vs + i];
                    w[i] = s;
                }
                if (threadIdx.x == 0) {
                    double hh = 0.0;
                    for (int j = 0; j <= k; ++j) hh += h2[j] * h2[j];
                    sc[0] = h2[k + 1] - hh;
                }
                __syncthreads();
            }
            if (threadIdx.x == 0 && sc[0] < 0.0) sc[0] = 0.0;
            __syncthreads();
            // Hessenberg column, rotations (every block, identically)
            if (threadIdx.x == 0) {
                double hn = sqrt(sc[0]);
                for (int q = 0; q <= k; ++q) H[q * GM_MAXV + k] = h1[q] + h2[q] + (q == k ? 1.0 : 0.0);
                double hk1 = hn;
                for (int q = 0; q < k; ++q) {
                    double a = H[q * GM_MAXV + k], bb = H[(q + 1) * GM_MAXV + k];
                    H[q * GM_MAXV + k] = cs[q] * a + sn[q] * bb;
                    H[(q + 1) * GM_MAXV + k] = -sn[q] * a + cs[q] * bb;
                }
                double a = H[k * GM_MAXV + k];
                double rr = sqrt(a * a + hk1 * hk1);
                double c = rr > 0 ? a / rr : 1.0, s = rr > 0 ? hk1 / rr : 0.0;
                cs[k] = c; sn[k] = s;
                H[k * GM_MAXV + k] = rr;
                double gk = gv[k];
                gv[k] = c * gk;
                gv[k + 1] = -s * gk;
                sc[1] = (fabs(gv[k + 1]) <= A.rtol * bn || hn == 0.0) ? 1.0 : 0.0;
                sc[2] = hn > 0.0 ? 1.0 / hn : 0.0;
            }
            __syncthreads();
            hscale = sc[2];
            wprev = w;
            kused = k + 1;
            if (sc[1] != 0.0) break;
        }
        // y = H^{-1} g, x += Dinv V y (own rows)
        if (threadIdx.x == 0) {
            for (int q = kused - 1; q >= 0; --q) {
                double s = gv[q];
                for (int t = q + 1; t < kused; ++t) s -= H[q * GM_MAXV + t] * y[t];
                double d = H[q * GM_MAXV + q];
                y[q] = d != 0.0 ? s / d : 0.0;
            }
        }
        __syncthreads();
        for (int i = r0 + (int)threadIdx.x; i < r1; i += GM_THREADS) {
            double s = 0.0;
            for (int j = 0; j < kused; ++j) s += y[j] * A.V[(size_t)j * vs + i];
            A.x[i] += A.dinv[i] * s;
        }
        grid_barrier(A);   // x complete before the next residual
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        A.out[0] = total;
        A.out[1] = conv ? 1 : 0;
    }
}

// dst[c][r] = src[r][c] for a rows x cols matrix of doubles, 32 x 32 tiles through LDS
__global__ void k_transpose(int rows, int cols, const double *__restrict__ src, double *__restrict__ dst) {
    __shared__ double t[32][33];
    const int tiles_r = (rows + 31) / 32;
    const int r0 = (int)(blockIdx.x % tiles_r) * 32, c0 = (int)(blockIdx.x / tiles_r) * 32;
    for (int j = threadIdx.y; j < 32; j += 8) {
        const int r = r0 + j, c = c0 + threadIdx.x;
        if (r < rows && c < cols) t[j][threadIdx.x] = src[(size_t)r * cols + c];
    }
    __syncthreads();
    for (int j = threadIdx.y; j < 32; j += 8) {
        const int c = c0 + j, r = r0 + threadIdx.x;
        if (r < rows && c < cols) dst[(size_t)c * rows + r] = t[threadIdx.x][j];
    }
}

static void transpose(int rows, int cols, const double *src, double *dst, hipStream_t s) {
    const unsigned tiles = (unsigned)((rows + 31) / 32) * (unsigned)((cols + 31) / 32);
    hipLaunchKernelGGL(k_transpose, dim3(tiles), dim3(32, 8), 0, s, rows, cols, src, dst);
}

static size_t sys_work(int ne) { return (size_t)(GM_MAXV + 2) * ne + (size_t)2 * GM_MAXBLK * GM_MAXV; }

// Launch the cooperative solves of every right-hand side ([ne][nrhs] vectors b
// and x; x holds the initial guess on entry).  Several systems share the
// resident blocks, at least one each, and are launched in groups when they do
// not all fit.  The status
// words of system r are C->d_iflag[4r..4r+2].  Returns false if the device
// cannot co-schedule the grid (the caller then uses the host-driven solver).
// fill of 32-bit words (clears barrier words without a memset node)
__global__ void k_fill_u32(int64_t n, unsigned v, unsigned *p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

bool gmres_coop_launch_ws(tdbem_ctx *C, const double *b, double *x, double rtol, int maxit, hipStream_t s,
                          double *work, int *iflag, unsigned *gbar);

bool gmres_coop_launch(tdbem_ctx *C, const double *b, double *x, double rtol, int maxit, hipStream_t s) {
    return gmres_coop_launch_ws(C, b, x, rtol, maxit, s, C->d_work, C->d_iflag, C->d_gbar);
}

// The same solve with its workspace (Krylov vectors, transposes, partial sums),
// status words and barrier words given by the caller.
bool gmres_coop_launch_ws(tdbem_ctx *C, const double *b, double *x, double rtol, int maxit, hipStream_t s,
                          double *work_in, int *iflag, unsigned *gbar) {
    int dev = 0;
    TD_HIP(hipGetDevice(&dev));
    int coop = 0;
    TD_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) return false;
    int per_cu = 0;
    TD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_gmres_coop, GM_THREADS, 0));
    int ncu = 0;
    TD_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int resident = per_cu * ncu;
    const int nr = C->nrhs, ne = C->ne;
    // blocks per system: C->gmres_blocks if set; else for one system enough
    // blocks (at least 64) to hold its rows in LDS, for several an equal share
    const int cap = C->gmres_blocks > 0 ? std::min(C->gmres_blocks, GM_MAXBLK) : GM_MAXBLK;
    int nbx;
    if (nr == 1)
        nbx = C->gmres_blocks > 0 ? cap : std::min(GM_MAXBLK, std::max(64, (ne + 32 * GM_RU - 1) / (32 * GM_RU)));
    else
        nbx = std::max(1, std::min(cap, resident / nr));
    nbx = std::min(nbx, resident);
    if (nbx < 1 || resident < 1) return false;
    const int per_launch = std::max(1, resident / nbx);
    const int m = std::min(GM_MAXV - 1, std::max(1, std::min(maxit, C->cfg.gmres_restart)));
    double *work = work_in;
    const double *bs = b;
    double *xs = x;
    if (nr > 1) {                       // systems contiguous: [nrhs][ne]
        double *bt = work, *xt = work + (size_t)ne * nr;
        work = xt + (size_t)ne * nr;
        transpose(ne, nr, b, bt, s);
        transpose(ne, nr, x, xt, s);
        bs = bt;
        xs = xt;
    }
    GmresArgs A;
    A.ne = ne; A.m = m; A.maxit = maxit; A.rtol = rtol;
    A.ptr = C->d_z0_ptr; A.col = C->d_z0_col; A.val = C->d_z0_val; A.dinv = C->d_z0_dinv; A.vald = C->d_z0_vald;
    A.sys_ws = sys_work(ne);
    for (int r0 = 0; r0 < nr; r0 += per_launch) {
        const int cnt = std::min(per_launch, nr - r0);
        A.b = bs + (size_t)r0 * ne;
        A.x = xs + (size_t)r0 * ne;
        A.V = work + (size_t)r0 * A.sys_ws;
        A.w0 = A.V + (size_t)(m + 1) * ne;
        A.w1 = A.w0 + ne;
        A.part = A.w1 + ne;
        A.out = iflag + 4 * r0;
        A.bar = gbar + (size_t)GMRES_BAR_WORDS * r0;
        void *args[] = {&A};
        TD_HIP(hipLaunchCooperativeKernel((const void *)k_gmres_coop, dim3(nbx, cnt), dim3(GM_THREADS), args, 0, s));
    }
    if (nr > 1) transpose(nr, ne, xs, x, s);
    TD_HIP(hipGetLastError());
    return true;
}

size_t gmres_coop_work_doubles(int ne, int nrhs) {
    return (size_t)nrhs * sys_work(ne) + (nrhs > 1 ? (size_t)2 * ne * nrhs : 0);
}

// ---------------------------------------------- allocation-free workspace
// tdbem_step_noalloc takes the device solve's workspace, status words and
// barrier words from this file-scope array instead of the context's
// allocations (every call on a device shares that device's copy, which keeps
// the last call's contents; overlapping calls on one device race).  In host
// code the array's name is not a device address: its address is taken per
// device with hipGetSymbolAddress (the device current at the time) and only
// that address is used.
static constexpr size_t NOALLOC_DOUBLES = (size_t)2 << 20;      // 16 MiB
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];
static constexpr int NOALLOC_MAX_DEVICES = 64;
static double *g_scratch[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

double *noalloc_scratch(size_t *capacity) {
    int dev = 0;
    TD_HIP(hipGetDevice(&dev));
    TD_REQUIRE(dev >= 0 && dev < NOALLOC_MAX_DEVICES, TDBEM_EINVAL, "device index beyond the static workspace table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        TD_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch[dev] = (double *)ptr;
    }
    if (capacity) *capacity = NOALLOC_DOUBLES;
    return g_scratch[dev];
}

// doubles of the static workspace one solve of C needs: barrier words, status
// words, then the solve's own workspace
size_t noalloc_need(const tdbem_ctx *C) {
    const size_t nr = C->nrhs;
    return (GMRES_BAR_WORDS * nr + 1) / 2 + (4 * nr + 1) / 2 + gmres_coop_work_doubles(C->ne, C->nrhs);
}

// the solve of one step on the static workspace: barrier words cleared by a
// fill kernel, then the cooperative launch; status words left in *iflag_out
bool gmres_coop_launch_static(tdbem_ctx *C, const double *b, double *x, double rtol, int maxit, hipStream_t s,
                              int **iflag_out) {
    size_t cap = 0;
    double *base = noalloc_scratch(&cap);
    const size_t nr = C->nrhs;
    const size_t bar_d = (GMRES_BAR_WORDS * nr + 1) / 2, flag_d = (4 * nr + 1) / 2;
    TD_REQUIRE(noalloc_need(C) <= cap, TDBEM_EINVAL, "the allocation-free step's workspace does not fit");
    unsigned *gbar = (unsigned *)base;
    int *iflag = (int *)(base + bar_d);
    double *work = base + bar_d + flag_d;
    const int64_t nb = (int64_t)GMRES_BAR_WORDS * nr;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, nb, 0u, gbar);
    TD_HIP(hipGetLastError());
    *iflag_out = iflag;
    return gmres_coop_launch_ws(C, b, x, rtol, maxit, s, work, iflag, gbar);
}

}  // namespace tdbem
