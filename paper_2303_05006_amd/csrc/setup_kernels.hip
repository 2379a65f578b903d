// Setup kernels (FP64): exact lag ranges of near pairs, the J-form coefficients
// Zt^(g)_ij (Sections 2.3-2.4), and the tested incident field (Eq. v_i).
//
// Inner integrals over a flat source triangle, for one field point x and one
// lag g, use polar coordinates about the projection x0 of x on the source
// plane (r dr = rho drho).  The radial integrals of the retarded kernels are
// closed forms in tau = g - r/(c dt):
//   Qa   = -c dt B'(tau)       (d/dr Qa = B'')
//   Qphi = -c dt Bint(tau)     (d/dr Qphi = B)
//   Qp   = F(tau)/r, F = B'(tau)/dt + zeta B(tau)   ((1/r) d/dr Qp = psi, grad(F/r) = (y-x) psi)
// The angular integral over each edge's signed sub-triangle is taken in
// v = asinh(s/|d|) (smooth in a strip of half-width pi/2), split where the
// light-cone circles r = (g-k) c dt cross the edge; in-plane vector moments use
// the surface gradient theorem as line integrals in w = asinh(s/rho).
#include <hip/hip_runtime.h>

#include <cmath>

#include "tdbem_internal.h"

namespace tdbem {

#define TD_HD __device__ __forceinline__
#define TD_CONST __constant__
#include "zt_integrals.inl"

__global__ void k_lag_range(GeoDev G, int64_t npairs, const int *pi, const int *pj, int *g_lo, int *g_hi) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    int lo, hi;
    pair_lag_range(G, pi[p], pj[p], lo, hi);
    g_lo[p] = lo;
    g_hi[p] = hi;
}

// one thread per stored coefficient: pair found by binary search on offsets
__global__ void k_zfill(GeoDev G, int64_t n, int64_t k0, int64_t npairs, const int *pi, const int *pj,
                        const int *g0, const int64_t *off, double *val) {
    // coefficients k0 .. k0 + n - 1 of the pair-major store
    int64_t k = k0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= k0 + n) return;
    int64_t lo = 0, hi = npairs - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= k) lo = mid; else hi = mid - 1;
    }
    int g = g0[lo] + (int)(k - off[lo]);
    val[k] = zt_value(G, pi[lo], pj[lo], g);
}

void launch_lag_range(const GeoDev &G, int64_t npairs, const int *pi, const int *pj, int *lo, int *hi, hipStream_t s) {
    if (npairs <= 0) return;
    int bs = 256;
    hipLaunchKernelGGL(k_lag_range, dim3((unsigned)((npairs + bs - 1) / bs)), dim3(bs), 0, s, G, npairs, pi, pj, lo, hi);
    TD_HIP(hipGetLastError());
}

void launch_zfill(const GeoDev &G, int64_t n, int64_t k0, int64_t npairs, const int *pi, const int *pj, const int *g0,
                  const int64_t *off, double *val, hipStream_t s) {
    if (n <= 0) return;
    int bs = 128;
    hipLaunchKernelGGL(k_zfill, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, G, n, k0, npairs, pi, pj, g0, off,
                       val);
    TD_HIP(hipGetLastError());
}

// ---- tested incident field V_i^{alpha-1} at t (Eq. v_i), leaf-order edges,
// output layout [rhs][ne] in canonical order through perm.
__global__ void k_vinc(GeoDev G, int ne, int nrhs, const double *pulses, const int *perm, double t, double *V) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    int r = blockIdx.y;
    if (p >= ne) return;
    V[(size_t)r * ne + perm[p]] = vinc_value(G, p, pulses + 11 * r, t);
}

void launch_vinc(const GeoDev &G, int ne, int nrhs, const double *pulses, const int *perm, double t, double *V, hipStream_t s) {
    int bs = 256;
    hipLaunchKernelGGL(k_vinc, dim3((ne + bs - 1) / bs, nrhs), dim3(bs), 0, s, G, ne, nrhs, pulses, perm, t, V);
    TD_HIP(hipGetLastError());
}

// ---- small conversion / gather helpers
__global__ void k_to_f32(const double *src, float *dst, int64_t n) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = (float)src[k];
}
__global__ void k_gather_vals(const double *val, const int64_t *idx, int64_t n, double *out) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = val[idx[k]];
}
void launch_to_f32(const double *src, float *dst, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
    TD_HIP(hipGetLastError());
}
void launch_gather_vals(const double *val, const int64_t *idx, int64_t n, double *out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_vals, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, val, idx, n, out);
    TD_HIP(hipGetLastError());
}

}  // namespace tdbem

namespace tdbem {

// number of stored coefficients of the all-pairs problem: sum over every
// (i, j) of its exact lag range (the direct mode's storage); grid-stride over
// pairs, integer sums (exact, order-independent)
__global__ void __launch_bounds__(256) k_count_d0(GeoDev G, int ne, unsigned long long *count) {
    const int64_t np = (int64_t)ne * ne;
    unsigned long long s = 0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
        int lo, hi;
        pair_lag_range(G, (int)(p / ne), (int)(p % ne), lo, hi);
        if (hi >= lo) s += (unsigned long long)(hi - lo + 1);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(count, s);
}

void launch_count_d0(const GeoDev &G, int ne, unsigned long long *count, hipStream_t s) {
    hipLaunchKernelGGL(k_count_d0, dim3(2048), dim3(256), 0, s, G, ne, count);
    TD_HIP(hipGetLastError());
}

}  // namespace tdbem
