// M2L through the 4-D Fourier transform (Section 3.6.1: the M2L product is a
// discrete convolution and may be evaluated with a 4-D FFT).
//
// The interpolation nodes are equispaced in space and time, so between a target
// cell and a source cell the M2L operator entry depends on the node indices
// only through their differences: with a = target spatial node, m = target time
// node, b, n the source's,
//     K(a, m; b, n) = k(a - b, m - n),  k(d, e) = f(u) / r,
//     r = |g_s d - d_s o|,  u = c g_t ((p - 1) lag + e) - r,
// (o the cell offset, g_s and g_t the node spacings; f the kernel of the
// channel group as in the dense kernels).  The product y = K x is therefore a
// 4-D linear convolution of x (p^4 values) with k ((2p - 1)^4 values).  Both
// are embedded in a circular convolution of size N = 2p per axis: k at index
// d mod N (index p unused), x zero-padded.  Then
//     y = IDFT( DFT(k) . DFT(x) )  restricted to the first p indices per axis.
// All data are real, so only the time frequencies 0..p (N/2 + 1 of them) are
// kept: NF = N^3 (p + 1) complex values per transformed vector.
//
// Layout and flow per level and time gate k:
//   KH [used offset][lag][group][NF]   transformed kernels (set up once)
//   MH [cell][slot][variant][channel][rhs][NF]   transformed moments, a ring
//      like MM; the new interval's slot is transformed at its gate
//   LH [cell][channel][rhs][NF]   products summed over the interaction list
//      and the window in the frequency domain, then transformed back into LC
//      (plus the parent's pending contribution PEND).
// Transforms are separable: one pass per axis, each output a direct sum over
// the axis (N <= 16 terms), through two scratch buffers in chunks of vectors.
// The frequency-domain product is a diagonal product: lanes are frequencies, a
// block sums one target's interaction list and window for a group of columns
// (channel, rhs) - bound by memory traffic, not arithmetic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "far_internal.h"

namespace tdbem {

// base offset of vector v of a strided family: v = cell * per + w.  A pass
// works on the vectors v0 .. v0 + nvec - 1 of its family; a scratch buffer
// holds only that chunk (local: indexed from 0).
struct VecMap {
    int64_t per, cell_stride, off, vsize;
    int local;
    __device__ int64_t base(int64_t v0, int64_t v) const {
        const int64_t u = local ? v : v0 + v;
        return (u / per) * cell_stride + off + (u % per) * vsize;
    }
};
static VecMap scratch_map(int64_t vsize) { return VecMap{1, vsize, 0, vsize, 1}; }
static VecMap family_map(int64_t per, int64_t cell_stride, int64_t off, int64_t vsize) {
    return VecMap{per, cell_stride, off, vsize, 0};
}

__device__ __forceinline__ void twiddles(double2 *tw, int N) {
    // tw[j] = exp(-2 pi i j / N)
    if (threadIdx.x < N) {
        double s, c;
        sincospi(2.0 * threadIdx.x / N, &s, &c);
        tw[threadIdx.x] = make_double2(c, -s);
    }
    __syncthreads();
}

// real input, pass along the innermost (time) axis:
// out[v][a][f] = sum_{n < nin} in[v][a][n] exp(-2 pi i f n / N), f = 0..nout-1
__global__ void __launch_bounds__(256) k_dft_r2c(const double *__restrict__ in, VecMap mi, double2 *__restrict__ out,
                                                 VecMap mo, int64_t v0, int64_t nvec, int A, int nin, int nout, int N) {
    __shared__ double2 tw[16];
    twiddles(tw, N);
    const int64_t per = (int64_t)A * nout;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nvec * per) return;
    const int64_t v = t / per;
    const int a = (int)((t % per) / nout), f = (int)(t % nout);
    const double *x = in + mi.base(v0, v) + (int64_t)a * nin;
    double re = 0.0, im = 0.0;
    for (int n = 0; n < nin; ++n) {
        const double2 w = tw[(f * n) % N];
        re += x[n] * w.x;
        im += x[n] * w.y;
    }
    out[mo.base(v0, v) + (int64_t)a * nout + f] = make_double2(re, im);
}

// complex pass along a middle axis: in [v][A][nin][B] -> out [v][A][nout][B],
// out[f] = sum_j in[j] exp(sgn 2 pi i f j / N) (sgn = -1 forward, +1 inverse)
__global__ void __launch_bounds__(256) k_dft_c2c(const double2 *__restrict__ in, VecMap mi, double2 *__restrict__ out,
                                                 VecMap mo, int64_t v0, int64_t nvec, int A, int B, int nin, int nout,
                                                 int N, int sgn) {
    __shared__ double2 tw[16];
    twiddles(tw, N);
    const int64_t per = (int64_t)A * nout * B;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nvec * per) return;
    const int64_t v = t / per, r = t % per;
    const int a = (int)(r / ((int64_t)nout * B)), f = (int)((r / B) % nout), b = (int)(r % B);
    const double2 *x = in + mi.base(v0, v) + (int64_t)a * nin * B + b;
    double re = 0.0, im = 0.0;
    for (int j = 0; j < nin; ++j) {
        double2 w = tw[(f * j) % N];
        if (sgn > 0) w.y = -w.y;
        const double2 z = x[(int64_t)j * B];
        re += z.x * w.x - z.y * w.y;
        im += z.x * w.y + z.y * w.x;
    }
    out[mo.base(v0, v) + ((int64_t)a * nout + f) * B + b] = make_double2(re, im);
}

// last inverse pass, along the time axis, from the kept frequencies 0..N/2 of a
// real signal: y[v][a][m] = s (Z_0 + (-1)^m Z_{N/2} + 2 Re sum_{0<f<N/2} Z_f
// exp(2 pi i f m / N)) for m < P; LC = PEND + y.  Vectors are (target, channel,
// rhs) in LC's order.
__global__ void __launch_bounds__(256) k_dft_c2r_lc(const double2 *__restrict__ in, int64_t v0, int64_t nvec, int P,
                                                    int N, double s, int nchr, int parity, const double *__restrict__ PEND,
                                                    double *__restrict__ LC) {
    __shared__ double2 tw[16];
    twiddles(tw, N);
    const int NT = N / 2 + 1, P3 = P * P * P;
    const int64_t per = (int64_t)P3 * P;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nvec * per) return;
    const int64_t v = t / per;
    const int a = (int)((t % per) / P), m = (int)(t % P);
    const double2 *z = in + (v * P3 + a) * NT;
    double y = z[0].x + ((m & 1) ? -z[N / 2].x : z[N / 2].x);
    for (int f = 1; f < N / 2; ++f) {
        const double2 w = tw[(f * m) % N];           // exp(-i theta): Re(Z e^{+i theta}) = Zx wx + Zy wy
        y += 2.0 * (z[f].x * w.x + z[f].y * w.y);
    }
    const int64_t gv = v0 + v, O = gv / nchr, rest = gv % nchr;
    LC[gv * per + t % per] = s * y + PEND[((O * 2 + parity) * nchr + rest) * per + t % per];
}

// circularly embedded kernel samples of the used offsets: vector (slot, lag,
// group) holds c[i1][i2][i3][it] = k(d, e) with d_x = i_x (i_x < P) or i_x - N
// (i_x > P), zero at index P
__global__ void __launch_bounds__(256) k_fft_kernel_samples(const int *__restrict__ slot_code, int64_t v0, int64_t nvec,
                                                            int P, int W, int kindA, double gs, double ds, double cgt,
                                                            double c2, double *__restrict__ out) {
    const int N = 2 * P;
    const int64_t per = (int64_t)N * N * N * N;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nvec * per) return;
    const int64_t v = t / per, gv = v0 + v;
    const int grp = (int)(gv % 2), lag = (int)((gv / 2) % W) + 1, cs = (int)(gv / (2 * W));
    const int code = slot_code[cs];
    const int ox = code / 49 - 3, oy = (code / 7) % 7 - 3, oz = code % 7 - 3;
    const int64_t r0 = t % per;
    const int it = (int)(r0 % N), i3 = (int)((r0 / N) % N), i2 = (int)((r0 / (N * N)) % N), i1 = (int)(r0 / (N * N * N));
    double val = 0.0;
    if (i1 != P && i2 != P && i3 != P && it != P) {
        const int d1 = i1 < P ? i1 : i1 - N, d2 = i2 < P ? i2 : i2 - N, d3 = i3 < P ? i3 : i3 - N,
                  e = it < P ? it : it - N;
        const double x = gs * d1 - ds * ox, y = gs * d2 - ds * oy, z = gs * d3 - ds * oz;
        const double r = sqrt(x * x + y * y + z * z);
        const double u = cgt * ((P - 1) * lag + e) - r;
        const int kfun = grp == 0 ? kindA : 1;
        if (u > 0.0 && r > 0.0) val = (kfun == 0 ? c2 * u : kfun == 1 ? u * u : 0.5 * c2 * c2) * (1.0 / r);
    }
    out[t] = val;
}

// frequency-domain M2L: one block per (target, column group, 256 frequencies);
// LH[target][channel][rhs][f] = sum over the interaction list and the window's
// lags of KH[offset][lag][group][f] MH[source][slot][variant][channel][rhs][f]
template <int CG>
__global__ void __launch_bounds__(256) k_m2l_fft_prod(int NF, const int *__restrict__ il_off,
                                                      const int *__restrict__ il_src, const int *__restrict__ il_code,
                                                      const int *__restrict__ code_slot, const double2 *__restrict__ KH,
                                                      const double2 *__restrict__ MH, int WR, int NV, int W, int k,
                                                      int nrhs, int ngrp0, double2 *__restrict__ LH) {
    const int O = blockIdx.x;
    const int grp = (int)blockIdx.y < ngrp0 ? 0 : 1;
    const int g = (int)blockIdx.y - (grp ? ngrp0 : 0);
    const int c0 = grp ? 3 : 0, nc = grp ? 4 : 3;
    const int col0 = g * CG, ncl = min(CG, nc * nrhs - col0);
    const int f = blockIdx.z * 256 + threadIdx.x;
    if (f >= NF || ncl <= 0) return;
    int64_t coff[CG];
#pragma unroll
    for (int j = 0; j < CG; ++j) {
        const int col = min(col0 + j, nc * nrhs - 1);
        coff[j] = ((int64_t)(c0 + col / nrhs) * nrhs + col % nrhs) * NF + f;
    }
    double2 acc[CG];
#pragma unroll
    for (int j = 0; j < CG; ++j) acc[j] = make_double2(0.0, 0.0);
    const int nlag = min(W, k + 1);
    const int64_t vstride = (int64_t)NCH * nrhs * NF;
    for (int q = il_off[O]; q < il_off[O + 1]; ++q) {
        const double2 *kp = KH + ((int64_t)code_slot[il_code[q]] * W * 2 + grp) * NF + f;
        const int64_t sb = (int64_t)il_src[q] * WR * NV;
        for (int lag = 1; lag <= nlag; ++lag) {
            const int var = W - lag < NV - 1 ? W - lag + 1 : 0;     // the window's oldest intervals: truncated
            const double2 kh = kp[(int64_t)(lag - 1) * 2 * NF];
            const double2 *mp = MH + (sb + (int64_t)((k + 1 - lag) % WR) * NV + var) * vstride;
#pragma unroll
            for (int j = 0; j < CG; ++j) {
                if (j < ncl) {
                    const double2 m = mp[coff[j]];
                    acc[j].x += kh.x * m.x - kh.y * m.y;
                    acc[j].y += kh.x * m.y + kh.y * m.x;
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < CG; ++j)
        if (j < ncl) LH[(int64_t)O * vstride + coff[j]] = acc[j];
}

// ------------------------------------------------------------------ host side
static constexpr int FFT_CG = 4;                           // columns per product block
static constexpr int64_t FFT_SCRATCH = (int64_t)1 << 24;   // complex values per scratch buffer

static inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

// forward transform of nvec vectors of real nin^4 values (time fastest; nin = P
// for moments, zero-padded to N per axis, or N for kernel samples) into NF
// complex values; in and out are strided families
static void forward(const FarState *F, const double *in, VecMap mi, double2 *out, VecMap mo, int64_t nvec, int nin,
                    hipStream_t s) {
    const int P = F->P, N = 2 * P, NT = P + 1;
    const int64_t per_vec = (int64_t)nin * N * N * NT;   // largest intermediate
    const int64_t chunk = std::max<int64_t>(1, FFT_SCRATCH / per_vec);
    const int n2 = nin * nin, n3 = n2 * nin;
    for (int64_t v0 = 0; v0 < nvec; v0 += chunk) {
        const int64_t nv = std::min(chunk, nvec - v0);
        double2 *s1 = F->fft_s1, *s2 = F->fft_s2;
        // time axis: [nin^3][nin] real -> [nin^3][NT]
        hipLaunchKernelGGL(k_dft_r2c, dim3(blocks(nv * n3 * NT)), dim3(256), 0, s, in, mi, s1,
                           scratch_map((int64_t)n3 * NT), v0, nv, n3, nin, NT, N);
        // axis 3: [nin^2][nin][NT] -> [nin^2][N][NT]
        hipLaunchKernelGGL(k_dft_c2c, dim3(blocks(nv * n2 * N * NT)), dim3(256), 0, s, s1,
                           scratch_map((int64_t)n3 * NT), s2, scratch_map((int64_t)n2 * N * NT), v0, nv, n2, NT, nin,
                           N, N, -1);
        // axis 2: [nin][nin][N NT] -> [nin][N][N NT]
        hipLaunchKernelGGL(k_dft_c2c, dim3(blocks(nv * nin * N * N * NT)), dim3(256), 0, s, s2,
                           scratch_map((int64_t)n2 * N * NT), s1, scratch_map((int64_t)nin * N * N * NT), v0, nv, nin,
                           N * NT, nin, N, N, -1);
        // axis 1: [nin][N^2 NT] -> [N][N^2 NT]
        hipLaunchKernelGGL(k_dft_c2c, dim3(blocks(nv * N * N * N * NT)), dim3(256), 0, s, s1,
                           scratch_map((int64_t)nin * N * N * NT), out, mo, v0, nv, 1, N * N * NT, nin, N, N, -1);
    }
    TD_HIP(hipGetLastError());
}

// inverse transform of LH (vectors (target, channel, rhs)) into LC = PEND + y
static void inverse_to_lc(const tdbem_ctx *C, FarLevel &FL, int parity, hipStream_t s) {
    const FarState *F = C->far;
    const int P = F->P, N = 2 * P, NT = P + 1;
    const int64_t NF = F->NF, nvec = (int64_t)FL.n * NCH * C->nrhs;
    const int64_t per_vec = (int64_t)P * N * N * NT;
    const int64_t chunk = std::max<int64_t>(1, FFT_SCRATCH / per_vec);
    const double sc = 1.0 / ((double)N * N * N * N);
    for (int64_t v0 = 0; v0 < nvec; v0 += chunk) {
        const int64_t nv = std::min(chunk, nvec - v0);
        double2 *s1 = F->fft_s1, *s2 = F->fft_s2;
        // axis 1: [N][N^2 NT] -> [P][N^2 NT]
        hipLaunchKernelGGL(k_dft_c2c, dim3(blocks(nv * P * N * N * NT)), dim3(256), 0, s, FL.LH,
                           family_map(1, NF, 0, NF), s1, scratch_map((int64_t)P * N * N * NT), v0, nv, 1, N * N * NT,
                           N, P, N, 1);
        // axis 2: [P][N][N NT] -> [P][P][N NT]
        hipLaunchKernelGGL(k_dft_c2c, dim3(blocks(nv * P * P * N * NT)), dim3(256), 0, s, s1,
                           scratch_map((int64_t)P * N * N * NT), s2, scratch_map((int64_t)P * P * N * NT), v0, nv, P,
                           N * NT, N, P, N, 1);
        // axis 3: [P^2][N][NT] -> [P^2][P][NT]
        hipLaunchKernelGGL(k_dft_c2c, dim3(blocks(nv * P * P * P * NT)), dim3(256), 0, s, s2,
                           scratch_map((int64_t)P * P * N * NT), s1, scratch_map((int64_t)P * P * P * NT), v0, nv,
                           P * P, NT, N, P, N, 1);
        // time axis (real result) plus the pending parent contribution
        hipLaunchKernelGGL(k_dft_c2r_lc, dim3(blocks(nv * P * P * P * P)), dim3(256), 0, s, s1, v0, nv, P, N, sc,
                           NCH * C->nrhs, parity, FL.PEND, FL.LC);
    }
    TD_HIP(hipGetLastError());
}

// transformed moments of one ring slot (every cell, variant, channel, rhs)
void m2l_fft_moments(tdbem_ctx *C, FarLevel &FL, int slot, hipStream_t s) {
    const FarState *F = C->far;
    const int64_t per = (int64_t)FL.NV * NCH * C->nrhs, NN = F->NN, NF = F->NF;
    forward(F, FL.MM, family_map(per, FL.WR * per * NN, slot * per * NN, NN), FL.MH,
            family_map(per, FL.WR * per * NF, slot * per * NF, NF), (int64_t)FL.n * per, F->P, s);
}

void m2l_fft_setup(tdbem_ctx *C, FarLevel &FL, const std::vector<int> &il_code, int kindA) {
    FarState *F = C->far;
    const int P = F->P, N = 2 * P, NT = P + 1;
    const int64_t NF = (int64_t)N * N * N * NT;
    F->NF = NF;
    if (!F->fft_s1) {
        F->fft_s1 = (double2 *)far_alloc(C, FFT_SCRATCH * sizeof(double2));
        F->fft_s2 = (double2 *)far_alloc(C, FFT_SCRATCH * sizeof(double2));
    }
    // the offsets that occur at this level
    std::vector<int> cslot(343, -1), scode;
    for (int c : il_code)
        if (cslot[c] < 0) { cslot[c] = (int)scode.size(); scode.push_back(c); }
    if (scode.empty()) scode.push_back(0);
    FL.fft_code_slot = (int *)far_alloc(C, 343 * sizeof(int));
    TD_HIP(hipMemcpy(FL.fft_code_slot, cslot.data(), 343 * sizeof(int), hipMemcpyHostToDevice));
    int *d_scode = (int *)far_alloc(C, scode.size() * sizeof(int));
    TD_HIP(hipMemcpy(d_scode, scode.data(), scode.size() * sizeof(int), hipMemcpyHostToDevice));
    const int64_t nk = (int64_t)scode.size() * FL.W * 2;
    const int nr = C->nrhs;
    FL.KH = (double2 *)far_alloc(C, (size_t)nk * NF * sizeof(double2));
    FL.MH = (double2 *)far_alloc(C, (size_t)FL.n * FL.WR * FL.NV * NCH * nr * NF * sizeof(double2));
    FL.LH = (double2 *)far_alloc(C, (size_t)FL.n * NCH * nr * NF * sizeof(double2));
    // kernel samples (N^4 reals per vector) in chunks, then their forward transform
    const int64_t per = (int64_t)N * N * N * N;
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(nk, FFT_SCRATCH / per));
    double *samp = (double *)far_alloc(C, (size_t)chunk * per * sizeof(double));
    hipStream_t s = C->stream;
    const double gs = FL.hn * (2.0 / (P - 1)), cgt = C->c * FL.ht * (2.0 / (P - 1));
    for (int64_t v0 = 0; v0 < nk; v0 += chunk) {
        const int64_t nv = std::min(chunk, nk - v0);
        hipLaunchKernelGGL(k_fft_kernel_samples, dim3(blocks(nv * per)), dim3(256), 0, s, d_scode, v0, nv, P, FL.W,
                           kindA, gs, FL.ds, cgt, 2.0 * C->c, samp);
        TD_HIP(hipGetLastError());
        forward(F, samp, family_map(1, per, 0, per), FL.KH + v0 * NF, family_map(1, NF, 0, NF), nv, N, s);
    }
    TD_HIP(hipStreamSynchronize(s));
}

void m2l_fft_level(tdbem_ctx *C, FarLevel &FL, int k, hipStream_t s) {
    const FarState *F = C->far;
    const int nr = C->nrhs;
    PhaseScope ps(C->prof, TDBEM_PH_M2L, s);
    m2l_fft_moments(C, FL, k % FL.WR, s);       // the interval completed at this gate
    const int ngrp0 = (3 * nr + FFT_CG - 1) / FFT_CG, ngrp1 = (4 * nr + FFT_CG - 1) / FFT_CG;
    hipLaunchKernelGGL(k_m2l_fft_prod<FFT_CG>, dim3(FL.n, ngrp0 + ngrp1, blocks(F->NF)), dim3(256), 0, s, (int)F->NF,
                       FL.il_off, FL.il_src, FL.il_code, FL.fft_code_slot, FL.KH, FL.MH, FL.WR, FL.NV, FL.W, k, nr,
                       ngrp0, FL.LH);
    TD_HIP(hipGetLastError());
    inverse_to_lc(C, FL, (k + 1) & 1, s);
}

}  // namespace tdbem
