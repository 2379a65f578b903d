// Training kernels of the learned initial guess: loss gradient and Adam step.
//
// Network (the definition is in tdbem.h, next to tdbem_guess_weights):
//   o(x) = relu(relu(x W1 + b1) W2 + b2) . w3 + b3,  g(x) = (o(x) - o(-x)) / 2,
// trained on L = (1/n) sum_s (g(x_s) - y_s)^2 in FP32.  Backward, per branch
// sigma = +-1 with a1 = sigma x W1 + b1, h1 = relu(a1), a2 = h1 W2 + b2,
// h2 = relu(a2) and do = sigma dL/dg / 2:
//   dw3 += do h2,  da2 = do w3 [a2 > 0],  dW2 += h1^T da2,  db2 += da2,
//   dh1 = da2 W2^T,  da1 = dh1 [a1 > 0],  dW1 += sigma x^T da1,  db1 += da1,
// and db3 = 0 (b3 cancels in g).
#include <hip/hip_runtime.h>

#include "tdbem_internal.h"

namespace tdbem {

static constexpr int TF = 116;        // features
static constexpr int TH = 128;        // hidden width
static constexpr int TS = 32;         // samples per block
static constexpr int TPB = 256;       // threads: 128 columns x 2 sample halves

struct GuessParams {
    const float *W1, *b1, *W2, *b2, *w3;
    float b3;
};

// one block per TS samples; thread t owns column t % 128 and samples
// 16 (t / 128) .. 16 (t / 128) + 15
__global__ void __launch_bounds__(TPB) k_guess_grad(const float *__restrict__ P, const float *__restrict__ X,
                                                    const float *__restrict__ Y, int64_t n, float *__restrict__ G,
                                                    float *__restrict__ loss) {
    __shared__ float xs[TS][TF];
    __shared__ float h1[2][TS][TH];     // per branch; later reused for da2
    __shared__ float ored[2][2][TS];    // [branch][column half][sample] partial outputs
    __shared__ float dgs[TS];
    const float *W1 = P, *b1 = W1 + TF * TH, *W2 = b1 + TH, *b2 = W2 + TH * TH, *w3 = b2 + TH;
    const float b3 = w3[TH];
    float *gW1 = G, *gb1 = gW1 + TF * TH, *gW2 = gb1 + TH, *gb2 = gW2 + TH * TH, *gw3 = gb2 + TH;
    const int t = threadIdx.x, c = t & (TH - 1), half = t >> 7;
    const int64_t s0 = (int64_t)blockIdx.x * TS;
    const int ns = (int)min((int64_t)TS, n - s0);
    for (int q = t; q < TS * TF; q += TPB) {
        const int s = q / TF, f = q % TF;
        xs[s][f] = s < ns ? X[(s0 + s) * TF + f] : 0.0f;
    }
    __syncthreads();
    // layer 1 (p = x W1, both branches from it)
    float p[16];
    for (int i = 0; i < 16; ++i) p[i] = 0.0f;
    for (int f = 0; f < TF; ++f) {
        const float w = W1[f * TH + c];
        for (int i = 0; i < 16; ++i) p[i] += xs[16 * half + i][f] * w;
    }
    const float bb1 = b1[c];
    for (int i = 0; i < 16; ++i) {
        const float ap = p[i] + bb1, am = -p[i] + bb1;
        h1[0][16 * half + i][c] = ap > 0.0f ? ap : 0.0f;
        h1[1][16 * half + i][c] = am > 0.0f ? am : 0.0f;
    }
    __syncthreads();
    // layer 2 and the output partials
    float a2[2][16];
    for (int br = 0; br < 2; ++br)
        for (int i = 0; i < 16; ++i) a2[br][i] = 0.0f;
    for (int k = 0; k < TH; ++k) {
        const float w = W2[k * TH + c];
        for (int i = 0; i < 16; ++i) {
            a2[0][i] += h1[0][16 * half + i][k] * w;
            a2[1][i] += h1[1][16 * half + i][k] * w;
        }
    }
    const float bb2 = b2[c], ww3 = w3[c];
    const int lane = t & 63, colhalf = (t >> 6) & 1;   // the wavefront's 64 columns
    for (int br = 0; br < 2; ++br)
        for (int i = 0; i < 16; ++i) {
            a2[br][i] += bb2;
            float v = (a2[br][i] > 0.0f ? a2[br][i] : 0.0f) * ww3;
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) ored[br][colhalf][16 * half + i] = v;
        }
    __syncthreads();
    if (t < TS) {
        const int s = t;
        float dg = 0.0f, l = 0.0f;
        if (s < ns) {
            const float op = ored[0][0][s] + ored[0][1][s] + b3, om = ored[1][0][s] + ored[1][1][s] + b3;
            const float g = 0.5f * (op - om), e = g - Y[s0 + s];
            dg = 2.0f * e / (float)n;
            l = e * e / (float)n;
        }
        dgs[s] = dg;
        for (int o = 16; o > 0; o >>= 1) l += __shfl_xor(l, o, 32);
        if (s == 0) atomicAdd(loss, l);
    }
    __syncthreads();
    // dw3, db2, da2 (da2 kept in registers, h1 still needed for dW2)
    float gw = 0.0f, gb = 0.0f;
    for (int br = 0; br < 2; ++br)
        for (int i = 0; i < 16; ++i) {
            const float dob = (br == 0 ? 0.5f : -0.5f) * dgs[16 * half + i];
            const bool on = a2[br][i] > 0.0f;
            gw += dob * (on ? a2[br][i] : 0.0f);
            a2[br][i] = on ? dob * ww3 : 0.0f;      // now da2
            gb += a2[br][i];
        }
    atomicAdd(&gw3[c], gw);
    atomicAdd(&gb2[c], gb);
    // dW2[k][c] = sum_s h1[s][k] da2[s][c]
    for (int k = 0; k < TH; ++k) {
        float acc = 0.0f;
        for (int i = 0; i < 16; ++i) acc += h1[0][16 * half + i][k] * a2[0][i] + h1[1][16 * half + i][k] * a2[1][i];
        atomicAdd(&gW2[k * TH + c], acc);
    }
    // masks of layer 1 before h1 is overwritten: bit i of m[br] = [a1 > 0] at (sample 16 half + i, unit c)
    unsigned int m0 = 0, m1 = 0;
    for (int i = 0; i < 16; ++i) {
        if (h1[0][16 * half + i][c] > 0.0f) m0 |= 1u << i;
        if (h1[1][16 * half + i][c] > 0.0f) m1 |= 1u << i;
    }
    __syncthreads();
    for (int i = 0; i < 16; ++i) {
        h1[0][16 * half + i][c] = a2[0][i];
        h1[1][16 * half + i][c] = a2[1][i];
    }
    __syncthreads();
    // dh1[s][k] = sum_c da2[s][c] W2[k][c]; this thread now owns unit k = c
    const int k = c;
    float d[2][16];
    for (int br = 0; br < 2; ++br)
        for (int i = 0; i < 16; ++i) d[br][i] = 0.0f;
    for (int cc = 0; cc < TH; ++cc) {
        const float w = W2[k * TH + cc];
        for (int i = 0; i < 16; ++i) {
            d[0][i] += h1[0][16 * half + i][cc] * w;
            d[1][i] += h1[1][16 * half + i][cc] * w;
        }
    }
    float gb1v = 0.0f;
    for (int i = 0; i < 16; ++i) {
        d[0][i] = (m0 >> i) & 1u ? d[0][i] : 0.0f;     // da1, branch +
        d[1][i] = (m1 >> i) & 1u ? d[1][i] : 0.0f;     // da1, branch -
        gb1v += d[0][i] + d[1][i];
    }
    atomicAdd(&gb1[k], gb1v);
    // dW1[f][k] = sum_s x[s][f] (da1+ - da1-)[s][k]
    for (int i = 0; i < 16; ++i) d[0][i] -= d[1][i];
    for (int f = 0; f < TF; ++f) {
        float acc = 0.0f;
        for (int i = 0; i < 16; ++i) acc += xs[16 * half + i][f] * d[0][i];
        atomicAdd(&gW1[f * TH + k], acc);
    }
}

__global__ void k_guess_adam(int n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2,
                             float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_fill_f32(int64_t n, float v, float *x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

void guess_grad(const float *P, const float *X, const float *Y, int64_t n, float *G, float *loss, hipStream_t s) {
    TD_REQUIRE(P && X && Y && G && loss, TDBEM_EINVAL, "null argument");
    TD_REQUIRE(n > 0 && n <= ((int64_t)1 << 31) * TS, TDBEM_EINVAL, "batch size out of range");
    const int64_t np = TDBEM_GUESS_NPARAMS;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, np, 0.0f, G);
    hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(64), 0, s, (int64_t)1, 0.0f, loss);
    hipLaunchKernelGGL(k_guess_grad, dim3((unsigned)((n + TS - 1) / TS)), dim3(TPB), 0, s, P, X, Y, n, G, loss);
    TD_HIP(hipGetLastError());
}

void guess_adam(float *P, const float *G, float *M, float *V, int t, float lr, float b1, float b2, float eps,
                hipStream_t s) {
    TD_REQUIRE(P && G && M && V, TDBEM_EINVAL, "null argument");
    TD_REQUIRE(t >= 1, TDBEM_EINVAL, "the Adam step count starts at 1");
    const int np = TDBEM_GUESS_NPARAMS;
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_guess_adam, dim3((np + 255) / 256), dim3(256), 0, s, np, P, G, M, V, lr, b1, b2, eps, c1, c2);
    TD_HIP(hipGetLastError());
}

}  // namespace tdbem
