// learned_kernels.hip - kernels of the learned preconditioner.
//
// The preconditioner maps a residual block R to
//   W = D0 .* R + b1 (C E + a)^H E (C E + a) R
//     = (D0 + b1 a^2 E) .* R + 2 a b1 E .* C(E .* R) + b1 E .* C(E .* C(E .* R)),
// a diagonal term plus two spectral-convolution layers (b1 = max(beta1, 0),
// a = beta0, so the layers add a positive semidefinite term and W stays a
// Hermitian positive definite map, as LOBPCG requires), where C = F V F^{-1}
// is the potential block of H~ (the apply's lifted-FFT convolution with the
// kinetic term off) and
//   D0 = M .* (1 + exp(o0[shell(k)])) / 2,  E = M .* exp(o1[shell(k)])
// with M the diagonal of eq:precond and (o0, o1) the two outputs of a small
// MLP (3 hidden layers, GELU) evaluated once per kinetic-energy shell.  D0
// never drops below M/2, so every component of the residual keeps at least
// half of its plain-preconditioned weight.  MLP
// weights are stored in bfloat16; every product accumulates in float32 and the
// optimiser keeps float32 master weights (Adam).  Grid-sized arithmetic is in
// float64 like the rest of the eigensolver's block algebra.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "learned_dev.hpp"

namespace iwfpm {

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));  // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

// GELU(x) = x Phi(x) (exact form) and its derivative Phi(x) + x phi(x)
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
    float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
    float pdf = 0.39894228040143268f * expf(-0.5f * x * x);
    return cdf + x * pdf;
}

// ---------------------------------------------------------------------------
// dense layers (the MLP runs over ~10^3 shells: a few MFLOP per layer)
// ---------------------------------------------------------------------------

// one thread per output; weights read along o (coalesced across the wavefront)
__global__ void k_dense_fwd(const float* __restrict__ X, const uint16_t* __restrict__ W, const float* __restrict__ b,
                            float* __restrict__ Z, float* __restrict__ Y, int S, int in, int out, int act) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= S * out) return;
    int s = e / out, o = e - s * out;
    float acc = b[o];
    const float* x = X + (size_t)s * in;
    for (int i = 0; i < in; ++i) acc = fmaf(x[i], bf2f(W[(size_t)i * out + o]), acc);
    if (Z) Z[e] = acc;
    Y[e] = act ? gelu(acc) : acc;
}

__global__ void k_act_bwd(const float* __restrict__ dY, const float* __restrict__ Z, float* __restrict__ dZ, int n,
                          int act) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    dZ[e] = act ? dY[e] * gelu_grad(Z[e]) : dY[e];
}

// dX[s][i] = sum_o dZ[s][o] W[i][o]
__global__ void k_dense_bwd_data(const float* __restrict__ dZ, const uint16_t* __restrict__ W, float* __restrict__ dX,
                                 int S, int in, int out) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= S * in) return;
    int s = e / in, i = e - s * in;
    float acc = 0.f;
    const float* dz = dZ + (size_t)s * out;
    const uint16_t* w = W + (size_t)i * out;
    for (int o = 0; o < out; ++o) acc = fmaf(dz[o], bf2f(w[o]), acc);
    dX[e] = acc;
}

// dW[i][o] = sum_s X[s][i] dZ[s][o];  db[o] = sum_s dZ[s][o]  (fixed summation order)
__global__ void k_dense_bwd_weight(const float* __restrict__ X, const float* __restrict__ dZ, float* __restrict__ dW,
                                   float* __restrict__ db, int S, int in, int out) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < in * out) {
        int i = e / out, o = e - i * out;
        float acc = 0.f;
        for (int s = 0; s < S; ++s) acc = fmaf(X[(size_t)s * in + i], dZ[(size_t)s * out + o], acc);
        dW[e] = acc;
    } else if (e < in * out + out) {
        int o = e - in * out;
        float acc = 0.f;
        for (int s = 0; s < S; ++s) acc += dZ[(size_t)s * out + o];
        db[o] = acc;
    }
}

__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ g,
                       uint16_t* __restrict__ wbf, int n, float lr, float b1, float b2, float c1, float c2, float eps) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float gg = g[e];
    float mm = b1 * m[e] + (1.f - b1) * gg;
    float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    float nw = w[e] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    w[e] = nw;
    wbf[e] = f2bf(nw);
}

__global__ void k_to_bf16(const float* __restrict__ w, uint16_t* __restrict__ wbf, int n) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) wbf[e] = f2bf(w[e]);
}

// ---------------------------------------------------------------------------
// grid-sized kernels (HBM-bound elementwise passes and reductions)
// ---------------------------------------------------------------------------

__global__ void k_expand(const double* __restrict__ M, const int* __restrict__ shell, const float* __restrict__ O,
                         double* __restrict__ D0, double* __restrict__ E, long long N) {
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (long long)gridDim.x * blockDim.x) {
        int s = shell[k];
        double mk = M[k];
        D0[k] = 0.5 * mk * (1.0 + exp((double)O[2 * s]));
        E[k] = mk * exp((double)O[2 * s + 1]);
    }
}

__global__ void k_scale_cols(ColPtrs R, double2* __restrict__ Y, int m, const double* __restrict__ d, long long N) {
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (long long)gridDim.x * blockDim.x) {
        double s = d[k];
        for (int j = 0; j < m; ++j) {
            double2 a = R.p[j][k];
            Y[(size_t)j * N + k] = make_double2(s * a.x, s * a.y);
        }
    }
}

__global__ void k_scale(const double2* __restrict__ A, double2* __restrict__ Y, int m, const double* __restrict__ d,
                        long long N) {
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (long long)gridDim.x * blockDim.x) {
        double s = d[k];
        for (int j = 0; j < m; ++j) {
            double2 a = A[(size_t)j * N + k];
            Y[(size_t)j * N + k] = make_double2(s * a.x, s * a.y);
        }
    }
}

// coefficients of the expanded layers: E A (c0), E Cc (c1) and the extra diagonal E (dl)
struct LayerCoef {
    double a, b1, c0, c1, dl;
};
__device__ __forceinline__ LayerCoef layer_coef(const float* beta) {
    LayerCoef c;
    c.a = beta[0];
    c.b1 = beta[1] > 0.f ? (double)beta[1] : 0.0;
    c.c0 = 2.0 * c.a * c.b1;
    c.c1 = c.b1;
    c.dl = c.b1 * c.a * c.a;
    return c;
}

__global__ void k_combine(ColPtrs R, const double2* __restrict__ A, const double2* __restrict__ C, ColPtrs W, int m,
                          const double* __restrict__ D0, const double* __restrict__ E, const float* __restrict__ beta,
                          long long N) {
    const LayerCoef lc = layer_coef(beta);
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (long long)gridDim.x * blockDim.x) {
        double e = E[k], d = D0[k] + lc.dl * e;
        for (int j = 0; j < m; ++j) {
            double2 r = R.p[j][k], a = A[(size_t)j * N + k], c = C[(size_t)j * N + k];
            W.p[j][k] = make_double2(d * r.x + e * (lc.c0 * a.x + lc.c1 * c.x), d * r.y + e * (lc.c0 * a.y + lc.c1 * c.y));
        }
    }
}

// block sum of v over the block's wavefronts (blockDim.x = 256), result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double* sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    return t;
}

__device__ __forceinline__ double redot(double2 a, double2 b) { return a.x * b.x + a.y * b.y; }  // Re(conj(a) b)

__global__ void __launch_bounds__(256) k_shell_grad(const double2* __restrict__ G, const double2* __restrict__ R,
                                                    const double2* __restrict__ A, const double2* __restrict__ C,
                                                    const double2* __restrict__ B1, const double2* __restrict__ B2,
                                                    int m, const double* __restrict__ M,
                                                    const double* __restrict__ D0,
                                                    const double* __restrict__ E, const float* __restrict__ beta,
                                                    const int* __restrict__ shell, double* __restrict__ dO,
                                                    double* __restrict__ dbeta, long long N) {
    __shared__ double sh[4];
    const LayerCoef lc = layer_coef(beta);
    double gb0 = 0.0, gb1 = 0.0, gbd = 0.0;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (long long)gridDim.x * blockDim.x) {
        double dd = 0.0, de = 0.0, ga = 0.0, gc = 0.0;
        for (int j = 0; j < m; ++j) {
            const size_t o = (size_t)j * N + k;
            double2 g = G[o], r = R[o], a = A[o], c = C[o], p1 = B1[o], p2 = B2[o];
            double gr = redot(g, r), gA = redot(g, a), gC = redot(g, c);
            dd += gr;
            de += lc.c0 * (gA + redot(p1, r)) + lc.c1 * (gC + redot(p1, a) + redot(p2, r));
            ga += gA;
            gc += gC;
        }
        const double e = E[k];
        const int s = shell[k];
        atomicAdd(&dO[2 * s], dd * (D0[k] - 0.5 * M[k]));  // dD0/do0 = M exp(o0) / 2
        atomicAdd(&dO[2 * s + 1], (de + lc.dl * dd) * e);
        gb0 += ga * e;
        gb1 += gc * e;
        gbd += dd * e;
    }
    double v = block_sum(gb0, sh);
    if (threadIdx.x == 0) atomicAdd(&dbeta[0], v);
    v = block_sum(gb1, sh);
    if (threadIdx.x == 0) atomicAdd(&dbeta[1], v);
    v = block_sum(gbd, sh);
    if (threadIdx.x == 0) atomicAdd(&dbeta[2], v);
}

// (dL/dc0, dL/dc1, dL/ddl) -> gradient of (beta0, beta1); below zero beta1 passes
// the gradient of its positive side so that the optimiser can switch the layers on
__global__ void k_beta_grad(const double* __restrict__ dbeta, const float* __restrict__ beta, float* __restrict__ g) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const LayerCoef lc = layer_coef(beta);
    const double g0 = dbeta[0], g1 = dbeta[1], gd = dbeta[2];
    g[0] = (float)(2.0 * lc.b1 * g0 + 2.0 * lc.a * lc.b1 * gd);
    g[1] = (float)(2.0 * lc.a * g0 + g1 + lc.a * lc.a * gd);
}

__global__ void k_to_float(const double* __restrict__ a, float* __restrict__ b, int n, double scale) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) b[e] = (float)(a[e] * scale);
}

__global__ void k_nonfinite(const float* __restrict__ a, int n, int* __restrict__ flag) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n && !isfinite(a[e])) atomicOr(flag, 1);
}

__global__ void k_nonfinite_d(const double* __restrict__ a, long long n, int* __restrict__ flag) {
    bool bad = false;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
        bad = bad || !isfinite(a[k]);
    if (bad) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
static int blocks_for(long long n, int cap) {
    long long b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}
constexpr int kGridCap = 4096;
constexpr int kNoCap = 1 << 30;

hipError_t lp_dense_fwd(const float* X, const uint16_t* W, const float* b, float* Z, float* Y, int S, int in, int out,
                        int act, hipStream_t st) {
    k_dense_fwd<<<blocks_for((long long)S * out, kNoCap), 256, 0, st>>>(X, W, b, Z, Y, S, in, out, act);
    return hipGetLastError();
}
hipError_t lp_act_bwd(const float* dY, const float* Z, float* dZ, int n, int act, hipStream_t st) {
    k_act_bwd<<<blocks_for(n, kNoCap), 256, 0, st>>>(dY, Z, dZ, n, act);
    return hipGetLastError();
}
hipError_t lp_dense_bwd(const float* X, const float* dZ, const uint16_t* W, float* dX, float* dW, float* db, int S,
                        int in, int out, hipStream_t st) {
    if (dX) k_dense_bwd_data<<<blocks_for((long long)S * in, kNoCap), 256, 0, st>>>(dZ, W, dX, S, in, out);
    k_dense_bwd_weight<<<blocks_for((long long)in * out + out, kNoCap), 256, 0, st>>>(X, dZ, dW, db, S, in, out);
    return hipGetLastError();
}
hipError_t lp_adam(float* w, float* m, float* v, const float* g, uint16_t* wbf, int n, float lr, float b1, float b2,
                   float c1, float c2, float eps, hipStream_t st) {
    k_adam<<<blocks_for(n, kNoCap), 256, 0, st>>>(w, m, v, g, wbf, n, lr, b1, b2, c1, c2, eps);
    return hipGetLastError();
}
hipError_t lp_to_bf16(const float* w, uint16_t* wbf, int n, hipStream_t st) {
    k_to_bf16<<<blocks_for(n, kNoCap), 256, 0, st>>>(w, wbf, n);
    return hipGetLastError();
}
hipError_t lp_expand(const double* M, const int* shell, const float* O, double* D0, double* E, long long N,
                     hipStream_t st) {
    k_expand<<<blocks_for(N, kGridCap), 256, 0, st>>>(M, shell, O, D0, E, N);
    return hipGetLastError();
}
hipError_t lp_scale_cols(const ColPtrs& R, double2* Y, int m, const double* d, long long N, hipStream_t st) {
    k_scale_cols<<<blocks_for(N, kGridCap), 256, 0, st>>>(R, Y, m, d, N);
    return hipGetLastError();
}
hipError_t lp_scale(const double2* A, double2* Y, int m, const double* d, long long N, hipStream_t st) {
    k_scale<<<blocks_for(N, kGridCap), 256, 0, st>>>(A, Y, m, d, N);
    return hipGetLastError();
}
hipError_t lp_combine(const ColPtrs& R, const double2* A, const double2* C, const ColPtrs& W, int m, const double* D0,
                      const double* E, const float* beta, long long N, hipStream_t st) {
    k_combine<<<blocks_for(N, kGridCap), 256, 0, st>>>(R, A, C, W, m, D0, E, beta, N);
    return hipGetLastError();
}
hipError_t lp_shell_grad(const double2* G, const double2* R, const double2* A, const double2* C, const double2* B1,
                         const double2* B2, int m, const double* M, const double* D0, const double* E,
                         const float* beta, const int* shell, double* dO, double* dbeta, long long N,
                         hipStream_t st) {
    k_shell_grad<<<blocks_for(N, kGridCap), 256, 0, st>>>(G, R, A, C, B1, B2, m, M, D0, E, beta, shell, dO, dbeta,
                                                          N);
    return hipGetLastError();
}
hipError_t lp_beta_grad(const double* dbeta, const float* beta, float* g, hipStream_t st) {
    k_beta_grad<<<1, 64, 0, st>>>(dbeta, beta, g);
    return hipGetLastError();
}
hipError_t lp_to_float(const double* a, float* b, int n, double scale, hipStream_t st) {
    k_to_float<<<blocks_for(n, kNoCap), 256, 0, st>>>(a, b, n, scale);
    return hipGetLastError();
}
hipError_t lp_nonfinite_d(const double* a, long long n, int* flag, hipStream_t st) {
    k_nonfinite_d<<<blocks_for(n, kGridCap), 256, 0, st>>>(a, n, flag);
    return hipGetLastError();
}
hipError_t lp_nonfinite(const float* a, int n, int* flag, hipStream_t st) {
    k_nonfinite<<<blocks_for(n, kNoCap), 256, 0, st>>>(a, n, flag);
    return hipGetLastError();
}

}  // namespace iwfpm
