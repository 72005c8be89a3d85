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
// dense layers of the shell MLP on the matrix cores (v_mfma_f32_16x16x16_bf16,
// float32 accumulation).  The weights are bfloat16; an operand held in
// float32 (activations, gradients) is split into three bfloat16 terms
// x = h + m + l (each the round-to-nearest of what the previous ones left),
// which carry its full 24-bit significand, and products of bfloat16 terms are
// exact in float32, so each layer computes what a float32 loop over the
// bf16-rounded weights would, up to the order of the float32 additions.
// Lane l of a wave holds A[l%16][4(l/16) .. 4(l/16)+3] and
// B[4(l/16) .. 4(l/16)+3][l%16] of a 16 x 16 x 16 step and ends with
// D[4(l/16) + v][l%16], v < 4; one wave per 16 x 16 tile of the output.
// ---------------------------------------------------------------------------
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// operand element (r, c) at p[r * sr + c * sc], float32 or (bf16 != 0) bfloat16
struct MatOp {
    const void* p;
    int sr, sc, bf16;
};

__device__ __forceinline__ float op_at(const MatOp& o, int r, int c) {
    const size_t e = (size_t)r * o.sr + (size_t)c * o.sc;
    return o.bf16 ? bf2f(reinterpret_cast<const uint16_t*>(o.p)[e]) : reinterpret_cast<const float*>(o.p)[e];
}

// x = h + m + l in bfloat16 (exact for normal float32 x)
__device__ __forceinline__ void split3(float x, short& h, short& m, short& l) {
    const uint16_t a = f2bf(x);
    const float r1 = x - bf2f(a);
    const uint16_t b = f2bf(r1);
    const float r2 = r1 - bf2f(b);
    h = (short)a;
    m = (short)b;
    l = (short)f2bf(r2);
}

// C (M x N, row-major, ldc) = A (M x K) B (K x N) [+ bias[n]]; Z (optional)
// receives C, Y = act(C).  Terms: 3 for A (float32) x B (bfloat16), the six
// largest of the nine for float32 x float32 (what is left is below 2^-23 of
// each product).
__global__ void __launch_bounds__(256) k_mlp_gemm(MatOp A, MatOp B, const float* __restrict__ bias, float* __restrict__ Z,
                                                  float* __restrict__ Y, int M, int N, int K, int act) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tiles_n = (N + 15) >> 4;
    const int tile = blockIdx.x * 4 + wave;
    const int tm = tile / tiles_n, tn = tile - tm * tiles_n;
    if (tm * 16 >= M) return;
    const int li = lane & 15, lk = 4 * (lane >> 4);
    const int row = tm * 16 + li, col = tn * 16 + li;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x4 ah, am, al, bh, bm, bl;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = k0 + lk + q;
            const float a = (row < M && k < K) ? op_at(A, row, k) : 0.f;
            const float b = (col < N && k < K) ? op_at(B, k, col) : 0.f;
            short h, m, l;
            split3(a, h, m, l);
            ah[q] = h;
            am[q] = m;
            al[q] = l;
            split3(b, h, m, l);
            bh[q] = h;
            bm[q] = m;
            bl[q] = l;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
        if (!B.bf16) {
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bm, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am, bm, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = tm * 16 + lk + v, c = tn * 16 + li;
        if (r < M && c < N) {
            float z = acc[v] + (bias ? bias[c] : 0.f);
            const size_t e = (size_t)r * N + c;
            if (Z) Z[e] = z;
            Y[e] = act ? gelu(z) : z;
        }
    }
}

__global__ void k_act_bwd(const float* __restrict__ dY, const float* __restrict__ Z, float* __restrict__ dZ, int n,
                          int act) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    dZ[e] = act ? dY[e] * gelu_grad(Z[e]) : dY[e];
}

// db[o] = sum_s dZ[s][o] (fixed summation order)
__global__ void k_bias_grad(const float* __restrict__ dZ, float* __restrict__ db, int S, int out) {
    int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= out) return;
    float acc = 0.f;
    for (int s = 0; s < S; ++s) acc += dZ[(size_t)s * out + o];
    db[o] = acc;
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

static int mlp_blocks(int M, int N) {
    const long long tiles = (long long)((M + 15) / 16) * ((N + 15) / 16);
    return (int)((tiles + 3) / 4);
}

hipError_t lp_dense_fwd(const float* X, const uint16_t* W, const float* b, float* Z, float* Y, int S, int in, int out,
                        int act, hipStream_t st) {
    // A = X (S x in, row-major), B = W (in x out, row-major, bfloat16)
    const MatOp A{X, in, 1, 0}, B{W, out, 1, 1};
    k_mlp_gemm<<<mlp_blocks(S, out), 256, 0, st>>>(A, B, b, Z, Y, S, out, in, act);
    return hipGetLastError();
}
hipError_t lp_act_bwd(const float* dY, const float* Z, float* dZ, int n, int act, hipStream_t st) {
    k_act_bwd<<<blocks_for(n, kNoCap), 256, 0, st>>>(dY, Z, dZ, n, act);
    return hipGetLastError();
}
hipError_t lp_dense_bwd(const float* X, const float* dZ, const uint16_t* W, float* dX, float* dW, float* db, int S,
                        int in, int out, hipStream_t st) {
    if (dX) {
        // dX (S x in) = dZ (S x out) W^T: B[k][n] = W[n][k]
        const MatOp A{dZ, out, 1, 0}, B{W, 1, out, 1};
        k_mlp_gemm<<<mlp_blocks(S, in), 256, 0, st>>>(A, B, nullptr, nullptr, dX, S, in, out, 0);
    }
    {
        // dW (in x out) = X^T (in x S) dZ (S x out): A[r][k] = X[k][r]
        const MatOp A{X, 1, in, 0}, B{dZ, out, 1, 0};
        k_mlp_gemm<<<mlp_blocks(in, out), 256, 0, st>>>(A, B, nullptr, nullptr, dW, in, out, S, 0);
    }
    k_bias_grad<<<(out + 255) / 256, 256, 0, st>>>(dZ, db, S, out);
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
