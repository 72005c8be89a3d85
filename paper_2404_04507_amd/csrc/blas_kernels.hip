// blas_kernels.hip - float64 block algebra of the block LOBPCG eigensolver.
//
// All blocks are complex float64, one contiguous column of N entries per
// vector; kernels take lists of column pointers so that any subset of the
// X / W / P blocks can be combined without copies.
//
//   gram      C = L^H R            tall-skinny (p, q <= 64), two-stage
//                                  deterministic reduction
//   lincomb   Y = beta Y + A C     (p <= 64 inputs, q <= 32 outputs per call)
//   residual  R_j = HX_j - theta_j X_j
//   colnorm2  ||R_j||^2           two-stage deterministic reduction
//   precond   W_j = M .* R_j       diagonal preconditioner (eq:precond)
//   randn     counter-based complex normal start block

#include <hip/hip_runtime.h>

#include "blas.hpp"

namespace iwfpm {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ---------------------------------------------------------------------------
// gram: partial[b][j][i] = sum over rows of block b of conj(L_i[r]) R_j[r]
// Thread (ti, tj) of a 16 x 16 grid owns the 4 x 4 output tile
// i = 4 ti + a, j = 4 tj + b.  Rows are staged through LDS 16 at a time.
// ---------------------------------------------------------------------------
constexpr int kGramRows = 16;

__global__ void __launch_bounds__(256) k_gram(ColPtrs L, int p, ColPtrs R, int q, long long N, long long rows_per_block,
                                              double2* __restrict__ partial) {
    __shared__ double2 sL[kGramRows][kMaxCols + 1];
    __shared__ double2 sR[kGramRows][kMaxCols + 1];
    const int tid = threadIdx.x;
    const int ti = tid & 15, tj = tid >> 4;
    double2 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0.0, 0.0);
    const long long r0 = (long long)blockIdx.x * rows_per_block;
    const long long r1 = min(N, r0 + rows_per_block);
    for (long long rb = r0; rb < r1; rb += kGramRows) {
        const int nr = (int)min((long long)kGramRows, r1 - rb);
        // stage: column c, row rr; consecutive threads take consecutive rows
        for (int e = tid; e < kGramRows * p; e += 256) {
            int c = e / kGramRows, rr = e - c * kGramRows;
            sL[rr][c] = rr < nr ? L.p[c][rb + rr] : make_double2(0.0, 0.0);
        }
        for (int e = tid; e < kGramRows * q; e += 256) {
            int c = e / kGramRows, rr = e - c * kGramRows;
            sR[rr][c] = rr < nr ? R.p[c][rb + rr] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        if (4 * ti < p && 4 * tj < q) {
            for (int rr = 0; rr < nr; ++rr) {
                double2 l[4], r[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) l[a] = sL[rr][4 * ti + a];
#pragma unroll
                for (int b = 0; b < 4; ++b) r[b] = sR[rr][4 * tj + b];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        // conj(l) * r
                        acc[a][b].x += l[a].x * r[b].x + l[a].y * r[b].y;
                        acc[a][b].y += l[a].x * r[b].y - l[a].y * r[b].x;
                    }
            }
        }
        __syncthreads();
    }
    double2* out = partial + (size_t)blockIdx.x * p * q;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            int i = 4 * ti + a, j = 4 * tj + b;
            if (i < p && j < q) out[(size_t)j * p + i] = acc[a][b];
        }
}

// sum the partials of nb blocks in block order: C[j*p + i]
__global__ void k_reduce_partials(const double2* __restrict__ partial, int nb, int count, double2* __restrict__ C) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    double2 s = make_double2(0.0, 0.0);
    for (int b = 0; b < nb; ++b) {
        double2 v = partial[(size_t)b * count + e];
        s.x += v.x;
        s.y += v.y;
    }
    C[e] = s;
}

// ---------------------------------------------------------------------------
// lincomb: Y_j = beta Y_j + sum_i A_i C[j*p + i]   (q <= QB)
// ---------------------------------------------------------------------------
template <int QB>
__global__ void __launch_bounds__(256) k_lincomb(ColPtrs A, int p, ColPtrs Y, int q, const double2* __restrict__ C,
                                                 double beta, long long N) {
    __shared__ double2 sC[kMaxCols * 32];
    for (int e = threadIdx.x; e < p * q; e += blockDim.x) sC[e] = C[e];
    __syncthreads();
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (long long)gridDim.x * blockDim.x) {
        double2 acc[QB];
#pragma unroll
        for (int j = 0; j < QB; ++j) {
            if (j < q && beta != 0.0) {
                double2 y = Y.p[j][r];
                acc[j] = make_double2(beta * y.x, beta * y.y);
            } else {
                acc[j] = make_double2(0.0, 0.0);
            }
        }
        for (int i = 0; i < p; ++i) {
            double2 a = A.p[i][r];
#pragma unroll
            for (int j = 0; j < QB; ++j) {
                if (j < q) {
                    double2 c = sC[j * p + i];
                    acc[j].x += a.x * c.x - a.y * c.y;
                    acc[j].y += a.x * c.y + a.y * c.x;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < QB; ++j)
            if (j < q) Y.p[j][r] = acc[j];
    }
}

// ---------------------------------------------------------------------------
// residual, column norms, preconditioner, random start
// ---------------------------------------------------------------------------
__global__ void k_residual(ColPtrs HX, ColPtrs X, ColPtrs Rout, Reals theta, int m, long long N) {
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (long long)gridDim.x * blockDim.x) {
        for (int j = 0; j < m; ++j) {
            double2 h = HX.p[j][r], x = X.p[j][r];
            double t = theta.v[j];
            Rout.p[j][r] = make_double2(h.x - t * x.x, h.y - t * x.y);
        }
    }
}

__global__ void __launch_bounds__(256) k_colnorm2(ColPtrs V, int m, long long N, long long rows_per_block,
                                                  double* __restrict__ partial) {
    __shared__ double red[256];
    const long long r0 = (long long)blockIdx.x * rows_per_block;
    const long long r1 = min(N, r0 + rows_per_block);
    for (int j = 0; j < m; ++j) {
        double s = 0.0;
        for (long long r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
            double2 v = V.p[j][r];
            s += v.x * v.x + v.y * v.y;
        }
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(size_t)blockIdx.x * m + j] = red[0];
        __syncthreads();
    }
}

__global__ void k_reduce_real(const double* __restrict__ partial, int nb, int count, double* __restrict__ out) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[(size_t)b * count + e];
    out[e] = s;
}

__global__ void k_precond(ColPtrs R, ColPtrs W, int m, const double* __restrict__ M, long long N) {
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (long long)gridDim.x * blockDim.x) {
        double mm = M[r];
        for (int j = 0; j < m; ++j) {
            double2 v = R.p[j][r];
            W.p[j][r] = make_double2(mm * v.x, mm * v.y);
        }
    }
}

// splitmix64 (Steele, Lea, Flood 2014) as a counter-based generator; two
// uniforms -> one complex standard normal by the Box-Muller transform
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ void k_randn(double2* __restrict__ out, long long count, unsigned long long seed) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (long long)gridDim.x * blockDim.x) {
        unsigned long long a = splitmix64(seed ^ splitmix64(2ull * (unsigned long long)e));
        unsigned long long b = splitmix64(seed ^ splitmix64(2ull * (unsigned long long)e + 1ull));
        double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740993.0);  // (0, 1]
        double u2 = (b >> 11) * (1.0 / 9007199254740992.0);          // [0, 1)
        double rad = sqrt(-log(u1));                                  // variance 1/2 per part
        double s, c;
        sincospi(2.0 * u2, &s, &c);
        out[e] = make_double2(rad * c, rad * s);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static int grid_for(long long N, int threads, int cap = 4096) {
    long long b = (N + threads - 1) / threads;
    return (int)std::max(1LL, std::min<long long>(b, cap));
}

hipError_t gram(const ColPtrs& L, int p, const ColPtrs& R, int q, long long N, double2* partial, int max_blocks,
                double2* C, hipStream_t st) {
    if (p <= 0 || q <= 0) return hipSuccess;
    long long rpb = (N + max_blocks - 1) / max_blocks;
    rpb = ((rpb + kGramRows - 1) / kGramRows) * kGramRows;
    int nb = (int)((N + rpb - 1) / rpb);
    k_gram<<<nb, 256, 0, st>>>(L, p, R, q, N, rpb, partial);
    int cnt = p * q;
    k_reduce_partials<<<(cnt + 255) / 256, 256, 0, st>>>(partial, nb, cnt, C);
    return hipGetLastError();
}

hipError_t lincomb(const ColPtrs& A, int p, const ColPtrs& Y, int q, const double2* C, double beta, long long N,
                   hipStream_t st) {
    if (q <= 0) return hipSuccess;
    int nb = grid_for(N, 256, 2048);
    if (q <= 8) k_lincomb<8><<<nb, 256, 0, st>>>(A, p, Y, q, C, beta, N);
    else if (q <= 16) k_lincomb<16><<<nb, 256, 0, st>>>(A, p, Y, q, C, beta, N);
    else k_lincomb<32><<<nb, 256, 0, st>>>(A, p, Y, q, C, beta, N);
    return hipGetLastError();
}

hipError_t residual(const ColPtrs& HX, const ColPtrs& X, const ColPtrs& R, const Reals& theta, int m, long long N,
                    hipStream_t st) {
    k_residual<<<grid_for(N, 256), 256, 0, st>>>(HX, X, R, theta, m, N);
    return hipGetLastError();
}

hipError_t colnorm2(const ColPtrs& V, int m, long long N, double* partial, int max_blocks, double* out,
                    hipStream_t st) {
    if (m <= 0) return hipSuccess;
    long long rpb = (N + max_blocks - 1) / max_blocks;
    int nb = (int)((N + rpb - 1) / rpb);
    k_colnorm2<<<nb, 256, 0, st>>>(V, m, N, rpb, partial);
    k_reduce_real<<<(m + 255) / 256, 256, 0, st>>>(partial, nb, m, out);
    return hipGetLastError();
}

hipError_t precond(const ColPtrs& R, const ColPtrs& W, int m, const double* M, long long N, hipStream_t st) {
    k_precond<<<grid_for(N, 256), 256, 0, st>>>(R, W, m, M, N);
    return hipGetLastError();
}

hipError_t randn(double2* out, long long count, unsigned long long seed, hipStream_t st) {
    k_randn<<<grid_for(count, 256), 256, 0, st>>>(out, count, seed);
    return hipGetLastError();
}

}  // namespace iwfpm
