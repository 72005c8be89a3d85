// blas_kernels.hip - float64 block algebra of the block LOBPCG eigensolver.
//
// All blocks are complex float64, one contiguous column of N entries per
// vector; kernels take lists of column pointers so that any subset of the
// X / W / P blocks can be combined without copies.
//
//   gram      C = L^H R            tall-skinny (p, q <= 64) on the matrix
//                                  cores, operands straight from HBM;
//                                  two-stage deterministic reduction
//   lincomb   Y = beta Y + A C     (p <= 64 inputs, q <= 48 outputs per call);
//                                  up to 32 outputs with vector FMAs (two rows
//                                  per lane), wider on the matrix cores
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
// gram: partial[b][j*p + i] = sum over the rows of block b of
// conj(L_i[r]) R_j[r] on the matrix cores (v_mfma_f64_16x16x4f64), operands
// loaded straight from HBM into the MFMA register layout (no LDS staging).
// Lane l of a wave holds A[l%16][l/16] and B[l/16][l%16] and ends with result
// v in D[l/16 + 4v][l%16].  The K index runs over 4-row groups: lane l loads
// the complex entry at row 4g + l/16 of column 16t + l%16, so one 16-byte load
// feeds two products (re, then im parts):
//   Re C += Lr Rr + Li Ri,   Im C += Lr Ri - Li Rr.
// A workgroup has one wave per 16-column tile of L; every wave walks the same
// rows and multiplies its tile by all TQ tiles of R (the R loads of the other
// waves hit in L1), keeping 2 TQ accumulators.  Loads run D groups ahead.
// ---------------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int kGramDepth = 8;  // 4-row groups in flight per wave

template <int TQ>
__device__ __forceinline__ void gram_load(const double2* lp, const double2* const (&rp)[TQ], long long g, long long g1,
                                          long long N, int lk, double2& lv, double2 (&rv)[TQ]) {
    const long long row = 4 * g + lk;
    const bool ok = g < g1 && row < N;
    lv = (ok && lp) ? lp[row] : make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < TQ; ++t) rv[t] = (ok && rp[t]) ? rp[t][row] : make_double2(0.0, 0.0);
}

// PAIRS: every complex column holds two real vectors (real part, imaginary
// part) and the result is their real Gram, four accumulators per tile
// (rr, ri, ir, ii), written as real (2p x 2q, column-major) partials.
template <int TQ, bool PAIRS = false>
__device__ __forceinline__ void gram_body(const ColPtrs& L, int p, const ColPtrs& R, int q, long long N,
                                          long long groups_per_block, double2* __restrict__ partial, int bid) {
    constexpr int D = kGramDepth;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int cl = 16 * wave + li;
    const double2* lp = cl < p ? L.p[cl] : nullptr;
    const double2* rp[TQ];
#pragma unroll
    for (int t = 0; t < TQ; ++t) {
        const int c = 16 * t + li;
        rp[t] = c < q ? R.p[c] : nullptr;
    }
    dbl4 accr[TQ], acci[TQ], accx[PAIRS ? TQ : 1], accy[PAIRS ? TQ : 1];
#pragma unroll
    for (int b = 0; b < TQ; ++b) {
        accr[b] = dbl4{0.0, 0.0, 0.0, 0.0};
        acci[b] = dbl4{0.0, 0.0, 0.0, 0.0};
        if constexpr (PAIRS) {
            accx[b] = dbl4{0.0, 0.0, 0.0, 0.0};
            accy[b] = dbl4{0.0, 0.0, 0.0, 0.0};
        }
    }
    const long long G = (N + 3) >> 2;
    const long long g0 = (long long)bid * groups_per_block, g1 = min(G, g0 + groups_per_block);
    double2 lb[D], rb[D][TQ];
#pragma unroll
    for (int d = 0; d < D; ++d) gram_load<TQ>(lp, rp, g0 + d, g1, N, lk, lb[d], rb[d]);
    for (long long g = g0; g < g1; g += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double2 lv = lb[d];
            double2 rv[TQ];
#pragma unroll
            for (int t = 0; t < TQ; ++t) rv[t] = rb[d][t];
            gram_load<TQ>(lp, rp, g + d + D, g1, N, lk, lb[d], rb[d]);
#pragma unroll
            for (int b = 0; b < TQ; ++b) {
                accr[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(lv.x, rv[b].x, accr[b], 0, 0, 0);
                acci[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(lv.x, rv[b].y, acci[b], 0, 0, 0);
            }
            if constexpr (PAIRS) {
#pragma unroll
                for (int b = 0; b < TQ; ++b) {
                    accx[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(lv.y, rv[b].x, accx[b], 0, 0, 0);
                    accy[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(lv.y, rv[b].y, accy[b], 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int b = 0; b < TQ; ++b) {
                    accr[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(lv.y, rv[b].y, accr[b], 0, 0, 0);
                    acci[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(lv.y, -rv[b].x, acci[b], 0, 0, 0);
                }
            }
        }
    }
    if constexpr (PAIRS) {
        double* out = reinterpret_cast<double*>(partial) + (size_t)bid * 4 * p * q;
        const size_t ld = 2 * (size_t)p;
#pragma unroll
        for (int b = 0; b < TQ; ++b) {
            const int j = 16 * b + li;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * wave + lk + 4 * v;
                if (i < p && j < q) {
                    out[(2 * (size_t)j) * ld + 2 * i] = accr[b][v];          // re . re
                    out[(2 * (size_t)j + 1) * ld + 2 * i] = acci[b][v];      // re . im
                    out[(2 * (size_t)j) * ld + 2 * i + 1] = accx[b][v];      // im . re
                    out[(2 * (size_t)j + 1) * ld + 2 * i + 1] = accy[b][v];  // im . im
                }
            }
        }
    } else {
        double2* out = partial + (size_t)bid * p * q;
#pragma unroll
        for (int b = 0; b < TQ; ++b) {
            const int j = 16 * b + li;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * wave + lk + 4 * v;
                if (i < p && j < q) out[(size_t)j * p + i] = make_double2(accr[b][v], acci[b][v]);
            }
        }
    }
}

// one wave per 16 columns of L (blockDim = 64 ceil(p / 16))
template <int TQ>
__global__ void __launch_bounds__(256) k_gram(ColPtrs L, int p, ColPtrs R, int q, long long N, long long groups_per_block,
                                              double2* __restrict__ partial) {
    gram_body<TQ>(L, p, R, q, N, groups_per_block, partial, blockIdx.x);
}

template <int TQ>
__global__ void __launch_bounds__(256) k_gram_pairs(ColPtrs L, int p, ColPtrs R, int q, long long N,
                                                    long long groups_per_block, double2* __restrict__ partial) {
    gram_body<TQ, true>(L, p, R, q, N, groups_per_block, partial, blockIdx.x);
}

// C[e] = sum over the nb partials, one workgroup per entry, fixed summation order
__global__ void __launch_bounds__(256) k_reduce_partials(const double2* __restrict__ partial, int nb, int count,
                                                         double2* __restrict__ C) {
    __shared__ double2 red[256];
    const int e = blockIdx.x;
    double2 s = make_double2(0.0, 0.0);
    for (int b = threadIdx.x; b < nb; b += 256) {
        double2 v = partial[(size_t)b * count + e];
        s.x += v.x;
        s.y += v.y;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[threadIdx.x].x += red[threadIdx.x + w].x;
            red[threadIdx.x].y += red[threadIdx.x + w].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) C[e] = red[0];
}

// ---------------------------------------------------------------------------
// lincomb, q <= 32: the four wavefronts of a workgroup share a pair of 64-row
// strips (rows r and r + 64 per lane) and split the outputs, wave w taking
// columns [w qg, w qg + qg) with qg = ceil(q / 4).  C (column-major, C[j*p + i])
// is read at wave-uniform addresses: straight from global memory by scalar
// loads when it is a kernel argument, else from an LDS copy.  Two rows per
// lane halve the C reads per multiply-add and double the loads in flight.
// ---------------------------------------------------------------------------
// PAIRS: A and Y hold two real vectors per complex column and C is the real
// (2p x 2q, column-major) coefficient matrix: each (input, output) column pair
// takes a 2 x 2 real block.
template <int QG, bool PAIRS = false>
__device__ __forceinline__ void lincomb_rows_body(const ColPtrs& A, int p, const ColPtrs& Y, int q,
                                                  const double2* __restrict__ C, double beta, long long N, int bid,
                                                  int nb) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int qg = (q + 3) >> 2;
    const int j0 = wave * qg;
    const int nj = max(0, min(qg, q - j0));
    if (nj == 0) return;
    for (long long r = (long long)bid * 128 + lane; r < N; r += (long long)nb * 128) {
        const long long r2 = r + 64;
        const bool ok2 = r2 < N;
        double2 acc[QG], acc2[QG];
#pragma unroll
        for (int j = 0; j < QG; ++j) {
            acc[j] = make_double2(0.0, 0.0);
            acc2[j] = make_double2(0.0, 0.0);
            if (j < nj && beta != 0.0) {
                const double2 y = Y.p[j0 + j][r];
                acc[j] = make_double2(beta * y.x, beta * y.y);
                if (ok2) {
                    const double2 y2 = Y.p[j0 + j][r2];
                    acc2[j] = make_double2(beta * y2.x, beta * y2.y);
                }
            }
        }
        // The pair form reads four coefficients per (input, output) pair through
        // the scalar unit; with many outputs per wave an unrolled input loop
        // holds more of them than there are SGPRs (they spill to VGPR lanes),
        // so it runs one input at a time there and relies on occupancy.
        constexpr int kInUnroll = (PAIRS && QG >= 4) ? 1 : 4;
#pragma unroll kInUnroll
        for (int i = 0; i < p; ++i) {
            const double2 a = A.p[i][r];
            const double2 a2 = ok2 ? A.p[i][r2] : make_double2(0.0, 0.0);
            if constexpr (PAIRS) {
                // C real: rows 2i, 2i+1 of columns 2(j0+j), 2(j0+j)+1 (leading dimension 2p)
                const double2* ci = C + (size_t)(2 * j0) * p + i;
#pragma unroll
                for (int j = 0; j < QG; ++j) {
                    if (j < nj) {
                        const double2 c0 = ci[(size_t)(2 * j) * p];      // (C[2i][2k], C[2i+1][2k])
                        const double2 c1 = ci[(size_t)(2 * j + 1) * p];  // (C[2i][2k+1], C[2i+1][2k+1])
                        acc[j].x += a.x * c0.x + a.y * c0.y;
                        acc[j].y += a.x * c1.x + a.y * c1.y;
                        acc2[j].x += a2.x * c0.x + a2.y * c0.y;
                        acc2[j].y += a2.x * c1.x + a2.y * c1.y;
                    }
                }
            } else {
                const double2* ci = C + (size_t)j0 * p + i;
#pragma unroll
                for (int j = 0; j < QG; ++j) {
                    if (j < nj) {
                        const double2 c = ci[(size_t)j * p];
                        acc[j].x += a.x * c.x - a.y * c.y;
                        acc[j].y += a.x * c.y + a.y * c.x;
                        acc2[j].x += a2.x * c.x - a2.y * c.y;
                        acc2[j].y += a2.x * c.y + a2.y * c.x;
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < QG; ++j)
            if (j < nj) {
                Y.p[j0 + j][r] = acc[j];
                if (ok2) Y.p[j0 + j][r2] = acc2[j];
            }
    }
}

template <int QG>
__global__ void __launch_bounds__(256) k_lincomb_rows(ColPtrs A, int p, ColPtrs Y, int q,
                                                      const double2* __restrict__ C, double beta, long long N) {
    lincomb_rows_body<QG>(A, p, Y, q, C, beta, N, blockIdx.x, gridDim.x);
}

template <int QG>
__global__ void __launch_bounds__(256) k_lincomb_pairs(ColPtrs A, int p, ColPtrs Y, int q,
                                                       const double2* __restrict__ C, double beta, long long N) {
    lincomb_rows_body<QG, true>(A, p, Y, q, C, beta, N, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// lincomb, 32 < q <= 48: Y_j = beta Y_j + sum_i A_i C[j*p + i]
//
// On the matrix cores: with the K index over (input column i, re/im),
// Re Y = sum_k Ax[r][k] Bre[k][j] and Im Y = sum_k Ax[r][k] Bim[k][j],
// Bre = (Re C, -Im C), Bim = (Im C, Re C) interleaved by (i, re/im).  Each
// wavefront owns 16-row tiles (grid-stride); its A operand is read straight
// from HBM (lanes 0-31 cover 16 rows of one input column, 256 contiguous
// bytes) exactly once, 8 K steps (16 input columns) ahead of their use, the
// prefetch running on into the next tile; C is staged transposed in LDS
// (zero-padded to 64 inputs) and each lane ends with whole complex outputs:
// rows lk + 4v of the tile, column 16 tq + li.
// ---------------------------------------------------------------------------
template <int TQ>
__device__ __forceinline__ void lincomb_body(const ColPtrs& A, int p, const ColPtrs& Y, int q,
                                             const double2* __restrict__ C, double beta, long long N, int bid, int nb,
                                             double2* sCt) {
    const int ldq = 16 * TQ;
    for (int e = threadIdx.x; e < kMaxCols * ldq; e += blockDim.x) {
        const int i = e / ldq, j = e - i * ldq;
        sCt[e] = (i < p && j < q) ? C[(size_t)j * p + i] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int li = lane & 15, lk = lane >> 4, half = lk >> 1, part = lk & 1;
    const int nchunk = (p + 15) >> 4;  // 8 K steps = 16 input columns per chunk
    const long long ntiles = (N + 15) >> 4;
    const long long t0 = (long long)bid * nw + wave, ts = (long long)nb * nw;
    auto fetch = [&](long long t, int kc, double (&a)[8]) {
        const long long ra = (t << 4) + li;
        const bool rok = t < ntiles && ra < N;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = 16 * kc + 2 * u + half;
            a[u] = (rok && i < p) ? reinterpret_cast<const double*>(A.p[i])[2 * ra + part] : 0.0;
        }
    };
    double an[8];
    fetch(t0, 0, an);
    for (long long t = t0; t < ntiles; t += ts) {
        const long long r0 = t << 4;
        dbl4 yr[TQ], yi[TQ];
#pragma unroll
        for (int c = 0; c < TQ; ++c) {
            yr[c] = dbl4{0.0, 0.0, 0.0, 0.0};
            yi[c] = dbl4{0.0, 0.0, 0.0, 0.0};
        }
        for (int kc = 0; kc < nchunk; ++kc) {
            double a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = an[u];
            if (kc + 1 < nchunk) fetch(t, kc + 1, an);
            else fetch(t + ts, 0, an);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = 16 * kc + 2 * u + half;
#pragma unroll
                for (int c = 0; c < TQ; ++c) {
                    const double2 cv = sCt[i * ldq + 16 * c + li];
                    const double br = part ? -cv.y : cv.x;
                    const double bi = part ? cv.x : cv.y;
                    yr[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], br, yr[c], 0, 0, 0);
                    yi[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bi, yi[c], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < TQ; ++c) {
            const int j = 16 * c + li;
            if (j >= q) continue;
            double2* yc = Y.p[j];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const long long row = r0 + lk + 4 * v;
                if (row >= N) continue;
                double2 y = make_double2(yr[c][v], yi[c][v]);
                if (beta != 0.0) {
                    const double2 old = yc[row];
                    y.x += beta * old.x;
                    y.y += beta * old.y;
                }
                yc[row] = y;
            }
        }
    }
}

template <int TQ>
__global__ void __launch_bounds__(256) k_lincomb(ColPtrs A, int p, ColPtrs Y, int q, const double2* __restrict__ C,
                                                 double beta, long long N) {
    __shared__ double2 sCt[kMaxCols * 48];
    lincomb_body<TQ>(A, p, Y, q, C, beta, N, blockIdx.x, gridDim.x, sCt);
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

__global__ void __launch_bounds__(256) k_reduce_real(const double* __restrict__ partial, int nb, int count,
                                                     double* __restrict__ out) {
    __shared__ double red[256];
    const int e = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += partial[(size_t)b * count + e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[e] = red[0];
}

// R_j = HX_j - theta_j X_j and the block's partial sums of ||R_j||^2
__device__ __forceinline__ void residual_norm_body(const ColPtrs& HX, const ColPtrs& X, const ColPtrs& Rout,
                                                   const Reals& theta, int m, long long N, long long rows_per_block,
                                                   double* __restrict__ partial, int bid, double* red) {
    const long long r0 = (long long)bid * rows_per_block;
    const long long r1 = min(N, r0 + rows_per_block);
    for (int j = 0; j < m; ++j) {
        double s = 0.0;
        const double t = theta.v[j];
        for (long long r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
            double2 h = HX.p[j][r], x = X.p[j][r];
            double2 v = make_double2(h.x - t * x.x, h.y - t * x.y);
            Rout.p[j][r] = v;
            s += v.x * v.x + v.y * v.y;
        }
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(size_t)bid * m + j] = red[0];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_residual_norm(ColPtrs HX, ColPtrs X, ColPtrs Rout, Reals theta, int m,
                                                       long long N, long long rows_per_block,
                                                       double* __restrict__ partial) {
    __shared__ double red[256];
    residual_norm_body(HX, X, Rout, theta, m, N, rows_per_block, partial, blockIdx.x, red);
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

// two real vectors per complex column: R = HX - X diag(theta) with one theta
// per real vector (theta[2j] for the real parts of column j, theta[2j+1] for
// the imaginary parts) and one squared norm per real vector
__device__ __forceinline__ void residual_norm_pairs_body(const ColPtrs& HX, const ColPtrs& X, const ColPtrs& Rout,
                                                         const Reals& theta, int m, long long N,
                                                         long long rows_per_block, double* __restrict__ partial,
                                                         int bid, double (*red)[256]) {
    const long long r0 = (long long)bid * rows_per_block;
    const long long r1 = min(N, r0 + rows_per_block);
    for (int j = 0; j < m; ++j) {
        double s0 = 0.0, s1 = 0.0;
        const double t0 = theta.v[2 * j], t1 = theta.v[2 * j + 1];
        for (long long r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
            const double2 h = HX.p[j][r], x = X.p[j][r];
            const double2 v = make_double2(h.x - t0 * x.x, h.y - t1 * x.y);
            Rout.p[j][r] = v;
            s0 += v.x * v.x;
            s1 += v.y * v.y;
        }
        red[0][threadIdx.x] = s0;
        red[1][threadIdx.x] = s1;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                red[0][threadIdx.x] += red[0][threadIdx.x + w];
                red[1][threadIdx.x] += red[1][threadIdx.x + w];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            partial[(size_t)bid * 2 * m + 2 * j] = red[0][0];
            partial[(size_t)bid * 2 * m + 2 * j + 1] = red[1][0];
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_residual_norm_pairs(ColPtrs HX, ColPtrs X, ColPtrs Rout, Reals theta, int m,
                                                             long long N, long long rows_per_block,
                                                             double* __restrict__ partial) {
    __shared__ double red[2][256];
    residual_norm_pairs_body(HX, X, Rout, theta, m, N, rows_per_block, partial, blockIdx.x, red);
}

// packs n real vectors (vector v: part (bit v of parts) of column src[v]),
// scaled by M when given, two per destination column; the imaginary half of
// the last column is zero when n is odd
__device__ __forceinline__ void gather_pairs_body(const ColPtrs& src, unsigned long long parts, int n, const ColPtrs& dst,
                                                  const double* __restrict__ M, long long N, int bid, int nb) {
    const int nd = (n + 1) >> 1;
    for (long long r = (long long)bid * blockDim.x + threadIdx.x; r < N; r += (long long)nb * blockDim.x) {
        const double mm = M ? M[r] : 1.0;
        for (int d = 0; d < nd; ++d) {
            const int v0 = 2 * d, v1 = 2 * d + 1;
            const double2 a = src.p[v0][r];
            double b = 0.0;
            if (v1 < n) {
                const double2 t = src.p[v1][r];
                b = ((parts >> v1) & 1) ? t.y : t.x;
            }
            dst.p[d][r] = make_double2(mm * (((parts >> v0) & 1) ? a.y : a.x), mm * b);
        }
    }
}

__global__ void k_gather_pairs(ColPtrs src, unsigned long long parts, int n, ColPtrs dst,
                               const double* __restrict__ M, long long N) {
    gather_pairs_body(src, parts, n, dst, M, N, blockIdx.x, gridDim.x);
}

// complex column v = (real vector v, 0), vector v being part (bit v) of src[v]
__global__ void k_unpack_real(ColPtrs src, unsigned long long parts, int n, ColPtrs dst, long long N) {
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (long long)gridDim.x * blockDim.x) {
        for (int v = 0; v < n; ++v) {
            const double2 a = src.p[v][r];
            dst.p[v][r] = make_double2(((parts >> v) & 1) ? a.y : a.x, 0.0);
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
// batched forms: many independent jobs (one per eigenproblem of a sweep) in
// one launch; job j owns blocks [start, start + nb) of the grid
// ---------------------------------------------------------------------------

template <typename J>
__device__ __forceinline__ int find_job(const J* __restrict__ jobs, int njobs, int b) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].start <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// blockDim = 64 ceil(max p / 16); the waves beyond a job's own L tiles have nothing to do
template <int TQ>
__global__ void __launch_bounds__(256) k_gram_batched(const GramJob* __restrict__ jobs, int njobs,
                                                      double2* __restrict__ partial) {
    const int j = find_job(jobs, njobs, blockIdx.x);
    const GramJob& jb = jobs[j];
    if ((int)(threadIdx.x >> 6) * 16 >= jb.p) return;
    gram_body<TQ>(jb.L, jb.p, jb.R, jb.q, jb.N, jb.groups_per_block, partial + jb.part_off, blockIdx.x - jb.start);
}

// one workgroup per output entry over all jobs (job j's entries start at out_start)
__global__ void __launch_bounds__(256) k_reduce_batched(const GramJob* __restrict__ jobs, int njobs,
                                                        const double2* __restrict__ partial,
                                                        double2* __restrict__ C) {
    __shared__ double2 red[256];
    const int e = blockIdx.x;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].out_start <= e) lo = mid;
        else hi = mid - 1;
    }
    const GramJob& jb = jobs[lo];
    const int le = e - jb.out_start, cnt = jb.p * jb.q * jb.width;
    double2 s = make_double2(0.0, 0.0);
    for (int b = threadIdx.x; b < jb.nb; b += 256) {
        double2 v = partial[jb.part_off + (size_t)b * cnt + le];
        s.x += v.x;
        s.y += v.y;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[threadIdx.x].x += red[threadIdx.x + w].x;
            red[threadIdx.x].y += red[threadIdx.x + w].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) C[e] = red[0];
}

template <int TQ>
__global__ void __launch_bounds__(256) k_lincomb_batched(const LinJob* __restrict__ jobs, int njobs) {
    __shared__ double2 sCt[kMaxCols * 48];
    const int j = find_job(jobs, njobs, blockIdx.x);
    const LinJob& jb = jobs[j];
    lincomb_body<TQ>(jb.A, jb.p, jb.Y, jb.q, jb.C, jb.beta, jb.N, blockIdx.x - jb.start, jb.nb, sCt);
}

template <int QG>
__global__ void __launch_bounds__(256) k_lincomb_rows_batched(const LinJob* __restrict__ jobs, int njobs) {
    __shared__ double2 sC[kMaxCols * 32];
    const int j = find_job(jobs, njobs, blockIdx.x);
    const LinJob& jb = jobs[j];
    for (int e = threadIdx.x; e < jb.p * jb.q; e += blockDim.x) sC[e] = jb.C[e];
    __syncthreads();
    lincomb_rows_body<QG>(jb.A, jb.p, jb.Y, jb.q, sC, jb.beta, jb.N, blockIdx.x - jb.start, jb.nb);
}

__global__ void __launch_bounds__(256) k_residual_norm_batched(const ResJob* __restrict__ jobs, int njobs,
                                                               double* __restrict__ partial) {
    __shared__ double red[256];
    const int j = find_job(jobs, njobs, blockIdx.x);
    const ResJob& jb = jobs[j];
    residual_norm_body(jb.HX, jb.X, jb.R, jb.theta, jb.m, jb.N, jb.rows_per_block, partial + jb.part_off,
                       blockIdx.x - jb.start, red);
}

// out[j's entries] = sums of the residual-norm partials
__global__ void __launch_bounds__(256) k_reduce_res_batched(const ResJob* __restrict__ jobs, int njobs,
                                                            const double* __restrict__ partial,
                                                            double* __restrict__ out) {
    __shared__ double red[256];
    const int e = blockIdx.x;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].out_start <= e) lo = mid;
        else hi = mid - 1;
    }
    const ResJob& jb = jobs[lo];
    const int le = e - jb.out_start;
    double s = 0.0;
    for (int b = threadIdx.x; b < jb.nb; b += 256) s += partial[jb.part_off + (size_t)b * (jb.m * jb.width) + le];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[e] = red[0];
}

template <int TQ>
__global__ void __launch_bounds__(256) k_gram_batched_pairs(const GramJob* __restrict__ jobs, int njobs,
                                                            double2* __restrict__ partial) {
    const int j = find_job(jobs, njobs, blockIdx.x);
    const GramJob& jb = jobs[j];
    if ((int)(threadIdx.x >> 6) * 16 >= jb.p) return;
    gram_body<TQ, true>(jb.L, jb.p, jb.R, jb.q, jb.N, jb.groups_per_block, partial + jb.part_off,
                        blockIdx.x - jb.start);
}

template <int QG>
__global__ void __launch_bounds__(256) k_lincomb_pairs_batched(const LinJob* __restrict__ jobs, int njobs) {
    __shared__ double2 sC[kLinPairsLds];
    const int j = find_job(jobs, njobs, blockIdx.x);
    const LinJob& jb = jobs[j];
    // the host rejects jobs with 2 p q > kLinPairsLds
    for (int e = threadIdx.x; e < 2 * jb.p * jb.q; e += blockDim.x) sC[e] = jb.C[e];
    __syncthreads();
    lincomb_rows_body<QG, true>(jb.A, jb.p, jb.Y, jb.q, sC, jb.beta, jb.N, blockIdx.x - jb.start, jb.nb);
}

__global__ void __launch_bounds__(256) k_residual_norm_pairs_batched(const ResJob* __restrict__ jobs, int njobs,
                                                                     double* __restrict__ partial) {
    __shared__ double red[2][256];
    const int j = find_job(jobs, njobs, blockIdx.x);
    const ResJob& jb = jobs[j];
    residual_norm_pairs_body(jb.HX, jb.X, jb.R, jb.theta, jb.m, jb.N, jb.rows_per_block, partial + jb.part_off,
                             blockIdx.x - jb.start, red);
}

__global__ void __launch_bounds__(256) k_gather_pairs_batched(const GatherJob* __restrict__ jobs, int njobs) {
    const int j = find_job(jobs, njobs, blockIdx.x);
    const GatherJob& jb = jobs[j];
    gather_pairs_body(jb.src, jb.parts, jb.n, jb.dst, jb.M, jb.N, blockIdx.x - jb.start, jb.nb);
}

__global__ void __launch_bounds__(256) k_precond_batched(const PreJob* __restrict__ jobs, int njobs) {
    const int j = find_job(jobs, njobs, blockIdx.x);
    const PreJob& jb = jobs[j];
    const int bid = blockIdx.x - jb.start;
    for (long long r = (long long)bid * blockDim.x + threadIdx.x; r < jb.N; r += (long long)jb.nb * blockDim.x) {
        double mm = jb.M[r];
        for (int c = 0; c < jb.m; ++c) {
            double2 v = jb.R.p[c][r];
            jb.W.p[c][r] = make_double2(mm * v.x, mm * v.y);
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static int grid_for(long long N, int threads, int cap = 4096) {
    long long b = (N + threads - 1) / threads;
    return (int)std::max(1LL, std::min<long long>(b, cap));
}

// Workgroups of a single tall Gram: max_blocks, or more for very tall ones.
// Each wave's loads in flight shrink with the number of columns (every 4-row
// group moves 64 bytes per column), so a tall Gram with few columns (tens of
// millions of rows, a handful of vectors) needs more waves to keep HBM busy:
// one block per 1024 groups (4096 rows), up to 8192 waves and what the partial
// buffer (max_blocks x kMaxCols^2 complex entries) holds at `per_block`
// entries each.  At 589,824 rows this stays at max_blocks, which measured
// faster there than more, smaller blocks.
static int gram_single_blocks(int p, int per_block, long long N, int max_blocks, long long* gpb) {
    const int TP = (p + 15) >> 4;
    const long long G = (N + 3) >> 2;
    const long long cap = (long long)max_blocks * kMaxCols * kMaxCols / std::max(1, per_block);
    const long long tall = std::max<long long>(max_blocks, G / 1024);
    const int want = (int)std::max<long long>(1, std::min<long long>({cap, 8192LL / TP, tall}));
    return gram_job_blocks(p, N, want, gpb);
}

hipError_t gram(const ColPtrs& L, int p, const ColPtrs& R, int q, long long N, double2* partial, int max_blocks,
                double2* C, hipStream_t st) {
    if (p <= 0 || q <= 0) return hipSuccess;
    // one wave per 16 columns of L
    const int TP = (p + 15) >> 4, TQ = (q + 15) >> 4;
    long long gpb;
    const int nb = gram_single_blocks(p, p * q, N, max_blocks, &gpb);
    switch (TQ) {
        case 1: k_gram<1><<<nb, 64 * TP, 0, st>>>(L, p, R, q, N, gpb, partial); break;
        case 2: k_gram<2><<<nb, 64 * TP, 0, st>>>(L, p, R, q, N, gpb, partial); break;
        case 3: k_gram<3><<<nb, 64 * TP, 0, st>>>(L, p, R, q, N, gpb, partial); break;
        default: k_gram<4><<<nb, 64 * TP, 0, st>>>(L, p, R, q, N, gpb, partial); break;
    }
    int cnt = p * q;
    k_reduce_partials<<<cnt, 256, 0, st>>>(partial, nb, cnt, C);
    return hipGetLastError();
}

hipError_t lincomb(const ColPtrs& A, int p, const ColPtrs& Y, int q, const double2* C, double beta, long long N,
                   hipStream_t st) {
    if (q <= 0) return hipSuccess;
    const int nb = (int)std::min<long long>(4096, std::max<long long>(1, (N + 127) / 128));
    if (q <= 32) {
        const int qg = (q + 3) >> 2;
        if (qg <= 2) k_lincomb_rows<2><<<nb, 256, 0, st>>>(A, p, Y, q, C, beta, N);
        else if (qg <= 4) k_lincomb_rows<4><<<nb, 256, 0, st>>>(A, p, Y, q, C, beta, N);
        else k_lincomb_rows<8><<<nb, 256, 0, st>>>(A, p, Y, q, C, beta, N);
    } else {
        // 16-row tiles, four per workgroup per sweep
        const int nt = (int)std::min<long long>(2048, std::max<long long>(1, (N + 63) / 64));
        k_lincomb<3><<<nt, 256, 0, st>>>(A, p, Y, q, C, beta, N);
    }
    return hipGetLastError();
}

hipError_t gram_pairs(const ColPtrs& L, int p, const ColPtrs& R, int q, long long N, double2* partial, int max_blocks,
                      double* C, hipStream_t st) {
    if (p <= 0 || q <= 0) return hipSuccess;
    const int TP = (p + 15) >> 4, TQ = (q + 15) >> 4;
    long long gpb;
    const int nb = gram_single_blocks(p, 2 * p * q, N, max_blocks, &gpb);
    switch (TQ) {
        case 1: k_gram_pairs<1><<<nb, 64 * TP, 0, st>>>(L, p, R, q, N, gpb, partial); break;
        case 2: k_gram_pairs<2><<<nb, 64 * TP, 0, st>>>(L, p, R, q, N, gpb, partial); break;
        case 3: k_gram_pairs<3><<<nb, 64 * TP, 0, st>>>(L, p, R, q, N, gpb, partial); break;
        default: k_gram_pairs<4><<<nb, 64 * TP, 0, st>>>(L, p, R, q, N, gpb, partial); break;
    }
    // 4pq real entries per block, reduced as 2pq pairs
    const int cnt = 2 * p * q;
    k_reduce_partials<<<cnt, 256, 0, st>>>(partial, nb, cnt, reinterpret_cast<double2*>(C));
    return hipGetLastError();
}

hipError_t lincomb_pairs(const ColPtrs& A, int p, const ColPtrs& Y, int q, const double* C, double beta, long long N,
                         hipStream_t st) {
    if (q <= 0) return hipSuccess;
    if (q > 32) return hipErrorInvalidValue;
    const int nb = (int)std::min<long long>(4096, std::max<long long>(1, (N + 127) / 128));
    const int qg = (q + 3) >> 2;
    const double2* C2 = reinterpret_cast<const double2*>(C);
    // accumulators sized to the outputs per wave (fewer registers, more waves)
    if (qg <= 2) k_lincomb_pairs<2><<<nb, 256, 0, st>>>(A, p, Y, q, C2, beta, N);
    else if (qg <= 3) k_lincomb_pairs<3><<<nb, 256, 0, st>>>(A, p, Y, q, C2, beta, N);
    else if (qg <= 4) k_lincomb_pairs<4><<<nb, 256, 0, st>>>(A, p, Y, q, C2, beta, N);
    else if (qg <= 6) k_lincomb_pairs<6><<<nb, 256, 0, st>>>(A, p, Y, q, C2, beta, N);
    else k_lincomb_pairs<8><<<nb, 256, 0, st>>>(A, p, Y, q, C2, beta, N);
    return hipGetLastError();
}

hipError_t residual_norm_pairs(const ColPtrs& HX, const ColPtrs& X, const ColPtrs& R, const Reals& theta, int m,
                               long long N, double* partial, int max_blocks, double* out, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    if (2 * m > kMaxCols) return hipErrorInvalidValue;
    long long rpb = (N + max_blocks - 1) / max_blocks;
    int nb = (int)((N + rpb - 1) / rpb);
    k_residual_norm_pairs<<<nb, 256, 0, st>>>(HX, X, R, theta, m, N, rpb, partial);
    k_reduce_real<<<2 * m, 256, 0, st>>>(partial, nb, 2 * m, out);
    return hipGetLastError();
}

hipError_t gather_pairs(const ColPtrs& src, unsigned long long parts, int n, const ColPtrs& dst, const double* M,
                        long long N, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_gather_pairs<<<grid_for(N, 256), 256, 0, st>>>(src, parts, n, dst, M, N);
    return hipGetLastError();
}

hipError_t unpack_real(const ColPtrs& src, unsigned long long parts, int n, const ColPtrs& dst, long long N,
                       hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_unpack_real<<<grid_for(N, 256), 256, 0, st>>>(src, parts, n, dst, N);
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
    k_reduce_real<<<m, 256, 0, st>>>(partial, nb, m, out);
    return hipGetLastError();
}

hipError_t residual_norm(const ColPtrs& HX, const ColPtrs& X, const ColPtrs& R, const Reals& theta, int m, long long N,
                         double* partial, int max_blocks, double* out, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    long long rpb = (N + max_blocks - 1) / max_blocks;
    int nb = (int)((N + rpb - 1) / rpb);
    k_residual_norm<<<nb, 256, 0, st>>>(HX, X, R, theta, m, N, rpb, partial);
    k_reduce_real<<<m, 256, 0, st>>>(partial, nb, m, out);
    return hipGetLastError();
}

hipError_t precond(const ColPtrs& R, const ColPtrs& W, int m, const double* M, long long N, hipStream_t st) {
    k_precond<<<grid_for(N, 256), 256, 0, st>>>(R, W, m, M, N);
    return hipGetLastError();
}

int gram_job_blocks(int p, long long N, int max_blocks, long long* groups_per_block) {
    const int TP = (p + 15) >> 4;
    const long long G = (N + 3) >> 2;
    const int want = std::max(1, std::min(max_blocks, (8192 + TP - 1) / TP));
    long long gpb = (G + want - 1) / want;
    gpb = std::max<long long>(kGramDepth, ((gpb + kGramDepth - 1) / kGramDepth) * kGramDepth);
    *groups_per_block = gpb;
    return (int)std::max<long long>(1, (G + gpb - 1) / gpb);
}

hipError_t gram_batched(const GramJob* jobs, int njobs, int total_blocks, int total_out, int maxp, int maxq,
                        double2* partial, double2* C, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    const int threads = 64 * ((maxp + 15) >> 4), TQ = (maxq + 15) >> 4;
    switch (TQ) {
        case 1: k_gram_batched<1><<<total_blocks, threads, 0, st>>>(jobs, njobs, partial); break;
        case 2: k_gram_batched<2><<<total_blocks, threads, 0, st>>>(jobs, njobs, partial); break;
        case 3: k_gram_batched<3><<<total_blocks, threads, 0, st>>>(jobs, njobs, partial); break;
        default: k_gram_batched<4><<<total_blocks, threads, 0, st>>>(jobs, njobs, partial); break;
    }
    k_reduce_batched<<<total_out, 256, 0, st>>>(jobs, njobs, partial, C);
    return hipGetLastError();
}

hipError_t lincomb_batched(const LinJob* jobs, int njobs, int total_blocks, int maxq, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    const int qg = (maxq + 3) >> 2;
    if (maxq <= 32) {
        if (qg <= 2) k_lincomb_rows_batched<2><<<total_blocks, 256, 0, st>>>(jobs, njobs);
        else if (qg <= 4) k_lincomb_rows_batched<4><<<total_blocks, 256, 0, st>>>(jobs, njobs);
        else k_lincomb_rows_batched<8><<<total_blocks, 256, 0, st>>>(jobs, njobs);
    } else {
        k_lincomb_batched<3><<<total_blocks, 256, 0, st>>>(jobs, njobs);
    }
    return hipGetLastError();
}

hipError_t residual_norm_batched(const ResJob* jobs, int njobs, int total_blocks, int total_out, double* partial,
                                 double* out, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    k_residual_norm_batched<<<total_blocks, 256, 0, st>>>(jobs, njobs, partial);
    k_reduce_res_batched<<<total_out, 256, 0, st>>>(jobs, njobs, partial, out);
    return hipGetLastError();
}

hipError_t gram_batched_pairs(const GramJob* jobs, int njobs, int total_blocks, int total_out, int maxp, int maxq,
                              double2* partial, double2* C, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    const int threads = 64 * ((maxp + 15) >> 4), TQ = (maxq + 15) >> 4;
    switch (TQ) {
        case 1: k_gram_batched_pairs<1><<<total_blocks, threads, 0, st>>>(jobs, njobs, partial); break;
        case 2: k_gram_batched_pairs<2><<<total_blocks, threads, 0, st>>>(jobs, njobs, partial); break;
        case 3: k_gram_batched_pairs<3><<<total_blocks, threads, 0, st>>>(jobs, njobs, partial); break;
        default: k_gram_batched_pairs<4><<<total_blocks, threads, 0, st>>>(jobs, njobs, partial); break;
    }
    k_reduce_batched<<<total_out, 256, 0, st>>>(jobs, njobs, partial, C);
    return hipGetLastError();
}

hipError_t lincomb_pairs_batched(const LinJob* jobs, int njobs, int total_blocks, int maxq, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    if (maxq > 32) return hipErrorInvalidValue;
    const int qg = (maxq + 3) >> 2;
    if (qg <= 2) k_lincomb_pairs_batched<2><<<total_blocks, 256, 0, st>>>(jobs, njobs);
    else if (qg <= 3) k_lincomb_pairs_batched<3><<<total_blocks, 256, 0, st>>>(jobs, njobs);
    else if (qg <= 4) k_lincomb_pairs_batched<4><<<total_blocks, 256, 0, st>>>(jobs, njobs);
    else if (qg <= 6) k_lincomb_pairs_batched<6><<<total_blocks, 256, 0, st>>>(jobs, njobs);
    else k_lincomb_pairs_batched<8><<<total_blocks, 256, 0, st>>>(jobs, njobs);
    return hipGetLastError();
}

hipError_t residual_norm_pairs_batched(const ResJob* jobs, int njobs, int total_blocks, int total_out, double* partial,
                                       double* out, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    k_residual_norm_pairs_batched<<<total_blocks, 256, 0, st>>>(jobs, njobs, partial);
    k_reduce_res_batched<<<total_out, 256, 0, st>>>(jobs, njobs, partial, out);
    return hipGetLastError();
}

hipError_t gather_pairs_batched(const GatherJob* jobs, int njobs, int total_blocks, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    k_gather_pairs_batched<<<total_blocks, 256, 0, st>>>(jobs, njobs);
    return hipGetLastError();
}

hipError_t precond_batched(const PreJob* jobs, int njobs, int total_blocks, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    k_precond_batched<<<total_blocks, 256, 0, st>>>(jobs, njobs);
    return hipGetLastError();
}

hipError_t randn(double2* out, long long count, unsigned long long seed, hipStream_t st) {
    k_randn<<<grid_for(count, 256), 256, 0, st>>>(out, count, seed);
    return hipGetLastError();
}

}  // namespace iwfpm
