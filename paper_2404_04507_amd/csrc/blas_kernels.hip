// blas_kernels.hip - float64 block algebra of the block LOBPCG eigensolver.
//
// All blocks are complex float64, one contiguous column of N entries per
// vector; kernels take lists of column pointers so that any subset of the
// X / W / P blocks can be combined without copies.
//
//   gram      C = L^H R            tall-skinny (p, q <= 64), wide ones on the
//                                  matrix cores; two-stage deterministic
//                                  reduction
//   lincomb   Y = beta Y + A C     (p <= 64 inputs, q <= 48 outputs per call);
//                                  outputs beyond 32 on the matrix cores
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
// gram for small blocks (p + q < 48, and every batched call): the p x q output
// is cut into 4 x 4 tiles; with ntile tiles, the 256 threads form 256 / ntile
// row groups, each summing its own subset of the staged rows for its tile.
// Rows are staged through LDS `rows` at a time; the row groups are summed in a
// fixed order at the end (deterministic).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void gram_vec_body(const ColPtrs& L, int p, const ColPtrs& R, int q, long long N,
                                          long long rows_per_block, int rows, double2* __restrict__ partial, int bid,
                                          unsigned char* smem) {
    const int pl = p | 1, pr = q | 1;  // odd pitches
    double2* sL = reinterpret_cast<double2*>(smem);
    double2* sR = sL + rows * pl;
    const int tid = threadIdx.x;
    const int TP = (p + 3) >> 2, TQ = (q + 3) >> 2, ntile = TP * TQ;
    const int ngroups = 256 / ntile;
    const int grp = tid / ntile, tile = tid - grp * ntile;
    const bool active = grp < ngroups;
    const int ti = tile % TP, tj = tile / TP;
    double2 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0.0, 0.0);
    const long long r0 = (long long)bid * rows_per_block;
    const long long r1 = min(N, r0 + rows_per_block);
    for (long long rb = r0; rb < r1; rb += rows) {
        const int nr = (int)min((long long)rows, r1 - rb);
        for (int e = tid; e < rows * p; e += 256) {
            int c = e / rows, rr = e - c * rows;
            sL[rr * pl + c] = rr < nr ? L.p[c][rb + rr] : make_double2(0.0, 0.0);
        }
        for (int e = tid; e < rows * q; e += 256) {
            int c = e / rows, rr = e - c * rows;
            sR[rr * pr + c] = rr < nr ? R.p[c][rb + rr] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        if (active) {
            for (int rr = grp; rr < nr; rr += ngroups) {
                double2 l[4], r[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    int i = 4 * ti + a;
                    l[a] = i < p ? sL[rr * pl + i] : make_double2(0.0, 0.0);
                }
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    int j = 4 * tj + b;
                    r[b] = j < q ? sR[rr * pr + j] : make_double2(0.0, 0.0);
                }
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        acc[a][b].x += l[a].x * r[b].x + l[a].y * r[b].y;
                        acc[a][b].y += l[a].x * r[b].y - l[a].y * r[b].x;
                    }
            }
        }
        __syncthreads();
    }
    // sum the row groups: red[grp][tile][16]
    double2* red = reinterpret_cast<double2*>(smem);
    if (active) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) red[((size_t)grp * ntile + tile) * 16 + a * 4 + b] = acc[a][b];
    }
    __syncthreads();
    double2* out = partial + (size_t)bid * p * q;
    for (int e = tid; e < ntile * 16; e += 256) {
        int t = e >> 4, ab = e & 15;
        int i = 4 * (t % TP) + (ab >> 2), j = 4 * (t / TP) + (ab & 3);
        if (i >= p || j >= q) continue;
        double2 sum = make_double2(0.0, 0.0);
        for (int g = 0; g < ngroups; ++g) {
            double2 v = red[((size_t)g * ntile + t) * 16 + ab];
            sum.x += v.x;
            sum.y += v.y;
        }
        out[(size_t)j * p + i] = sum;
    }
}

// ---------------------------------------------------------------------------
// gram for wide blocks: partial[b][j*p + i] = sum over the rows of block b of
// conj(L_i[r]) R_j[r], on the matrix cores (v_mfma_f64_16x16x4f64).  With the K index running over
// (row, re/im) pairs, Re C = sum_k Lx[k][i] Rx[k][j] and Im C = sum_k Lx[k][i]
// Ry[k][j], where Lx, Rx hold (re, im) of each row and Ry holds (im, -re): two
// real 16x16x4 products per 16x16 complex output tile and K step of two rows,
// sharing the A operand.  Lane l of a wave holds A[l%16][l/16], B[l/16][l%16]
// and result v in D[l/16 + 4v][l%16], so each lane ends with whole complex
// entries.  Rows are staged through LDS kGramRows at a time (odd pitches),
// the next chunk's loads in flight in registers while the current one is
// multiplied; the 4 wavefronts split the output tiles.
// ---------------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int kGramRows = 24;   // rows staged per chunk (12 K steps)
constexpr int kGramTilesPerWave = 4;

// registers of one thread's share of one staged matrix (kGramRows rows of at
// most 64 padded columns)
constexpr int kGramRegs = (kGramRows * 64 + 255) / 256;

// load this thread's entries e = tid + 256 u of the chunk at row rb of X
// (zero beyond nr rows and p columns)
__device__ __forceinline__ void fetch_chunk(const ColPtrs& X, int p, int pitch, long long rb, int nr, int tid,
                                            double2 (&v)[kGramRegs]) {
    const int total = kGramRows * (pitch - 1);
#pragma unroll
    for (int u = 0; u < kGramRegs; ++u) {
        const int e = tid + 256 * u;
        const int c = e / kGramRows, rr = e - c * kGramRows;
        v[u] = (e < total && rr < nr && c < p) ? X.p[c][rb + rr] : make_double2(0.0, 0.0);
    }
}

__device__ __forceinline__ void put_chunk(int pitch, double2* __restrict__ s, int tid, const double2 (&v)[kGramRegs]) {
    const int total = kGramRows * (pitch - 1);
#pragma unroll
    for (int u = 0; u < kGramRegs; ++u) {
        const int e = tid + 256 * u;
        const int c = e / kGramRows, rr = e - c * kGramRows;
        if (e < total) s[rr * pitch + c] = v[u];
    }
}

__device__ __forceinline__ void gram_body(const ColPtrs& L, int p, const ColPtrs& R, int q, long long N,
                                          long long rows_per_block, double2* __restrict__ partial, int bid,
                                          unsigned char* smem) {
    const int TP = (p + 15) >> 4, TQ = (q + 15) >> 4, ntile = TP * TQ;
    const int pl = 16 * TP + 1, pr = 16 * TQ + 1;  // odd pitches (complex entries)
    double2* sL = reinterpret_cast<double2*>(smem);
    double2* sR = sL + kGramRows * pl;
    const double* dL = reinterpret_cast<const double*>(sL);
    const double* dR = reinterpret_cast<const double*>(sR);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;  // A row / B column, and K index 0..3
    const int half = lk >> 1, part = lk & 1;   // staged row within the K step, re/im
    dbl4 accr[kGramTilesPerWave], acci[kGramTilesPerWave];
#pragma unroll
    for (int t = 0; t < kGramTilesPerWave; ++t) {
        accr[t] = dbl4{0.0, 0.0, 0.0, 0.0};
        acci[t] = dbl4{0.0, 0.0, 0.0, 0.0};
    }
    const long long r0 = (long long)bid * rows_per_block;
    const long long r1 = min(N, r0 + rows_per_block);
    // software pipeline: the next chunk's loads are in flight while the
    // matrix cores work on the staged one
    double2 nL[kGramRegs], nR[kGramRegs];
    if (r0 < r1) {
        const int nr0 = (int)min((long long)kGramRows, r1 - r0);
        fetch_chunk(L, p, pl, r0, nr0, tid, nL);
        fetch_chunk(R, q, pr, r0, nr0, tid, nR);
    }
    for (long long rb = r0; rb < r1; rb += kGramRows) {
        put_chunk(pl, sL, tid, nL);
        put_chunk(pr, sR, tid, nR);
        __syncthreads();
        const long long rn = rb + kGramRows;
        if (rn < r1) {
            const int nrn = (int)min((long long)kGramRows, r1 - rn);
            fetch_chunk(L, p, pl, rn, nrn, tid, nL);
            fetch_chunk(R, q, pr, rn, nrn, tid, nR);
        }
#pragma unroll
        for (int t = 0; t < kGramTilesPerWave; ++t) {
            const int tile = wave + 4 * t;
            if (tile < ntile) {  // uniform across the wave
                const int ti = tile % TP, tj = tile / TP;
#pragma unroll 4
                for (int ks = 0; ks < kGramRows / 2; ++ks) {
                    const int row = 2 * ks + half;
                    const double a = dL[2 * (row * pl + 16 * ti + li) + part];
                    const double2 rv = sR[row * pr + 16 * tj + li];
                    const double br = part ? rv.y : rv.x;
                    const double bi = part ? -rv.x : rv.y;
                    accr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, br, accr[t], 0, 0, 0);
                    acci[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bi, acci[t], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    (void)dR;
    double2* out = partial + (size_t)bid * p * q;
#pragma unroll
    for (int t = 0; t < kGramTilesPerWave; ++t) {
        const int tile = wave + 4 * t;
        if (tile < ntile) {
            const int ti = tile % TP, tj = tile / TP;
            const int j = 16 * tj + li;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * ti + lk + 4 * v;
                if (i < p && j < q) out[(size_t)j * p + i] = make_double2(accr[t][v], acci[t][v]);
            }
        }
    }
}

__global__ void __launch_bounds__(256) k_gram(ColPtrs L, int p, ColPtrs R, int q, long long N, long long rows_per_block,
                                              double2* __restrict__ partial) {
    extern __shared__ __align__(16) unsigned char smem[];
    gram_body(L, p, R, q, N, rows_per_block, partial, blockIdx.x, smem);
}

__global__ void __launch_bounds__(256) k_gram_vec(ColPtrs L, int p, ColPtrs R, int q, long long N,
                                                  long long rows_per_block, int rows, double2* __restrict__ partial) {
    extern __shared__ __align__(16) unsigned char smem[];
    gram_vec_body(L, p, R, q, N, rows_per_block, rows, partial, blockIdx.x, smem);
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
// lincomb, q <= 32: one row per thread, all q outputs in registers, C in LDS
// (broadcast reads); wider outputs go to the matrix-core version below.
// ---------------------------------------------------------------------------
template <int QB>
__device__ __forceinline__ void lincomb_vec_body(const ColPtrs& A, int p, const ColPtrs& Y, int q,
                                             const double2* __restrict__ C, double beta, long long N, int bid, int nb,
                                             double2* sC) {
    for (int e = threadIdx.x; e < p * q; e += blockDim.x) sC[e] = C[e];
    __syncthreads();
    for (long long r = (long long)bid * blockDim.x + threadIdx.x; r < N; r += (long long)nb * blockDim.x) {
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
// lincomb, 32 < q <= 48: Y_j = beta Y_j + sum_i A_i C[j*p + i]
//
// On the matrix cores, like gram: with the K index over (input column i,
// re/im), Re Y = sum_k Ax[r][k] Bre[k][j] and Im Y = sum_k Ax[r][k] Bim[k][j],
// Bre = (Re C, -Im C), Bim = (Im C, Re C) interleaved by (i, re/im).  Each
// wavefront owns 16-row tiles (grid-stride); its A operand is read straight
// from HBM (lanes 0-31 cover 16 rows of one input column, 256 contiguous
// bytes) exactly once, C is staged transposed in LDS, and each lane ends with
// whole complex outputs: rows lk + 4v of the tile, column 16 tq + li.
// ---------------------------------------------------------------------------
template <int TQ>
__device__ __forceinline__ void lincomb_body(const ColPtrs& A, int p, const ColPtrs& Y, int q,
                                             const double2* __restrict__ C, double beta, long long N, int bid, int nb,
                                             double2* sCt) {
    const int ldq = 16 * TQ;
    for (int e = threadIdx.x; e < p * ldq; e += blockDim.x) {
        const int i = e / ldq, j = e - i * ldq;
        sCt[e] = j < q ? C[(size_t)j * p + i] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int li = lane & 15, lk = lane >> 4, half = lk >> 1, part = lk & 1;
    const int ksteps = (p + 1) >> 1;
    const long long ntiles = (N + 15) >> 4;
    for (long long t = (long long)bid * nw + wave; t < ntiles; t += (long long)nb * nw) {
        const long long r0 = t << 4;
        const long long ra = r0 + li;
        const bool rok = ra < N;
        dbl4 yr[TQ], yi[TQ];
#pragma unroll
        for (int c = 0; c < TQ; ++c) {
            yr[c] = dbl4{0.0, 0.0, 0.0, 0.0};
            yi[c] = dbl4{0.0, 0.0, 0.0, 0.0};
        }
#pragma unroll 4
        for (int ks = 0; ks < ksteps; ++ks) {
            const int i = 2 * ks + half;
            const bool iok = i < p;
            const double a = (iok && rok) ? reinterpret_cast<const double*>(A.p[i])[2 * ra + part] : 0.0;
            const int ic = iok ? i : 0;
#pragma unroll
            for (int c = 0; c < TQ; ++c) {
                double2 cv = sCt[ic * ldq + 16 * c + li];
                if (!iok) cv = make_double2(0.0, 0.0);
                const double br = part ? -cv.y : cv.x;
                const double bi = part ? cv.x : cv.y;
                yr[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, br, yr[c], 0, 0, 0);
                yi[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bi, yi[c], 0, 0, 0);
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

template <int QB>
__global__ void __launch_bounds__(256) k_lincomb_vec(ColPtrs A, int p, ColPtrs Y, int q,
                                                     const double2* __restrict__ C, double beta, long long N) {
    __shared__ double2 sC[kMaxCols * 32];
    lincomb_vec_body<QB>(A, p, Y, q, C, beta, N, blockIdx.x, gridDim.x, sC);
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

__global__ void __launch_bounds__(256) k_gram_batched(const GramJob* __restrict__ jobs, int njobs,
                                                      double2* __restrict__ partial) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int j = find_job(jobs, njobs, blockIdx.x);
    const GramJob& jb = jobs[j];
    gram_vec_body(jb.L, jb.p, jb.R, jb.q, jb.N, jb.rows_per_block, jb.rows, partial + jb.part_off,
                  blockIdx.x - jb.start, smem);
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
    const int le = e - jb.out_start, cnt = jb.p * jb.q;
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

template <int QB>
__global__ void __launch_bounds__(256) k_lincomb_vec_batched(const LinJob* __restrict__ jobs, int njobs) {
    __shared__ double2 sC[kMaxCols * 32];
    const int j = find_job(jobs, njobs, blockIdx.x);
    const LinJob& jb = jobs[j];
    lincomb_vec_body<QB>(jb.A, jb.p, jb.Y, jb.q, jb.C, jb.beta, jb.N, blockIdx.x - jb.start, jb.nb, sC);
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
    for (int b = threadIdx.x; b < jb.nb; b += 256) s += partial[jb.part_off + (size_t)b * jb.m + le];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[e] = red[0];
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

static size_t gram_lds(int p, int q) {
    return (size_t)kGramRows * (16 * ((p + 15) / 16) + 1 + 16 * ((q + 15) / 16) + 1) * sizeof(double2);
}

hipError_t gram(const ColPtrs& L, int p, const ColPtrs& R, int q, long long N, double2* partial, int max_blocks,
                double2* C, hipStream_t st) {
    if (p <= 0 || q <= 0) return hipSuccess;
    int nb;
    if (p + q >= 48) {
        long long rpb = (N + max_blocks - 1) / max_blocks;
        rpb = ((rpb + kGramRows - 1) / kGramRows) * kGramRows;
        nb = (int)((N + rpb - 1) / rpb);
        k_gram<<<nb, 256, gram_lds(p, q), st>>>(L, p, R, q, N, rpb, partial);
    } else {
        long long rpb;
        int rows;
        size_t lds;
        nb = gram_job_blocks(p, q, N, max_blocks, &rpb, &rows, &lds);
        k_gram_vec<<<nb, 256, lds, st>>>(L, p, R, q, N, rpb, rows, partial);
    }
    int cnt = p * q;
    k_reduce_partials<<<cnt, 256, 0, st>>>(partial, nb, cnt, C);
    return hipGetLastError();
}

hipError_t lincomb(const ColPtrs& A, int p, const ColPtrs& Y, int q, const double2* C, double beta, long long N,
                   hipStream_t st) {
    if (q <= 0) return hipSuccess;
    if (q <= 32) {
        int nb = grid_for(N, 256, 2048);
        if (q <= 8) k_lincomb_vec<8><<<nb, 256, 0, st>>>(A, p, Y, q, C, beta, N);
        else if (q <= 16) k_lincomb_vec<16><<<nb, 256, 0, st>>>(A, p, Y, q, C, beta, N);
        else k_lincomb_vec<32><<<nb, 256, 0, st>>>(A, p, Y, q, C, beta, N);
    } else {
        // 16-row tiles, four per workgroup per sweep
        int nb = (int)std::min<long long>(2048, std::max<long long>(1, (N + 63) / 64));
        k_lincomb<3><<<nb, 256, 0, st>>>(A, p, Y, q, C, beta, N);
    }
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

int gram_job_blocks(int p, int q, long long N, int max_blocks, long long* rows_per_block, int* rows, size_t* lds) {
    const int pl = p | 1, pr = q | 1;
    int r = (int)std::min<long long>(128, (48 * 1024) / ((pl + pr) * (long long)sizeof(double2)));
    r = std::max(r, 8);
    long long rpb = (N + max_blocks - 1) / max_blocks;
    rpb = ((rpb + r - 1) / r) * r;
    int ntile = ((p + 3) / 4) * ((q + 3) / 4);
    *rows_per_block = rpb;
    *rows = r;
    *lds = std::max((size_t)r * (pl + pr) * sizeof(double2), (size_t)(256 / ntile) * ntile * 16 * sizeof(double2));
    return (int)((N + rpb - 1) / rpb);
}

hipError_t gram_batched(const GramJob* jobs, int njobs, int total_blocks, int total_out, size_t lds,
                        double2* partial, double2* C, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    k_gram_batched<<<total_blocks, 256, lds, st>>>(jobs, njobs, partial);
    k_reduce_batched<<<total_out, 256, 0, st>>>(jobs, njobs, partial, C);
    return hipGetLastError();
}

hipError_t lincomb_batched(const LinJob* jobs, int njobs, int total_blocks, int maxq, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    if (maxq <= 8) k_lincomb_vec_batched<8><<<total_blocks, 256, 0, st>>>(jobs, njobs);
    else if (maxq <= 16) k_lincomb_vec_batched<16><<<total_blocks, 256, 0, st>>>(jobs, njobs);
    else if (maxq <= 32) k_lincomb_vec_batched<32><<<total_blocks, 256, 0, st>>>(jobs, njobs);
    else k_lincomb_batched<3><<<total_blocks, 256, 0, st>>>(jobs, njobs);
    return hipGetLastError();
}

hipError_t residual_norm_batched(const ResJob* jobs, int njobs, int total_blocks, int total_out, double* partial,
                                 double* out, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    k_residual_norm_batched<<<total_blocks, 256, 0, st>>>(jobs, njobs, partial);
    k_reduce_res_batched<<<total_out, 256, 0, st>>>(jobs, njobs, partial, out);
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
