// blas.hpp - float64 block-algebra kernels of the eigensolver (blas_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

namespace iwfpm {

constexpr int kMaxCols = 64;
// double2 entries of the coefficient array the batched real-pair combination
// stages in LDS (2 p q of them for p input and q output columns)
constexpr int kLinPairsLds = kMaxCols * 32;

// up to kMaxCols column pointers, passed by value as a kernel argument
struct ColPtrs {
    double2* p[kMaxCols];
};
struct Reals {
    double v[kMaxCols];
};

// C (p x q, column-major, C[j*p + i]) = L^H R; `partial` holds max_blocks*p*q entries
hipError_t gram(const ColPtrs& L, int p, const ColPtrs& R, int q, long long N, double2* partial, int max_blocks,
                double2* C, hipStream_t st);
// Y_j = beta Y_j + sum_i A_i C[j*p + i], q <= 48
hipError_t lincomb(const ColPtrs& A, int p, const ColPtrs& Y, int q, const double2* C, double beta, long long N,
                   hipStream_t st);
// Two real vectors per complex column (real part, imaginary part):
//   gram_pairs     C (2p x 2q real, column-major) = real Gram of the 2p real vectors in L
//                  with the 2q in R; `partial` holds max_blocks*4pq doubles
//   lincomb_pairs  Y = beta Y + A C with C the real (2p x 2q, column-major) coefficients, q <= 32
//   residual_norm_pairs  R = HX - X diag(theta) (one theta per real vector, 2m of them),
//                  out[v] = ||R_v||^2 per real vector; `partial` holds max_blocks*2m doubles
//   gather_pairs   packs n real vectors (part of src[v] given by bit v of parts), times M
//                  when M is not null, into ceil(n/2) columns (a zero half when n is odd)
//   unpack_real    complex column v = (real vector v, 0)
hipError_t gram_pairs(const ColPtrs& L, int p, const ColPtrs& R, int q, long long N, double2* partial, int max_blocks,
                      double* C, hipStream_t st);
hipError_t lincomb_pairs(const ColPtrs& A, int p, const ColPtrs& Y, int q, const double* C, double beta, long long N,
                         hipStream_t st);
hipError_t residual_norm_pairs(const ColPtrs& HX, const ColPtrs& X, const ColPtrs& R, const Reals& theta, int m,
                               long long N, double* partial, int max_blocks, double* out, hipStream_t st);
hipError_t gather_pairs(const ColPtrs& src, unsigned long long parts, int n, const ColPtrs& dst, const double* M,
                        long long N, hipStream_t st);
hipError_t unpack_real(const ColPtrs& src, unsigned long long parts, int n, const ColPtrs& dst, long long N,
                       hipStream_t st);
hipError_t residual(const ColPtrs& HX, const ColPtrs& X, const ColPtrs& R, const Reals& theta, int m, long long N,
                    hipStream_t st);
// out[j] = ||V_j||^2; `partial` holds max_blocks*m doubles
hipError_t colnorm2(const ColPtrs& V, int m, long long N, double* partial, int max_blocks, double* out,
                    hipStream_t st);
// R_j = HX_j - theta_j X_j and out[j] = ||R_j||^2
hipError_t residual_norm(const ColPtrs& HX, const ColPtrs& X, const ColPtrs& R, const Reals& theta, int m, long long N,
                         double* partial, int max_blocks, double* out, hipStream_t st);
hipError_t precond(const ColPtrs& R, const ColPtrs& W, int m, const double* M, long long N, hipStream_t st);
hipError_t randn(double2* out, long long count, unsigned long long seed, hipStream_t st);

// batched jobs (device-resident tables); job j owns grid blocks [start, start + nb)
struct GramJob {
    ColPtrs L, R;
    int p, q;
    long long N, groups_per_block;  // 4-row groups per block
    int nb, start, out_start;
    long long part_off;  // offset of this job's partials (entries)
    int width = 1;       // entries per (column, column) pair: 1 complex, 2 for a real 2 x 2 block
};
struct LinJob {
    ColPtrs A, Y;
    const double2* C;  // p x q coefficients (device)
    double beta;
    long long N;
    int p, q, nb, start;
};
struct ResJob {
    ColPtrs HX, X, R;
    Reals theta;
    long long N, rows_per_block;
    int m, nb, start, out_start;
    long long part_off;
    int width = 1;  // norms per column: 1, or 2 with two real vectors per column
};
struct GatherJob {
    ColPtrs src, dst;
    unsigned long long parts;
    const double* M;
    long long N;
    int n, nb, start;
};
struct PreJob {
    ColPtrs R, W;
    const double* M;
    long long N;
    int m, nb, start;
};

// blocks (at most max_blocks) and 4-row groups per block of one gram over N rows with p columns on the left
int gram_job_blocks(int p, long long N, int max_blocks, long long* groups_per_block);
// maxp, maxq: the widest p and q over the jobs
hipError_t gram_batched(const GramJob* jobs, int njobs, int total_blocks, int total_out, int maxp, int maxq,
                        double2* partial, double2* C, hipStream_t st);
hipError_t lincomb_batched(const LinJob* jobs, int njobs, int total_blocks, int maxq, hipStream_t st);
hipError_t residual_norm_batched(const ResJob* jobs, int njobs, int total_blocks, int total_out, double* partial,
                                 double* out, hipStream_t st);
hipError_t precond_batched(const PreJob* jobs, int njobs, int total_blocks, hipStream_t st);
// batched forms of the pair kernels (jobs: width 2; LinJob.C real 2p x 2q as pairs of doubles)
hipError_t gram_batched_pairs(const GramJob* jobs, int njobs, int total_blocks, int total_out, int maxp, int maxq,
                              double2* partial, double2* C, hipStream_t st);
hipError_t lincomb_pairs_batched(const LinJob* jobs, int njobs, int total_blocks, int maxq, hipStream_t st);
hipError_t residual_norm_pairs_batched(const ResJob* jobs, int njobs, int total_blocks, int total_out, double* partial,
                                       double* out, hipStream_t st);
hipError_t gather_pairs_batched(const GatherJob* jobs, int njobs, int total_blocks, hipStream_t st);

}  // namespace iwfpm
