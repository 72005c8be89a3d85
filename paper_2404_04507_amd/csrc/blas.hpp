// blas.hpp - float64 block-algebra kernels of the eigensolver (blas_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

namespace iwfpm {

constexpr int kMaxCols = 64;

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

}  // namespace iwfpm
