// learned_dev.hpp - launchers of the learned preconditioner's kernels
// (learned_kernels.hip).  Blocks of m complex columns are contiguous
// (column j at base + j*N) unless passed as ColPtrs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "blas.hpp"

namespace iwfpm {

// ---- dense layers of the shell MLP: bfloat16 weights on the bf16 matrix cores, float32 accumulation ----
// Y[s][o] = act(sum_i X[s][i] W[i][o] + b[o]) for s < S; Z (optional) keeps the pre-activation
hipError_t lp_dense_fwd(const float* X, const uint16_t* W, const float* b, float* Z, float* Y, int S, int in, int out,
                        int act, hipStream_t st);
// dZ = dY .* act'(Z)
hipError_t lp_act_bwd(const float* dY, const float* Z, float* dZ, int n, int act, hipStream_t st);
// dX = dZ W^T (skipped when dX is null), dW = X^T dZ, db = column sums of dZ
hipError_t lp_dense_bwd(const float* X, const float* dZ, const uint16_t* W, float* dX, float* dW, float* db, int S,
                        int in, int out, hipStream_t st);
// Adam on float32 master weights w (moments m, v) with bias corrections c1, c2;
// refreshes the bfloat16 copy wbf
hipError_t lp_adam(float* w, float* m, float* v, const float* g, uint16_t* wbf, int n, float lr, float b1, float b2,
                   float c1, float c2, float eps, hipStream_t st);
// wbf = bfloat16(w), round to nearest even
hipError_t lp_to_bf16(const float* w, uint16_t* wbf, int n, hipStream_t st);

// ---- grid-sized pieces ----
// D0 = M (1 + exp(O[shell][0])) / 2, E = M exp(O[shell][1])
hipError_t lp_expand(const double* M, const int* shell, const float* O, double* D0, double* E, long long N,
                     hipStream_t st);
// Y_j = d .* R_j (R as column pointers, Y contiguous)
hipError_t lp_scale_cols(const ColPtrs& R, double2* Y, int m, const double* d, long long N, hipStream_t st);
// Y = d .* A (contiguous blocks)
hipError_t lp_scale(const double2* A, double2* Y, int m, const double* d, long long N, hipStream_t st);
// W_j = (D0 + b1 a^2 E) .* R_j + E .* (2 a b1 A_j + b1 C_j), a = beta[0], b1 = max(beta[1], 0);
// beta is a device pointer
hipError_t lp_combine(const ColPtrs& R, const double2* A, const double2* C, const ColPtrs& W, int m, const double* D0,
                      const double* E, const float* beta, long long N, hipStream_t st);
// per-point parameter gradients of the preconditioner, reduced into shells:
//   dO[s][0] += (D0 - M/2) sum_j Re(conj(G_j) R_j)
//   dO[s][1] += E  sum_j c0 (Re(conj(G) A) + Re(conj(B1) R)) + c1 (Re(conj(G) C) + Re(conj(B1) A)
//                                 + Re(conj(B2) R)) + dl Re(conj(G) R)
//   dbeta[0] += sum Re(conj(G) E A),  dbeta[1] += sum Re(conj(G) E C),  dbeta[2] += sum Re(conj(G) E R)
// with (c0, c1, dl) = (2 a b1, b1, b1 a^2)
hipError_t lp_shell_grad(const double2* G, const double2* R, const double2* A, const double2* C, const double2* B1,
                         const double2* B2, int m, const double* M, const double* D0, const double* E,
                         const float* beta, const int* shell, double* dO, double* dbeta, long long N,
                         hipStream_t st);
// g[0..1] = gradient of (beta0, beta1) from the three sums of lp_shell_grad
hipError_t lp_beta_grad(const double* dbeta, const float* beta, float* g, hipStream_t st);
// b[i] = float(a[i] * scale)
hipError_t lp_to_float(const double* a, float* b, int n, double scale, hipStream_t st);
// flag[0] = 1 if any of the n floats is not finite (flag zeroed by the caller)
hipError_t lp_nonfinite(const float* a, int n, int* flag, hipStream_t st);
hipError_t lp_nonfinite_d(const double* a, long long n, int* flag, hipStream_t st);

}  // namespace iwfpm
