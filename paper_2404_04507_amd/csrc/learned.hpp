// learned.hpp - learned preconditioner used inside the block LOBPCG.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <vector>

#include "../../include/iwfpm.h"
#include "blas.hpp"

struct iwfpm_plan_s;

namespace iwfpm {

struct LearnedPrecond;

// true when a network is attached and its weights are usable
bool learned_ready(const LearnedPrecond* lp, const iwfpm_plan_s* p);
// W_j = T(R_j) for j < m; returns IWFPM_OK or an error (the caller falls back to M)
int learned_apply(LearnedPrecond* lp, iwfpm_plan_s* p, const ColPtrs& R, const ColPtrs& W, int m, hipStream_t st);
void learned_free(LearnedPrecond* lp);

// Iterates recorded by a plain solve (training data): every `stride`
// iterations, the first ncol columns of X (and, when R is not empty, of
// R = HX - X theta) are copied into slot `got` (contiguous ncol x N blocks
// supplied by the caller).
struct Capture {
    int stride = 8;
    int ncol = 0;
    std::vector<double2*> X, R;            // one pair per slot
    std::vector<std::vector<double>> eta;  // backward errors at the time of recording
    int got = 0;
    int last_it = -1;
};

// plain LOBPCG solve that fills `cap` (lobpcg.cpp); evecs: device, N x nev
int eigs_capture(iwfpm_plan_s* p, const iwfpm_eigs_opts& o, Capture* cap, double* evals, void* evecs,
                 hipStream_t st);
// diagonal of eq:precond for H~ + sigma I in vector order (lobpcg.cpp)
void precond_diagonal(const iwfpm_plan_s* p, std::vector<double>& M);

// small dense Hermitian helpers of the eigensolver (lobpcg.cpp), column-major:
// A = V diag(w) V^H with w ascending; and for a Gram matrix G (k x k) the
// k x rank map T with T^H G T = I, dropping directions below eps (relative)
void heev(const std::vector<std::complex<double>>& A, int n, std::vector<double>& w,
          std::vector<std::complex<double>>& V);
int svqb(const std::vector<std::complex<double>>& G, int k, std::vector<std::complex<double>>& T, double eps = 1e-12);

}  // namespace iwfpm
