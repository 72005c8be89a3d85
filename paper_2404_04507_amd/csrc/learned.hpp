// learned.hpp - learned preconditioner used inside the block LOBPCG.
#pragma once

#include <hip/hip_runtime.h>

#include "blas.hpp"

struct iwfpm_plan_s;

namespace iwfpm {

struct LearnedPrecond;

// true when weights are loaded and match the plan's geometry
bool learned_ready(const LearnedPrecond* lp, const iwfpm_plan_s* p);
// W_j = g(R_j) for j < m; returns IWFPM_OK or an error (the caller falls back)
int learned_apply(LearnedPrecond* lp, iwfpm_plan_s* p, const ColPtrs& R, const ColPtrs& W, int m, hipStream_t st);
void learned_free(LearnedPrecond* lp);

}  // namespace iwfpm
