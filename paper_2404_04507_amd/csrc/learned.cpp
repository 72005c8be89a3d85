// learned.cpp - learned preconditioner (weights not yet supported in this build)
#include "learned.hpp"

#include "../../include/iwfpm.h"

namespace iwfpm {

struct LearnedPrecond {
    int dummy = 0;
};

bool learned_ready(const LearnedPrecond* lp, const iwfpm_plan_s*) { return lp != nullptr && false; }
int learned_apply(LearnedPrecond*, iwfpm_plan_s*, const ColPtrs&, const ColPtrs&, int, hipStream_t) {
    return IWFPM_ERR_WEIGHTS;
}
void learned_free(LearnedPrecond* lp) { delete lp; }

}  // namespace iwfpm
