"""The allocation-free apply (iwfpm_apply_noalloc) against iwfpm_apply.

The entry point stages the multi-pass schedules' intermediate grid in the
library's static device array instead of the plan's workspace; the kernels
are the same, so on the same inputs it must give iwfpm_apply's output bit for
bit.  Two calls in a row, the second with a smaller input, check that the
shared array's leftover contents from the first call never leak into the
second; sizes beyond the array are refused with IWFPM_ERR_TOO_LARGE.
"""

import ctypes

import numpy as np
import pytest
import torch

import paper_2404_04507_amd as lib
from paper_2404_04507_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(X):
    return torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda:0")


def _noalloc(plan, X):
    so = lib.load_library()
    Y = torch.empty_like(X)
    st = so.iwfpm_apply_noalloc(plan._h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                X.shape[0], ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, Y


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_matches_apply_twice(prec):
    big = W.c2_2d(lam=5.0)                      # 589,824 points, three passes
    small = W.paper_example_2d(0.8 * 3.141592653589793, 0.2 * 3.141592653589793, 6, 20)  # 5,760 points
    print(f"case: noalloc {prec} 2d_lifted_4d x16 then ex4.2 x3", flush=True)
    for prob, nvec, seed in ((big, 16, 3), (small, 3, 4)):
        with lib.Plan.from_problem(prob, precision=prec, schedule="threepass") as p:
            X = _dev(W.random_block(prob.N, nvec, seed=seed))
            ref = p.apply(X)
            st, Y = _noalloc(p, X)
            torch.cuda.synchronize()
            assert st == 0, lib.load_library().iwfpm_status_string(st)
            assert torch.equal(Y, ref)


def test_noalloc_fused_and_empty():
    prob = W.c1_1d()
    print("case: noalloc fused c1 + nvec 0", flush=True)
    with lib.Plan.from_problem(prob) as p:
        X = _dev(W.random_block(prob.N, 5, seed=9))
        st, Y = _noalloc(p, X)
        torch.cuda.synchronize()
        assert st == 0 and torch.equal(Y, p.apply(X))
        st, _ = _noalloc(p, X[:0])
        assert st == 0


def test_noalloc_refuses_beyond_scratch():
    """A 16^6 grid in float64 needs a 256 MiB intermediate per vector, more than
    the static array: refused before any device work, and the array still
    serves a fitting call afterwards (16^6 in float32, 128 MiB per vector)."""
    so = lib.load_library()
    assert so.iwfpm_noalloc_scratch_bytes() == 128 << 20
    prob = W.c3_3d()
    print("case: noalloc 3d_lifted_6d fp64 refused, fp32 one vector", flush=True)
    with lib.Plan.from_problem(prob, precision="fp64") as p:
        X = torch.zeros((1, prob.N), dtype=torch.complex128, device="cuda:0")
        st, _ = _noalloc(p, X)
        assert st == -11
    with lib.Plan.from_problem(prob, precision="fp32") as p:
        X = _dev(W.random_block(prob.N, 1, seed=5))
        st, Y = _noalloc(p, X)
        torch.cuda.synchronize()
        assert st == 0 and torch.equal(Y, p.apply(X))
