"""GPU parity of axes longer than one register pencil (more than 64 points, or
an extent with no compiled pencil), against the CPU oracle.

Such an axis is transformed in two or three in-place stages whose output is
left in the stages' digit order between the inverse and the forward
transform.  These tests put long axes in every place of every schedule: the
leading and the last axis of the fused kernel, the trailing slabs of passes
1/3, the middle pass's convolution axis and its other leading axes, the
further pass of the five-pass schedule; both potential paths (per-axis tables
and the full potential grid, where the digit order must be undone before V is
read); grid and window order; float64 and float32.  The grids are the paper's
own: Table 2's L = 40 and 60 (80- and 120-point axes), Table 3's PM rectangle
(120 x 84), Table 6's IWFPM window (100 x 12 x 12), Table 9's reference L = 40
(80^3 x 10^3), and the 8192-point axis of Tables 4, 7 and 8's references.

Tolerances as in test_apply_gpu.py (derived there from the arithmetic).
"""

import math

import numpy as np
import pytest

from paper_2404_04507_amd import workloads as W
from test_apply_gpu import check_full, sampled_check

pytestmark = pytest.mark.gpu


def _complex_oblique(P, d, K, L, seed=3):
    """Complex conjugate-pair coefficients on modes off the axes: the
    potential-grid path, where every V lookup crosses the digit order."""
    n = P.shape[1]
    rng = np.random.default_rng(seed)
    modes, vhat = [[0] * n], [0.9]
    for _ in range(3):
        m = rng.integers(-2, 3, size=n)
        if not m.any():
            continue
        c = complex(rng.standard_normal(), rng.standard_normal())
        modes += [list(m), list(-m)]
        vhat += [c, c.conjugate()]
    return W.Problem("oblique", d, P, K, L, np.array(modes), np.array(vhat))


@pytest.mark.parametrize("order", ["grid", "window"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("L", [40, 60])
def test_table2_grids_fused(L, prec, order):
    """Ex. 4.1 at IWFPM K = 5, L = 40 / 60: 80 x 10 and 120 x 10 grids, the
    long axis leading in the fused kernel."""
    prob = W.paper_example_1d(2.5, 5, L)
    print(f"case: ex4.1 K=5 L={L} fused {prec} {order}", flush=True)
    check_full(prob, prec, order=order, schedule="fused")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_long_last_axis_fused(prec):
    """K = 42, L = 3 (6 x 84): the long axis is the fused kernel's last
    (convolution) axis."""
    prob = W.paper_example_1d(2.5, 42, 3)
    print(f"case: ex4.1 K=42 L=3 fused {prec}", flush=True)
    check_full(prob, prec, schedule="fused")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("window", ["pm", "exact"])
def test_table3_rectangle_threepass(window, prec):
    """Table 3's projection-method truncation K = 42, L = 60 (120 x 84): long
    trailing slabs in passes 1/3 and a long convolution axis in pass 2."""
    prob = W.paper_example_1d(2.5, 42, 60)
    print(f"case: ex4.1 K=42 L=60 {window} threepass {prec}", flush=True)
    check_full(prob, prec, window=window, schedule="threepass")


@pytest.mark.parametrize("order", ["grid", "window"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("split", [1, 2])
def test_table6_window_threepass(split, prec, order):
    """Table 6's IWFPM window (Ex. 4.2 case I, K = 6, L = 50: 100 x 12 x 12).
    split 1: the 100-point axis is the middle pass's convolution axis; split 2:
    it is a leading axis transformed beside a short convolution axis."""
    if order == "window" and split == 2:
        pytest.skip("window order keeps the k_I axes in one slab (split <= n - d = 1)")
    prob = W.paper_example_2d(0.8 * math.pi, 0.2 * math.pi, 6, 50)
    print(f"case: ex4.2 K=6 L=50 split={split} {prec} {order}", flush=True)
    check_full(prob, prec, order=order, schedule="threepass", split=split)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_three_stage_axis_in_middle_pass(prec):
    """2L = 8192 (8 x 32 x 32, the axis of the paper's L = 4096 references)
    as the middle pass's convolution axis, 8192 x 6 grid."""
    prob = W.paper_example_1d(3.0, 3, 4096)
    print(f"case: ex4.1 K=3 L=4096 threepass {prec}", flush=True)
    check_full(prob, prec, schedule="threepass", nvec=2)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_three_stage_axis_in_slabs(prec):
    """2K = 8192 as the trailing slab of passes 1 and 3 (2 x 8192 grid)."""
    prob = W.paper_example_1d(3.0, 4096, 1)
    print(f"case: ex4.1 K=4096 L=1 threepass {prec}", flush=True)
    check_full(prob, prec, schedule="threepass", nvec=2)


@pytest.mark.parametrize("schedule", ["fused", "threepass"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_long_axes_potential_grid(schedule, prec):
    """Oblique complex modes (the potential grid) on an 80 x 84 grid, both axes
    long: every V lookup undoes the digit order of both axes."""
    prob = _complex_oblique(np.array([[1.0, W.GOLDEN]]), 1, [42], [40])
    print(f"case: oblique potential 80x84 {schedule} {prec}", flush=True)
    check_full(prob, prec, schedule=schedule)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gap_extents(prec):
    """Extents below 64 without a compiled pencil of their own (34, 50, 62,
    44), in two stages, on a 2D/4D window."""
    P = W.rot_pair_P()
    modes, vhat = W.cosine_modes(4, [1.5, 1.5, 1.5, 1.5])
    prob = W.Problem("gaps", 2, P, [2, 25], [17, 3], modes, vhat)  # 34 x 6 x 4 x 50
    print(f"case: gap extents 34x6x4x50 {prec}", flush=True)
    check_full(prob, prec, schedule="threepass")
    prob = W.Problem("gaps", 2, P, [31, 2], [3, 22], modes, vhat)  # 6 x 44 x 62 x 4
    check_full(prob, prec, schedule="threepass")


@pytest.mark.timeout(600)
def test_table9_reference_grid_five_pass_sampled():
    """Ex. 4.3 at K = 5, L = 40 (80^3 x 10^3 = 512,000,000 points), the paper's
    reference truncation for Table 9: five passes, the 80-point axes in the
    middle pass (with the potential) and the further pass.  One vector, float32
    convolution, sampled entries against the oracle's row-by-row apply."""
    prob = W.paper_example_3d(math.pi, 5, 40)
    print(f"case: ex4.3 K=5 L=40 N={prob.N} fp32 five-pass", flush=True)
    sampled_check(prob, "fp32", nvec=1, nsample=300)
