// internal.hpp - descriptors shared by the host plan and the HIP kernels.
#pragma once

#include <cstdint>

namespace iwfpm {

constexpr int kMaxAxes = 8;
constexpr int kMaxFactors = 3;

// Geometry of the lifted grid K*_{K,L} (Sec. 3.2) as the kernels see it.
// Storage axes: 0..n-d-1 are the k_II axes, n-d..n-1 the k_I axes (fastest).
struct DevGeom {
    int n, d;
    int order;                      // 0 grid order, 1 window order
    int vmode;                      // 0 per-axis potential tables, 1 potential grid
    int kin;                        // 1: add the kinetic term, 0: potential block only
    int ext[kMaxAxes];              // extents 2L..., 2K...
    int stride[kMaxAxes];           // row-major element strides
    int N;                          // grid points per vector (< 2^31)
    int nkI;                        // points per k_I slice (product of the d fastest extents)
    int voff[kMaxAxes];             // offset of axis ax's potential table
    double P1[kMaxAxes * kMaxAxes]; // 2 pi P_I, d x d row-major
    // Axes longer than one register pencil are transformed in nfac > 1
    // stages of fac[0] x fac[1] (x fac[2]) points; between the inverse and
    // the forward transform such an axis is stored in the stages' digit
    // order (see long_axis_perm).  twoff: offset of its twiddle table
    // e^{+2 pi i j / ext}, j < ext.  nfac = 1 for every other axis.
    int nfac[kMaxAxes];
    int fac[kMaxAxes][kMaxFactors];
    int twoff[kMaxAxes];
};

// Device pointers owned by the plan.
struct DevTabs {
    const int* slice_a;       // per k_II slice: lower window end a_j = -K_j - floor(q_j), nslice x d
    const double* slice_g;    // per k_II slice: 2 pi (P_II k_II)_j, nslice x d
    const float* vtab32;      // per-axis potential tables (already divided by N)
    const double* vtab64;
    const float* vgrid32;     // potential on G_{K,L} divided by N (vmode 1)
    const double* vgrid64;
    const float* tw32;        // twiddle tables of the long axes (complex, interleaved)
    const double* tw64;
};

// Three-pass schedule (see apply_kernels.hip).
struct PassDesc {
    int split;          // number of leading axes handled by the middle pass
    int s_in;           // product of the trailing n - split extents (slab size)
    int s_out;          // product of the leading split extents
    int slabs_per_wg;   // passes 1 and 3: slabs per workgroup
    int tile;           // pass 2: columns per workgroup (a power of two)
    int threads_inner;  // block size of passes 1 and 3
    int threads_outer;  // block size of pass 2
    int xcd_remap;      // remap workgroup ids so that one XCD walks adjacent tiles
    // grids whose leading block does not fit one workgroup: the middle pass
    // keeps axes [0, split_mid) (with the potential) and a further pass
    // transforms axes [split_mid, split) on its own, once before and once after
    // it (0: no such pass)
    int split_mid;
    int tile_mid;       // that pass: columns per workgroup (a power of two)
    int threads_mid;    // that pass: block size
};

// LDS layout of a tile whose last axis (extent sl) is padded to an odd pitch sp
struct RowGeom {
    int sl, sp;
};

// bytes of the per-row table (kinetic and window data) for `rows` rows, d k_I axes
inline int row_table_bytes(int rows, int d) { return rows * (8 * d + 12); }

}  // namespace iwfpm
