// apply_launch.hpp - host-side launchers of the apply kernels.  Each
// (kernel, precision) pair is compiled in its own translation unit
// (apply_tu.hip built once per pair) so that the build parallelises.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace iwfpm {

// padded row geometry of slab tiles: last extent sl, odd pitch sp
inline RowGeom row_geom(const DevGeom& g) {
    int sl = g.ext[g.n - 1];
    return RowGeom{sl, sl + ((sl & 1) ? 0 : 1)};
}
// dynamic LDS of the fused kernel and of passes 1/3 (tile + row table)
inline size_t lds_fused(const DevGeom& g, size_t esz) {
    RowGeom rg = row_geom(g);
    int rows = g.N / rg.sl;
    return (size_t)rows * rg.sp * esz + row_table_bytes(rows, g.d);
}
inline size_t lds_slabs(const DevGeom& g, const PassDesc& pd, size_t esz) {
    RowGeom rg = row_geom(g);
    int rows = pd.slabs_per_wg * pd.s_in / rg.sl;
    return (size_t)rows * rg.sp * esz + row_table_bytes(rows, g.d);
}
// pass 2 tile: rows of (last leading extent) x tile columns, padded by `tile`,
// then the potential's per-row and per-column sums (one real each)
inline size_t lds_columns(const DevGeom& g, const PassDesc& pd, size_t esz) {
    int El = g.ext[pd.split - 1];
    const size_t rows = (size_t)(pd.s_out / El);
    return rows * (El + 1) * pd.tile * esz + (rows + pd.tile) * (esz / 2);
}

// the further pass over axes [split_mid, split): rows of (extent of axis
// split - 1) x tile_mid columns, padded by tile_mid
inline size_t lds_mid(const DevGeom& g, const PassDesc& pd, size_t esz) {
    int El = g.ext[pd.split - 1];
    int mid = g.stride[pd.split_mid - 1] / pd.s_in;
    return (size_t)(mid / El) * (El + 1) * pd.tile_mid * esz;
}
// the middle pass's descriptor when a further pass takes axes [split_mid, split)
inline PassDesc middle_desc(const DevGeom& g, const PassDesc& pd) {
    PassDesc q = pd;
    if (pd.split_mid > 0) {
        q.split = pd.split_mid;
        q.s_in = g.stride[pd.split_mid - 1];
        q.s_out = g.N / q.s_in;
    }
    return q;
}

template <typename R, int MAXS>
hipError_t launch_fused(const DevGeom& g, const DevTabs& t, int threads, const void* psi, void* hpsi, int nvec,
                        hipStream_t st);
template <typename R, int MAXS>
hipError_t launch_pass1(const DevGeom& g, const DevTabs& t, const PassDesc& pd, const void* psi, void* ws,
                        int nvec, hipStream_t st);
template <typename R, int MAXS>
hipError_t launch_pass2(const DevGeom& g, const DevTabs& t, const PassDesc& pd, void* ws, int nvec, hipStream_t st);
template <typename R, int MAXS>
hipError_t launch_pass3(const DevGeom& g, const DevTabs& t, const PassDesc& pd, const void* psi, const void* ws,
                        void* hpsi, int nvec, hipStream_t st);
// the further pass (sign +1: inverse, -1: forward)
template <typename R, int MAXS>
hipError_t launch_passm(const DevGeom& g, const DevTabs& t, const PassDesc& pd, int sign, void* ws, int nvec,
                        hipStream_t st);
template <typename R, int MAXS>
hipError_t prepare_passm(int lds_bytes);
// persistent batched pass over the work table (head, items in device memory)
template <typename R, int MAXS>
hipError_t launch_batch(const void* head, const void* items, int grid, size_t lds, int pass, hipStream_t st);
template <typename R, int MAXS>
hipError_t prepare_batch(int lds_bytes);
template <typename R, int MAXS>
hipError_t occupancy_batch(size_t lds, int* blocks_per_cu);
// raise the dynamic-LDS limit of the kernel of this translation unit (current device)
template <typename R, int MAXS>
hipError_t prepare_fused(int lds_bytes);
template <typename R, int MAXS>
hipError_t prepare_pass1(int lds_bytes);
template <typename R, int MAXS>
hipError_t prepare_pass2(int lds_bytes);
template <typename R, int MAXS>
hipError_t prepare_pass3(int lds_bytes);

}  // namespace iwfpm
