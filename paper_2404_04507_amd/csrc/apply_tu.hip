// apply_tu.hip - one (kernel, precision) pair of the apply, selected at
// build time by IWFPM_TU_KERNEL (0 fused, 1 pass 1, 2 pass 2, 3 pass 3, 4 the
// persistent batched pass, 5 the further pass over the axes between the
// middle pass and pass 1) and
// IWFPM_TU_REAL (float or double) and IWFPM_TU_MAXS, the largest
// axis extent the instantiated kernels transform (16, 32 or 64).
#include "apply_kernels.hpp"
#include "apply_launch.hpp"

#ifndef IWFPM_TU_KERNEL
#error "IWFPM_TU_KERNEL must be defined"
#endif
#ifndef IWFPM_TU_REAL
#error "IWFPM_TU_REAL must be defined"
#endif
#ifndef IWFPM_TU_MAXS
#error "IWFPM_TU_MAXS must be defined"
#endif

namespace iwfpm {

using R = IWFPM_TU_REAL;
constexpr int M = IWFPM_TU_MAXS;

#if IWFPM_TU_KERNEL == 0
template <>
hipError_t launch_fused<R, M>(const DevGeom& g, const DevTabs& t, int threads, const void* psi, void* hpsi, int nvec,
                           hipStream_t st) {
    size_t lds = lds_fused(g, sizeof(cplx<R>));
    k_fused<R, M><<<dim3(nvec), dim3(threads), lds, st>>>(g, t, row_geom(g), reinterpret_cast<const double2*>(psi),
                                                           reinterpret_cast<double2*>(hpsi));
    return hipGetLastError();
}
template <>
hipError_t prepare_fused<R, M>(int lds_bytes) {
    return hipFuncSetAttribute((const void*)k_fused<R, M>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}
#elif IWFPM_TU_KERNEL == 1
template <>
hipError_t launch_pass1<R, M>(const DevGeom& g, const DevTabs& t, const PassDesc& pd, const void* psi, void* ws,
                           int nvec, hipStream_t st) {
    int nb = ((pd.s_out + pd.slabs_per_wg - 1) / pd.slabs_per_wg) * nvec;
    size_t lds = lds_slabs(g, pd, sizeof(cplx<R>));
    k_pass1<R, M><<<dim3(nb), dim3(pd.threads_inner), lds, st>>>(
        g, t, pd, row_geom(g), reinterpret_cast<const double2*>(psi), reinterpret_cast<cplx<R>*>(ws));
    return hipGetLastError();
}
template <>
hipError_t prepare_pass1<R, M>(int lds_bytes) {
    return hipFuncSetAttribute((const void*)k_pass1<R, M>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}
#elif IWFPM_TU_KERNEL == 2
template <>
hipError_t launch_pass2<R, M>(const DevGeom& g, const DevTabs& t, const PassDesc& pd, void* ws, int nvec,
                           hipStream_t st) {
    int ntile = (pd.s_in + pd.tile - 1) / pd.tile;
    size_t lds = lds_columns(g, pd, sizeof(cplx<R>));
    k_pass2<R, M><<<dim3(ntile * nvec), dim3(pd.threads_outer), lds, st>>>(g, t, pd,
                                                                            reinterpret_cast<cplx<R>*>(ws));
    return hipGetLastError();
}
template <>
hipError_t prepare_pass2<R, M>(int lds_bytes) {
    return hipFuncSetAttribute((const void*)k_pass2<R, M>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}
#elif IWFPM_TU_KERNEL == 3
template <>
hipError_t launch_pass3<R, M>(const DevGeom& g, const DevTabs& t, const PassDesc& pd, const void* psi, const void* ws,
                           void* hpsi, int nvec, hipStream_t st) {
    int nb = ((pd.s_out + pd.slabs_per_wg - 1) / pd.slabs_per_wg) * nvec;
    size_t lds = lds_slabs(g, pd, sizeof(cplx<R>));
    k_pass3<R, M><<<dim3(nb), dim3(pd.threads_inner), lds, st>>>(
        g, t, pd, row_geom(g), reinterpret_cast<const double2*>(psi), reinterpret_cast<const cplx<R>*>(ws),
        reinterpret_cast<double2*>(hpsi));
    return hipGetLastError();
}
template <>
hipError_t prepare_pass3<R, M>(int lds_bytes) {
    return hipFuncSetAttribute((const void*)k_pass3<R, M>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}
#elif IWFPM_TU_KERNEL == 4
template <>
hipError_t launch_batch<R, M>(const void* head, const void* items, int grid, size_t lds, int pass, hipStream_t st) {
    k_batch_pass<R, M><<<dim3(grid), dim3(256), lds, st>>>(reinterpret_cast<const BatchHead*>(head),
                                                           reinterpret_cast<const BatchItem*>(items), pass);
    return hipGetLastError();
}
template <>
hipError_t prepare_batch<R, M>(int lds_bytes) {
    return hipFuncSetAttribute((const void*)k_batch_pass<R, M>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               lds_bytes);
}
template <>
hipError_t occupancy_batch<R, M>(size_t lds, int* blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch_pass<R, M>, 256, lds);
}
#elif IWFPM_TU_KERNEL == 5
template <>
hipError_t launch_passm<R, M>(const DevGeom& g, const DevTabs& t, const PassDesc& pd, int sign, void* ws, int nvec,
                              hipStream_t st) {
    const int cols = pd.s_in;
    const int outer = g.N / g.stride[pd.split_mid - 1];
    const long long nb = (long long)((cols + pd.tile_mid - 1) / pd.tile_mid) * outer * nvec;
    if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    size_t lds = lds_mid(g, pd, sizeof(cplx<R>));
    if (sign > 0)
        k_passm<1, R, M><<<dim3((unsigned)nb), dim3(pd.threads_mid), lds, st>>>(g, t, pd,
                                                                               reinterpret_cast<cplx<R>*>(ws));
    else
        k_passm<-1, R, M><<<dim3((unsigned)nb), dim3(pd.threads_mid), lds, st>>>(g, t, pd,
                                                                                reinterpret_cast<cplx<R>*>(ws));
    return hipGetLastError();
}
template <>
hipError_t prepare_passm<R, M>(int lds_bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)k_passm<1, R, M>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       lds_bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_passm<-1, R, M>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}
#else
#error "IWFPM_TU_KERNEL out of range"
#endif

}  // namespace iwfpm
