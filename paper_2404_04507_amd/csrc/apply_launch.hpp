// apply_launch.hpp - host-side launchers of the apply kernels.  Each
// (kernel, precision) pair is compiled in its own translation unit
// (apply_tu.hip built once per pair) so that the build parallelises.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace iwfpm {

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
