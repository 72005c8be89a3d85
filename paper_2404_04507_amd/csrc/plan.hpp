// plan.hpp - the plan object behind iwfpm_plan_t (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/iwfpm.h"
#include "internal.hpp"

namespace iwfpm {

struct DeviceBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};

struct Schedule {
    bool ok = false;
    bool fused = false;
    PassDesc pd{};
    int maxs_fused = 0, maxs_inner = 0, maxs_outer = 0;  // extent classes (16, 32, 64)
    int threads_fused = 256;
};

struct LearnedPrecond;  // learned.cpp

// Per-kernel timing of applies: HIP events recorded on the apply's stream
// around each kernel, read back lazily so that recording never blocks.
struct ApplyProfiler {
    bool on = false;
    struct Slot {
        hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
        int kind = 0;            // 0 fused (ev0..ev1), 1 three-pass (ev0..ev3)
        long long points = 0;    // grid points processed by each kernel
        bool pending = false;
    };
    std::vector<Slot> ring;
    size_t head = 0;
    double ms[4] = {0, 0, 0, 0};        // fused, pass 1, pass 2, pass 3
    long long launches[4] = {0, 0, 0, 0};
    long long points[4] = {0, 0, 0, 0};
};

}  // namespace iwfpm

struct iwfpm_plan_s {
    // problem
    int d = 0, n = 0;
    std::vector<double> P;        // d x n
    std::vector<int> K, L;
    std::vector<int> modes;       // n_modes x n (merged duplicates)
    std::vector<double> vre, vim; // coefficients
    iwfpm_opts opts{};
    // geometry (host)
    iwfpm::DevGeom geom{};
    std::vector<double> Q;        // d x (n-d)
    long long nslice = 0;
    std::vector<int> slice_a;     // nslice x d
    std::vector<double> slice_g;  // nslice x d
    std::vector<double> vtab;     // per-axis tables / N (vmode 0)
    std::vector<double> vgrid;    // V on the grid / N (vmode 1)
    std::vector<double> tw;       // twiddle tables of the long axes (re, im interleaved)
    double vhat0 = 0.0;           // coefficient of the zero mode
    double vsum_nonzero = 0.0;    // sum over m != 0 of |Vhat_m|
    double vsum_abs = 0.0;        // sum over all m of |Vhat_m|
    double lam_max = 0.0;
    // schedules per precision: [0] float64, [1] float32
    iwfpm::Schedule sched[2];
    // device
    bool host_only = true;
    iwfpm::DeviceBuf d_slice_a, d_slice_g, d_vtab32, d_vtab64, d_vgrid32, d_vgrid64, d_tw32, d_tw64;
    iwfpm::DeviceBuf d_ws;        // apply workspace
    iwfpm::DeviceBuf d_ef_freq;   // eigenfunction output: (P k)_j per window point (d x N)
    iwfpm::DeviceBuf d_ef_ws;     // eigenfunction output: per-axis tables and slice partials
    iwfpm::DevTabs tabs{};
    iwfpm::ApplyProfiler prof;
    // eigensolver state (lobpcg.cpp)
    void* solver = nullptr;
    iwfpm::LearnedPrecond* learned = nullptr;
};

namespace iwfpm {

// host helpers shared by plan.cpp and lobpcg.cpp
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

int dev_alloc(DeviceBuf& b, size_t bytes);
void dev_free(DeviceBuf& b);

// grow the plan's apply workspace for nvec vectors of precision prec
int plan_ensure_ws(iwfpm_plan_s* p, int nvec, int prec, hipStream_t st);
int extent_class_of(int e);
// stages of an axis transform (fac[0..return)), 0 if the extent is unsupported
int axis_factors(int e, int* fac);
// extent class (16, 32, 64) of the register pencils axis ax needs
int axis_class(const DevGeom& g, int ax);

// apply on a plan (precision 0 = float64 convolution, 1 = float32), with the
// plan's own workspace (grown as needed)
int plan_apply(iwfpm_plan_s* p, const void* psi, void* hpsi, int nvec, int precision, hipStream_t st, int kinetic = 1);
// the same with a caller's workspace of ws_bytes (vectors applied in chunks
// whose intermediate grids fit; ERR_ARG if one vector's does not); allocates
// nothing
int plan_apply_ws(iwfpm_plan_s* p, const void* psi, void* hpsi, int nvec, int precision, hipStream_t st,
                  int kinetic, void* ws, size_t ws_bytes);

// grid position -> true label k (paper order) and vector position
void host_label(const iwfpm_plan_s* p, long long gpos, int* k_out);
long long host_grid_to_vec(const iwfpm_plan_s* p, long long gpos);
double host_kinetic(const iwfpm_plan_s* p, const int* k);

}  // namespace iwfpm
