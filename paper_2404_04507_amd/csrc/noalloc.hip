// noalloc.hip - the Hamiltonian apply for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).
//
// The multi-pass schedules stage the intermediate grid in a workspace
// (the fused one needs none).  Here that workspace is a file-scope device
// array of kScratchBytes, which each GPU the library runs on holds until the
// process ends.  Host code never passes the array's own name to a kernel (on
// the host it is a stand-in, not a device address): the first call on a
// device, with that device current, resolves the array's address there with
// hipGetSymbolAddress and keeps it per device, and the kernels receive that
// pointer as they receive the plan's own workspace.
//
// Every call on one GPU shares that GPU's array.  Nothing in it has to start
// at zero (every pass writes the part of the grid it later reads), but calls
// that overlap in time on one GPU - on different streams, or from several
// threads - race for it.

#include <hip/hip_runtime.h>

#include <mutex>

#include "plan.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)128 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on `dev` (the current device)
int scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return IWFPM_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return IWFPM_ERR_DEVICE;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return IWFPM_OK;
}

}  // namespace

extern "C" {

int64_t iwfpm_noalloc_scratch_bytes(void) { return (int64_t)kScratchBytes; }

int iwfpm_apply_noalloc(iwfpm_plan_t p, const void* psi, void* hpsi, int nvec, void* stream) {
    if (!p || nvec < 0) return IWFPM_ERR_ARG;
    if (nvec > 0 && (!psi || !hpsi)) return IWFPM_ERR_ARG;
    if (p->host_only) return IWFPM_ERR_NODEVICE;
    if (nvec == 0) return IWFPM_OK;
    const size_t bytes = (size_t)nvec * (size_t)p->geom.N * 16;
    const char* a = (const char*)psi;
    const char* b = (const char*)hpsi;
    if (a < b + bytes && b < a + bytes) return IWFPM_ERR_ARG;  // overlapping buffers
    const int prec = p->opts.precision == IWFPM_PREC_FP32 ? 1 : 0;
    const iwfpm::Schedule& sc = p->sched[prec];
    if (!sc.ok) return IWFPM_ERR_UNSUPPORTED;
    // one vector's intermediate grid must fit; more vectors are applied in
    // chunks that fit
    if (!sc.fused && (size_t)p->geom.N * (prec ? 8 : 16) > kScratchBytes) return IWFPM_ERR_TOO_LARGE;
    iwfpm::DeviceGuard guard(p->opts.device);
    if (!guard.ok) return IWFPM_ERR_DEVICE;
    void* ws = nullptr;
    int rc = scratch_address(p->opts.device, &ws);
    if (rc != IWFPM_OK) return rc;
    return iwfpm::plan_apply_ws(p, psi, hpsi, nvec, p->opts.precision, (hipStream_t)stream, 1, ws, kScratchBytes);
}

}  // extern "C"
