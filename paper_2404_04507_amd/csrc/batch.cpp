// batch.cpp - ragged batches of plans applied by one persistent launch per
// pass (e.g. a sweep of couplings whose windows differ), optionally replayed
// from a captured hipGraph.
//
// The work table (per instance: geometry, tables, schedule, vector and
// workspace pointers, and the first work item of each pass) lives in device
// memory and is refreshed by an asynchronous copy before every apply; the
// launches (and the captured graph) only see its address, so one graph
// serves every apply of the batch.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "apply_kernels.hpp"
#include "apply_launch.hpp"
#include "plan.hpp"

using namespace iwfpm;

struct iwfpm_batch_s {
    int B = 0;
    int prec = 0;
    int device = 0;
    std::vector<iwfpm_plan_s*> plans;
    DeviceBuf d_table;           // BatchHead followed by B BatchItems
    unsigned char* h_table = nullptr;  // pinned staging
    size_t table_bytes = 0;
    hipEvent_t staged = nullptr;  // the last copy out of the staging buffer
    int maxs = 16;
    size_t lds = 0;
    int grid = 0;
    bool use_graph = false;
    hipGraphExec_t gexec = nullptr;
    hipStream_t gstream = nullptr;
};

static size_t items_offset() { return (sizeof(BatchHead) + 255) / 256 * 256; }

template <typename R>
static hipError_t launch_passes(iwfpm_batch_s* b, hipStream_t st) {
    const void* head = b->d_table.ptr;
    const void* items = (const unsigned char*)b->d_table.ptr + items_offset();
    for (int pass = 0; pass < 3; ++pass) {
        hipError_t e;
        switch (b->maxs) {
            case 16: e = launch_batch<R, 16>(head, items, b->grid, b->lds, pass, st); break;
            case 32: e = launch_batch<R, 32>(head, items, b->grid, b->lds, pass, st); break;
            default: e = launch_batch<R, 64>(head, items, b->grid, b->lds, pass, st); break;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename R>
static hipError_t occupancy(int maxs, size_t lds, int* n) {
    switch (maxs) {
        case 16: return occupancy_batch<R, 16>(lds, n);
        case 32: return occupancy_batch<R, 32>(lds, n);
        default: return occupancy_batch<R, 64>(lds, n);
    }
}

extern "C" {

int iwfpm_batch_create(int B, const iwfpm_plan_t* plans, int precision, int use_graph, iwfpm_batch_t* out) {
    if (!out || B < 1 || !plans) return IWFPM_ERR_ARG;
    *out = nullptr;
    if (precision != IWFPM_PREC_FP64 && precision != IWFPM_PREC_FP32) return IWFPM_ERR_ARG;
    const int prec = precision == IWFPM_PREC_FP32 ? 1 : 0;
    const size_t esz = prec ? 8 : 16;
    int dev = -1, maxe = 1;
    size_t lds = 0;
    for (int i = 0; i < B; ++i) {
        iwfpm_plan_s* p = plans[i];
        if (!p) return IWFPM_ERR_ARG;
        if (p->host_only) return IWFPM_ERR_NODEVICE;
        for (int j = 0; j < i; ++j)
            if (plans[j] == p) return IWFPM_ERR_ARG;  // each plan owns one workspace
        if (dev < 0) dev = p->opts.device;
        if (p->opts.device != dev) return IWFPM_ERR_ARG;  // one device per batch
        const Schedule& sc = p->sched[prec];
        if (!sc.ok) return IWFPM_ERR_UNSUPPORTED;
        if (!sc.fused && sc.pd.split_mid > 0) return IWFPM_ERR_UNSUPPORTED;  // five-pass grids: apply one by one
        for (int ax = 0; ax < p->n; ++ax) maxe = std::max(maxe, axis_class(p->geom, ax));
        if (sc.fused) lds = std::max(lds, lds_fused(p->geom, esz));
        else lds = std::max({lds, lds_slabs(p->geom, sc.pd, esz), lds_columns(p->geom, sc.pd, esz)});
    }
    DeviceGuard guard(dev);
    if (!guard.ok) return IWFPM_ERR_DEVICE;
    iwfpm_batch_s* b = new (std::nothrow) iwfpm_batch_s();
    if (!b) return IWFPM_ERR_ALLOC;
    b->B = B;
    b->prec = prec;
    b->device = dev;
    b->plans.assign(plans, plans + B);
    b->maxs = extent_class_of(maxe);
    b->lds = lds;
    b->use_graph = use_graph != 0;
    b->table_bytes = items_offset() + (size_t)B * sizeof(BatchItem);
    int rc = dev_alloc(b->d_table, b->table_bytes);
    if (rc == IWFPM_OK && hipHostMalloc((void**)&b->h_table, b->table_bytes) != hipSuccess) rc = IWFPM_ERR_ALLOC;
    if (rc == IWFPM_OK && hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess)
        rc = IWFPM_ERR_DEVICE;
    int per_cu = 0, cus = 0;
    if (rc == IWFPM_OK) {
        hipError_t e = prec ? occupancy<float>(b->maxs, lds, &per_cu) : occupancy<double>(b->maxs, lds, &per_cu);
        if (e != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            rc = IWFPM_ERR_DEVICE;
    }
    if (rc != IWFPM_OK) {
        iwfpm_batch_destroy(b);
        return rc;
    }
    b->grid = std::max(1, per_cu) * std::max(1, cus);
    *out = b;
    return IWFPM_OK;
}

int iwfpm_batch_apply(iwfpm_batch_t b, const void* const* psi, void* const* hpsi, const int* nvec, void* stream) {
    if (!b || !psi || !hpsi || !nvec) return IWFPM_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    DeviceGuard guard(b->device);
    if (!guard.ok) return IWFPM_ERR_DEVICE;
    for (int i = 0; i < b->B; ++i) {
        if (nvec[i] < 0 || (nvec[i] > 0 && (!psi[i] || !hpsi[i]))) return IWFPM_ERR_ARG;
        if (nvec[i] > 0) {
            int rc = plan_ensure_ws(b->plans[i], nvec[i], b->prec, st);
            if (rc) return rc;
        }
    }
    // the staging buffer may still be read by the previous copy
    if (hipEventSynchronize(b->staged) != hipSuccess) return IWFPM_ERR_DEVICE;
    BatchHead* head = reinterpret_cast<BatchHead*>(b->h_table);
    BatchItem* items = reinterpret_cast<BatchItem*>(b->h_table + items_offset());
    int tot[3] = {0, 0, 0};
    for (int i = 0; i < b->B; ++i) {
        iwfpm_plan_s* p = b->plans[i];
        const Schedule& sc = p->sched[b->prec];
        BatchItem& it = items[i];
        std::memset(&it, 0, sizeof(it));
        it.g = p->geom;
        it.t = p->tabs;
        it.pd = sc.pd;
        it.rg = row_geom(p->geom);
        it.psi = reinterpret_cast<const double2*>(psi[i]);
        it.hpsi = reinterpret_cast<double2*>(hpsi[i]);
        it.ws = p->d_ws.ptr;
        it.fused = sc.fused ? 1 : 0;
        for (int k = 0; k < 3; ++k) it.start[k] = tot[k];
        const int nv = nvec[i];
        if (sc.fused) {
            tot[0] += nv;
        } else {
            const int bpv = (sc.pd.s_out + sc.pd.slabs_per_wg - 1) / sc.pd.slabs_per_wg;
            const int ntile = (sc.pd.s_in + sc.pd.tile - 1) / sc.pd.tile;
            tot[0] += bpv * nv;
            tot[1] += ntile * nv;
            tot[2] += bpv * nv;
        }
    }
    head->B = b->B;
    for (int k = 0; k < 3; ++k) head->total[k] = tot[k];
    if (hipMemcpyAsync(b->d_table.ptr, b->h_table, b->table_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
        return IWFPM_ERR_DEVICE;
    if (hipEventRecord(b->staged, st) != hipSuccess) return IWFPM_ERR_DEVICE;
    // graphs cannot be captured on the null stream: launch directly there
    if (!b->use_graph || st == nullptr)
        return (b->prec ? launch_passes<float>(b, st) : launch_passes<double>(b, st)) == hipSuccess ? IWFPM_OK
                                                                                                   : IWFPM_ERR_DEVICE;
    if (!b->gexec || b->gstream != st) {
        if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return IWFPM_ERR_DEVICE;
        hipError_t e = b->prec ? launch_passes<float>(b, st) : launch_passes<double>(b, st);
        hipError_t e2 = hipStreamEndCapture(st, &graph);
        if (e != hipSuccess || e2 != hipSuccess || !graph) return IWFPM_ERR_DEVICE;
        e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            b->gexec = nullptr;
            return IWFPM_ERR_DEVICE;
        }
        b->gstream = st;
    }
    return hipGraphLaunch(b->gexec, st) == hipSuccess ? IWFPM_OK : IWFPM_ERR_DEVICE;
}

int iwfpm_batch_destroy(iwfpm_batch_t b) {
    if (!b) return IWFPM_ERR_ARG;
    {
        DeviceGuard guard(b->device);
        if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
        if (b->staged) (void)hipEventSynchronize(b->staged);
        if (b->staged) (void)hipEventDestroy(b->staged);
        (void)hipDeviceSynchronize();
        dev_free(b->d_table);
        if (b->h_table) (void)hipHostFree(b->h_table);
    }
    delete b;
    return IWFPM_OK;
}

}  // extern "C"
