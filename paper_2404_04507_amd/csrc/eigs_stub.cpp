// temporary: eigensolver entry points until lobpcg.cpp lands
#include "plan.hpp"
extern "C" {
void iwfpm_default_eigs_opts(iwfpm_eigs_opts* o) {
    if (!o) return;
    o->nev = 8; o->block = 0; o->tol = 1e-8; o->maxit = 500; o->precond = IWFPM_PRECOND_PLAIN; o->seed = 2404045070ull; o->polish = 1;
}
int iwfpm_eigs(iwfpm_plan_t, const iwfpm_eigs_opts*, const void*, double*, void*, double*, iwfpm_stats*, void*) {
    return IWFPM_ERR_UNSUPPORTED;
}
int iwfpm_destroy(iwfpm_plan_t p) {
    if (!p) return IWFPM_ERR_ARG;
    if (!p->host_only) {
        iwfpm::DeviceGuard g(p->opts.device);
        (void)hipDeviceSynchronize();
        iwfpm::dev_free(p->d_slice_a); iwfpm::dev_free(p->d_slice_g);
        iwfpm::dev_free(p->d_vtab32); iwfpm::dev_free(p->d_vtab64);
        iwfpm::dev_free(p->d_vgrid32); iwfpm::dev_free(p->d_vgrid64);
        iwfpm::dev_free(p->d_ws);
        for (auto& sl : p->prof.ring)
            for (auto& e : sl.ev)
                if (e) (void)hipEventDestroy(e);
    }
    delete p;
    return IWFPM_OK;
}
}
