// Entry points whose device implementation is not in this library version.
#include "host.h"

using namespace d2d;

extern "C" d2d_status d2d_batch_create(d2d_ctx* ctx, d2d_sb* const* sbs, int n, d2d_batch** out) {
    (void)ctx; (void)sbs; (void)n;
    if (out) *out = nullptr;
    set_error("d2d_batch_create is not built in this library version");
    return D2D_EINVAL;
}
extern "C" d2d_status d2d_batch_destroy(d2d_batch* b) { (void)b; return D2D_OK; }
extern "C" d2d_status d2d_batch_hv(d2d_batch* b, int prec, const void* const* v, void* const* w) {
    (void)b; (void)prec; (void)v; (void)w;
    set_error("d2d_batch_hv is not built in this library version");
    return D2D_EINVAL;
}
extern "C" d2d_status d2d_batch_lanczos(d2d_batch* b, const d2d_lanczos_opts* opts, const double* const* v0,
                                        double* energies, double* const* psi, d2d_lanczos_stats* per_problem) {
    (void)b; (void)opts; (void)v0; (void)energies; (void)psi; (void)per_problem;
    set_error("d2d_batch_lanczos is not built in this library version");
    return D2D_EINVAL;
}
