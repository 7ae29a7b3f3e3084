// Local observables of a superblock state (the paper's stripe analysis,
// Eqs. (2)-(4)): site densities on the two explicit columns.
#include <algorithm>
#include <vector>

#include "host.h"

using namespace d2d;

extern "C" d2d_status d2d_column_densities(d2d_sb* sb, const double* psi, double* out) {
    if (!sb || !psi || !out) {
        set_error("d2d_column_densities: NULL argument");
        return D2D_EINVAL;
    }
    const int legs = sb->model.legs;
    const bool fermi = sb->model.kind == D2D_HUBBARD;
    const int nbits = fermi ? 2 * legs : legs;
    if (nbits > DENS_SLOTS - 1) {
        set_error("d2d_column_densities: %d occupation bits per column exceed %d", nbits, DENS_SLOTS - 1);
        return D2D_EINVAL;
    }
    d2d_ctx* ctx = sb->ctx;
    const int np = (int)sb->pairs.size();
    int64_t maxe = 0;
    for (const auto& p : sb->pairs) maxe = std::max<int64_t>(maxe, (int64_t)p.dL * p.dR);
    const int gx = (int)std::max<int64_t>(1, std::min<int64_t>(64, (maxe + 4095) / 4096));
    constexpr int S = 2 * DENS_SLOTS;
    const size_t nbytes = (size_t)np * gx * S * sizeof(double);
    double* part = nullptr;
    D2D_CHECK(ctx->alloc((void**)&part, nbytes));
    std::vector<double> h((size_t)np * gx * S);
    hipError_t e = launch_col_dens(sb->d_sec, np, gx, sb->d_rowsL, sb->d_colsR, sb->m, nbits, psi, part, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), part, nbytes, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    ctx->free(part, nbytes);
    if (e != hipSuccess) {
        set_error("d2d_column_densities: %s", hipGetErrorString(e));
        return D2D_EDEVICE;
    }
    // fixed-order sum of the partials
    double tot[S] = {};
    for (size_t b = 0; b < (size_t)np * gx; ++b)
        for (int k = 0; k < S; ++k) tot[k] += h[b * S + k];
    for (int c = 0; c < 2; ++c) {
        const double* t = tot + c * DENS_SLOTS;
        const double wsum = t[DENS_SLOTS - 1];
        for (int y = 0; y < legs; ++y) {
            double up, dn;
            if (fermi) {
                up = t[2 * y];
                dn = t[2 * y + 1];
            } else {
                up = t[y];
                dn = wsum - t[y];
            }
            out[(c * legs + y) * 2 + 0] = up;
            out[(c * legs + y) * 2 + 1] = dn;
        }
    }
    return D2D_OK;
}
