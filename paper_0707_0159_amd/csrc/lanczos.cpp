// Ground state of the superblock by restarted Lanczos with FP64 residual
// correction (the exact-diagonalisation routine of the DMRG step).
//
// Restart j:  w = H_64 x_j,  theta_j = x_j.w,  r = w - theta_j x_j,
//             rho_j = |r|  -> host (the only synchronisation per restart).
// Inner:      Lanczos started from x_j: q_0 = x_j, alpha_0 = theta_j,
//             beta_1 = rho_j, q_1 = r / rho_j (all FP64-exact), then k-1
//             steps with Hv in the working precision (FP64 / FP32 / BF16
//             inputs, FP32 accumulation), full reorthogonalisation by
//             classical Gram-Schmidt twice in FP64, the lowest eigenpair of the
//             k x k tridiagonal on the device, x_{j+1} = Q y / |Q y|.
// The fixed point is an eigenvector of the FP64 operator because the residual
// that drives every restart is computed with the FP64 Hv.
#include <chrono>
#include <cmath>
#include <cstring>

#include "host.h"

using namespace d2d;

struct LanczosWork {
    int kmax = 0;
    int64_t N = 0;
    int nb = 0;
    double* Q = nullptr;
    double* X = nullptr;
    double* W = nullptr;
    float* wlo = nullptr;
    float* vlo = nullptr;        // FP32 input (BF16 uses the first half as uint16)
    double* partial = nullptr;
    double* scal = nullptr;
    double* host_res = nullptr;  // pinned
    hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
    hipGraph_t graph[3] = {nullptr, nullptr, nullptr};
    int graph_k[3] = {0, 0, 0};
};

namespace {
constexpr int S_ALPHA = 0, S_BETA = 130, S_C1 = 260, S_C2 = 390, S_NRM = 520, S_THETA = 524, S_Y = 528,
              S_TWORK = 660, S_RES = 1300, S_FLAGS = 1304, S_LEN = 1400;
constexpr int PARTIAL_ROWS = 130;
// second partial-sum buffer of the fused step kernels (33 rows x 256 blocks), after the first
constexpr int64_t PARTIAL2_ROWS = 34;
}  // namespace

// partial-sum area: PARTIAL_ROWS x nb for the general kernels, of which the
// first 34 x 256 also serve the fused step kernels, then a second 34 x 256 buffer
static size_t partial_len(int nb) {
    const size_t a = (size_t)PARTIAL_ROWS * (nb > 256 ? nb : 256);
    return a + (size_t)PARTIAL2_ROWS * 256;
}
#define PARTIAL2 ((int64_t)PARTIAL_ROWS * (w->nb > 256 ? w->nb : 256))

namespace d2d {

void free_lanczos(d2d_sb* sb) {
    LanczosWork* lw = sb->lz;
    if (!lw) return;
    d2d_ctx* c = sb->ctx;
    for (int p = 0; p < 3; ++p) {
        if (lw->exec[p]) (void)hipGraphExecDestroy(lw->exec[p]);
        if (lw->graph[p]) (void)hipGraphDestroy(lw->graph[p]);
    }
    c->free(lw->Q, (size_t)(lw->kmax + 1) * lw->N * 8);
    c->free(lw->X, (size_t)lw->N * 8);
    c->free(lw->W, (size_t)lw->N * 8);
    c->free(lw->wlo, (size_t)lw->N * 4);
    c->free(lw->vlo, (size_t)lw->N * 4);
    c->free(lw->partial, partial_len(lw->nb) * 8);
    c->free(lw->scal, (size_t)S_LEN * 8);
    if (lw->host_res) (void)hipHostFree(lw->host_res);
    delete lw;
    sb->lz = nullptr;
}

}  // namespace d2d

static d2d_status ensure_work(d2d_sb* sb, int kmax) {
    if (sb->lz && sb->lz->kmax >= kmax) return D2D_OK;
    free_lanczos(sb);
    d2d_ctx* c = sb->ctx;
    LanczosWork* w = new LanczosWork();
    w->kmax = kmax;
    w->N = sb->N;
    w->nb = lz_nblocks(sb->N);
    sb->lz = w;
    D2D_CHECK(c->alloc((void**)&w->Q, (size_t)(kmax + 1) * w->N * 8));
    D2D_CHECK(c->alloc((void**)&w->X, (size_t)w->N * 8));
    D2D_CHECK(c->alloc((void**)&w->W, (size_t)w->N * 8));
    D2D_CHECK(c->alloc((void**)&w->wlo, (size_t)w->N * 4));
    D2D_CHECK(c->alloc((void**)&w->vlo, (size_t)w->N * 4));
    D2D_CHECK(c->alloc((void**)&w->partial, partial_len(w->nb) * 8));
    D2D_CHECK(c->alloc((void**)&w->scal, (size_t)S_LEN * 8));
    D2D_HIP(hipMemset(w->scal, 0, (size_t)S_LEN * 8));
    D2D_HIP(hipHostMalloc((void**)&w->host_res, 8 * sizeof(double), hipHostMallocDefault));
    return D2D_OK;
}

// FP64 residual of X: W = H X, theta = X.W, W <- W - theta X, rho = |W|;
// alpha[0] = theta, beta[1] = rho; (theta, rho) copied to pinned host memory.
static d2d_status residual_step(d2d_sb* sb, hipStream_t s) {
    LanczosWork* w = sb->lz;
    double* sc = w->scal;
    D2D_CHECK(sb_hv(sb, D2D_FP64, w->X, w->W, s));
    D2D_HIP(launch_lz_residual(w->X, w->W, w->N, w->partial, w->partial + PARTIAL2, sc + S_ALPHA, sc + S_BETA,
                               sc + S_RES, s));
    D2D_HIP(hipMemcpyAsync(w->host_res, sc + S_RES, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    return D2D_OK;
}

// One inner Lanczos of k vectors started from X (needs residual_step before),
// ending with X = Ritz vector, normalised.
static d2d_status inner_loop(d2d_sb* sb, int prec, int k, hipStream_t s) {
    LanczosWork* w = sb->lz;
    double* sc = w->scal;
    const int64_t N = w->N;
    void* lo = prec == D2D_FP64 ? nullptr : (void*)w->vlo;
    D2D_HIP(launch_copy_f64(w->X, w->Q, N, s));
    D2D_HIP(launch_scale_store(w->W, sc + S_BETA + 1, w->Q + N, lo, prec, N, s));
    for (int i = 1; i < k; ++i) {
        double* qi = w->Q + (int64_t)i * N;
        const int nq = i + 1;
        if (nq <= 32) {
            // fused step: three kernels with in-kernel reductions
            if (prec == D2D_FP64) D2D_CHECK(sb_hv(sb, D2D_FP64, qi, w->W, s));
            else D2D_CHECK(sb_hv(sb, prec, w->vlo, w->wlo, s));
            LzStepArgs a{};
            a.Q = w->Q;
            a.n = N;
            a.nq = nq;
            a.i = i;
            a.upcast = prec != D2D_FP64;
            a.w32 = w->wlo;
            a.w = w->W;
            a.partial = w->partial;
            a.partial2 = w->partial + PARTIAL2;
            a.alpha = sc + S_ALPHA;
            a.beta = sc + S_BETA;
            a.qnext = i + 1 < k ? w->Q + (int64_t)(i + 1) * N : nullptr;
            a.lo = lo;
            a.lo_prec = prec;
            D2D_HIP(launch_lz_step(a, s));
            continue;
        }
        if (prec == D2D_FP64) {
            D2D_CHECK(sb_hv(sb, D2D_FP64, qi, w->W, s));
            D2D_HIP(launch_dots_f64(w->Q, N, nq, w->W, N, w->partial, s));
        } else {
            D2D_CHECK(sb_hv(sb, prec, w->vlo, w->wlo, s));
            D2D_HIP(launch_upcast_dots(w->Q, N, nq, w->wlo, w->W, N, w->partial, s));
        }
        D2D_HIP(launch_reduce(w->partial, nq, w->nb, sc + S_C1, s));
        D2D_HIP(launch_update(w->Q, N, nq, sc + S_C1, w->W, N, nullptr, s));
        D2D_HIP(launch_dots_f64(w->Q, N, nq, w->W, N, w->partial, s));
        D2D_HIP(launch_reduce(w->partial, nq, w->nb, sc + S_C2, s));
        D2D_HIP(launch_update(w->Q, N, nq, sc + S_C2, w->W, N, w->partial, s));
        D2D_HIP(launch_reduce(w->partial, 1, w->nb, sc + S_NRM, s));
        D2D_HIP(launch_step_scalars(i, sc + S_C1, sc + S_C2, sc + S_NRM, sc + S_ALPHA, sc + S_BETA, sc + S_FLAGS, s));
        if (i + 1 < k) D2D_HIP(launch_scale_store(w->W, sc + S_BETA + i + 1, w->Q + (int64_t)(i + 1) * N, lo, prec, N, s));
    }
    D2D_HIP(launch_tridiag(sc + S_ALPHA, sc + S_BETA, k, sc + S_THETA + 1, sc + S_Y, sc + S_TWORK, s));
    D2D_HIP(launch_lz_ritz(w->Q, N, k, sc + S_Y, w->X, N, w->partial, s));
    return D2D_OK;
}

static d2d_status restart(d2d_sb* sb, int prec, int k, bool use_graph, hipStream_t s) {
    LanczosWork* w = sb->lz;
    if (!use_graph || s == nullptr) {
        D2D_CHECK(inner_loop(sb, prec, k, s));
        return residual_step(sb, s);
    }
    if (!w->exec[prec] || w->graph_k[prec] != k) {
        if (w->exec[prec]) (void)hipGraphExecDestroy(w->exec[prec]);
        if (w->graph[prec]) (void)hipGraphDestroy(w->graph[prec]);
        w->exec[prec] = nullptr;
        w->graph[prec] = nullptr;
        // work lists must exist before capture (their creation copies memory)
        WorkItem* dummy;
        int nw;
        const int shape_p = sb->tile_sel[prec] >= 0 ? sb->tile_sel[prec] : sb_auto_tile(sb, prec);
        const int shape_64 = sb->tile_sel[0] >= 0 ? sb->tile_sel[0] : sb_auto_tile(sb, D2D_FP64);
        D2D_CHECK(sb_work(sb, shape_p, &dummy, &nw));
        D2D_CHECK(sb_work(sb, shape_64, &dummy, &nw));
        const int64_t saved[3] = {sb->hv_count[0], sb->hv_count[1], sb->hv_count[2]};
        D2D_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        d2d_status st = inner_loop(sb, prec, k, s);
        if (st == D2D_OK) st = residual_step(sb, s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        for (int i = 0; i < 3; ++i) sb->hv_count[i] = saved[i];
        if (st != D2D_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) {
            set_error("graph capture failed: %s", hipGetErrorString(e));
            return D2D_EDEVICE;
        }
        w->graph[prec] = g;
        D2D_HIP(hipGraphInstantiate(&w->exec[prec], g, nullptr, nullptr, 0));
        w->graph_k[prec] = k;
    }
    D2D_HIP(hipGraphLaunch(w->exec[prec], s));
    sb->hv_count[prec] += k - 1;
    sb->hv_count[D2D_FP64] += 1;
    return D2D_OK;
}

extern "C" d2d_status d2d_lanczos(d2d_sb* sb, const d2d_lanczos_opts* opts, const double* v0, double* energy,
                                  double* psi, d2d_lanczos_stats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    if (!sb || !opts || !v0 || !energy) {
        set_error("d2d_lanczos: NULL argument");
        return D2D_EINVAL;
    }
    if (opts->k_in < 2 || opts->k_in > 128 || opts->max_restarts < 0 || !(opts->tol_res > 0.0) ||
        opts->prec < 0 || opts->prec > 2) {
        set_error("d2d_lanczos: bad options (k_in 2..128, tol_res > 0, prec 0..2)");
        return D2D_EINVAL;
    }
    if (!(sb->prec_mask & (1u << opts->prec)) || !sb->HL[opts->prec]) {
        set_error("d2d_lanczos: precision %d not kept by this superblock", opts->prec);
        return D2D_EINVAL;
    }
    hipStream_t s = sb->ctx->stream;
    const int k = (int)std::min<int64_t>(opts->k_in, sb->N);
    D2D_CHECK(ensure_work(sb, std::max(k, 2)));
    LanczosWork* w = sb->lz;
    const int64_t cnt0[3] = {sb->hv_count[0], sb->hv_count[1], sb->hv_count[2]};
    // x_0 = v0 / |v0|
    D2D_HIP(launch_dots_f64(v0, w->N, 1, v0, w->N, w->partial, s));
    D2D_HIP(launch_reduce(w->partial, 1, w->nb, w->scal + S_NRM, s));
    D2D_HIP(hipMemcpyAsync(w->host_res, w->scal + S_NRM, sizeof(double), hipMemcpyDeviceToHost, s));
    D2D_HIP(hipStreamSynchronize(s));
    const double n0 = w->host_res[0];
    if (!std::isfinite(n0) || !(n0 > 0.0)) {
        set_error("d2d_lanczos: start vector is zero or not finite");
        return D2D_EINVAL;
    }
    D2D_HIP(launch_scale_copy(v0, w->scal + S_NRM, w->X, w->N, s));
    D2D_CHECK(residual_step(sb, s));
    D2D_HIP(hipStreamSynchronize(s));
    double theta = w->host_res[0], rho = w->host_res[1], rho_prev = -1.0;
    int prec = opts->prec;
    int j = 0;
    d2d_lanczos_stats st{};
    d2d_status result = D2D_ENOCONV;
    for (;;) {
        const double tsec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (!std::isfinite(theta) || !std::isfinite(rho)) {
            set_error("d2d_lanczos: non-finite Rayleigh quotient at restart %d", j);
            result = D2D_EDEVICE;
            break;
        }
        if (rho_prev >= 0.0 && prec != D2D_FP64 && opts->escalate > 0.0 && rho > opts->escalate * rho_prev) {
            // raise to the next precision this superblock keeps
            int np = prec == D2D_BF16 ? D2D_FP32 : D2D_FP64;
            if (!(sb->prec_mask & (1u << np)) || !sb->HL[np]) np = D2D_FP64;
            prec = np;
        }
        if (st.nlog < D2D_LOG_MAX) {
            st.log_t[st.nlog] = tsec;
            st.log_theta[st.nlog] = theta;
            st.log_rho[st.nlog] = rho;
            st.log_prec[st.nlog] = prec;
            st.nlog++;
        }
        if (rho <= opts->tol_res * std::fabs(theta) || rho == 0.0 || k < 2) {
            result = D2D_OK;
            break;
        }
        if (j >= opts->max_restarts) {
            set_error("d2d_lanczos: no convergence after %d restarts (rho = %g)", j, rho);
            result = D2D_ENOCONV;
            break;
        }
        D2D_CHECK(restart(sb, prec, k, opts->use_graph != 0, s));
        D2D_HIP(hipStreamSynchronize(s));
        rho_prev = rho;
        theta = w->host_res[0];
        rho = w->host_res[1];
        ++j;
    }
    *energy = theta;
    if (psi) {
        D2D_HIP(hipMemcpyAsync(psi, w->X, (size_t)w->N * 8, hipMemcpyDeviceToDevice, s));
        D2D_HIP(hipStreamSynchronize(s));
    }
    st.restarts = j;
    for (int i = 0; i < 3; ++i) st.hv_count[i] = sb->hv_count[i] - cnt0[i];
    st.residual = rho;
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    return result;
}
