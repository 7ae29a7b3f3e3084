// Ground state of one superblock or of a set of superblocks by restarted
// Lanczos with FP64 residual correction (the exact-diagonalisation routine of
// the DMRG step).
//
// Restart j:  w = H_64 x_j,  theta_j = x_j.w,  r = w - theta_j x_j,
//             rho_j = |r|  -> host (the only synchronisation per restart).
// Inner:      Lanczos started from x_j: q_0 = x_j, alpha_0 = theta_j,
//             beta_1 = rho_j, q_1 = r / rho_j (all FP64-exact), then k-1
//             steps with Hv in the working precision (FP64 / FP32 / BF16
//             inputs, FP32 accumulation), reorthogonalisation by classical
//             Gram-Schmidt twice in FP64, the lowest eigenpair of the k x k
//             tridiagonal on the device, x_{j+1} = Q y / |Q y| with q_0 = x_j
//             taken in FP64 (below FP64 the basis is stored in the products'
//             input precision).
// The fixed point is an eigenvector of the FP64 operator because the residual
// that drives every restart is computed with the FP64 Hv.
//
// A set of problems (a batch) runs in lockstep: their vectors are
// concatenated, the vector kernels are segmented per problem, the Hv is one
// grouped launch over all of them, and a converged problem leaves the launches
// at the next restart.  A problem whose restarts fall short because of the
// working precision waits until the others are done at that precision, and
// the waiting problems then go on one precision higher.  One superblock is
// the set of one.
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>

#include "host.h"

using namespace d2d;

namespace d2d {

void free_lanczos_work(d2d_ctx* c, LanczosWork*& lw) {
    if (!lw) return;
    for (int p = 0; p < 2 * D2D_NPREC; ++p) {
        if (lw->exec[p]) (void)hipGraphExecDestroy(lw->exec[p]);
        if (lw->graph[p]) (void)hipGraphDestroy(lw->graph[p]);
    }
    const size_t nt = (size_t)lw->ntot;
    c->free(lw->Q, (size_t)(lw->kmax + 1) * lw->ldq * 8);
    c->free(lw->X, nt * 8);
    c->free(lw->W, nt * 8);
    c->free(lw->wlo, nt * 4);
    c->free(lw->vlo, nt * 4);
    c->free(lw->partial, (size_t)2 * 34 * lw->NB * 8);
    c->free(lw->scal, (size_t)lw->nprob * S_LEN * 8);
    c->free(lw->res, (size_t)3 * lw->nprob * 8);
    c->free(lw->bt, (size_t)lw->NB * sizeof(LzSeg));
    c->free(lw->prange, (size_t)lw->nprob * sizeof(int2));
    c->free(lw->active, (size_t)lw->nprob * sizeof(int));
    if (lw->res_host) (void)hipHostFree(lw->res_host);
    delete lw;
    lw = nullptr;
}

void free_lanczos(d2d_sb* sb) { free_lanczos_work(sb->ctx, sb->lz); }

// Workspace for problems of lengths len[] (concatenated in order), k vectors.
d2d_status ensure_lanczos_work(d2d_ctx* c, LanczosWork*& lw, const std::vector<int64_t>& len, int kmax) {
    int64_t ntot = 0;
    for (int64_t n : len) ntot += n;
    if (lw && lw->kmax >= kmax && lw->ntot == ntot && lw->nprob == (int)len.size()) return D2D_OK;
    free_lanczos_work(c, lw);
    lw = new LanczosWork();
    LanczosWork* w = lw;
    w->kmax = kmax;
    w->ntot = ntot;
    w->nprob = (int)len.size();
    // block table: every problem gets its own blocks (at most 256)
    std::vector<LzSeg> bt;
    std::vector<int2> pr(w->nprob);
    int64_t off = 0;
    for (int p = 0; p < w->nprob; ++p) {
        const int nb = lz_step_blocks(len[p]);
        const int b0 = (int)bt.size();
        const int64_t per = (len[p] + nb - 1) / nb;
        for (int b = 0; b < nb; ++b) {
            LzSeg sg{};
            sg.prob = p;
            sg.act = 1;
            sg.pb0 = b0;
            sg.pb1 = b0 + nb;
            sg.lo = off + std::min<int64_t>((int64_t)b * per, len[p]);
            sg.hi = off + std::min<int64_t>((int64_t)(b + 1) * per, len[p]);
            bt.push_back(sg);
        }
        pr[p] = make_int2(b0, b0 + nb);
        off += len[p];
    }
    w->NB = (int)bt.size();
    w->h_bt = bt;
    for (const LzSeg& sg : bt) w->max_seg = std::max<int64_t>(w->max_seg, sg.hi - sg.lo);
    w->seg_off.resize(w->nprob);
    w->seg_len = len;
    off = 0;
    for (int p = 0; p < w->nprob; ++p) {
        w->seg_off[p] = off;
        off += len[p];
    }
    const size_t nt = (size_t)ntot;
    // every basis vector starts on a 128-byte boundary (64 elements of 2 bytes or more)
    w->ldq = (ntot + 63) / 64 * 64;
    D2D_CHECK(c->alloc((void**)&w->Q, (size_t)(kmax + 1) * w->ldq * 8));
    D2D_CHECK(c->alloc((void**)&w->X, nt * 8));
    D2D_CHECK(c->alloc((void**)&w->W, nt * 8));
    D2D_CHECK(c->alloc((void**)&w->wlo, nt * 4));
    D2D_CHECK(c->alloc((void**)&w->vlo, nt * 4));
    D2D_CHECK(c->alloc((void**)&w->partial, (size_t)2 * 34 * w->NB * 8));
    D2D_CHECK(c->alloc((void**)&w->scal, (size_t)w->nprob * S_LEN * 8));
    D2D_CHECK(c->alloc((void**)&w->res, (size_t)3 * w->nprob * 8));
    D2D_CHECK(c->alloc((void**)&w->bt, bt.size() * sizeof(LzSeg)));
    D2D_CHECK(c->alloc((void**)&w->prange, pr.size() * sizeof(int2)));
    D2D_CHECK(c->alloc((void**)&w->active, (size_t)w->nprob * sizeof(int)));
    D2D_HIP(hipMemset(w->scal, 0, (size_t)w->nprob * S_LEN * 8));
    D2D_HIP(hipMemcpy(w->bt, bt.data(), bt.size() * sizeof(LzSeg), hipMemcpyHostToDevice));
    D2D_HIP(hipMemcpy(w->prange, pr.data(), pr.size() * sizeof(int2), hipMemcpyHostToDevice));
    D2D_HIP(hipMemset(w->res, 0, (size_t)3 * w->nprob * 8));
    D2D_HIP(hipHostMalloc((void**)&w->res_host, (size_t)3 * w->nprob * 8, hipHostMallocDefault));
    return D2D_OK;
}

}  // namespace d2d

namespace {

// active flags per problem, and the same flags in every block-table entry
d2d_status set_active_flags(LanczosWork* w, const std::vector<int>& act) {
    for (auto& sg : w->h_bt) sg.act = act[sg.prob] ? 1 : 0;
    D2D_HIP(hipMemcpy(w->active, act.data(), act.size() * sizeof(int), hipMemcpyHostToDevice));
    D2D_HIP(hipMemcpy(w->bt, w->h_bt.data(), w->h_bt.size() * sizeof(LzSeg), hipMemcpyHostToDevice));
    return D2D_OK;
}

LzSet set_of(LanczosWork* w) {
    LzSet z{};
    z.nprob = w->nprob;
    z.NB = w->NB;
    z.ntot = w->ntot;
    z.bt = w->bt;
    z.prange = w->prange;
    z.active = w->active;
    z.partial = w->partial;
    z.partial2 = w->partial + (size_t)34 * w->NB;
    z.scal = w->scal;
    z.res = w->res;
    return z;
}

// FP64 residual of X; (theta, rho) of every problem and the last Ritz residual
// estimates copied to pinned host memory.
d2d_status residual_step(LanczosWork* w, HvOps& hv, hipStream_t s) {
    const LzSet z = set_of(w);
    D2D_CHECK(hv.hv(D2D_FP64, w->X, w->W, s));
    D2D_HIP(launch_lz_residual(z, w->X, w->W, s));
    D2D_HIP(hipMemcpyAsync(w->res_host, w->res, (size_t)3 * w->nprob * 8, hipMemcpyDeviceToHost, s));
    return D2D_OK;
}

// Bytes per basis element: basis 0 stores the basis in the products' input
// precision (FP64, FP32 for FP32 and BF16x3, BF16 for BF16), 1 in FP64, 2 in
// FP32 below FP64.
int basis_bytes(int prec, int basis) {
    if (prec == D2D_FP64 || basis == 1) return 8;
    if (prec == D2D_BF16 && basis == 0) return 2;
    return 4;
}

// One inner Lanczos of k vectors from X (after residual_step); X <- Ritz vector.
// X enters the Ritz vector in FP64, so the rounding of a narrow basis only
// touches the correction sum_{j>=1} y_j q_j, which shrinks with the residual.
// A basis vector in the products' input precision is the product's input
// itself; otherwise the step writes an input copy (lo).
// coop: the Gram step may run as one cooperative kernel (not under capture);
// it does where every block's segment fits the kernel's registers and the
// grid fits the device at once.
// what a call did besides its products (reported in the statistics)
struct RunCounters {
    int captures = 0;          // restarts captured as graphs
    int64_t coop_steps = 0;    // steps run as the one-kernel (cooperative) step
};

d2d_status inner_loop(LanczosWork* w, HvOps& hv, int prec, int k, int window, bool fused, bool plain_cgs2,
                      int basis, bool coop, hipStream_t s, RunCounters* rc) {
    const LzSet z = set_of(w);
    const int64_t ldq = w->ldq;
    const int qb = basis_bytes(prec, basis);
    const bool one_kernel = coop && w->max_seg <= lz_coop_segment_max() &&
                            lz_coop_fits(z.NB, prec != D2D_FP64, qb);
    const size_t qs = (size_t)qb;
    char* Q = (char*)w->Q;
    const int in_bytes = prec == D2D_FP64 ? 8 : (prec == D2D_BF16 ? 2 : 4);
    void* lo = qb == in_bytes ? nullptr : (void*)w->vlo;
    D2D_HIP(launch_lz_first(z, w->X, w->W, Q, qb, ldq, lo, prec, s));
    for (int i = 1; i < k; ++i) {
        const void* qi = Q + (size_t)i * ldq * qs;
        // fused GEMM + central launch; the step's first kernel adds the parts
        HvParts parts{};
        const void* hin = lo ? (const void*)lo : qi;
        void* hout = prec == D2D_FP64 ? (void*)w->W : (void*)w->wlo;
        if (fused) D2D_CHECK(hv.hv_fused(prec, hin, hout, s, &parts));
        else D2D_CHECK(hv.hv(prec, hin, hout, s));
        LzStepArgs a{};
        a.bt = z.bt;
        // projection against q_{i-nq+1} .. q_i (all of them for full reorthogonalisation)
        const int nq = window >= 2 ? std::min(i + 1, window) : i + 1;
        a.Q = Q + (size_t)(i + 1 - nq) * ldq * qs;
        a.qbytes = qb;
        a.ldq = ldq;
        a.nq = nq;
        a.i = i;
        a.upcast = prec != D2D_FP64;
        a.gram = !plain_cgs2 && window >= 2 && window <= 4;
        a.coop = a.gram && one_kernel;
        a.w32 = w->wlo;
        a.w = w->W;
        for (int q = 0; q < 3; ++q) a.wpart[q] = parts.x[q];
        a.wpart[3] = parts.central;
        a.partial = z.partial;
        a.partial2 = z.partial2;
        a.NB = z.NB;
        a.scal = z.scal;
        a.qnext = i + 1 < k ? (void*)(Q + (size_t)(i + 1) * ldq * qs) : nullptr;
        a.lo = lo;
        a.lo_prec = prec;
        D2D_HIP(launch_lz_step(a, s));
        if (a.coop && rc) rc->coop_steps++;
    }
    D2D_HIP(launch_lz_tridiag(z, k, s));
    D2D_HIP(launch_lz_ritz(z, Q, qb, ldq, k, w->X, s));
    return D2D_OK;
}

void drop_graphs(LanczosWork* w) {
    for (int p = 0; p < 2 * D2D_NPREC; ++p) {
        if (w->exec[p]) (void)hipGraphExecDestroy(w->exec[p]);
        if (w->graph[p]) (void)hipGraphDestroy(w->graph[p]);
        w->exec[p] = nullptr;
        w->graph[p] = nullptr;
    }
}

// A restart (its inner Lanczos and the FP64 residual) launched directly, or
// captured once as a hipGraph and replayed.  A capture stays valid, across
// calls too, while the workspace lives and nothing it recorded changes: the
// precision, cycle length, window, fusion, Gram form and basis storage, the
// launch stream and the operator's launch configuration (its fingerprint).
d2d_status restart(LanczosWork* w, HvOps& hv, int prec, int k, bool full, int window, bool fused,
                   bool plain_cgs2, int basis, bool coop, bool use_graph, hipStream_t s, RunCounters* rc) {
    if (!use_graph || s == nullptr) {
        D2D_CHECK(inner_loop(w, hv, prec, k, window, fused, plain_cgs2, basis, coop, s, rc));
        D2D_CHECK(residual_step(w, hv, s));
        hv.count(prec, k - 1);
        hv.count(D2D_FP64, 1);
        return D2D_OK;
    }
    const int g = 2 * prec + (full ? 0 : 1);
    D2D_CHECK(hv.prepare(prec));          // launch tables exist before the fingerprint and any capture
    D2D_CHECK(hv.prepare(D2D_FP64));
    uint64_t key = hv.fingerprint();
    for (uint64_t x : {(uint64_t)k, (uint64_t)window, (uint64_t)fused, (uint64_t)plain_cgs2, (uint64_t)basis,
                       (uint64_t)(uintptr_t)s})
        key = fnv_mix(key, x);
    if (!w->exec[g] || w->graph_key[g] != key) {
        if (w->exec[g]) (void)hipGraphExecDestroy(w->exec[g]);
        if (w->graph[g]) (void)hipGraphDestroy(w->graph[g]);
        w->exec[g] = nullptr;
        w->graph[g] = nullptr;
        w->graph_key[g] = 0;
        D2D_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        d2d_status st = inner_loop(w, hv, prec, k, window, fused, plain_cgs2, basis, false, s, nullptr);
        if (st == D2D_OK) st = residual_step(w, hv, s);
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamEndCapture(s, &gr);
        if (st != D2D_OK) {
            if (gr) (void)hipGraphDestroy(gr);
            return st;
        }
        if (e != hipSuccess) {
            set_error("graph capture failed: %s", hipGetErrorString(e));
            return D2D_EDEVICE;
        }
        w->graph[g] = gr;
        D2D_HIP(hipGraphInstantiate(&w->exec[g], gr, nullptr, nullptr, 0));
        w->graph_key[g] = key;
        if (rc) rc->captures++;
    }
    D2D_HIP(hipGraphLaunch(w->exec[g], s));
    hv.count(prec, k - 1);
    hv.count(D2D_FP64, 1);
    return D2D_OK;
}

}  // namespace

namespace d2d {

d2d_status check_lanczos_opts(const d2d_lanczos_opts* o) {
    // the tridiagonal solve and the scalar layout take k <= 128; a projection
    // covers at most 32 basis vectors (full reorthogonalisation: k <= 32)
    const int kb = o ? (o->k_in_bf16 > 0 ? o->k_in_bf16 : o->k_in) : 0;
    if (!o || o->k_in < 2 || o->k_in > 128 || (o->reorth_window == 0 && o->k_in > 32) || o->k_in_bf16 < 0 ||
        kb < 2 || kb > 128 || (o->reorth_window == 0 && kb > 32) || o->max_restarts < 0 ||
        !(o->tol_res > 0.0) || o->prec < 0 || o->prec >= D2D_NPREC || o->reorth_window < 0 ||
        o->reorth_window == 1 || o->reorth_window > 32 || o->separate_central < 0 ||
        o->separate_central > 1 || !(o->tol_rel_e >= 0.0) || o->plain_cgs2 < 0 || o->plain_cgs2 > 1 ||
        o->basis < 0 || o->basis > 2 || o->fixed_cycles < 0 || o->fixed_cycles > 1 || o->one_kernel_step < 0 ||
        o->one_kernel_step > 1) {
        set_error("Lanczos options: k_in and k_in_bf16 (0 or) 2..128 (2..32 with full reorthogonalisation), "
                  "max_restarts >= 0, "
                  "tol_res > 0, prec 0..3, reorth_window 0 or 2..32, "
                  "separate_central 0 or 1, tol_rel_e >= 0, plain_cgs2 0 or 1, basis 0..2, "
                  "fixed_cycles 0 or 1, one_kernel_step 0 or 1");
        return D2D_EINVAL;
    }
    return D2D_OK;
}

d2d_status run_lanczos(d2d_ctx* ctx, LanczosWork*& lw, HvOps& hv, const d2d_lanczos_opts* opts,
                       const std::vector<int64_t>& len, const double* const* v0, double* energies,
                       double* const* psi, d2d_lanczos_stats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = ctx->stream;
    const int np = (int)len.size();
    int64_t nmin = len[0];
    for (int64_t n : len) nmin = std::min(nmin, n);
    // Krylov size per precision (BF16 cycles may be shorter), at most the
    // smallest problem's dimension (an exhausted space needs no more)
    auto k_of = [&](int prec) {
        const int kk = prec == D2D_BF16 && opts->k_in_bf16 > 0 ? opts->k_in_bf16 : opts->k_in;
        return (int)std::min<int64_t>(kk, std::max<int64_t>(nmin, 2));
    };
    const int kmax = std::max(k_of(D2D_BF16), k_of(D2D_FP64));
    D2D_CHECK(ensure_lanczos_work(ctx, lw, len, kmax));
    LanczosWork* w = lw;
    const LzSet z = set_of(w);
    std::vector<int> act(np, 1);
    D2D_CHECK(set_active_flags(w, act));
    {
        // restarts captured by an earlier call are replayed while they hold
        // (see restart); a rebuilt work list invalidates them
        bool rebuilt = false;
        D2D_CHECK(hv.set_active(act, &rebuilt));
        if (rebuilt) drop_graphs(w);
    }
    for (int p = 0; p < np; ++p) {
        if (v0 && v0[p])
            D2D_HIP(hipMemcpyAsync(w->X + w->seg_off[p], v0[p], (size_t)len[p] * 8, hipMemcpyDeviceToDevice, s));
        else
            D2D_HIP(launch_seeded_normal(w->X + w->seg_off[p], len[p], opts->seed + (uint64_t)p, s));
    }
    D2D_HIP(launch_lz_norms(z, w->X, s));
    D2D_HIP(hipMemcpyAsync(w->res_host, w->res, (size_t)2 * np * 8, hipMemcpyDeviceToHost, s));
    D2D_HIP(hipStreamSynchronize(s));
    for (int p = 0; p < np; ++p) {
        const double n0 = w->res_host[2 * p];
        if (!std::isfinite(n0) || !(n0 > 0.0)) {
            set_error("Lanczos: start vector %d is zero or not finite", p);
            return D2D_EINVAL;
        }
    }
    D2D_HIP(launch_lz_normalize_into(z, w->X, w->X, s));
    D2D_CHECK(residual_step(w, hv, s));
    hv.count(D2D_FP64, 1);
    D2D_HIP(hipStreamSynchronize(s));
    std::vector<double> theta(np), rho(np), rho_prev(np, -1.0), theta_prev(np, 0.0), pred(np, 0.0);
    std::vector<int> have_prev(np, 0);
    // residual reduction per inner step of each problem's last cycle (log10; 0: unknown)
    std::vector<double> rate(np, 0.0);
    std::vector<d2d_lanczos_stats> st(np);
    std::memset(st.data(), 0, sizeof(d2d_lanczos_stats) * np);
    // deferred: the problem's restarts need a higher precision; it waits until
    // the problems still converging at this precision are done
    std::vector<int> done(np, 0), restarts(np, 0), deferred(np, 0);
    // Hv applications to each problem by precision (the initial FP64 residual included)
    std::vector<std::array<int64_t, D2D_NPREC>> hvc(np);
    for (int p = 0; p < np; ++p) {
        theta[p] = w->res_host[2 * p];
        rho[p] = w->res_host[2 * p + 1];
        hvc[p].fill(0);
        hvc[p][D2D_FP64] = 1;
    }
    int prec = opts->prec;
    int j = 0;
    d2d_status result = D2D_OK;
    RunCounters rc;
    for (;;) {
        const double tsec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        bool changed = false, any = false;
        for (int p = 0; p < np; ++p) {
            if (done[p] || deferred[p]) continue;
            if (!std::isfinite(theta[p]) || !std::isfinite(rho[p])) {
                set_error("Lanczos: non-finite Rayleigh quotient (problem %d, restart %d)", p, j);
                return D2D_EDEVICE;
            }
            // A restart is short of what it should achieve because of the
            // low-precision products when it both made poor progress and shows
            // their error: the Rayleigh quotient rose (exact arithmetic never
            // lets it), or the true residual is well above the one the Krylov
            // recurrence predicted.  Slow convergence of the Krylov space itself
            // (the estimate matches) keeps the precision.
            const bool shortfall = rho_prev[p] >= 0.0 && opts->escalate > 0.0 && rho[p] > opts->escalate * rho_prev[p] &&
                                   (theta[p] > theta_prev[p] + 1e-13 * std::fabs(theta_prev[p]) || rho[p] > 4.0 * pred[p]);
            d2d_lanczos_stats& sp = st[p];
            if (sp.nlog < D2D_LOG_MAX) {
                sp.log_t[sp.nlog] = tsec;
                sp.log_theta[sp.nlog] = theta[p];
                sp.log_rho[sp.nlog] = rho[p];
                sp.log_pred[sp.nlog] = pred[p];
                sp.log_prec[sp.nlog] = prec;
                sp.nlog++;
            }
            const bool e_stop = opts->tol_rel_e > 0.0 && have_prev[p] &&
                                std::fabs(theta[p] - theta_prev[p]) <= opts->tol_rel_e * std::fabs(theta[p]);
            if (rho[p] <= opts->tol_res * std::fabs(theta[p]) || rho[p] == 0.0 || e_stop) {
                done[p] = 1;
                changed = true;
                sp.seconds = tsec;
                if (psi && psi[p])
                    D2D_HIP(hipMemcpyAsync(psi[p], w->X + w->seg_off[p], (size_t)len[p] * 8,
                                           hipMemcpyDeviceToDevice, s));
            } else if (shortfall && prec != D2D_FP64) {
                deferred[p] = 1;
                changed = true;
            } else {
                any = true;
            }
        }
        if (!any) {
            // nothing left at this precision: the deferred problems go on one
            // step higher (BF16 -> BF16x3 when kept -> FP32 when kept -> FP64)
            bool wait = false;
            for (int p = 0; p < np; ++p) wait = wait || deferred[p];
            if (!wait) break;
            int nxt = D2D_FP64;
            if (prec == D2D_BF16 && hv.has(D2D_BF16X3)) nxt = D2D_BF16X3;
            else if ((prec == D2D_BF16 || prec == D2D_BF16X3) && hv.has(D2D_FP32)) nxt = D2D_FP32;
            prec = nxt;
            for (int p = 0; p < np; ++p) deferred[p] = 0;
            changed = true;
        }
        if (j >= opts->max_restarts) {
            set_error("Lanczos: no convergence after %d restarts", j);
            result = D2D_ENOCONV;
            for (int p = 0; p < np; ++p)
                if (!done[p] && psi && psi[p])
                    D2D_HIP(hipMemcpyAsync(psi[p], w->X + w->seg_off[p], (size_t)len[p] * 8,
                                           hipMemcpyDeviceToDevice, s));
            break;
        }
        std::vector<int> a(np);
        for (int p = 0; p < np; ++p) a[p] = done[p] || deferred[p] ? 0 : 1;
        if (changed) {
            D2D_HIP(hipStreamSynchronize(s));
            D2D_CHECK(set_active_flags(w, a));
            bool rebuilt = false;
            D2D_CHECK(hv.set_active(a, &rebuilt));
            if (rebuilt) drop_graphs(w);
        }
        // Cycle length: k_of(prec), or shorter when every iterating problem's
        // last cycle reduced the residual at a rate that reaches the residual
        // bar in fewer steps (1.25 x the steps plus 4, for the slower start of
        // a cycle); with an energy-change stop the cycles stay full.
        const int kfull = k_of(prec);
        int k = kfull;
        if (!opts->fixed_cycles && opts->tol_rel_e == 0.0) {
            int need = 2;
            for (int p = 0; p < np && need < kfull; ++p) {
                if (!a[p]) continue;
                const double bar = opts->tol_res * std::fabs(theta[p]);
                if (!(rate[p] > 0.0) || !(bar > 0.0)) {
                    need = kfull;
                    break;
                }
                // (capped before the conversion: a tiny rate gives a huge count)
                const double steps = std::log10(rho[p] / bar) / rate[p];
                need = std::max(need, (int)std::min<double>(kfull, std::ceil(1.25 * steps) + 5));
            }
            k = std::min(kfull, need);
        }
        D2D_CHECK(restart(w, hv, prec, k, k == kfull, opts->reorth_window, opts->separate_central == 0,
                          opts->plain_cgs2 != 0, opts->basis, opts->one_kernel_step != 0, opts->use_graph != 0, s,
                          &rc));
        for (int p = 0; p < np; ++p)
            if (a[p]) {
                hvc[p][prec] += k - 1;
                hvc[p][D2D_FP64] += 1;
            }
        D2D_HIP(hipStreamSynchronize(s));
        ++j;
        for (int p = 0; p < np; ++p) {
            if (!a[p]) continue;
            rho_prev[p] = rho[p];
            theta_prev[p] = theta[p];
            have_prev[p] = 1;
            theta[p] = w->res_host[2 * p];
            rho[p] = w->res_host[2 * p + 1];
            pred[p] = w->res_host[2 * np + p];
            restarts[p] += 1;   // the restarts that included the problem
            rate[p] = rho[p] > 0.0 && rho[p] < rho_prev[p] ? std::log10(rho_prev[p] / rho[p]) / (k - 1) : 0.0;
        }
    }
    D2D_HIP(hipStreamSynchronize(s));
    const double total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int p = 0; p < np; ++p) {
        energies[p] = theta[p];
        st[p].restarts = restarts[p];
        st[p].residual = rho[p];
        if (!done[p]) st[p].seconds = total;
        for (int i = 0; i < D2D_NPREC; ++i) st[p].hv_count[i] = hvc[p][i];
        st[p].graph_captures = rc.captures;
        st[p].coop_steps = rc.coop_steps;
        if (stats) stats[p] = st[p];
    }
    if (np == 1 && stats) stats[0].seconds = total;
    return result;
}

}  // namespace d2d

namespace {

// Hv operations of one superblock.
struct SbHv : HvOps {
    d2d_sb* sb;
    explicit SbHv(d2d_sb* b) : sb(b) {}
    d2d_status hv(int prec, const void* v, void* w, hipStream_t s) override {
        return sb_hv_nocount(sb, prec, v, w, s);
    }
    d2d_status hv_fused(int prec, const void* v, void* w, hipStream_t s, HvParts* parts) override {
        if (!sb->fuse[prec]) {
            *parts = HvParts{};
            return sb_hv_nocount(sb, prec, v, w, s);
        }
        return sb_hv_parts(sb, prec, v, w, s, HV_ALL, parts);
    }
    d2d_status prepare(int prec) override {
        const WorkList* wl = nullptr;
        const int shape = sb->tile_sel[prec] >= 0 ? sb->tile_sel[prec] : sb_auto_tile(sb, prec);
        D2D_CHECK(sb_ensure_parts(sb, sb->split[prec], true));
        return sb_work(sb, shape, sb->split[prec], sb->xcd[prec], sb->dense[prec], &wl);
    }
    d2d_status set_active(const std::vector<int>&, bool* rebuilt) override {
        if (rebuilt) *rebuilt = false;
        return D2D_OK;
    }
    bool has(int prec) override { return (sb->prec_mask & (1u << prec)) && sb->HL[prec]; }
    void count(int prec, int64_t n) override { sb->hv_count[prec] += n; }
    int64_t counter(int prec) override { return sb->hv_count[prec]; }
    uint64_t fingerprint() override {
        return config_fingerprint(sb->tile_sel, sb->split, sb->fuse, sb->xcd, sb->dense, sb->persist, sb->d_x, sb->d_w2, 0);
    }
};

}  // namespace

extern "C" d2d_status d2d_lanczos(d2d_sb* sb, const d2d_lanczos_opts* opts, const double* v0, double* energy,
                                  double* psi, d2d_lanczos_stats* stats) {
    if (!sb || !opts || !energy) {
        set_error("d2d_lanczos: NULL argument");
        return D2D_EINVAL;
    }
    D2D_CHECK(check_lanczos_opts(opts));
    if (!(sb->prec_mask & (1u << opts->prec)) || !sb->HL[opts->prec]) {
        set_error("d2d_lanczos: precision %d not kept by this superblock", opts->prec);
        return D2D_EINVAL;
    }
    SbHv hv(sb);
    const std::vector<int64_t> len{sb->N};
    const double* v[1] = {v0};
    double* p[1] = {psi};
    return run_lanczos(sb->ctx, sb->lz, hv, opts, len, v, energy, p, stats);
}
