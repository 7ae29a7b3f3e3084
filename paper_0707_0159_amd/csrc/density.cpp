// Reduced density matrix of one half of the superblock state and the block
// of the next DMRG step: the paper's density-matrix formation (DMF), its
// diagonalisation (DMD), and the renormalisation of the enlarged half's
// operators onto the kept states.
//
//   side 0: rho_L[q_L] = V[q] V[q]^T  over block 1 (x) column 2
//   side 1: rho_R[q_R] = V[q]^T V[q]  over column 3 (x) block 4
//
// DMF: every sector's rho is one problem of a grouped FP64 matrix-core GEMM
// (one launch).  DMD: each sector is diagonalised on the device (rocSOLVER
// dsyevd, FP64).  Its tridiagonal reduction and divide and conquer are long
// chains of small dependent launches, so the sectors are spread over a few
// streams of their own (largest first, each to the least loaded stream by
// d^3), each fed by a host thread of its own, which run concurrently and
// join the context's stream before one host synchronisation; the m_keep eigenvectors of largest weight are kept (ties:
// sector ascending, then index in the sector ascending).  Renormalisation:
// the kept columns are gathered on the device with their sign fixed (entry of
// largest modulus positive), H' = U^T (H U) per sector as two grouped GEMM
// launches, and the new edge column's operators (one nonzero per row in the
// half basis) as a row gather G = O U_from followed by E' = U_to^T G, one
// grouped launch for all of them.  Only the small results (H', E') come back
// to the host, where the block object lives.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <thread>

#include "host.h"

using namespace d2d;

namespace {

// A device buffer charged to the context, freed at scope exit.
template <typename T>
struct DevBuf {
    d2d_ctx* ctx;
    T* p = nullptr;
    size_t n = 0;
    explicit DevBuf(d2d_ctx* c) : ctx(c) {}
    d2d_status alloc(size_t count) {
        n = std::max<size_t>(count, 1);
        return ctx->alloc((void**)&p, n * sizeof(T));
    }
    d2d_status upload(const std::vector<T>& h) {
        D2D_CHECK(alloc(h.size()));
        if (!h.empty()) D2D_HIP(hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
        return D2D_OK;
    }
    ~DevBuf() {
        if (p) ctx->free(p, n * sizeof(T));
    }
};

// Tiles of a list of GEMM problems (64 x 64 output tiles, problem-major).
std::vector<int4> gemm_tiles(const std::vector<GemmProb>& probs) {
    std::vector<int4> t;
    for (size_t i = 0; i < probs.size(); ++i)
        for (int j = 0; j < (probs[i].N + 63) / 64; ++j)
            for (int r = 0; r < (probs[i].M + 63) / 64; ++r) t.push_back(make_int4((int)i, r, j, 0));
    return t;
}

d2d_status grouped_gemm(d2d_ctx* ctx, const std::vector<GemmProb>& probs, hipStream_t s) {
    if (probs.empty()) return D2D_OK;
    const std::vector<int4> tiles = gemm_tiles(probs);
    DevBuf<GemmProb> dp(ctx);
    DevBuf<int4> dt(ctx);
    D2D_CHECK(dp.upload(probs));
    D2D_CHECK(dt.upload(tiles));
    D2D_HIP(launch_gemm_f64(dp.p, dt.p, (int)tiles.size(), s));
    D2D_HIP(hipStreamSynchronize(s));   // the tables are freed at return
    return D2D_OK;
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

// Streams of the density-matrix eigensolver, owned by the context: each with
// its rocBLAS handle, a device workspace of the library's own that the handle
// uses (sized before any work is queued, so that no call allocates while
// others run) and an event that joins it back to the context's stream.
struct EigLanes {
    int n = 0;
    hipStream_t s[EIG_LANES] = {};
    rocblas_handle h[EIG_LANES] = {};
    hipEvent_t done[EIG_LANES] = {};
    hipEvent_t start = nullptr;
    void* ws[EIG_LANES] = {};
    size_t ws_bytes[EIG_LANES] = {};
};

void free_eig_lanes(d2d_ctx* ctx) {
    EigLanes* L = ctx->eig;
    if (!L) return;
    for (int i = 0; i < L->n; ++i) {
        if (L->s[i]) (void)hipStreamSynchronize(L->s[i]);
        if (L->h[i]) rocblas_destroy_handle(L->h[i]);
        if (L->ws[i]) ctx->free(L->ws[i], L->ws_bytes[i]);
        if (L->done[i]) (void)hipEventDestroy(L->done[i]);
        if (L->s[i]) (void)hipStreamDestroy(L->s[i]);
    }
    if (L->start) (void)hipEventDestroy(L->start);
    delete L;
    ctx->eig = nullptr;
}

static d2d_status eig_lanes(d2d_ctx* ctx, EigLanes** out) {
    if (!ctx->eig) {
        EigLanes* L = new EigLanes();
        ctx->eig = L;
        if (hipEventCreateWithFlags(&L->start, hipEventDisableTiming) != hipSuccess) {
            set_error("hipEventCreateWithFlags failed");
            return D2D_EDEVICE;
        }
        for (int i = 0; i < EIG_LANES; ++i) {
            // default priority, like every stream of the library
            if (hipStreamCreateWithFlags(&L->s[i], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&L->done[i], hipEventDisableTiming) != hipSuccess ||
                rocblas_create_handle(&L->h[i]) != rocblas_status_success ||
                rocblas_set_stream(L->h[i], L->s[i]) != rocblas_status_success) {
                L->n = i + 1;
                set_error("density-matrix eigensolver streams: creation failed");
                return D2D_EDEVICE;
            }
            L->n = i + 1;
        }
    }
    *out = ctx->eig;
    return D2D_OK;
}

namespace {

// One half's density matrix between the phases: its sectors' rho (then
// their eigenvectors, in place), eigenvalues and the selection.
struct Half {
    d2d_sb* sb;
    int side, np;
    std::vector<int> dim;
    std::vector<int64_t> roff;
    std::vector<size_t> evoff;
    size_t nev = 0;
    DevBuf<double> rho, ev, offd;
    DevBuf<rocblas_int> info;
    std::vector<double> evh;
    std::vector<std::vector<int>> kept;
    int keep = 0;
    Half(d2d_sb* s, int sd)
        : sb(s), side(sd), np((int)s->pairs.size()), rho(s->ctx), ev(s->ctx), offd(s->ctx), info(s->ctx) {}
};

// DMF: rho of every sector of the half, one grouped GEMM launch.
d2d_status half_rho(Half& h, const double* psi) {
    d2d_sb* sb = h.sb;
    const int np = h.np, side = h.side;
    h.dim.assign(np, 0);
    h.roff.assign(np + 1, 0);
    h.evoff.assign(np, 0);
    h.nev = 0;
    for (int p = 0; p < np; ++p) {
        h.dim[p] = side == 0 ? sb->pairs[p].dL : sb->pairs[p].dR;
        h.roff[p + 1] = h.roff[p] + (int64_t)h.dim[p] * h.dim[p];
        h.evoff[p] = h.nev;
        h.nev += h.dim[p];
    }
    D2D_CHECK(h.rho.alloc((size_t)h.roff[np]));
    std::vector<GemmProb> probs;
    for (int p = 0; p < np; ++p) {
        const SectorDev& q = sb->pairs[p];
        GemmProb g{};
        g.A = psi + q.off;
        g.B = psi + q.off;
        g.C = h.rho.p + h.roff[p];
        g.M = g.N = h.dim[p];
        g.K = side == 0 ? q.dR : q.dL;
        g.lda = g.ldb = q.dL;
        g.ldc = h.dim[p];
        g.ta = side == 0 ? 0 : 1;   // side 0: V V^T; side 1: V^T V
        g.tb = side == 0 ? 1 : 0;
        probs.push_back(g);
    }
    return grouped_gemm(sb->ctx, probs, sb->ctx->stream);
}

// DMD: the eigenpairs of every sector of the given halves (ascending
// eigenvalues, vectors in place of rho), all sectors of all halves spread over
// the context's eigensolver streams together; the eigenvalues come back to
// the host.
d2d_status halves_eig(d2d_ctx* ctx, const std::vector<Half*>& hs) {
    hipStream_t s = ctx->stream;
    EigLanes* lanes = nullptr;
    D2D_CHECK(eig_lanes(ctx, &lanes));
    struct Job {
        Half* h;
        int p, d;
    };
    std::vector<Job> jobs;
    for (Half* h : hs) {
        D2D_CHECK(h->ev.alloc(h->nev));
        D2D_CHECK(h->offd.alloc(h->nev));   // each sector's off-diagonal workspace, at its eigenvalues' offset
        D2D_CHECK(h->info.alloc((size_t)h->np));
        for (int p = 0; p < h->np; ++p) jobs.push_back({h, p, h->dim[p]});
    }
    const int nj = (int)jobs.size();
    // sectors to lanes: largest first, each to the lane with the least d^3 so far
    std::stable_sort(jobs.begin(), jobs.end(), [](const Job& x, const Job& y) { return x.d > y.d; });
    std::vector<int> lane_of(nj, 0);
    double load[EIG_LANES] = {};
    int big[EIG_LANES] = {};
    const int nl = std::min(lanes->n, std::max(nj, 1));
    for (int j = 0; j < nj; ++j) {
        const int l = (int)(std::min_element(load, load + nl) - load);
        lane_of[j] = l;
        load[l] += (double)jobs[j].d * jobs[j].d * jobs[j].d;
        big[l] = std::max(big[l], jobs[j].d);
    }
    auto syevd = [&](int j) {
        Half& h = *jobs[j].h;
        const int p = jobs[j].p;
        return rocsolver_dsyevd(lanes->h[lane_of[j]], rocblas_evect_original, rocblas_fill_lower, h.dim[p],
                                h.rho.p + h.roff[p], h.dim[p], h.ev.p + h.evoff[p], h.offd.p + h.evoff[p],
                                h.info.p + p);
    };
    // each lane's workspace, for the largest sector it gets, before any work is queued
    for (int l = 0; l < nl; ++l) {
        int j0 = -1;
        for (int j = 0; j < nj; ++j)
            if (lane_of[j] == l) {
                j0 = j;
                break;
            }
        if (j0 < 0) continue;
        rocblas_handle h = lanes->h[l];
        if (rocblas_start_device_memory_size_query(h) != rocblas_status_success) {
            set_error("rocblas_start_device_memory_size_query failed");
            return D2D_EDEVICE;
        }
        const rocblas_status q = syevd(j0);
        size_t need = 0;
        if ((q != rocblas_status_size_increased && q != rocblas_status_size_unchanged &&
             q != rocblas_status_success) ||
            rocblas_stop_device_memory_size_query(h, &need) != rocblas_status_success) {
            set_error("rocsolver_dsyevd workspace query failed (dim %d)", big[l]);
            return D2D_EDEVICE;
        }
        if (need > lanes->ws_bytes[l] || !lanes->ws[l]) {
            // the lane is idle here: the previous call ended with a host synchronisation
            if (lanes->ws[l]) ctx->free(lanes->ws[l], lanes->ws_bytes[l]);
            lanes->ws[l] = nullptr;
            lanes->ws_bytes[l] = 0;
            const size_t bytes = std::max<size_t>(need, 256);
            D2D_CHECK(ctx->alloc(&lanes->ws[l], bytes));
            lanes->ws_bytes[l] = bytes;
            if (rocblas_set_workspace(h, lanes->ws[l], bytes) != rocblas_status_success) {
                set_error("rocblas_set_workspace(%zu bytes) failed", bytes);
                return D2D_EDEVICE;
            }
        }
    }
    D2D_HIP(hipEventRecord(lanes->start, s));   // rho is formed
    for (int l = 0; l < nl; ++l) D2D_HIP(hipStreamWaitEvent(lanes->s[l], lanes->start, 0));
    // Every lane's sectors are queued by a host thread of its own.  The
    // eigensolver issues several kernels per matrix column, most of them a few
    // microseconds long, so one thread queuing all sectors in turn keeps the
    // device waiting on the host's launch rate.  (The error message is kept
    // per thread, so the workers only record which sector failed.)
    std::vector<int> failed(nl, -1);
    auto run_lane = [&](int l) {
        if (hipSetDevice(ctx->device) != hipSuccess) {
            failed[l] = nj;
            return;
        }
        for (int j = 0; j < nj; ++j)
            if (lane_of[j] == l && syevd(j) != rocblas_status_success) {
                failed[l] = j;
                return;
            }
    };
    {
        // a lane whose thread cannot be started is queued by this thread
        // (nothing may throw across the C interface)
        std::vector<std::thread> workers;
        std::vector<int> inline_lanes;
        for (int l = 1; l < nl; ++l) {
            try {
                workers.emplace_back(run_lane, l);
            } catch (...) {
                inline_lanes.push_back(l);
            }
        }
        run_lane(0);
        for (int l : inline_lanes) run_lane(l);
        for (auto& w : workers) w.join();
    }
    for (int l = 0; l < nl; ++l)
        if (failed[l] >= 0) {
            if (failed[l] == nj) set_error("hipSetDevice(%d) failed in an eigensolver thread", ctx->device);
            else
                set_error("rocsolver_dsyevd failed on sector %d (dim %d)", jobs[failed[l]].p, jobs[failed[l]].d);
            for (int k = 0; k < nl; ++k) (void)hipStreamSynchronize(lanes->s[k]);
            return D2D_EDEVICE;
        }
    for (int l = 0; l < nl; ++l) {
        D2D_HIP(hipEventRecord(lanes->done[l], lanes->s[l]));
        D2D_HIP(hipStreamWaitEvent(s, lanes->done[l], 0));
    }
    std::vector<std::vector<rocblas_int>> infoh(hs.size());
    for (size_t k = 0; k < hs.size(); ++k) {
        Half& h = *hs[k];
        h.evh.assign(h.nev, 0.0);
        infoh[k].assign(h.np, 0);
        D2D_HIP(hipMemcpyAsync(h.evh.data(), h.ev.p, h.nev * 8, hipMemcpyDeviceToHost, s));
        D2D_HIP(hipMemcpyAsync(infoh[k].data(), h.info.p, sizeof(rocblas_int) * h.np, hipMemcpyDeviceToHost, s));
    }
    D2D_HIP(hipStreamSynchronize(s));
    for (size_t k = 0; k < hs.size(); ++k)
        for (int p = 0; p < hs[k]->np; ++p)
            if (infoh[k][p] != 0) {
                set_error("density-matrix eigensolve of sector %d (dim %d) did not converge (info %d)", p,
                          hs[k]->dim[p], (int)infoh[k][p]);
                return D2D_EDEVICE;
            }
    return D2D_OK;
}

// The kept states of a half: the m_keep eigenvectors of largest weight, ties
// by (sector ascending, index ascending); inside a sector rocSOLVER's order is
// ascending, so index i of the descending list is column dim-1-i.  Pairs are
// in ascending q_L, so on side 1 q_R = Q - q_L descends along them.
void half_select(Half& h, int m_keep, double* trunc_err, double* spectrum, int64_t* spectrum_len) {
    const int np = h.np;
    std::vector<int> rank(np);
    for (int p = 0; p < np; ++p) rank[p] = h.side == 0 ? p : np - 1 - p;
    struct Cand {
        double w;
        int p, i;
    };
    std::vector<Cand> cand;
    cand.reserve(h.nev);
    for (int p = 0; p < np; ++p)
        for (int i = 0; i < h.dim[p]; ++i) cand.push_back({h.evh[h.evoff[p] + h.dim[p] - 1 - i], p, i});
    std::stable_sort(cand.begin(), cand.end(), [&](const Cand& a, const Cand& b) {
        if (a.w != b.w) return a.w > b.w;
        if (a.p != b.p) return rank[a.p] < rank[b.p];
        return a.i < b.i;
    });
    if (spectrum_len) {
        const int64_t cap = *spectrum_len;
        if (spectrum)
            for (int64_t i = 0; i < cap && i < (int64_t)cand.size(); ++i) spectrum[i] = cand[i].w;
        *spectrum_len = (int64_t)cand.size();
    }
    h.keep = (int)std::min<size_t>((size_t)m_keep, cand.size());
    h.kept.assign(np, {});
    double wsum = 0.0;
    for (int k = 0; k < h.keep; ++k) {
        h.kept[cand[k].p].push_back(cand[k].i);
        wsum += cand[k].w;
    }
    *trunc_err = std::max(0.0, 1.0 - wsum);
}

// Renormalisation: the new block of a half from its kept eigenvectors.
d2d_status half_block(Half& h, d2d_block** new_block) {
    d2d_sb* sb = h.sb;
    d2d_ctx* ctx = sb->ctx;
    hipStream_t s = ctx->stream;
    const int side = h.side, np = h.np, keep = h.keep;
    const std::vector<int>& dim = h.dim;
    const std::vector<int64_t>& roff = h.roff;
    DevBuf<double>& rho = h.rho;
    std::vector<std::vector<int>>& kept = h.kept;
    // ---- renormalisation
    // the half's sectors in ascending quantum number: the pairs in order (side
    // 0) or in reverse order (side 1)
    std::vector<int> order(np);
    std::iota(order.begin(), order.end(), 0);
    if (side == 1) std::reverse(order.begin(), order.end());
    std::vector<int> start(np, 0), cnt(np, 0);
    std::vector<int64_t> uoff(np + 1, 0), hoff(np + 1, 0);
    const Column col = make_column(sb->model);
    const int n = sb->n, m = sb->m;
    auto nb = std::make_unique<d2d_block>();
    nb->ctx = ctx;
    nb->model = sb->model;
    nb->side = side;
    nb->m = keep;
    nb->H = Mat(keep, keep);
    nb->keys = col.keys;
    nb->ops.assign(col.keys.size(), Mat(keep, keep));
    int pos = 0;
    std::vector<int4> sel;
    std::vector<int64_t> seloff;
    for (int oi = 0; oi < np; ++oi) {
        const int p = order[oi];
        std::sort(kept[p].begin(), kept[p].end());
        start[p] = pos;
        cnt[p] = (int)kept[p].size();
        pos += cnt[p];
        const QN q = side == 0 ? sb->pair_q[p] : QN{sb->Q[0] - sb->pair_q[p].first, sb->Q[1] - sb->pair_q[p].second};
        for (int c = 0; c < cnt[p]; ++c) nb->qn.push_back(q);
    }
    for (int p = 0; p < np; ++p) {
        uoff[p + 1] = uoff[p] + (int64_t)dim[p] * cnt[p];
        hoff[p + 1] = hoff[p] + (int64_t)cnt[p] * cnt[p];
        for (int c = 0; c < cnt[p]; ++c) {
            sel.push_back(make_int4(dim[p], dim[p] - 1 - kept[p][c], (int)(seloff.size() / 2), 0));
            seloff.push_back(roff[p]);
            seloff.push_back(uoff[p] + (int64_t)c * dim[p]);
        }
    }
    DevBuf<double> U(ctx), T(ctx), Hp(ctx);
    D2D_CHECK(U.alloc((size_t)uoff[np]));
    D2D_CHECK(T.alloc((size_t)uoff[np]));
    D2D_CHECK(Hp.alloc((size_t)hoff[np]));
    {
        DevBuf<int4> dsel(ctx);
        DevBuf<int64_t> doff(ctx);
        D2D_CHECK(dsel.upload(sel));
        D2D_CHECK(doff.upload(seloff));
        D2D_HIP(launch_pick_columns(dsel.p, (int)sel.size(), doff.p, rho.p, U.p, s));
        D2D_HIP(hipStreamSynchronize(s));
    }
    // the block keeps its transformation from the enlarged half (sector by
    // sector, rows in the sector's half indices) and its lineage, for the
    // wavefunction transformation of finite-system sweeps
    {
        std::vector<double> uh((size_t)uoff[np]);
        if (uoff[np] > 0) D2D_HIP(hipMemcpy(uh.data(), U.p, (size_t)uoff[np] * 8, hipMemcpyDeviceToHost));
        const std::vector<int32_t>* hv = side == 0 ? sb->rowsL.data() : sb->colsR.data();
        for (int oi = 0; oi < np; ++oi) {
            const int p = order[oi];
            if (!cnt[p]) continue;
            USector u;
            u.rows = hv[p];
            u.col0 = start[p];
            u.ncols = cnt[p];
            u.v.assign(uh.begin() + uoff[p], uh.begin() + uoff[p + 1]);
            nb->U.push_back(std::move(u));
        }
        nb->id = new_block_id();
        nb->parent = side == 0 ? sb->id1 : sb->id4;
        nb->u_dim = (int64_t)n * m;
    }
    // H' = U^T (H U): H_l as stored (column-major), H_r through its stored transpose
    {
        std::vector<GemmProb> p1, p2;
        for (int p = 0; p < np; ++p) {
            if (!cnt[p]) continue;
            const int d = dim[p];
            GemmProb g{};
            g.A = side == 0 ? (const double*)sb->HL[0] + sb->pairs[p].hl_off
                            : (const double*)sb->HR[0] + sb->pairs[p].hr_off;
            g.B = U.p + uoff[p];
            g.C = T.p + uoff[p];
            g.M = d;
            g.N = cnt[p];
            g.K = d;
            g.lda = g.ldb = g.ldc = d;
            g.ta = side;
            g.tb = 0;
            p1.push_back(g);
            GemmProb g2{};
            g2.A = U.p + uoff[p];
            g2.B = T.p + uoff[p];
            g2.C = Hp.p + hoff[p];
            g2.M = g2.N = cnt[p];
            g2.K = d;
            g2.lda = g2.ldb = d;
            g2.ldc = cnt[p];
            g2.ta = 1;
            g2.tb = 0;
            p2.push_back(g2);
        }
        D2D_CHECK(grouped_gemm(ctx, p1, s));
        D2D_CHECK(grouped_gemm(ctx, p2, s));
    }
    // edge operators: for operator o and target sector pt, G = O U_from (rows
    // of the half basis gathered from the source sector pf with the
    // operator's value, times the block parity for a left Hubbard block),
    // then E'[pt, pf] = U_pt^T G.  The same gathers carry the half
    // Hamiltonian's part that the stored sector operators leave out, the
    // column's off-diagonal terms (pieces of one nonzero per row, even in
    // the fermions: no parity), into H'.
    const std::vector<int32_t>* halves = side == 0 ? sb->rowsL.data() : sb->colsR.data();
    std::vector<int> sector_of_half((size_t)m * n, -1), pos_of_half((size_t)m * n, -1);
    for (int p = 0; p < np; ++p)
        for (size_t i = 0; i < halves[p].size(); ++i) {
            sector_of_half[halves[p][i]] = p;
            pos_of_half[halves[p][i]] = (int)i;
        }
    const std::vector<QN>& bq = side == 0 ? sb->qn1 : sb->qn4;
    struct Entry {
        int o, pt, pf;
    };
    std::vector<Entry> ents;
    std::vector<int4> ent4;
    std::vector<int64_t> eoffs;          // per entry: row map offset, U_from offset, G offset
    std::vector<int32_t> rmap;
    std::vector<double> rval;
    std::vector<int64_t> goff(1, 0), eout(1, 0);
    int64_t maxn = 0;
    const std::vector<Mat> hops = offdiagonal_pieces(col.H);
    const size_t nedge = col.keys.size();
    for (size_t o = 0; o < nedge + hops.size(); ++o) {
        const bool edge = o < nedge;
        const Mat& cop = edge ? col.ops[o] : hops[o - nedge];
        std::vector<int> src(n, -1);
        std::vector<double> val(n, 0.0);
        for (int a = 0; a < n; ++a)
            for (int a2 = 0; a2 < n; ++a2)
                if (cop(a, a2) != 0.0) {
                    src[a] = a2;
                    val[a] = cop(a, a2);
                }
        for (int pt = 0; pt < np; ++pt) {
            if (!cnt[pt]) continue;
            const int dt = dim[pt];
            // the source sectors the rows of pt reach (one, since the operator
            // shifts the quantum numbers by a fixed amount; grouped anyway)
            std::vector<int> rows_pf(dt, -1), rows_pos(dt, -1);
            std::vector<double> rows_v(dt, 0.0);
            std::vector<int> pfs;
            for (int r = 0; r < dt; ++r) {
                const int hrow = halves[pt][r], a = hrow / m, b = hrow % m;
                if (src[a] < 0) continue;
                double v = val[a];
                if (edge && sb->model.kind == D2D_HUBBARD && side == 0)
                    v *= ((bq[b].first + bq[b].second) & 1) ? -1.0 : 1.0;
                const int hsrc = src[a] * m + b;
                const int pf = sector_of_half[hsrc];
                if (pf < 0 || !cnt[pf]) continue;
                rows_pf[r] = pf;
                rows_pos[r] = pos_of_half[hsrc];
                rows_v[r] = v;
                if (std::find(pfs.begin(), pfs.end(), pf) == pfs.end()) pfs.push_back(pf);
            }
            for (int pf : pfs) {
                const int64_t mo = (int64_t)rmap.size();
                for (int r = 0; r < dt; ++r) {
                    rmap.push_back(rows_pf[r] == pf ? rows_pos[r] : -1);
                    rval.push_back(rows_pf[r] == pf ? rows_v[r] : 0.0);
                }
                const int e = (int)ents.size();
                ents.push_back({(int)o, pt, pf});
                ent4.push_back(make_int4(dt, cnt[pf], e, dim[pf]));
                eoffs.push_back(mo);
                eoffs.push_back(uoff[pf]);
                eoffs.push_back(goff.back());
                maxn = std::max<int64_t>(maxn, (int64_t)dt * cnt[pf]);
                goff.push_back(goff.back() + (int64_t)dt * cnt[pf]);
                eout.push_back(eout.back() + (int64_t)cnt[pt] * cnt[pf]);
            }
        }
    }
    DevBuf<double> G(ctx), E(ctx);
    D2D_CHECK(G.alloc((size_t)goff.back()));
    D2D_CHECK(E.alloc((size_t)eout.back()));
    {
        DevBuf<int4> dent(ctx);
        DevBuf<int64_t> doffs(ctx);
        DevBuf<int32_t> dmap(ctx);
        DevBuf<double> dval(ctx);
        D2D_CHECK(dent.upload(ent4));
        D2D_CHECK(doffs.upload(eoffs));
        D2D_CHECK(dmap.upload(rmap));
        D2D_CHECK(dval.upload(rval));
        D2D_HIP(launch_gather_rows(dent.p, (int)ent4.size(), maxn, doffs.p, dmap.p, dval.p, U.p, G.p, s));
        std::vector<GemmProb> pe;
        for (size_t e = 0; e < ents.size(); ++e) {
            const Entry& x = ents[e];
            GemmProb g{};
            g.A = U.p + uoff[x.pt];
            g.B = G.p + goff[e];
            g.C = E.p + eout[e];
            g.M = cnt[x.pt];
            g.N = cnt[x.pf];
            g.K = dim[x.pt];
            g.lda = g.ldb = dim[x.pt];
            g.ldc = cnt[x.pt];
            g.ta = 1;
            g.tb = 0;
            pe.push_back(g);
        }
        D2D_CHECK(grouped_gemm(ctx, pe, s));
    }
    // results to the host block
    std::vector<double> hh((size_t)hoff[np]), eh((size_t)eout.back());
    if (!hh.empty()) D2D_HIP(hipMemcpyAsync(hh.data(), Hp.p, hh.size() * 8, hipMemcpyDeviceToHost, s));
    if (!eh.empty()) D2D_HIP(hipMemcpyAsync(eh.data(), E.p, eh.size() * 8, hipMemcpyDeviceToHost, s));
    D2D_HIP(hipStreamSynchronize(s));
    for (int p = 0; p < np; ++p)
        for (int j = 0; j < cnt[p]; ++j)
            for (int i = 0; i < cnt[p]; ++i) nb->H(start[p] + i, start[p] + j) = hh[hoff[p] + (int64_t)j * cnt[p] + i];
    for (size_t e = 0; e < ents.size(); ++e) {
        const Entry& x = ents[e];
        Mat& M = x.o < (int)nedge ? nb->ops[x.o] : nb->H;   // a column off-diagonal piece adds to H'
        for (int j = 0; j < cnt[x.pf]; ++j)
            for (int i = 0; i < cnt[x.pt]; ++i)
                M(start[x.pt] + i, start[x.pf] + j) += eh[eout[e] + (int64_t)j * cnt[x.pt] + i];
    }
    // sectors of the new block
    for (int i = 0; i < nb->m; ++i) {
        if (i == 0 || nb->qn[i] != nb->qn[i - 1]) {
            nb->sec_qn.push_back(nb->qn[i]);
            nb->sec_dim.push_back(0);
            nb->sec_start.push_back(i);
        }
        nb->sec_dim.back()++;
    }
    nb->ncols = (side == 0 ? sb->ncols1 : sb->ncols4) + 1;
    ctx->children++;
    *new_block = nb.release();
    return D2D_OK;
}

}  // namespace

static d2d_status density_impl(d2d_sb* sb, const double* psi, int side, int m_keep, d2d_block** new_block,
                               double* trunc_err, double* spectrum, int64_t* spectrum_len, double* ms) {
    if (!sb || !psi || !new_block || !trunc_err || (side != 0 && side != 1) || m_keep < 1) {
        set_error("d2d_density_matrix: bad argument");
        return D2D_EINVAL;
    }
    *new_block = nullptr;
    D2D_HIP(hipStreamSynchronize(sb->ctx->stream));   // phases are timed from here
    auto t0 = std::chrono::steady_clock::now();
    Half h(sb, side);
    D2D_CHECK(half_rho(h, psi));
    const double t_dmf = seconds_since(t0);
    auto t1 = std::chrono::steady_clock::now();
    D2D_CHECK(halves_eig(sb->ctx, {&h}));
    half_select(h, m_keep, trunc_err, spectrum, spectrum_len);
    const double t_dmd = seconds_since(t1);
    auto t2 = std::chrono::steady_clock::now();
    D2D_CHECK(half_block(h, new_block));
    if (ms) {
        ms[0] = t_dmf * 1e3;
        ms[1] = t_dmd * 1e3;
        ms[2] = seconds_since(t2) * 1e3;
    }
    return D2D_OK;
}

extern "C" d2d_status d2d_density_matrix_both(d2d_sb* sb, const double* psi, int m_keep, d2d_block** new_left,
                                              d2d_block** new_right, double trunc_err[2], double ms[3]) {
    if (!sb || !psi || !new_left || !new_right || !trunc_err || m_keep < 1) {
        set_error("d2d_density_matrix_both: bad argument");
        return D2D_EINVAL;
    }
    *new_left = *new_right = nullptr;
    D2D_HIP(hipStreamSynchronize(sb->ctx->stream));
    auto t0 = std::chrono::steady_clock::now();
    Half h0(sb, 0), h1(sb, 1);
    D2D_CHECK(half_rho(h0, psi));
    D2D_CHECK(half_rho(h1, psi));
    const double t_dmf = seconds_since(t0);
    auto t1 = std::chrono::steady_clock::now();
    D2D_CHECK(halves_eig(sb->ctx, {&h0, &h1}));
    half_select(h0, m_keep, &trunc_err[0], nullptr, nullptr);
    half_select(h1, m_keep, &trunc_err[1], nullptr, nullptr);
    const double t_dmd = seconds_since(t1);
    auto t2 = std::chrono::steady_clock::now();
    D2D_CHECK(half_block(h0, new_left));
    const d2d_status st = half_block(h1, new_right);
    if (st != D2D_OK) {
        d2d_block_destroy(*new_left);
        *new_left = nullptr;
        return st;
    }
    if (ms) {
        ms[0] = t_dmf * 1e3;
        ms[1] = t_dmd * 1e3;
        ms[2] = seconds_since(t2) * 1e3;
    }
    return D2D_OK;
}

extern "C" d2d_status d2d_density_matrix(d2d_sb* sb, const double* psi, int side, int m_keep, d2d_block** new_block,
                                         double* trunc_err, double* spectrum, int64_t* spectrum_len) {
    return density_impl(sb, psi, side, m_keep, new_block, trunc_err, spectrum, spectrum_len, nullptr);
}

extern "C" d2d_status d2d_density_matrix_timed(d2d_sb* sb, const double* psi, int side, int m_keep,
                                               d2d_block** new_block, double* trunc_err, double* spectrum,
                                               int64_t* spectrum_len, double ms[3]) {
    if (!ms) {
        set_error("d2d_density_matrix_timed: ms is NULL");
        return D2D_EINVAL;
    }
    return density_impl(sb, psi, side, m_keep, new_block, trunc_err, spectrum, spectrum_len, ms);
}

// ---------------------------------------------------------------- wavefunction transformation
namespace {

// Dense column-major rows x cols matrix of a block's transformation (its
// sectors scattered into the enlarged half's full basis).
std::vector<double> dense_u(const std::vector<USector>& U, int64_t rows, int cols) {
    std::vector<double> out((size_t)rows * cols, 0.0);
    for (const USector& u : U) {
        const size_t d = u.rows.size();
        for (int c = 0; c < u.ncols; ++c)
            for (size_t i = 0; i < d; ++i) out[(size_t)u.rows[i] + (size_t)(u.col0 + c) * rows] = u.v[c * d + i];
    }
    return out;
}

}  // namespace

extern "C" d2d_status d2d_wavefunction_transform(d2d_sb* from, const double* psi_from, d2d_sb* to, double* psi_to,
                                                 int direction) {
    if (!from || !psi_from || !to || !psi_to || (direction != 0 && direction != 1)) {
        set_error("d2d_wavefunction_transform: bad argument");
        return D2D_EINVAL;
    }
    if (from->ctx != to->ctx || from->n != to->n || from->model.kind != to->model.kind ||
        from->model.legs != to->model.legs) {
        set_error("d2d_wavefunction_transform: superblocks of different contexts or models");
        return D2D_EINVAL;
    }
    const int n = from->n, m = from->m, m2 = to->m;
    const int64_t D = (int64_t)n * m, D2 = (int64_t)n * m2;
    // direction 0: to's block 1 grew from from's left half, and from's block 4
    // from to's right half; direction 1: the mirror image
    const bool ok = direction == 0
                        ? (to->parent1 == from->id1 && to->u_dim1 == D && from->parent4 == to->id4 && from->u_dim4 == D2)
                        : (to->parent4 == from->id4 && to->u_dim4 == D && from->parent1 == to->id1 && from->u_dim1 == D2);
    if (!ok) {
        set_error("d2d_wavefunction_transform: the superblocks' blocks are not one sweep step apart in direction %d",
                  direction);
        return D2D_EINVAL;
    }
    d2d_ctx* ctx = from->ctx;
    hipStream_t s = ctx->stream;
    // the new block's transformation (D x m2) and the old neighbour's (D2 x m)
    const std::vector<double> Unew = dense_u(direction == 0 ? to->U1 : to->U4, D, m2);
    const std::vector<double> Uold = dense_u(direction == 0 ? from->U4 : from->U1, D2, m);
    DevBuf<double> full(ctx), mid(ctx), out(ctx), un(ctx), uo(ctx);
    D2D_CHECK(full.alloc((size_t)(D * D)));
    D2D_CHECK(mid.alloc((size_t)(m2 * D)));
    D2D_CHECK(out.alloc((size_t)(D2 * D2)));
    D2D_CHECK(un.upload(Unew));
    D2D_CHECK(uo.upload(Uold));
    D2D_CHECK(d2d_unpack(from, psi_from, full.p));
    std::vector<GemmProb> first, second;
    GemmProb g{};
    if (direction == 0) {
        // X = Unew^T Psi (m2 x D): rows the new block's states, columns (i3, i4)
        g.A = un.p;
        g.B = full.p;
        g.C = mid.p;
        g.M = m2;
        g.N = (int)D;
        g.K = (int)D;
        g.lda = (int)D;
        g.ldb = (int)D;
        g.ldc = m2;
        g.ta = 1;
        first.push_back(g);
        // Psi'[(i3, j1), (j3, j4)] = sum_i4 X[j1, (i3, i4)] Uold[(j3, j4), i4], one problem per i3
        for (int i3 = 0; i3 < n; ++i3) {
            GemmProb h{};
            h.A = mid.p + (int64_t)i3 * m * m2;
            h.B = uo.p;
            h.C = out.p + (int64_t)i3 * m2;
            h.M = m2;
            h.N = (int)D2;
            h.K = m;
            h.lda = m2;
            h.ldb = (int)D2;
            h.ldc = (int)D2;
            h.tb = 1;
            second.push_back(h);
        }
    } else {
        // Y = Psi Unew (D x m2): rows (i2, i1), columns the new block's states
        g.A = full.p;
        g.B = un.p;
        g.C = mid.p;
        g.M = (int)D;
        g.N = m2;
        g.K = (int)D;
        g.lda = (int)D;
        g.ldb = (int)D;
        g.ldc = (int)D;
        first.push_back(g);
        // Psi'[(j2, j1), (i2, j4)] = sum_i1 Uold[(j2, j1), i1] Y[(i2, i1), j4], one problem per i2
        for (int i2 = 0; i2 < n; ++i2) {
            GemmProb h{};
            h.A = uo.p;
            h.B = mid.p + (int64_t)i2 * m;
            h.C = out.p + (int64_t)i2 * m2 * D2;
            h.M = (int)D2;
            h.N = m2;
            h.K = m;
            h.lda = (int)D2;
            h.ldb = (int)D;
            h.ldc = (int)D2;
            second.push_back(h);
        }
    }
    D2D_CHECK(grouped_gemm(ctx, first, s));
    D2D_CHECK(grouped_gemm(ctx, second, s));
    D2D_CHECK(d2d_pack(to, out.p, psi_to));
    D2D_HIP(hipStreamSynchronize(s));   // the work buffers are freed at return
    return D2D_OK;
}
