// Reduced density matrix of one half of the superblock state and the block
// of the next DMRG step (the paper's density-matrix formation and
// diagonalisation routines, DMF and DMD).
//
//   side 0: rho_L[q_L] = V[q] V[q]^T  over block 1 (x) column 2
//   side 1: rho_R[q_R] = V[q]^T V[q]  over column 3 (x) block 4
//
// Each sector of rho is formed and diagonalised on the device (rocSOLVER
// dsyevd, FP64).  The m_keep eigenvectors of largest weight are kept (ties:
// sector ascending, then index in the sector ascending); the enlarged half's
// Hamiltonian is projected on the device, H' = U^T H U, and the operators of
// the new edge column (one nonzero per row) by a gather on the host.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <numeric>

#include "host.h"

using namespace d2d;

namespace {

struct DevVec {
    d2d_ctx* ctx;
    double* p = nullptr;
    size_t n = 0;
    explicit DevVec(d2d_ctx* c) : ctx(c) {}
    d2d_status alloc(size_t count) {
        n = count;
        return ctx->alloc((void**)&p, n * 8);
    }
    ~DevVec() {
        if (p) ctx->free(p, n * 8);
    }
};

}  // namespace

extern "C" d2d_status d2d_density_matrix(d2d_sb* sb, const double* psi, int side, int m_keep, d2d_block** new_block,
                                         double* trunc_err, double* spectrum, int64_t* spectrum_len) {
    if (!sb || !psi || !new_block || !trunc_err || (side != 0 && side != 1) || m_keep < 1) {
        set_error("d2d_density_matrix: bad argument");
        return D2D_EINVAL;
    }
    *new_block = nullptr;
    d2d_ctx* ctx = sb->ctx;
    hipStream_t s = ctx->stream;
    const int np = (int)sb->pairs.size();
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) {
        set_error("rocblas_create_handle failed");
        return D2D_EDEVICE;
    }
    struct HGuard {
        rocblas_handle h;
        ~HGuard() { rocblas_destroy_handle(h); }
    } hg{h};
    rocblas_set_stream(h, s);

    // 1. rho per sector and its eigendecomposition (ascending eigenvalues)
    std::vector<int> dim(np);
    std::vector<size_t> roff(np + 1, 0);
    for (int p = 0; p < np; ++p) {
        dim[p] = side == 0 ? sb->pairs[p].dL : sb->pairs[p].dR;
        roff[p + 1] = roff[p] + (size_t)dim[p] * dim[p];
    }
    int dmax = *std::max_element(dim.begin(), dim.end());
    DevVec rho(ctx), ev(ctx), work(ctx);
    D2D_CHECK(rho.alloc(roff[np]));
    size_t nev = 0;
    for (int p = 0; p < np; ++p) nev += dim[p];
    D2D_CHECK(ev.alloc(nev));
    D2D_CHECK(work.alloc((size_t)dmax + 1));
    rocblas_int* info = nullptr;
    D2D_CHECK(ctx->alloc((void**)&info, sizeof(rocblas_int) * 4));
    struct IGuard {
        d2d_ctx* c;
        rocblas_int* p;
        ~IGuard() { c->free(p, sizeof(rocblas_int) * 4); }
    } ig{ctx, info};
    size_t eoff = 0;
    std::vector<size_t> evoff(np);
    for (int p = 0; p < np; ++p) {
        const SectorDev& q = sb->pairs[p];
        D2D_HIP(launch_syrk_f64(psi + q.off, q.dL, q.dR, side, rho.p + roff[p], s));
        evoff[p] = eoff;
        if (rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_lower, dim[p], rho.p + roff[p], dim[p],
                             ev.p + eoff, work.p, info) != rocblas_status_success) {
            set_error("rocsolver_dsyevd failed on sector %d (dim %d)", p, dim[p]);
            return D2D_EDEVICE;
        }
        eoff += dim[p];
    }
    std::vector<double> evh(nev);
    D2D_HIP(hipMemcpyAsync(evh.data(), ev.p, nev * 8, hipMemcpyDeviceToHost, s));
    D2D_HIP(hipStreamSynchronize(s));

    // 2. selection: descending weight, ties by (sector ascending, index ascending);
    //    inside a sector rocSOLVER's order is ascending, so index i of the
    //    descending list is column dim-1-i
    // rank of each pair's half sector in ascending quantum number: pairs are in
    // ascending q_L, so q_R = Q - q_L descends along them
    std::vector<int> rank(np);
    for (int p = 0; p < np; ++p) rank[p] = side == 0 ? p : np - 1 - p;
    struct Cand {
        double w;
        int p, i;
    };
    std::vector<Cand> cand;
    cand.reserve(nev);
    for (int p = 0; p < np; ++p)
        for (int i = 0; i < dim[p]; ++i) cand.push_back({evh[evoff[p] + dim[p] - 1 - i], p, i});
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
    const int keep = (int)std::min<size_t>((size_t)m_keep, cand.size());
    std::vector<std::vector<int>> kept(np);
    double wsum = 0.0;
    for (int k = 0; k < keep; ++k) {
        kept[cand[k].p].push_back(cand[k].i);
        wsum += cand[k].w;
    }
    *trunc_err = std::max(0.0, 1.0 - wsum);
    // the half's sectors in ascending quantum number are the pairs in order (side 0)
    // or in reverse order (side 1: q_R = Q - q_L descends as q_L ascends)
    std::vector<int> order(np);
    std::iota(order.begin(), order.end(), 0);
    if (side == 1) std::reverse(order.begin(), order.end());

    // 3. U columns per kept sector (host copies), H' = U^T H U on the device
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
    std::vector<int> start(np, 0), cnt(np, 0);
    std::vector<std::vector<double>> U(np);     // dim x cnt, column-major
    int pos = 0;
    for (int oi = 0; oi < np; ++oi) {
        const int p = order[oi];
        std::sort(kept[p].begin(), kept[p].end());
        start[p] = pos;
        cnt[p] = (int)kept[p].size();
        if (cnt[p] == 0) continue;
        const int d = dim[p];
        std::vector<double> Z((size_t)d * d);
        D2D_HIP(hipMemcpy(Z.data(), rho.p + roff[p], (size_t)d * d * 8, hipMemcpyDeviceToHost));
        U[p].resize((size_t)d * cnt[p]);
        for (int c = 0; c < cnt[p]; ++c) {
            const int srccol = d - 1 - kept[p][c];
            // sign: largest-modulus component positive
            double best = 0.0;
            int bi = 0;
            for (int r = 0; r < d; ++r)
                if (std::fabs(Z[(size_t)srccol * d + r]) > std::fabs(best)) {
                    best = Z[(size_t)srccol * d + r];
                    bi = r;
                }
            (void)bi;
            const double sg = best < 0.0 ? -1.0 : 1.0;
            for (int r = 0; r < d; ++r) U[p][(size_t)c * d + r] = sg * Z[(size_t)srccol * d + r];
        }
        const QN q = side == 0 ? sb->pair_q[p] : QN{sb->Q[0] - sb->pair_q[p].first, sb->Q[1] - sb->pair_q[p].second};
        for (int c = 0; c < cnt[p]; ++c) nb->qn.push_back(q);
        // H' block on the device: T = H U, H' = U^T T  (H_r is stored transposed; it is symmetric)
        const double* Hd = side == 0 ? (const double*)sb->HL[0] + sb->pairs[p].hl_off
                                     : (const double*)sb->HR[0] + sb->pairs[p].hr_off;
        DevVec Ud(ctx), T(ctx), Hp(ctx);
        D2D_CHECK(Ud.alloc((size_t)d * cnt[p]));
        D2D_CHECK(T.alloc((size_t)d * cnt[p]));
        D2D_CHECK(Hp.alloc((size_t)cnt[p] * cnt[p]));
        D2D_HIP(hipMemcpy(Ud.p, U[p].data(), (size_t)d * cnt[p] * 8, hipMemcpyHostToDevice));
        D2D_HIP(launch_gemm_nn_f64(Hd, d, Ud.p, d, T.p, d, d, cnt[p], d, side == 1 ? 1 : 0, s));
        D2D_HIP(launch_gemm_nn_f64(Ud.p, d, T.p, d, Hp.p, cnt[p], cnt[p], cnt[p], d, 1, s));
        std::vector<double> hp((size_t)cnt[p] * cnt[p]);
        D2D_HIP(hipMemcpyAsync(hp.data(), Hp.p, hp.size() * 8, hipMemcpyDeviceToHost, s));
        D2D_HIP(hipStreamSynchronize(s));
        for (int j = 0; j < cnt[p]; ++j)
            for (int i = 0; i < cnt[p]; ++i) nb->H(pos + i, pos + j) = hp[(size_t)j * cnt[p] + i];
        pos += cnt[p];
    }
    // 4. edge operators of the new block: the new column's site operators in the
    //    half basis (left: c (x) P_block with the block's string; right: c (x) 1),
    //    projected: E'[to, from] = U_to^T O U_from.  O has one nonzero per row.
    const std::vector<int32_t>* halves = side == 0 ? sb->rowsL.data() : sb->colsR.data();
    std::vector<std::vector<int32_t>> posin(np);
    std::vector<int> sector_of_half((size_t)m * n, -1), pos_of_half((size_t)m * n, -1);
    for (int p = 0; p < np; ++p)
        for (size_t i = 0; i < halves[p].size(); ++i) {
            sector_of_half[halves[p][i]] = p;
            pos_of_half[halves[p][i]] = (int)i;
        }
    // parity of the block states of this half (block 1 for side 0)
    const std::vector<QN>& bq = side == 0 ? sb->qn1 : sb->qn4;
    for (size_t o = 0; o < col.keys.size(); ++o) {
        const Mat& cop = col.ops[o];
        // row map of the column operator
        std::vector<int> src(n, -1);
        std::vector<double> val(n, 0.0);
        for (int a = 0; a < n; ++a)
            for (int a2 = 0; a2 < n; ++a2)
                if (cop(a, a2) != 0.0) {
                    src[a] = a2;
                    val[a] = cop(a, a2);
                }
        Mat& E = nb->ops[o];
        for (int pt = 0; pt < np; ++pt) {
            if (!cnt[pt]) continue;
            const int dt = dim[pt];
            // T[row, c] = O[row, :] U_from[:, c] for every source sector
            for (int r = 0; r < dt; ++r) {
                const int hrow = halves[pt][r], a = hrow / m, b = hrow % m;
                if (src[a] < 0) continue;
                double v = val[a];
                if (sb->model.kind == D2D_HUBBARD && side == 0)
                    v *= ((bq[b].first + bq[b].second) & 1) ? -1.0 : 1.0;
                const int hsrc = src[a] * m + b;
                const int pf = sector_of_half[hsrc];
                if (pf < 0 || !cnt[pf]) continue;
                const int rf = pos_of_half[hsrc];
                // E'[start[pt]+i, start[pf]+j] += U_to[r, i] * v * U_from[rf, j]
                for (int i = 0; i < cnt[pt]; ++i) {
                    const double ut = U[pt][(size_t)i * dt + r] * v;
                    if (ut == 0.0) continue;
                    for (int j = 0; j < cnt[pf]; ++j)
                        E(start[pt] + i, start[pf] + j) += ut * U[pf][(size_t)j * dim[pf] + rf];
                }
            }
        }
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
