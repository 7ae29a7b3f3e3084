// Superblock of the direct 2-D DMRG (Eq. (1)): sector enumeration, packed
// layout, device assembly of the dense sector operators, central-term gather
// tables, grouped-GEMM work lists and the Hv entry point.
#include <algorithm>
#include <map>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <numeric>

#include "host.h"

using namespace d2d;

namespace {

template <typename T>
d2d_status upload(d2d_ctx* ctx, const std::vector<T>& h, T** d) {
    *d = nullptr;
    if (h.empty()) return D2D_OK;
    D2D_CHECK(ctx->alloc((void**)d, h.size() * sizeof(T)));
    hipError_t e = hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        ctx->free(*d, h.size() * sizeof(T));
        *d = nullptr;
        set_error("hipMemcpy H2D failed: %s", hipGetErrorString(e));
        return D2D_EDEVICE;
    }
    return D2D_OK;
}

template <typename T>
void release(d2d_ctx* ctx, T*& p, size_t count) {
    if (p) ctx->free((void*)p, count * sizeof(T));
    p = nullptr;
}

// Assemble one half (slow = column state a, fast = block state b) for every
// pair's sector into dense blocks at out (+offsets), optionally transposed.
d2d_status assemble_half(d2d_sb* sb, const d2d_block* blk, const Column& col, const std::vector<BondTerm>& terms,
                         bool left, double* out) {
    d2d_ctx* ctx = sb->ctx;
    const int m = blk->m, n = col.n, T = (int)terms.size();
    const auto& rows = left ? sb->rowsL : sb->colsR;
    const int np = (int)rows.size();
    std::vector<int64_t> rows_off(np + 1, 0), out_off(np);
    std::vector<int32_t> rows_cat;
    int64_t max_d2 = 0;
    for (int p = 0; p < np; ++p) {
        rows_off[p + 1] = rows_off[p] + (int64_t)rows[p].size();
        out_off[p] = left ? sb->pairs[p].hl_off : sb->pairs[p].hr_off;
        rows_cat.insert(rows_cat.end(), rows[p].begin(), rows[p].end());
        max_d2 = std::max<int64_t>(max_d2, (int64_t)rows[p].size() * rows[p].size());
    }
    std::vector<double> S((size_t)T * n * n), F((size_t)T * m * m), coef(T);
    for (int t = 0; t < T; ++t) {
        // left: S_t = column factor B, F_t = block factor A; right: S_t = A (column), F_t = B (block)
        const Mat& sm = left ? terms[t].B : terms[t].A;
        const Mat& fm = left ? terms[t].A : terms[t].B;
        std::copy(sm.a.begin(), sm.a.end(), S.begin() + (size_t)t * n * n);
        std::copy(fm.a.begin(), fm.a.end(), F.begin() + (size_t)t * m * m);
        coef[t] = terms[t].coef;
    }
    int64_t *d_rows_off = nullptr, *d_out_off = nullptr;
    int32_t* d_rows = nullptr;
    double *d_F0 = nullptr, *d_S0 = nullptr, *d_S = nullptr, *d_F = nullptr, *d_coef = nullptr;
    d2d_status st = D2D_OK;
    if ((st = upload(ctx, rows_off, &d_rows_off)) == D2D_OK && (st = upload(ctx, out_off, &d_out_off)) == D2D_OK &&
        (st = upload(ctx, rows_cat, &d_rows)) == D2D_OK && (st = upload(ctx, blk->H.a, &d_F0)) == D2D_OK &&
        (st = upload(ctx, col.H.a, &d_S0)) == D2D_OK && (st = upload(ctx, S, &d_S)) == D2D_OK &&
        (st = upload(ctx, F, &d_F)) == D2D_OK && (st = upload(ctx, coef, &d_coef)) == D2D_OK) {
        AssembleArgs a{np, d_rows_off, d_rows, d_out_off, m, n, T, d_F0, d_S0, d_S, d_F, d_coef, out, max_d2};
        a.transpose = left ? 0 : 1;
        hipError_t e = launch_assemble(a, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) {
            set_error("operator assembly failed: %s", hipGetErrorString(e));
            st = D2D_EDEVICE;
        }
    }
    release(ctx, d_rows_off, rows_off.size());
    release(ctx, d_out_off, out_off.size());
    release(ctx, d_rows, rows_cat.size());
    release(ctx, d_F0, blk->H.a.size());
    release(ctx, d_S0, col.H.a.size());
    release(ctx, d_S, S.size());
    release(ctx, d_F, F.size());
    release(ctx, d_coef, coef.size());
    return st;
}

bool same_model(const d2d_model& a, const d2d_model& b) {
    return a.kind == b.kind && a.legs == b.legs && a.t == b.t && a.U == b.U && a.J == b.J;
}

}  // namespace

d2d_sb::~d2d_sb() {
    free_lanczos(this);
    if (!ctx) return;
    const size_t np = pairs.size();
    release(ctx, d_sec, np);
    const size_t hls[D2D_NPREC] = {(size_t)hl_len * 8, (size_t)hl_len * 4, (size_t)hl16_len * 2,
                                   (size_t)hl16_len * 4};
    const size_t hrs[D2D_NPREC] = {(size_t)hr_len * 8, (size_t)hr_len * 4, (size_t)hr16_len * 2,
                                   (size_t)hr16_len * 4};
    for (int p = 0; p < D2D_NPREC; ++p) {
        if (HL[p]) ctx->free(HL[p], hls[p]);
        if (HR[p]) ctx->free(HR[p], hrs[p]);
        HL[p] = HR[p] = nullptr;
    }
    for (int i = 0; i < 3; ++i) {
        if (d_x[i]) ctx->free(d_x[i], (size_t)N * 8);
        d_x[i] = nullptr;
    }
    if (d_w2) ctx->free(d_w2, (size_t)N * 8);
    d_w2 = nullptr;
    release(ctx, d_vp, (size_t)vp_len * vparts);
    release(ctx, d_vt, (size_t)vt_len * vparts);
    release(ctx, d_ptiles, (size_t)n_ptiles);
    release(ctx, d_cunits, h_cunits.size());
    release(ctx, d_cterms, h_cterms.size());
    release(ctx, d_rowsL, (size_t)Drows);
    release(ctx, d_colsR, (size_t)Dcols);
    for (auto& kv : work) free_work(ctx, kv.second);
    work.clear();
}

namespace d2d {

int sb_auto_tile(const d2d_sb* sb, int prec) {
    const int D = std::max(sb->max_dl, sb->max_dr);
    if (prec == D2D_FP64) return D <= 64 ? 0 : (D <= 768 ? 1 : 2);
    if (prec == D2D_FP32) return D <= 64 ? 3 : (D <= 768 ? 4 : 5);
    if (prec == D2D_BF16) return D <= 64 ? 17 : (D <= 512 ? 14 : 15);
    if (prec == D2D_BF16X3) return D <= 64 ? 30 : (D <= 512 ? 28 : 29);
    return -1;
}

// K-step lists of one pair for a tile shape: for every row tile the steps of
// H_l V, for every column tile the steps of V H_r^T (appended to ks), and the
// flops a step executes per output element of the tile.
struct PairSteps {
    std::vector<int32_t> row_off, row_n, col_off, col_n;
};

static PairSteps pair_steps(const SectorDev& sd, const TileShape& ts, const uint8_t* nzl, const uint8_t* nzr,
                            std::vector<int32_t>& ks) {
    PairSteps ps;
    const bool b16 = ts.prec == D2D_BF16 || ts.prec == D2D_BF16X3;
    const int dL = sd.dL, dR = sd.dR;
    // the K-loops run over the padded lengths of the BF16 operands (zero padding)
    const int KL = b16 ? sd.dLp : dL, KR = b16 ? sd.dRp : dR;
    const int cl = (dL + NZ_CELL - 1) / NZ_CELL, cr = (dR + NZ_CELL - 1) / NZ_CELL;
    // stored operator (column-major d x d): cell (i / NZ_CELL, j / NZ_CELL) at cells[j_cell * c + i_cell]
    auto any = [](const uint8_t* cells, int c, int i0, int i1, int j0, int j1) {
        for (int j = j0; j < j1; ++j)
            for (int i = i0; i < i1; ++i)
                if (cells[(size_t)j * c + i]) return true;
        return false;
    };
    const int tm = (dL + ts.BM - 1) / ts.BM, tn = (dR + ts.BN - 1) / ts.BN;
    for (int i = 0; i < tm; ++i) {
        ps.row_off.push_back((int32_t)ks.size());
        // H_l stored as (row r, column k): rows of the tile x columns of the step
        const int r0 = i * ts.BM / NZ_CELL, r1 = (std::min((i + 1) * ts.BM, dL) + NZ_CELL - 1) / NZ_CELL;
        for (int k0 = 0; k0 < KL; k0 += ts.BK) {
            const int c0 = k0 / NZ_CELL, c1 = std::min((std::min(k0 + ts.BK, dL) + NZ_CELL - 1) / NZ_CELL, cl);
            if (!nzl || (c0 < c1 && any(nzl, cl, r0, r1, c0, c1))) ks.push_back(k0);
        }
        ps.row_n.push_back((int32_t)ks.size() - ps.row_off.back());
    }
    for (int j = 0; j < tn; ++j) {
        ps.col_off.push_back((int32_t)ks.size());
        // H_r^T stored as (row k, column c): rows of the step x columns of the tile
        const int q0 = j * ts.BN / NZ_CELL, q1 = (std::min((j + 1) * ts.BN, dR) + NZ_CELL - 1) / NZ_CELL;
        for (int k0 = 0; k0 < KR; k0 += ts.BK) {
            const int c0 = k0 / NZ_CELL, c1 = std::min((std::min(k0 + ts.BK, dR) + NZ_CELL - 1) / NZ_CELL, cr);
            if (!nzr || (c0 < c1 && any(nzr, cr, c0, c1, q0, q1))) ks.push_back(k0);
        }
        ps.col_n.push_back((int32_t)ks.size() - ps.col_off.back());
    }
    return ps;
}

// flops of the steps ks[off .. off+n) of one K-loop for an output tile of
// rows x cols, clipped to the true (unpadded) K extent d
static double steps_flops(const std::vector<int32_t>& ks, int off, int n, int BK, int d, int rows, int cols) {
    double f = 0;
    for (int q = off; q < off + n; ++q) f += 2.0 * rows * cols * std::max(0, std::min(BK, d - ks[q]));
    return f;
}

// Items of one pair: for every K-loop variant of the split level, the tiles
// i0..i1 x j0..j1 in raster order (rows fastest), with their step counts as
// costs.  Halves of a K-loop cut its step list in two.
static void pair_items(int p, const SectorDev& sd, const TileShape& ts, const PairSteps& ps,
                       const std::vector<int32_t>& ks, int split, int i0, int i1, int j0, int j1,
                       std::vector<std::pair<int, WorkItem>>& w, double& flops) {
    const int nv = split == 2 ? 4 : (split == 1 ? 2 : 1);
    for (int v = 0; v < nv; ++v)
        for (int j = j0; j < j1; ++j)
            for (int i = i0; i < i1; ++i) {
                const int rows = std::min(ts.BM, sd.dL - i * ts.BM), cols = std::min(ts.BN, sd.dR - j * ts.BN);
                const int ro = ps.row_off[i], rn = ps.row_n[i], co = ps.col_off[j], cn = ps.col_n[j];
                WorkItem it{(int32_t)p, i, j, 0, {ro, co}, {0, 0}};
                if (split == 2) {
                    // slots: W (H_l V, 1st half), X0 (2nd half), X1 (V H_r^T, 1st half), X2 (2nd half)
                    const int rh = (rn + 1) / 2, ch = (cn + 1) / 2;
                    const int part[4] = {1 | (0 << 2) | (1 << 4) | (0 << 5), 1 | (1 << 2) | (1 << 4) | (1 << 5),
                                         2 | (2 << 2) | (1 << 4) | (0 << 5), 2 | (3 << 2) | (1 << 4) | (1 << 5)};
                    it.part = part[v];
                    if (v < 2) {
                        it.ks[0] = v == 0 ? ro : ro + rh;
                        it.kn[0] = v == 0 ? rh : rn - rh;
                    } else {
                        it.ks[1] = v == 2 ? co : co + ch;
                        it.kn[1] = v == 2 ? ch : cn - ch;
                    }
                } else if (split == 1) {
                    it.part = v == 0 ? (1 | (0 << 2)) : (2 | (1 << 2));
                    if (v == 0) it.kn[0] = rn;
                    else it.kn[1] = cn;
                } else {
                    it.kn[0] = rn;
                    it.kn[1] = cn;
                }
                flops += steps_flops(ks, it.ks[0], it.kn[0], ts.BK, sd.dL, rows, cols) +
                         steps_flops(ks, it.ks[1], it.kn[1], ts.BK, sd.dR, rows, cols);
                w.push_back({it.kn[0] + it.kn[1], it});
            }
}

void make_work(const std::vector<SectorDev>& pairs, const std::vector<int>* keep, const TileShape& ts, int split,
               int xcd, const NzCells* nz, WorkHost& out, const TileShape* ts1, bool all_steps) {
    out.items.clear();
    out.ksteps.clear();
    out.flops = 0;
    out.n0 = -1;
    if (split == 3) {
        // Asymmetric split: the H_l V items in ts, then the V H_r^T items in
        // ts1; each part longest K-loops first.  With the operators' runs
        // known, an H_l V item covers a segment of at most BM rows inside one
        // run of rows with one column-2 state, and its K steps are those
        // whose BK columns hold a nonzero in exactly those rows (row-exact
        // pattern); a V H_r^T item likewise covers a segment of at most BN
        // columns inside one run of column-3 states.  The rows of a run couple
        // only to the runs of the column states its column Hamiltonian and
        // bond operators reach, so an aligned segment runs only those K steps.
        // each item with its place in its sector's item grid: for H_l V items
        // a = row segment (operator panel), b = column tile (input panel);
        // for V H_r^T items a = column segment, b = row tile
        struct Ent {
            int klen;
            WorkItem it;
            int a, b;
        };
        std::vector<Ent> w0, w1;
        const bool runs = nz && !nz->runsL.empty();
        // steps of BK columns over a K extent KL (padded for BF16) whose
        // 16-column cells are set in any of the rows [r0, r1) of mask (nc cells per row)
        auto seg_steps = [&](const uint8_t* mask, int nc, int r0, int r1, int KL, int BK) {
            const int off = (int)out.ksteps.size();
            for (int k0 = 0; k0 < KL; k0 += BK) {
                bool any = all_steps || !mask;
                const int c0 = k0 / NZ_CELL, c1 = std::min((k0 + BK + NZ_CELL - 1) / NZ_CELL, nc);
                for (int r = r0; r < r1 && !any; ++r)
                    for (int c = c0; c < c1 && !any; ++c) any = mask[(size_t)r * nc + c] != 0;
                if (any) out.ksteps.push_back(k0);
            }
            return std::make_pair(off, (int)out.ksteps.size() - off);
        };
        for (size_t p = 0; p < pairs.size(); ++p) {
            if (keep && !(*keep)[p]) continue;
            const SectorDev& sd = pairs[p];
            const bool b16 = ts.prec == D2D_BF16 || ts.prec == D2D_BF16X3;
            const int KL = b16 ? sd.dLp : sd.dL, KR = b16 ? sd.dRp : sd.dR;
            if (!runs) {
                const uint8_t* nl = nz && !all_steps ? nz->L[p] : nullptr;
                const uint8_t* nr = nz && !all_steps ? nz->R[p] : nullptr;
                const PairSteps p0 = pair_steps(sd, ts, nl, nr, out.ksteps);
                const PairSteps p1 = pair_steps(sd, *ts1, nl, nr, out.ksteps);
                for (int j = 0; j < (sd.dR + ts.BN - 1) / ts.BN; ++j)
                    for (int i = 0; i < (sd.dL + ts.BM - 1) / ts.BM; ++i) {
                        WorkItem it{(int32_t)p, i, j, 1 | (0 << 2), {p0.row_off[i], 0}, {p0.row_n[i], 0}};
                        const int rows = std::min(ts.BM, sd.dL - i * ts.BM), cols = std::min(ts.BN, sd.dR - j * ts.BN);
                        out.flops += steps_flops(out.ksteps, it.ks[0], it.kn[0], ts.BK, sd.dL, rows, cols);
                        w0.push_back({it.kn[0], it, i, j});
                    }
                for (int j = 0; j < (sd.dR + ts1->BN - 1) / ts1->BN; ++j)
                    for (int i = 0; i < (sd.dL + ts1->BM - 1) / ts1->BM; ++i) {
                        WorkItem it{(int32_t)p, i, j, 2 | (1 << 2), {0, p1.col_off[j]}, {0, p1.col_n[j]}};
                        const int rows = std::min(ts1->BM, sd.dL - i * ts1->BM), cols = std::min(ts1->BN, sd.dR - j * ts1->BN);
                        out.flops += steps_flops(out.ksteps, it.ks[1], it.kn[1], ts1->BK, sd.dR, rows, cols);
                        w1.push_back({it.kn[1], it, j, i});
                    }
                continue;
            }
            const int cL = (sd.dL + NZ_CELL - 1) / NZ_CELL, cR = (sd.dR + NZ_CELL - 1) / NZ_CELL;
            const std::vector<int>& rl = *nz->runsL[p];
            int seg = 0;
            for (size_t q = 0; q + 1 < rl.size(); ++q)
                for (int t0 = rl[q]; t0 < rl[q + 1]; t0 += ts.BM, ++seg) {
                    const int t1 = std::min(rl[q + 1], t0 + ts.BM);
                    const auto st = seg_steps(nz->rowL[p], cL, t0, t1, KL, ts.BK);
                    for (int j = 0; j < (sd.dR + ts.BN - 1) / ts.BN; ++j) {
                        WorkItem it{(int32_t)p, t0, j, 1 | (0 << 2) | ITEM_ALIGNED, {st.first, 0}, {st.second, t1 - t0}};
                        const int cols = std::min(ts.BN, sd.dR - j * ts.BN);
                        out.flops += steps_flops(out.ksteps, it.ks[0], it.kn[0], ts.BK, sd.dL, t1 - t0, cols);
                        w0.push_back({it.kn[0], it, seg, j});
                    }
                }
            const std::vector<int>& rr = *nz->runsR[p];
            seg = 0;
            for (size_t q = 0; q + 1 < rr.size(); ++q)
                for (int t0 = rr[q]; t0 < rr[q + 1]; t0 += ts1->BN, ++seg) {
                    const int t1 = std::min(rr[q + 1], t0 + ts1->BN);
                    const auto st = seg_steps(nz->colR[p], cR, t0, t1, KR, ts1->BK);
                    for (int i = 0; i < (sd.dL + ts1->BM - 1) / ts1->BM; ++i) {
                        WorkItem it{(int32_t)p, i, t0, 2 | (1 << 2) | ITEM_ALIGNED, {0, st.first}, {t1 - t0, st.second}};
                        const int rows = std::min(ts1->BM, sd.dL - i * ts1->BM);
                        out.flops += steps_flops(out.ksteps, it.ks[1], it.kn[1], ts1->BK, sd.dR, rows, t1 - t0);
                        w1.push_back({it.kn[1], it, seg, i});
                    }
                }
        }
        if (xcd) {
            // XCD-aware order per launch (work-group b runs on XCD b mod 8):
            // each sector's item grid is cut into 8 rectangles, 2 bands of
            // a (operator segments) x 4 bands of b (input panels) when the
            // grid allows, else 8 runs of its a-major order; XCD x takes
            // rectangle x of every sector, sectors in order of decreasing
            // work, each rectangle a-major so that an XCD's work-groups in
            // flight share their operator segments and input panels in its
            // L2.  Lists are padded with empty items (p = -1) to one length.
            auto order_xcd = [&](std::vector<Ent>& w) {
                constexpr int NX = 8;
                std::vector<std::vector<WorkItem>> bins(NX);
                std::map<int, std::vector<Ent>> by_p;
                for (auto& e : w) by_p[e.it.p].push_back(e);
                std::vector<std::pair<double, int>> ps;
                for (auto& kv : by_p) {
                    double work = 0;
                    for (auto& e : kv.second) work += e.klen;
                    ps.push_back({work, kv.first});
                }
                std::stable_sort(ps.begin(), ps.end(), [](const std::pair<double, int>& x, const std::pair<double, int>& y) {
                    return x.first > y.first;
                });
                for (auto& pw : ps) {
                    std::vector<Ent>& v = by_p[pw.second];
                    int na = 0, nb = 0;
                    for (auto& e : v) {
                        na = std::max(na, e.a + 1);
                        nb = std::max(nb, e.b + 1);
                    }
                    std::stable_sort(v.begin(), v.end(), [](const Ent& x, const Ent& y) {
                        return x.a != y.a ? x.a < y.a : x.b < y.b;
                    });
                    if (na >= 2 && nb >= 4) {
                        for (auto& e : v) bins[(e.a * 2 / na) * 4 + e.b * 4 / nb].push_back(e.it);
                    } else {
                        const size_t n = v.size();
                        for (int x = 0; x < NX; ++x)
                            for (size_t q = x * n / NX; q < (x + 1) * n / NX; ++q) bins[x].push_back(v[q].it);
                    }
                }
                size_t len = 0;
                for (auto& b : bins) len = std::max(len, b.size());
                for (size_t j = 0; j < len; ++j)
                    for (int x = 0; x < NX; ++x)
                        out.items.push_back(j < bins[x].size() ? bins[x][j] : WorkItem{-1, 0, 0, 0, {0, 0}, {0, 0}});
            };
            order_xcd(w0);
            out.n0 = (int)out.items.size();
            order_xcd(w1);
            return;
        }
        auto lpt = [](const Ent& a, const Ent& b) { return a.klen > b.klen; };
        std::stable_sort(w0.begin(), w0.end(), lpt);
        std::stable_sort(w1.begin(), w1.end(), lpt);
        for (auto& x : w0) out.items.push_back(x.it);
        out.n0 = (int)out.items.size();
        for (auto& x : w1) out.items.push_back(x.it);
        return;
    }
    std::vector<PairSteps> ps(pairs.size());
    for (size_t p = 0; p < pairs.size(); ++p) {
        if (keep && !(*keep)[p]) continue;
        ps[p] = pair_steps(pairs[p], ts, nz ? nz->L[p] : nullptr, nz ? nz->R[p] : nullptr, out.ksteps);
    }
    if (xcd) {
        // XCD-aware order.  Work-groups go to the 8 XCDs round-robin by index,
        // and each XCD has its own L2: cut every pair's tile grid into 8
        // rectangles (2 row bands x 4 column bands when the grid allows, else
        // 8 runs of its raster order), give rectangle x to XCD x, and
        // interleave the 8 lists so that item b runs on XCD b mod 8.  An XCD
        // then re-reads the operator panels of its own rows and the input
        // panels of its own columns only.  Pairs go in order of decreasing
        // work; the lists are padded with empty items (p = -1) to one length.
        constexpr int NX = 8;
        std::vector<int> order;
        for (size_t p = 0; p < pairs.size(); ++p)
            if (!keep || (*keep)[p]) order.push_back((int)p);
        auto work_of = [&](int p) {
            const double a = pairs[p].dL, b = pairs[p].dR;
            return a * a * b + a * b * b;
        };
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work_of(a) > work_of(b); });
        std::vector<std::vector<WorkItem>> bins(NX);
        for (int p : order) {
            const SectorDev& sd = pairs[p];
            const int tm = (sd.dL + ts.BM - 1) / ts.BM, tn = (sd.dR + ts.BN - 1) / ts.BN;
            if (tm >= 2 && tn >= 4) {
                for (int x = 0; x < NX; ++x) {
                    const int rb = x / 4, cb = x % 4;
                    std::vector<std::pair<int, WorkItem>> w;
                    pair_items(p, sd, ts, ps[p], out.ksteps, split, rb * tm / 2, (rb + 1) * tm / 2, cb * tn / 4,
                               (cb + 1) * tn / 4, w, out.flops);
                    for (auto& e : w) bins[x].push_back(e.second);
                }
            } else {
                std::vector<std::pair<int, WorkItem>> w;
                pair_items(p, sd, ts, ps[p], out.ksteps, split, 0, tm, 0, tn, w, out.flops);
                const size_t n = w.size();
                for (int x = 0; x < NX; ++x)
                    for (size_t q = x * n / NX; q < (x + 1) * n / NX; ++q) bins[x].push_back(w[q].second);
            }
        }
        size_t len = 0;
        for (auto& b : bins) len = std::max(len, b.size());
        for (size_t j = 0; j < len; ++j)
            for (int x = 0; x < NX; ++x)
                out.items.push_back(j < bins[x].size() ? bins[x][j] : WorkItem{-1, 0, 0, 0, {0, 0}, {0, 0}});
        return;
    }
    std::vector<std::pair<int, WorkItem>> w;
    for (size_t p = 0; p < pairs.size(); ++p) {
        if (keep && !(*keep)[p]) continue;
        const int tm = (pairs[p].dL + ts.BM - 1) / ts.BM, tn = (pairs[p].dR + ts.BN - 1) / ts.BN;
        pair_items((int)p, pairs[p], ts, ps[p], out.ksteps, split, 0, tm, 0, tn, w, out.flops);
    }
    // longest K-loops first
    std::stable_sort(w.begin(), w.end(), [](const std::pair<int, WorkItem>& a, const std::pair<int, WorkItem>& b) {
        return a.first > b.first;
    });
    for (auto& x : w) out.items.push_back(x.second);
}

d2d_status upload_work(d2d_ctx* ctx, const WorkHost& h, WorkList& wl) {
    if (h.items.size() > wl.cap_items) {
        if (wl.items) ctx->free(wl.items, wl.cap_items * sizeof(WorkItem));
        wl.items = nullptr;
        wl.cap_items = 0;
        D2D_CHECK(ctx->alloc((void**)&wl.items, h.items.size() * sizeof(WorkItem)));
        wl.cap_items = h.items.size();
    }
    if (h.ksteps.size() > wl.cap_steps || !wl.ksteps) {
        if (wl.ksteps) ctx->free(wl.ksteps, wl.cap_steps * sizeof(int32_t));
        wl.ksteps = nullptr;
        wl.cap_steps = 0;
        const size_t cap = std::max<size_t>(h.ksteps.size(), 1);
        D2D_CHECK(ctx->alloc((void**)&wl.ksteps, cap * sizeof(int32_t)));
        wl.cap_steps = cap;
    }
    if (!wl.ctr) {
        // counters of persistent launches: each launch leaves them zero
        D2D_CHECK(ctx->alloc((void**)&wl.ctr, 4 * sizeof(int)));
        D2D_HIP(hipMemset(wl.ctr, 0, 4 * sizeof(int)));
    }
    if (!h.items.empty())
        D2D_HIP(hipMemcpy(wl.items, h.items.data(), h.items.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
    if (!h.ksteps.empty())
        D2D_HIP(hipMemcpy(wl.ksteps, h.ksteps.data(), h.ksteps.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    wl.n = (int)h.items.size();
    wl.nsteps = (int)h.ksteps.size();
    wl.flops = h.flops;
    wl.n0 = h.n0;
    return D2D_OK;
}

void free_work(d2d_ctx* ctx, WorkList& wl) {
    if (wl.items) ctx->free(wl.items, wl.cap_items * sizeof(WorkItem));
    if (wl.ksteps) ctx->free(wl.ksteps, wl.cap_steps * sizeof(int32_t));
    if (wl.ctr) ctx->free(wl.ctr, 4 * sizeof(int));
    wl = WorkList{};
}

NzCells sb_nz(const d2d_sb* sb) {
    NzCells nz;
    for (size_t p = 0; p < sb->pairs.size(); ++p) {
        nz.L.push_back(sb->nzL[p].data());
        nz.R.push_back(sb->nzR[p].data());
        nz.rowL.push_back(sb->nzRowL[p].data());
        nz.colR.push_back(sb->nzColR[p].data());
        nz.runsL.push_back(&sb->runsL[p]);
        nz.runsR.push_back(&sb->runsR[p]);
    }
    return nz;
}

d2d_status sb_work(d2d_sb* sb, int shape, int split, int xcd, int dense, const WorkList** out) {
    const int key = shape | (split << 16) | (xcd << 18) | (dense << 19);
    auto it = sb->work.find(key);
    if (it != sb->work.end()) {
        *out = &it->second;
        return D2D_OK;
    }
    WorkHost h;
    const NzCells nz = sb_nz(sb);
    // the asymmetric split places its items on the runs even when it runs every step
    make_work(sb->pairs, nullptr, tile_shape(shape), split, xcd, (dense && split != 3) ? nullptr : &nz, h,
              split == 3 ? &tile_shape(asym_partner(shape)) : nullptr, dense != 0);
    WorkList wl;
    const d2d_status st = upload_work(sb->ctx, h, wl);
    if (st != D2D_OK) {
        free_work(sb->ctx, wl);
        return st;
    }
    sb->work[key] = wl;
    *out = &sb->work[key];
    return D2D_OK;
}

d2d_status hv_launch(const HvTables& t, int prec, int shape, const WorkList& wl, const void* v, void* w,
                     hipStream_t s, int stages) {
    // a split work list (passed together with its partial outputs x) writes
    // shares of the K-loops there; the central term adds them, or, fused,
    // leaves them to the consumer
    HvGemmArgs g{wl.items, wl.n, wl.ksteps, t.sec, t.HL[prec], t.HR[prec], v, w, {t.x[0], t.x[1], t.x[2]}, nullptr};
    if (t.persist) {
        if (!wl.ctr) {
            set_error("persistent launch without the work list's counters");
            return D2D_ESTATE;
        }
        g.ctr = wl.ctr;
    }
    CentralArgs c{};
    c.units = t.cunits;
    c.nunits = t.n_cunits;
    c.terms = t.cterms;
    c.V = v;   // the unpadded input in every precision
    if (t.w2) {
        c.W = t.w2;
        g.fuse = &c;
    } else {
        c.W = w;
        for (int i = 0; i < 3; ++i) c.X[i] = t.x[i];
    }
    if (prec == D2D_BF16 || prec == D2D_BF16X3) {
        if (stages & HV_PACK) {
            if (prec == D2D_BF16)
                D2D_HIP(launch_pack_bf16(t.ptiles, t.n_ptiles, t.sec, (const bf16_t*)v, t.vp, t.vt, s));
            else
                D2D_HIP(launch_pack_bf16x3(t.ptiles, t.n_ptiles, t.sec, (const float*)v, t.vp, t.vt, t.lo[2],
                                           t.lo[3], s));
        }
        g.V = t.vp;
        if (prec == D2D_BF16X3)
            for (int i = 0; i < 4; ++i) g.lo[i] = t.lo[i];
    }
    if (stages & HV_GEMM) {
        const bool b16 = prec == D2D_BF16 || prec == D2D_BF16X3;
        if (wl.n0 >= 0) {
            // asymmetric split: the H_l V items in the lead shape, then the
            // V H_r^T items in its partner (the fused central term rides on the second)
            HvGemmArgs g0 = g, g1 = g;
            g0.nwork = wl.n0;
            g0.fuse = nullptr;
            g1.work = wl.items + wl.n0;
            g1.nwork = wl.n - wl.n0;
            if (g.ctr) g1.ctr = g.ctr + 2;   // the second launch counts on its own pair
            const int shape1 = asym_partner(shape);
            if (b16) {
                D2D_HIP(launch_hv_gemm_bf16(shape, g0, t.vt, s));
                D2D_HIP(launch_hv_gemm_bf16(shape1, g1, t.vt, s));
            } else {
                D2D_HIP(launch_hv_gemm(shape, g0, s));
                D2D_HIP(launch_hv_gemm(shape1, g1, s));
            }
        } else if (b16) {
            D2D_HIP(launch_hv_gemm_bf16(shape, g, t.vt, s));
        } else {
            D2D_HIP(launch_hv_gemm(shape, g, s));
        }
    }
    if (!t.w2 && (stages & HV_CENTRAL)) D2D_HIP(launch_central(prec, c, s));
    return D2D_OK;
}

static HvTables tables_of(d2d_sb* sb) {
    HvTables t{};
    t.sec = sb->d_sec;
    t.npairs = (int)sb->pairs.size();
    for (int p = 0; p < D2D_NPREC; ++p) {
        t.HL[p] = sb->HL[p];
        t.HR[p] = sb->HR[p];
    }
    t.lo[0] = sb->hl16_len;
    t.lo[1] = sb->hr16_len;
    t.lo[2] = sb->vp_len;
    t.lo[3] = sb->vt_len;
    t.cunits = sb->d_cunits;
    t.n_cunits = (int)sb->h_cunits.size();
    t.cterms = sb->d_cterms;
    t.ptiles = sb->d_ptiles;
    t.n_ptiles = sb->n_ptiles;
    t.vp = sb->d_vp;
    t.vt = sb->d_vt;
    return t;
}

d2d_status sb_ensure_parts(d2d_sb* sb, int split, bool central) {
    for (int i = 0; i < split_parts(split); ++i)
        if (!sb->d_x[i]) D2D_CHECK(sb->ctx->alloc(&sb->d_x[i], (size_t)sb->N * 8));
    if (central && !sb->d_w2) D2D_CHECK(sb->ctx->alloc(&sb->d_w2, (size_t)sb->N * 8));
    return D2D_OK;
}

d2d_status sb_hv_parts(d2d_sb* sb, int prec, const void* v, void* w, hipStream_t s, int stages,
                       HvParts* parts) {
    if (prec < 0 || prec >= D2D_NPREC || !(sb->prec_mask & (1u << prec)) || !sb->HL[prec]) {
        set_error("precision %d not available on this superblock", prec);
        return D2D_EINVAL;
    }
    const int shape = sb->tile_sel[prec] >= 0 ? sb->tile_sel[prec] : sb_auto_tile(sb, prec);
    const int split = sb->split[prec];
    const WorkList* wl = nullptr;
    D2D_CHECK(sb_work(sb, shape, split, sb->xcd[prec], sb->dense[prec], &wl));
    HvTables t = tables_of(sb);
    t.persist = sb->persist[prec];
    D2D_CHECK(sb_ensure_parts(sb, split, parts != nullptr));
    for (int i = 0; i < split_parts(split); ++i) t.x[i] = sb->d_x[i];
    if (parts) {
        t.w2 = sb->d_w2;
        for (int i = 0; i < 3; ++i) parts->x[i] = t.x[i];
        parts->central = t.w2;
    }
    return hv_launch(t, prec, shape, *wl, v, w, s, stages);
}

d2d_status sb_hv_nocount(d2d_sb* sb, int prec, const void* v, void* w, hipStream_t s) {
    return sb_hv_parts(sb, prec, v, w, s);
}

d2d_status sb_hv(d2d_sb* sb, int prec, const void* v, void* w, hipStream_t s) {
    D2D_CHECK(sb_hv_parts(sb, prec, v, w, s));
    sb->hv_count[prec]++;
    return D2D_OK;
}

}  // namespace d2d

extern "C" d2d_status d2d_sb_create(d2d_ctx* ctx, const d2d_block* b1, const d2d_block* b4, const d2d_model* model,
                                    const int64_t target_q[2], unsigned prec_mask, d2d_sb** out) {
    if (!ctx || !b1 || !b4 || !model || !target_q || !out) {
        set_error("d2d_sb_create: NULL argument");
        return D2D_EINVAL;
    }
    *out = nullptr;
    if (!same_model(b1->model, *model) || !same_model(b4->model, *model)) {
        set_error("d2d_sb_create: blocks were built for a different model");
        return D2D_EINVAL;
    }
    if (b1->side != 0 || b4->side != 1) {
        set_error("d2d_sb_create: block 1 must be a left block and block 4 a right block");
        return D2D_EINVAL;
    }
    if (b1->m != b4->m) {
        set_error("d2d_sb_create: blocks 1 and 4 must have the same number of states (%d vs %d)", b1->m, b4->m);
        return D2D_EINVAL;
    }
    if (prec_mask & ~15u) {
        set_error("d2d_sb_create: unknown precision bits 0x%x", prec_mask);
        return D2D_EINVAL;
    }
    prec_mask |= 1u << D2D_FP64;   // the FP64 operators are always kept (residuals, restarts)
    D2D_HIP(hipSetDevice(ctx->device));
    const Column col = make_column(*model);
    const int m = b1->m, n = col.n;
    const int64_t mn = (int64_t)m * n;
    if (mn > (1ll << 30)) {
        set_error("half dimension m*n = %lld too large", (long long)mn);
        return D2D_EINVAL;
    }
    auto sb = std::make_unique<d2d_sb>();
    sb->ctx = ctx;
    sb->model = *model;
    sb->m = m;
    sb->n = n;
    sb->Q[0] = target_q[0];
    sb->Q[1] = target_q[1];
    sb->prec_mask = prec_mask;
    sb->qn1 = b1->qn;
    sb->qn4 = b4->qn;
    sb->ncols1 = b1->ncols;
    sb->ncols4 = b4->ncols;
    sb->id1 = b1->id;
    sb->parent1 = b1->parent;
    sb->u_dim1 = b1->u_dim;
    sb->U1 = b1->U;
    sb->id4 = b4->id;
    sb->parent4 = b4->parent;
    sb->u_dim4 = b4->u_dim;
    sb->U4 = b4->U;
    ctx->children++;   // undone by the destructor path below on failure
    struct Guard {
        std::unique_ptr<d2d_sb>* p;
        d2d_ctx* c;
        ~Guard() {
            if (*p) c->children--;
        }
    } guard{&sb, ctx};

    // a1: sectors of the two enlarged halves, half index = column state * m + block state
    std::map<QN, std::vector<int32_t>> left, right;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < m; ++b) {
            left[{col.qn[a].first + b1->qn[b].first, col.qn[a].second + b1->qn[b].second}].push_back(a * m + b);
            right[{col.qn[a].first + b4->qn[b].first, col.qn[a].second + b4->qn[b].second}].push_back(a * m + b);
        }
    std::map<QN, int> pair_of;
    int64_t off = 0, hl = 0, hr = 0, rb = 0, cb = 0;
    for (auto& kv : left) {
        const QN qr{target_q[0] - kv.first.first, target_q[1] - kv.first.second};
        auto it = right.find(qr);
        if (it == right.end()) continue;
        SectorDev s{};
        s.dL = (int32_t)kv.second.size();
        s.dR = (int32_t)it->second.size();
        s.off = off;
        s.hl_off = hl;
        s.hr_off = hr;
        s.row_base = rb;
        s.col_base = cb;
        s.dLp = (s.dL + 7) / 8 * 8;
        s.dRp = (s.dR + 7) / 8 * 8;
        s.hl16_off = sb->hl16_len;
        s.hr16_off = sb->hr16_len;
        s.vp_off = sb->vp_len;
        s.vt_off = sb->vt_len;
        sb->hl16_len += (int64_t)s.dLp * s.dL;
        sb->hr16_len += (int64_t)s.dRp * s.dR;
        sb->vp_len += (int64_t)s.dLp * s.dR;
        sb->vt_len += (int64_t)s.dRp * s.dL;
        off += (int64_t)s.dL * s.dR;
        hl += (int64_t)s.dL * s.dL;
        hr += (int64_t)s.dR * s.dR;
        rb += s.dL;
        cb += s.dR;
        pair_of[kv.first] = (int)sb->pairs.size();
        sb->pairs.push_back(s);
        sb->pair_q.push_back(kv.first);
        sb->rowsL.push_back(kv.second);
        sb->colsR.push_back(it->second);
        sb->max_dl = std::max(sb->max_dl, (int)s.dL);
        sb->max_dr = std::max(sb->max_dr, (int)s.dR);
        sb->max_elems = std::max<int64_t>(sb->max_elems, (int64_t)s.dL * s.dR);
        sb->flops_exec += 2.0 * s.dL * (double)s.dL * s.dR + 2.0 * s.dL * (double)s.dR * s.dR;
    }
    if (sb->pairs.empty()) {
        set_error("d2d_sb_create: the target sector (%lld,%lld) is empty", (long long)target_q[0],
                  (long long)target_q[1]);
        return D2D_EINVAL;
    }
    sb->N = off;
    sb->hl_len = hl;
    sb->hr_len = hr;
    sb->Drows = rb;
    sb->Dcols = cb;
    D2D_CHECK(upload(ctx, sb->pairs, &sb->d_sec));

    // a2: dense sector operators, FP64 master copies
    D2D_CHECK(ctx->alloc(&sb->HL[D2D_FP64], (size_t)hl * 8));
    D2D_CHECK(ctx->alloc(&sb->HR[D2D_FP64], (size_t)hr * 8));
    const std::vector<BondTerm> tl = bond_terms(*model, b1->keys, b1->ops, b1->parity(), col.keys, col.ops);
    const std::vector<BondTerm> tr = bond_terms(*model, col.keys, col.ops, col.parity, b4->keys, b4->ops);
    // the dense sector operators carry the column Hamiltonian's diagonal
    // only; its off-diagonal part joins the central term (a5 below)
    Column cdiag = col;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (i != j) cdiag.H(i, j) = 0.0;
    D2D_CHECK(assemble_half(sb.get(), b1, cdiag, tl, true, (double*)sb->HL[D2D_FP64]));
    D2D_CHECK(assemble_half(sb.get(), b4, cdiag, tr, false, (double*)sb->HR[D2D_FP64]));
    // nonzero count of the sector operators (the method's sparse flop count)
    {
        std::vector<double> h(hl), r(hr);
        D2D_HIP(hipMemcpy(h.data(), sb->HL[D2D_FP64], hl * 8, hipMemcpyDeviceToHost));
        D2D_HIP(hipMemcpy(r.data(), sb->HR[D2D_FP64], hr * 8, hipMemcpyDeviceToHost));
        // and the zero pattern in cells, for the K steps the grouped GEMM can leave out
        auto cells = [](const double* a, int d, std::vector<uint8_t>& out, int64_t& nnz) {
            const int c = (d + NZ_CELL - 1) / NZ_CELL;
            out.assign((size_t)c * c, 0);
            for (int j = 0; j < d; ++j)
                for (int i = 0; i < d; ++i)
                    if (a[i + (int64_t)j * d] != 0.0) {
                        out[(size_t)(j / NZ_CELL) * c + i / NZ_CELL] = 1;
                        ++nnz;
                    }
        };
        // row-exact patterns: per row of H_l (per column of the stored H_r^T)
        // the 16-wide cells of the other index that hold a nonzero
        auto lines = [](const double* a, int d, bool by_row, std::vector<uint8_t>& out) {
            const int c = (d + NZ_CELL - 1) / NZ_CELL;
            out.assign((size_t)d * c, 0);
            for (int j = 0; j < d; ++j)
                for (int i = 0; i < d; ++i)
                    if (a[i + (int64_t)j * d] != 0.0) {
                        if (by_row) out[(size_t)i * c + j / NZ_CELL] = 1;
                        else out[(size_t)j * c + i / NZ_CELL] = 1;
                    }
        };
        // starts of the runs of one column state (half index / m) along a sector
        auto run_starts = [m](const std::vector<int32_t>& idx, std::vector<int>& out) {
            out.clear();
            for (size_t i = 0; i < idx.size(); ++i)
                if (i == 0 || idx[i] / m != idx[i - 1] / m) out.push_back((int)i);
            out.push_back((int)idx.size());
        };
        const size_t npp = sb->pairs.size();
        sb->nzL.resize(npp);
        sb->nzR.resize(npp);
        sb->nzRowL.resize(npp);
        sb->nzColR.resize(npp);
        sb->runsL.resize(npp);
        sb->runsR.resize(npp);
        for (size_t p = 0; p < npp; ++p) {
            const SectorDev& s = sb->pairs[p];
            int64_t nl = 0, nr = 0;
            cells(h.data() + s.hl_off, s.dL, sb->nzL[p], nl);
            cells(r.data() + s.hr_off, s.dR, sb->nzR[p], nr);
            lines(h.data() + s.hl_off, s.dL, true, sb->nzRowL[p]);
            lines(r.data() + s.hr_off, s.dR, false, sb->nzColR[p]);
            run_starts(sb->rowsL[p], sb->runsL[p]);
            run_starts(sb->colsR[p], sb->runsR[p]);
            sb->flops_nnz += 2.0 * nl * s.dR + 2.0 * nr * s.dL;
        }
    }
    if (prec_mask & (1u << D2D_FP32)) {
        D2D_CHECK(ctx->alloc(&sb->HL[D2D_FP32], (size_t)hl * 4));
        D2D_CHECK(ctx->alloc(&sb->HR[D2D_FP32], (size_t)hr * 4));
        D2D_HIP(launch_cast_f64_f32((const double*)sb->HL[0], (float*)sb->HL[1], hl, ctx->stream));
        D2D_HIP(launch_cast_f64_f32((const double*)sb->HR[0], (float*)sb->HR[1], hr, ctx->stream));
    }
    const bool want16 = (prec_mask & (1u << D2D_BF16)) != 0, want3 = (prec_mask & (1u << D2D_BF16X3)) != 0;
    if (want16 || want3) {
        // BF16 operators: one copy (BF16) and / or hi and lo copies (BF16x3,
        // lo at hl16_len / hr16_len elements after hi); the padded input
        // copies VP / VT hold the lo parts after the hi parts when BF16x3 is kept
        const size_t h16 = (size_t)sb->hl16_len * 2, r16 = (size_t)sb->hr16_len * 2;
        sb->vparts = want3 ? 2 : 1;
        for (int kind : {D2D_BF16, D2D_BF16X3}) {
            if (!(prec_mask & (1u << kind))) continue;
            const size_t np = kind == D2D_BF16X3 ? 2 : 1;
            D2D_CHECK(ctx->alloc(&sb->HL[kind], h16 * np));
            D2D_CHECK(ctx->alloc(&sb->HR[kind], r16 * np));
            // padding of every K-major operand is zero and stays zero
            D2D_HIP(hipMemset(sb->HL[kind], 0, h16 * np));
            D2D_HIP(hipMemset(sb->HR[kind], 0, r16 * np));
        }
        D2D_CHECK(ctx->alloc((void**)&sb->d_vp, (size_t)sb->vp_len * 2 * sb->vparts));
        D2D_CHECK(ctx->alloc((void**)&sb->d_vt, (size_t)sb->vt_len * 2 * sb->vparts));
        D2D_HIP(hipMemset(sb->d_vp, 0, (size_t)sb->vp_len * 2 * sb->vparts));
        D2D_HIP(hipMemset(sb->d_vt, 0, (size_t)sb->vt_len * 2 * sb->vparts));
        const int npp = (int)sb->pairs.size();
        std::vector<int64_t> so_l(npp), so_r(npp), do_l(npp), do_r(npp);
        std::vector<int32_t> dl(npp), dlp(npp), dr(npp), drp(npp);
        int64_t mx = 0;
        for (int p = 0; p < npp; ++p) {
            const SectorDev& q = sb->pairs[p];
            so_l[p] = q.hl_off; so_r[p] = q.hr_off; do_l[p] = q.hl16_off; do_r[p] = q.hr16_off;
            dl[p] = q.dL; dlp[p] = q.dLp; dr[p] = q.dR; drp[p] = q.dRp;
            mx = std::max<int64_t>(mx, std::max<int64_t>((int64_t)q.dL * q.dL, (int64_t)q.dR * q.dR));
        }
        int64_t *a1 = nullptr, *a2 = nullptr, *a3 = nullptr, *a4 = nullptr;
        int32_t *b1 = nullptr, *b2 = nullptr, *b3 = nullptr, *b4 = nullptr;
        d2d_status st = D2D_OK;
        if ((st = upload(ctx, so_l, &a1)) == D2D_OK && (st = upload(ctx, so_r, &a2)) == D2D_OK &&
            (st = upload(ctx, do_l, &a3)) == D2D_OK && (st = upload(ctx, do_r, &a4)) == D2D_OK &&
            (st = upload(ctx, dl, &b1)) == D2D_OK && (st = upload(ctx, dlp, &b2)) == D2D_OK &&
            (st = upload(ctx, dr, &b3)) == D2D_OK && (st = upload(ctx, drp, &b4)) == D2D_OK) {
            hipError_t e = hipSuccess;
            for (int kind : {D2D_BF16, D2D_BF16X3}) {
                if (!(prec_mask & (1u << kind))) continue;
                for (int part = 0; part < (kind == D2D_BF16X3 ? 2 : 1) && e == hipSuccess; ++part) {
                    e = launch_op_bf16(a1, a3, b1, b2, npp, 1, part, (const double*)sb->HL[0],
                                       (bf16_t*)sb->HL[kind] + part * sb->hl16_len, mx, ctx->stream);
                    if (e == hipSuccess)
                        e = launch_op_bf16(a2, a4, b3, b4, npp, 0, part, (const double*)sb->HR[0],
                                           (bf16_t*)sb->HR[kind] + part * sb->hr16_len, mx, ctx->stream);
                }
            }
            if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
            if (e != hipSuccess) {
                set_error("BF16 operator conversion failed: %s", hipGetErrorString(e));
                st = D2D_EDEVICE;
            }
        }
        release(ctx, a1, so_l.size()); release(ctx, a2, so_r.size());
        release(ctx, a3, do_l.size()); release(ctx, a4, do_r.size());
        release(ctx, b1, dl.size()); release(ctx, b2, dlp.size());
        release(ctx, b3, dr.size()); release(ctx, b4, drp.size());
        D2D_CHECK(st);
        std::vector<int4> pt;
        for (int p = 0; p < npp; ++p) {
            const int tr = (sb->pairs[p].dL + 63) / 64, tc = (sb->pairs[p].dR + 63) / 64;
            for (int j = 0; j < tc; ++j)
                for (int i = 0; i < tr; ++i) pt.push_back(make_int4(p, i, j, 0));
        }
        sb->n_ptiles = (int)pt.size();
        D2D_CHECK(upload(ctx, pt, &sb->d_ptiles));
    }

    // a5: central bond terms sum_k c_k A_k (x) B_k, A_k on column 2, B_k on column 3,
    // then the columns' own off-diagonal terms: piece (x) 1 for column 2
    // (part of H_l) and 1 (x) piece for column 3 (part of H_r)
    std::vector<BondTerm> tc = bond_terms(*model, col.keys, col.ops, col.parity, col.keys, col.ops);
    sb->K = (int)tc.size();
    {
        const Mat id = mat_identity(n);
        for (const Mat& pc : offdiagonal_pieces(col.H)) {
            tc.push_back({1.0, pc, id});
            tc.push_back({1.0, id, pc});
        }
    }
    const int K = (int)tc.size(), np = (int)sb->pairs.size();
    // position of every half index inside its sector
    std::vector<int32_t> posL(mn, -1), posR(mn, -1);
    for (auto& kv : left)
        for (size_t i = 0; i < kv.second.size(); ++i) posL[kv.second[i]] = (int32_t)i;
    for (auto& kv : right)
        for (size_t i = 0; i < kv.second.size(); ++i) posR[kv.second[i]] = (int32_t)i;
    // the nonzero of every row of A_k and B_k, and the change of quantum numbers
    struct TermMap {
        std::vector<int> ra, rb;
        std::vector<double> av, bv;
        QN dA{0, 0};
        bool live = false;
    };
    std::vector<TermMap> tmap(K);
    for (int k = 0; k < K; ++k) {
        const Mat& A = tc[k].A;
        const Mat& B = tc[k].B;
        TermMap& t = tmap[k];
        t.ra.assign(n, -1);
        t.rb.assign(n, -1);
        t.av.assign(n, 0.0);
        t.bv.assign(n, 0.0);
        QN dB{0, 0};
        bool seenA = false, seenB = false;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                if (A(i, j) != 0.0) {
                    if (t.ra[i] >= 0) {
                        set_error("central operator with two nonzeros in a row");
                        return D2D_EINVAL;
                    }
                    t.ra[i] = j;
                    t.av[i] = A(i, j);
                    t.dA = {col.qn[i].first - col.qn[j].first, col.qn[i].second - col.qn[j].second};
                    seenA = true;
                }
                if (B(i, j) != 0.0) {
                    if (t.rb[i] >= 0) {
                        set_error("central operator with two nonzeros in a row");
                        return D2D_EINVAL;
                    }
                    t.rb[i] = j;
                    t.bv[i] = B(i, j);
                    dB = {col.qn[i].first - col.qn[j].first, col.qn[i].second - col.qn[j].second};
                    seenB = true;
                }
            }
        if (!seenA || !seenB) continue;
        if (t.dA.first + dB.first != 0 || t.dA.second + dB.second != 0) {
            set_error("central term does not conserve the quantum numbers");
            return D2D_EINVAL;
        }
        t.live = true;
    }
    // Rectangles: within a pair block, a run of rows with one column-2 state
    // i2 times a run of columns with one column-3 state i3.  Term k maps the
    // rectangle onto the rectangle of (A_k's column for i2, B_k's column for
    // i3) in the pair shifted by its change of quantum numbers, with the same
    // block-1 and block-4 states in the same order, times one coefficient.
    struct Run {
        int start, len, col, first;   // first packed index, length, column state, block state of the first
    };
    auto runs_of = [&](const std::vector<int32_t>& idx) {
        std::vector<Run> out;
        for (int i = 0; i < (int)idx.size(); ++i) {
            const int a = idx[i] / m;
            if (out.empty() || out.back().col != a) out.push_back({i, 0, a, idx[i] % m});
            out.back().len++;
        }
        return out;
    };
    std::vector<CentralUnit>& units = sb->h_cunits;
    std::vector<CentralTerm>& terms = sb->h_cterms;
    int64_t gathers = 0;
    for (int p = 0; p < np; ++p) {
        const SectorDev& s = sb->pairs[p];
        const std::vector<Run> rr = runs_of(sb->rowsL[p]), cr = runs_of(sb->colsR[p]);
        for (const Run& R : rr)
            for (const Run& C : cr) {
                std::vector<CentralTerm> list;
                double self = 0.0;
                for (int k = 0; k < K; ++k) {
                    const TermMap& t = tmap[k];
                    if (!t.live || t.ra[R.col] < 0 || t.rb[C.col] < 0) continue;
                    auto it = pair_of.find(QN{sb->pair_q[p].first - t.dA.first, sb->pair_q[p].second - t.dA.second});
                    if (it == pair_of.end()) continue;
                    const int p2 = it->second;
                    const double coef = tc[k].coef * t.av[R.col] * t.bv[C.col];
                    if (coef == 0.0) continue;
                    const int sr = posL[(int64_t)t.ra[R.col] * m + R.first];
                    const int sc = posR[(int64_t)t.rb[C.col] * m + C.first];
                    // the run maps onto consecutive rows / columns of the source block
                    for (int i = 0; i < R.len; ++i)
                        if (posL[(int64_t)t.ra[R.col] * m + sb->rowsL[p][R.start + i] % m] != sr + i) {
                            set_error("central term: a row run does not map onto consecutive rows");
                            return D2D_EINVAL;
                        }
                    for (int i = 0; i < C.len; ++i)
                        if (posR[(int64_t)t.rb[C.col] * m + sb->colsR[p][C.start + i] % m] != sc + i) {
                            set_error("central term: a column run does not map onto consecutive columns");
                            return D2D_EINVAL;
                        }
                    gathers += (int64_t)R.len * C.len;
                    const SectorDev& s2 = sb->pairs[p2];
                    if (p2 == p && sr == R.start && sc == C.start) {
                        self += coef;   // terms mapping the rectangle onto itself act as one
                        continue;
                    }
                    CentralTerm e{};
                    e.base = s2.off + sr + (int64_t)sc * s2.dL;
                    e.ld = s2.dL;
                    e.c64 = coef;
                    e.c32 = (float)coef;
                    list.push_back(e);
                }
                if (self != 0.0) {
                    CentralTerm e{};
                    e.base = s.off + R.start + (int64_t)C.start * s.dL;
                    e.ld = s.dL;
                    e.c64 = self;
                    e.c32 = (float)self;
                    list.insert(list.begin(), e);
                }
                const int tofs = (int)terms.size(), nt = (int)list.size();
                terms.insert(terms.end(), list.begin(), list.end());
                // work units of one wave: up to 64 rows x CENTRAL_CS * (64 / rows) columns
                for (int ru = 0; ru < R.len; ru += 64) {
                    const int nr = std::min(64, R.len - ru);
                    const int span = CENTRAL_CS * (64 / nr);
                    for (int cu = 0; cu < C.len; cu += span) {
                        CentralUnit u{};
                        u.off = s.off + R.start + (int64_t)C.start * s.dL;
                        u.ldw = s.dL;
                        u.ru = ru;
                        u.nr = nr;
                        u.cu = cu;
                        u.nc = std::min(span, C.len - cu);
                        u.tofs = tofs;
                        u.nt = nt;
                        u.p = p;
                        units.push_back(u);
                    }
                }
            }
    }
    sb->flops_central = 2.0 * (double)gathers;
    // every index a unit's wave forms (W and each term's source, at the
    // unit's first and last row and column) inside the packed vector
    for (const CentralUnit& u : units) {
        const int64_t lo = u.ru + (int64_t)u.cu * u.ldw, hi = u.ru + u.nr - 1 + (int64_t)(u.cu + u.nc - 1) * u.ldw;
        bool ok = u.nr >= 1 && u.nr <= 64 && u.nc >= 1 && u.nc <= CENTRAL_CS * (64 / u.nr) && u.off + lo >= 0 &&
                  u.off + hi < sb->N && u.tofs >= 0 && u.tofs + u.nt <= (int)terms.size();
        for (int t = 0; ok && t < u.nt; ++t) {
            const CentralTerm& e = terms[u.tofs + t];
            ok = e.base + u.ru + (int64_t)u.cu * e.ld >= 0 &&
                 e.base + u.ru + u.nr - 1 + (int64_t)(u.cu + u.nc - 1) * e.ld < sb->N;
        }
        if (!ok) {
            set_error("central term: a work unit reaches outside the vector");
            return D2D_EINVAL;
        }
    }
    D2D_CHECK(upload(ctx, units, &sb->d_cunits));
    D2D_CHECK(upload(ctx, terms, &sb->d_cterms));
    {
        // half indices of the packed rows and columns (full-space conversion)
        std::vector<int32_t> hr, hc;
        for (size_t p = 0; p < sb->pairs.size(); ++p) {
            hr.insert(hr.end(), sb->rowsL[p].begin(), sb->rowsL[p].end());
            hc.insert(hc.end(), sb->colsR[p].begin(), sb->colsR[p].end());
        }
        D2D_CHECK(upload(ctx, hr, &sb->d_rowsL));
        D2D_CHECK(upload(ctx, hc, &sb->d_colsR));
    }
    // work lists of the default launch configuration of every kept precision
    for (int p = 0; p < D2D_NPREC; ++p) {
        if (!(prec_mask & (1u << p)) || !sb->HL[p]) continue;
        const WorkList* wl = nullptr;
        D2D_CHECK(sb_work(sb.get(), sb_auto_tile(sb.get(), p), 0, 0, 0, &wl));
    }
    D2D_HIP(hipStreamSynchronize(ctx->stream));
    *out = sb.release();
    return D2D_OK;
}

extern "C" d2d_status d2d_sb_destroy(d2d_sb* sb) {
    if (!sb) return D2D_OK;
    d2d_ctx* c = sb->ctx;
    if (c) (void)hipStreamSynchronize(c->stream);
    delete sb;
    if (c) c->children--;
    return D2D_OK;
}

extern "C" d2d_status d2d_sb_info(const d2d_sb* sb, d2d_sb_info_t* info) {
    if (!sb || !info) {
        set_error("d2d_sb_info: NULL argument");
        return D2D_EINVAL;
    }
    std::memset(info, 0, sizeof(*info));
    info->n = sb->N;
    info->npairs = (int32_t)sb->pairs.size();
    info->m = sb->m;
    info->ncol = sb->n;
    info->nterms = sb->K;
    info->max_dl = sb->max_dl;
    info->max_dr = sb->max_dr;
    info->flops_exec = sb->flops_exec;
    info->flops_nnz = sb->flops_nnz + sb->flops_central;
    info->flops_central = sb->flops_central;
    const double ops = (double)(sb->hl_len + sb->hr_len);
    info->op_entries = sb->hl_len + sb->hr_len;
    const double N = (double)sb->N;
    info->bytes_min_fp64 = 3.0 * N * 8 + ops * 8;
    info->bytes_min_fp32 = 3.0 * N * 4 + ops * 4;
    info->bytes_min_bf16 = 2.0 * N * 2 + N * 4 + ops * 2;
    info->bytes_min_bf16x3 = 2.0 * N * 4 + N * 4 + ops * 4;
    return D2D_OK;
}

extern "C" d2d_status d2d_sb_sectors(const d2d_sb* sb, int64_t* qL, int64_t* dL, int64_t* dR, int64_t* offset) {
    if (!sb || !qL || !dL || !dR || !offset) {
        set_error("d2d_sb_sectors: NULL argument");
        return D2D_EINVAL;
    }
    for (size_t p = 0; p < sb->pairs.size(); ++p) {
        qL[2 * p] = sb->pair_q[p].first;
        qL[2 * p + 1] = sb->pair_q[p].second;
        dL[p] = sb->pairs[p].dL;
        dR[p] = sb->pairs[p].dR;
        offset[p] = sb->pairs[p].off;
    }
    return D2D_OK;
}

static d2d_status full_pack(d2d_sb* sb, int dir, const double* src, double* dst, const char* who) {
    if (!sb || !src || !dst) {
        set_error("%s: NULL argument", who);
        return D2D_EINVAL;
    }
    const int64_t D = (int64_t)sb->m * sb->n;
    hipStream_t s = sb->ctx->stream;
    if (dir == 1) D2D_HIP(launch_fill(dst, D2D_FP64, D * D, 0.0, s));
    D2D_HIP(launch_full_pack(sb->d_sec, (int)sb->pairs.size(), sb->max_elems, sb->d_rowsL, sb->d_colsR, D, dir, src,
                             dst, s));
    return D2D_OK;
}

extern "C" d2d_status d2d_pack(d2d_sb* sb, const double* full, double* packed) {
    return full_pack(sb, 0, full, packed, "d2d_pack");
}

extern "C" d2d_status d2d_unpack(d2d_sb* sb, const double* packed, double* full) {
    return full_pack(sb, 1, packed, full, "d2d_unpack");
}

extern "C" d2d_status d2d_hv(d2d_sb* sb, int prec, const void* v, void* w) {
    if (!sb || !v || !w) {
        set_error("d2d_hv: NULL argument");
        return D2D_EINVAL;
    }
    if (v == w) {
        set_error("d2d_hv: v and w must not overlap");
        return D2D_EINVAL;
    }
    return sb_hv(sb, prec, v, w, sb->ctx->stream);
}

// ------------------------------------------------------------------ Hv without allocation
// Partial outputs of split K-loops for d2d_hv_noalloc: a file-scope device
// array, one copy per GPU, held until the process ends.  In host code its
// name stands for a host-side shadow, not a device address: the address on a
// device comes from hipGetSymbolAddress with that device current, and only
// that address is ever passed to a kernel.
static __device__ __align__(256) unsigned char scratch[D2D_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on `device` (looked up once per device)
d2d_status scratch_on(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("d2d_hv_noalloc: device %d out of range", device);
        return D2D_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int prev = 0;
        D2D_HIP(hipGetDevice(&prev));
        D2D_HIP(hipSetDevice(device));
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        (void)hipSetDevice(prev);
        if (e != hipSuccess || !ptr) {
            set_error("d2d_hv_noalloc: hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            return D2D_EDEVICE;
        }
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return D2D_OK;
}
}  // namespace

extern "C" d2d_status d2d_hv_noalloc(d2d_sb* sb, int prec, const void* v, void* w) {
    if (!sb || !v || !w) {
        set_error("d2d_hv_noalloc: NULL argument");
        return D2D_EINVAL;
    }
    if (v == w) {
        set_error("d2d_hv_noalloc: v and w must not overlap");
        return D2D_EINVAL;
    }
    if (prec < 0 || prec >= D2D_NPREC || !(sb->prec_mask & (1u << prec)) || !sb->HL[prec]) {
        set_error("d2d_hv_noalloc: precision %d not available on this superblock", prec);
        return D2D_EINVAL;
    }
    const int shape = sb->tile_sel[prec] >= 0 ? sb->tile_sel[prec] : sb_auto_tile(sb, prec);
    const int split = sb->split[prec];
    const int key = shape | (split << 16) | (sb->xcd[prec] << 18) | (sb->dense[prec] << 19);
    auto it = sb->work.find(key);
    if (it == sb->work.end()) {
        set_error("d2d_hv_noalloc: the work list of the launch configuration of precision %d is not built "
                  "(d2d_sb_create, d2d_sb_set_tile and d2d_sb_autotune build it)", prec);
        return D2D_ESTATE;
    }
    // the partial outputs, in the product's output type, one after the other
    const int nparts = split_parts(split);
    const size_t elem = prec == D2D_FP64 ? 8 : 4;
    const size_t need = (size_t)nparts * (size_t)sb->N * elem;
    if (need > (size_t)D2D_NOALLOC_SCRATCH_BYTES) {
        set_error("d2d_hv_noalloc: %d partial outputs of %lld elements need %zu bytes, more than the %u bytes "
                  "of scratch", nparts, (long long)sb->N, need, (unsigned)D2D_NOALLOC_SCRATCH_BYTES);
        return D2D_EINVAL;
    }
    HvTables t = tables_of(sb);
    t.persist = sb->persist[prec];
    if (nparts > 0) {
        void* base = nullptr;
        D2D_CHECK(scratch_on(sb->ctx->device, &base));
        // every split work item stores every element of its tile into its
        // slot, so the parts need no clearing
        for (int i = 0; i < nparts; ++i) t.x[i] = (char*)base + (size_t)i * sb->N * elem;
    }
    D2D_CHECK(hv_launch(t, prec, shape, it->second, v, w, sb->ctx->stream));
    sb->hv_count[prec]++;
    return D2D_OK;
}

extern "C" d2d_status d2d_hv_count(const d2d_sb* sb, int64_t counts[D2D_NPREC]) {
    if (!sb || !counts) {
        set_error("d2d_hv_count: NULL argument");
        return D2D_EINVAL;
    }
    for (int i = 0; i < D2D_NPREC; ++i) counts[i] = sb->hv_count[i];
    return D2D_OK;
}

namespace d2d {

bool decode_tile(int prec, int tile, TileSel* out) {
    TileSel t;
    t.split = tile < 0 ? 0
                       : ((tile & D2D_TILE_ASYM) ? 3 : ((tile & D2D_TILE_SPLIT4) ? 2 : ((tile & D2D_TILE_SPLIT) ? 1 : 0)));
    t.fuse = tile >= 0 ? ((tile & D2D_TILE_FUSED) ? 1 : 0) : (prec != D2D_FP64 ? 1 : 0);
    t.xcd = tile >= 0 && (tile & D2D_TILE_XCD) ? 1 : 0;
    t.dense = tile >= 0 && (tile & D2D_TILE_DENSE) ? 1 : 0;
    t.persist = tile >= 0 && (tile & D2D_TILE_PERSIST) ? 1 : 0;
    t.shape = tile < 0 ? -1 : (tile & 0xFFFF);
    if (t.shape >= tile_shape_count() || (t.shape >= 0 && tile_shape(t.shape).prec != prec) ||
        (tile >= 0 && (tile & ~(0xFFFF | D2D_TILE_SPLIT | D2D_TILE_SPLIT4 | D2D_TILE_FUSED | D2D_TILE_XCD |
                                D2D_TILE_DENSE | D2D_TILE_ASYM | D2D_TILE_PERSIST))) ||
        (tile >= 0 && (tile & D2D_TILE_SPLIT) && (tile & D2D_TILE_SPLIT4)) ||
        // a persistent launch takes items in list order, which an XCD order cannot steer
        (t.persist && t.xcd) ||
        // the asymmetric split: a shape with a partner, no other split
        (t.split == 3 && (asym_partner(t.shape) < 0 || (tile & (D2D_TILE_SPLIT | D2D_TILE_SPLIT4)))))
        return false;
    *out = t;
    return true;
}

int encode_tile(const TileSel& t) {
    return t.shape | (t.split == 1 ? D2D_TILE_SPLIT : 0) | (t.split == 2 ? D2D_TILE_SPLIT4 : 0) |
           (t.split == 3 ? D2D_TILE_ASYM : 0) |
           (t.fuse ? D2D_TILE_FUSED : 0) | (t.xcd ? D2D_TILE_XCD : 0) | (t.dense ? D2D_TILE_DENSE : 0) |
           (t.persist ? D2D_TILE_PERSIST : 0);
}

}  // namespace d2d

extern "C" d2d_status d2d_sb_set_tile(d2d_sb* sb, int prec, int tile) {
    if (!sb || prec < 0 || prec >= D2D_NPREC) {
        set_error("d2d_sb_set_tile: bad argument");
        return D2D_EINVAL;
    }
    TileSel t;
    if (!decode_tile(prec, tile, &t)) {
        set_error("d2d_sb_set_tile: tile %d is not a shape of precision %d", tile, prec);
        return D2D_EINVAL;
    }
    sb->tile_sel[prec] = t.shape;
    sb->split[prec] = t.split;
    sb->fuse[prec] = t.fuse;
    sb->xcd[prec] = t.xcd;
    sb->dense[prec] = t.dense;
    sb->persist[prec] = t.persist;
    // the work list of the configuration is built here, so that products in
    // it (d2d_hv_noalloc among them) need no allocation
    if ((sb->prec_mask & (1u << prec)) && sb->HL[prec]) {
        const WorkList* wl = nullptr;
        D2D_CHECK(sb_work(sb, t.shape >= 0 ? t.shape : sb_auto_tile(sb, prec), t.split, t.xcd, t.dense, &wl));
    }
    return D2D_OK;
}

extern "C" d2d_status d2d_sb_gemm_flops(d2d_sb* sb, int prec, double* flops) {
    if (!sb || !flops || prec < 0 || prec >= D2D_NPREC) {
        set_error("d2d_sb_gemm_flops: bad argument");
        return D2D_EINVAL;
    }
    if (!(sb->prec_mask & (1u << prec)) || !sb->HL[prec]) {
        set_error("d2d_sb_gemm_flops: precision %d not kept by this superblock", prec);
        return D2D_EINVAL;
    }
    const int shape = sb->tile_sel[prec] >= 0 ? sb->tile_sel[prec] : sb_auto_tile(sb, prec);
    const WorkList* wl = nullptr;
    D2D_CHECK(sb_work(sb, shape, sb->split[prec], sb->xcd[prec], sb->dense[prec], &wl));
    *flops = wl->flops;
    return D2D_OK;
}

extern "C" d2d_status d2d_tile_shapes(int* count, int* desc) {
    if (!count) {
        set_error("d2d_tile_shapes: NULL count");
        return D2D_EINVAL;
    }
    *count = tile_shape_count();
    if (desc)
        for (int i = 0; i < *count; ++i) {
            const TileShape& t = tile_shape(i);
            desc[5 * i] = t.prec;
            desc[5 * i + 1] = t.BM;
            desc[5 * i + 2] = t.BN;
            desc[5 * i + 3] = t.BK;
            desc[5 * i + 4] = t.PF;
        }
    return D2D_OK;
}

extern "C" d2d_status d2d_hv_profile(d2d_sb* sb, int prec, const void* v, void* w, int reps, double* ms_gemm,
                                     double* ms_central) {
    if (!sb || !v || !w || !ms_gemm || !ms_central || reps < 1 || reps > 100000) {
        set_error("d2d_hv_profile: bad argument");
        return D2D_EINVAL;
    }
    hipStream_t s = sb->ctx->stream;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    d2d_status st = D2D_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            set_error("hipEventCreate failed");
            st = D2D_EDEVICE;
            break;
        }
    // one whole product (work list, BF16 copies of v), the GEMM launches back
    // to back, the central-term launches back to back, and a last whole
    // product so that w = H v on return
    if (st == D2D_OK) st = sb_hv(sb, prec, v, w, s);
    if (st == D2D_OK && hipEventRecord(ev[0], s) != hipSuccess) st = D2D_EDEVICE;
    for (int r = 0; r < reps && st == D2D_OK; ++r) st = sb_hv_parts(sb, prec, v, w, s, HV_GEMM);
    if (st == D2D_OK && hipEventRecord(ev[1], s) != hipSuccess) st = D2D_EDEVICE;
    for (int r = 0; r < reps && st == D2D_OK; ++r) st = sb_hv_parts(sb, prec, v, w, s, HV_CENTRAL);
    if (st == D2D_OK && hipEventRecord(ev[2], s) != hipSuccess) st = D2D_EDEVICE;
    if (st == D2D_OK) st = sb_hv(sb, prec, v, w, s);
    float a = 0.f, c = 0.f;
    if (st == D2D_OK && (hipStreamSynchronize(s) != hipSuccess || hipEventElapsedTime(&a, ev[0], ev[1]) != hipSuccess ||
                         hipEventElapsedTime(&c, ev[1], ev[2]) != hipSuccess)) {
        set_error("d2d_hv_profile: HIP event timing failed");
        st = D2D_EDEVICE;
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (st != D2D_OK) return st;
    *ms_gemm = a / reps;
    *ms_central = c / reps;
    return D2D_OK;
}

// ------------------------------------------------------------------ autotuner
static uint64_t sector_key(const d2d_sb* sb, int prec) {
    uint64_t h = 1469598103934665603ull ^ (uint64_t)prec;
    auto mix = [&](uint64_t v) {
        h ^= v;
        h *= 1099511628211ull;
    };
    mix(sb->pairs.size());
    for (const auto& p : sb->pairs) {
        mix((uint64_t)p.dL);
        mix((uint64_t)p.dR);
    }
    return h;
}

namespace d2d {

bool tune_cache_lookup(uint64_t key, int prec, TileSel* sel, int* tile, double* ms) {
    const char* cache = getenv("D2D_TUNE_CACHE");
    if (!cache || !*cache) return false;
    FILE* f = fopen(cache, "r");
    if (!f) return false;
    unsigned long long k;
    int t;
    double m;
    bool found = false;
    while (!found && fscanf(f, "%llx %d %lf", &k, &t, &m) == 3)
        if (k == key && t >= 0 && decode_tile(prec, t, sel)) {
            *tile = t;
            *ms = m;
            found = true;
        }
    fclose(f);
    return found;
}

void tune_cache_store(uint64_t key, int tile, double ms) {
    const char* cache = getenv("D2D_TUNE_CACHE");
    if (!cache || !*cache) return;
    FILE* f = fopen(cache, "a");
    if (!f) return;
    fprintf(f, "%llx %d %.6f\n", (unsigned long long)key, tile, ms);
    fclose(f);
}

d2d_status tune_configs(hipStream_t s, int prec, int reps, const std::function<d2d_status(const TileSel&)>& run,
                        TileSel* best, double* best_ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    d2d_status st = D2D_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        set_error("autotune: HIP event creation failed");
        st = D2D_EDEVICE;
    }
    bool any = false;
    double bms = 1e300;
    const int nsh = tile_shape_count();
    for (int tt = 0; tt < 32 * nsh && st == D2D_OK; ++tt) {
        TileSel c;
        c.shape = tt % nsh;
        c.split = (tt / nsh) % 4;
        c.fuse = (tt / (4 * nsh)) % 2;
        c.xcd = (tt / (8 * nsh)) % 2;
        c.persist = tt / (16 * nsh);
        if (tile_shape(c.shape).prec != prec) continue;
        if (c.split == 3 && asym_partner(c.shape) < 0) continue;
        if (c.persist && c.xcd) continue;
        st = run(c);   // warm-up (also builds the work list)
        if (st != D2D_OK) break;
        if (hipEventRecord(e0, s) != hipSuccess) st = D2D_EDEVICE;
        for (int r = 0; r < reps && st == D2D_OK; ++r) st = run(c);
        float ms = 0.f;
        if (st == D2D_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = D2D_EDEVICE;
        if (st == D2D_OK && ms / reps < bms) {
            bms = ms / reps;
            *best = c;
            any = true;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st == D2D_OK && !any) {
        set_error("autotune: no tile shape for precision %d", prec);
        st = D2D_EINVAL;
    }
    if (st == D2D_OK) *best_ms = bms;
    return st;
}

}  // namespace d2d

extern "C" d2d_status d2d_sb_autotune(d2d_sb* sb, int prec, int reps, int* best_tile, double* best_ms) {
    if (!sb || !best_tile || !best_ms || prec < 0 || prec >= D2D_NPREC || reps < 1 || reps > 10000) {
        set_error("d2d_sb_autotune: bad argument");
        return D2D_EINVAL;
    }
    if (!(sb->prec_mask & (1u << prec)) || !sb->HL[prec]) {
        set_error("d2d_sb_autotune: precision %d not kept by this superblock", prec);
        return D2D_EINVAL;
    }
    auto apply = [&](const TileSel& c) {
        sb->tile_sel[prec] = c.shape;
        sb->split[prec] = c.split;
        sb->fuse[prec] = c.fuse;
        sb->xcd[prec] = c.xcd;
        sb->dense[prec] = c.dense;
        sb->persist[prec] = c.persist;
    };
    const uint64_t key = sector_key(sb, prec);
    TileSel sel;
    if (tune_cache_lookup(key, prec, &sel, best_tile, best_ms)) {
        apply(sel);
        return D2D_OK;
    }
    d2d_ctx* ctx = sb->ctx;
    hipStream_t s = ctx->stream;
    const size_t in_sz = prec == D2D_FP64 ? 8 : (prec == D2D_BF16 ? 2 : 4);
    const size_t out_sz = prec == D2D_FP64 ? 8 : 4;
    void *v = nullptr, *w = nullptr;
    D2D_CHECK(ctx->alloc(&v, (size_t)sb->N * in_sz));
    d2d_status st = ctx->alloc(&w, (size_t)sb->N * out_sz);
    if (st != D2D_OK) {
        ctx->free(v, (size_t)sb->N * in_sz);
        return st;
    }
    const TileSel saved{sb->tile_sel[prec], sb->split[prec], sb->fuse[prec], sb->xcd[prec], sb->dense[prec],
                        sb->persist[prec]};
    if (launch_fill(v, prec, sb->N, 0.5, s) != hipSuccess) {
        set_error("d2d_sb_autotune: HIP setup failed");
        st = D2D_EDEVICE;
    }
    double bms = 0;
    if (st == D2D_OK)
        st = tune_configs(s, prec, reps, [&](const TileSel& c) {
            apply(c);
            HvParts parts{};
            D2D_CHECK(sb_hv_parts(sb, prec, v, w, s, HV_ALL, c.fuse ? &parts : nullptr));
            if (!c.fuse) return D2D_OK;
            // a fused product leaves its parts to the consumer: charge reading them
            const void* pp[4] = {parts.x[0], parts.x[1], parts.x[2], parts.central};
            D2D_HIP(launch_read_parts(pp, prec, sb->N, w, s));
            return D2D_OK;
        }, &sel, &bms);
    ctx->free(v, (size_t)sb->N * in_sz);
    ctx->free(w, (size_t)sb->N * out_sz);
    if (st != D2D_OK) {
        apply(saved);
        return st;
    }
    apply(sel);
    *best_tile = encode_tile(sel);
    *best_ms = bms;
    tune_cache_store(key, *best_tile, bms);
    return D2D_OK;
}
