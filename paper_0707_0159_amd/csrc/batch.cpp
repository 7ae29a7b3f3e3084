// Batches of independent superblocks of uneven size.  The sector tables,
// operators and central-term tables of all problems are concatenated, so one
// grouped-GEMM launch (work list sorted longest-first across problems) and one
// central-term launch cover every sector of every problem; the Lanczos vector
// kernels are segmented per problem.  Converged problems leave the work lists
// at the next restart.
#include <algorithm>
#include <cstring>

#include "host.h"

using namespace d2d;

struct d2d_batch {
    d2d_ctx* ctx = nullptr;
    std::vector<d2d_sb*> sbs;
    unsigned prec_mask = 0;
    std::vector<SectorDev> pairs;       // rebased
    std::vector<int> pair_prob;
    std::vector<int64_t> voff, len;
    int64_t ntot = 0;
    int max_dl = 0, max_dr = 0;
    SectorDev* d_sec = nullptr;
    void* HL[D2D_NPREC] = {nullptr, nullptr, nullptr, nullptr};
    void* HR[D2D_NPREC] = {nullptr, nullptr, nullptr, nullptr};
    size_t hl_bytes[D2D_NPREC] = {0, 0, 0, 0}, hr_bytes[D2D_NPREC] = {0, 0, 0, 0};
    int64_t h16_len = 0, r16_len = 0;   // BF16 operator lengths (the BF16x3 lo parts follow the hi parts)
    int vparts = 1;
    // central term: every problem's units and terms, rebased; the launch table
    // holds the units of the active problems
    std::vector<CentralUnit> cunits;
    std::vector<CentralTerm> cterms;
    CentralTerm* d_cterms = nullptr;
    CentralUnit* d_cunits = nullptr;
    int n_cunits = 0, cap_cunits = 0;
    int4* d_ptiles = nullptr;
    int n_ptiles = 0, cap_ptiles = 0;
    bf16_t *d_vp = nullptr, *d_vt = nullptr;
    int64_t vp_len = 0, vt_len = 0;
    // work_key(shape, split, xcd, dense) -> work list of the active problems
    std::map<int, WorkList> work;
    NzCells nz;                         // zero pattern of every pair's operators (owned by the superblocks)
    std::vector<int> active;
    int64_t hv_count[D2D_NPREC] = {0, 0, 0, 0};
    // launch configuration per precision (as on a single superblock)
    int tile_sel[D2D_NPREC] = {-1, -1, -1, -1};   // shape index, or -1 = by size
    int split[D2D_NPREC] = {0, 0, 0, 0};          // K-loop split level
    int fuse[D2D_NPREC] = {0, 1, 1, 1};           // central term inside the GEMM launch (inner steps)
    int xcd[D2D_NPREC] = {0, 0, 0, 0};            // XCD-aware work order
    int dense[D2D_NPREC] = {0, 0, 0, 0};          // every K step (no skipping of zero operator tiles)
    int persist[D2D_NPREC] = {0, 0, 0, 0};        // persistent grouped launch
    void* d_x[3] = {nullptr, nullptr, nullptr};   // ntot doubles each, partial outputs of split K-loops
    void* d_w2 = nullptr;               // ntot doubles, central-term part of fused launches
    void* stage_v = nullptr;
    void* stage_w = nullptr;
    uint64_t builds = 0;                // work lists built so far (a rebuild reshapes the launches)
    LanczosWork* lz = nullptr;
    ~d2d_batch();
};

namespace {

template <typename T>
void dfree(d2d_ctx* c, T*& p, size_t count) {
    if (p) c->free((void*)p, count * sizeof(T));
    p = nullptr;
}

template <typename T>
d2d_status dupload(d2d_ctx* c, const std::vector<T>& h, T** d) {
    *d = nullptr;
    if (h.empty()) return D2D_OK;
    D2D_CHECK(c->alloc((void**)d, h.size() * sizeof(T)));
    D2D_HIP(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return D2D_OK;
}

int batch_auto_tile(const d2d_batch* b, int prec) {
    const int D = std::max(b->max_dl, b->max_dr);
    if (prec == D2D_FP64) return D <= 64 ? 0 : (D <= 768 ? 1 : 2);
    if (prec == D2D_FP32) return D <= 64 ? 3 : (D <= 768 ? 4 : 5);
    if (prec == D2D_BF16X3) return D <= 64 ? 30 : (D <= 512 ? 28 : 29);
    return D <= 64 ? 17 : (D <= 512 ? 14 : 15);
}

int work_key(int shape, int split, int xcd, int dense) { return shape | split << 16 | xcd << 18 | dense << 19; }

int batch_shape(const d2d_batch* b, int prec) {
    return b->tile_sel[prec] >= 0 ? b->tile_sel[prec] : batch_auto_tile(b, prec);
}

// Launch tables of the active problems (work list of one shape, split level,
// order and step choice; central and pack tiles).
d2d_status build_work(d2d_batch* b, int key) {
    b->builds++;
    std::vector<int> keep(b->pairs.size());
    for (size_t p = 0; p < b->pairs.size(); ++p) keep[p] = b->active[b->pair_prob[p]];
    WorkHost h;
    const int split = (key >> 16) & 3;
    const bool dense = (key >> 19) & 1;
    make_work(b->pairs, &keep, tile_shape(key & 0xFFFF), split, (key >> 18) & 1,
              (dense && split != 3) ? nullptr : &b->nz, h,
              split == 3 ? &tile_shape(asym_partner(key & 0xFFFF)) : nullptr, dense);
    return upload_work(b->ctx, h, b->work[key]);
}

d2d_status build_tiles(d2d_batch* b) {
    std::vector<CentralUnit> ct;
    std::vector<int4> pt;
    std::vector<int> keep(b->pairs.size());
    for (size_t p = 0; p < b->pairs.size(); ++p) keep[p] = b->active[b->pair_prob[p]];
    for (const CentralUnit& u : b->cunits)
        if (keep[u.p]) ct.push_back(u);
    for (size_t p = 0; p < b->pairs.size(); ++p) {
        if (!keep[p]) continue;
        const int dL = b->pairs[p].dL, dR = b->pairs[p].dR;
        for (int j = 0; j < (dR + 63) / 64; ++j)
            for (int i = 0; i < (dL + 63) / 64; ++i) pt.push_back(make_int4((int)p, i, j, 0));
    }
    if ((int)ct.size() > b->cap_cunits) {
        dfree(b->ctx, b->d_cunits, (size_t)b->cap_cunits);
        b->cap_cunits = (int)std::max<size_t>(ct.size(), 1);
        D2D_CHECK(b->ctx->alloc((void**)&b->d_cunits, (size_t)b->cap_cunits * sizeof(CentralUnit)));
    }
    if ((int)pt.size() > b->cap_ptiles) {
        dfree(b->ctx, b->d_ptiles, (size_t)b->cap_ptiles);
        b->cap_ptiles = (int)std::max<size_t>(pt.size(), 1);
        D2D_CHECK(b->ctx->alloc((void**)&b->d_ptiles, (size_t)b->cap_ptiles * sizeof(int4)));
    }
    if (!ct.empty())
        D2D_HIP(hipMemcpy(b->d_cunits, ct.data(), ct.size() * sizeof(CentralUnit), hipMemcpyHostToDevice));
    if (!pt.empty()) D2D_HIP(hipMemcpy(b->d_ptiles, pt.data(), pt.size() * sizeof(int4), hipMemcpyHostToDevice));
    b->n_cunits = (int)ct.size();
    b->n_ptiles = (int)pt.size();
    return D2D_OK;
}

HvTables tables_of(d2d_batch* b) {
    HvTables t{};
    t.sec = b->d_sec;
    t.npairs = (int)b->pairs.size();
    for (int p = 0; p < D2D_NPREC; ++p) {
        t.HL[p] = b->HL[p];
        t.HR[p] = b->HR[p];
    }
    t.lo[0] = b->h16_len;
    t.lo[1] = b->r16_len;
    t.lo[2] = b->vp_len;
    t.lo[3] = b->vt_len;
    t.cunits = b->d_cunits;
    t.n_cunits = b->n_cunits;
    t.cterms = b->d_cterms;
    t.ptiles = b->d_ptiles;
    t.n_ptiles = b->n_ptiles;
    t.vp = b->d_vp;
    t.vt = b->d_vt;
    return t;
}

// Work list of the precision's current launch configuration (built on first use).
d2d_status batch_work(d2d_batch* b, int prec, int* shape, const WorkList** wl) {
    *shape = batch_shape(b, prec);
    const int key = work_key(*shape, b->split[prec], b->xcd[prec], b->dense[prec]);
    if (b->work.find(key) == b->work.end()) D2D_CHECK(build_work(b, key));
    *wl = &b->work[key];
    return D2D_OK;
}

d2d_status batch_hv(d2d_batch* b, int prec, const void* v, void* w, hipStream_t s, HvParts* parts = nullptr) {
    if (prec < 0 || prec >= D2D_NPREC || !(b->prec_mask & (1u << prec)) || !b->HL[prec]) {
        set_error("precision %d not kept by every superblock of the batch", prec);
        return D2D_EINVAL;
    }
    int shape = 0;
    const WorkList* wl = nullptr;
    D2D_CHECK(batch_work(b, prec, &shape, &wl));
    HvTables t = tables_of(b);
    for (int i = 0; i < split_parts(b->split[prec]); ++i) {
        if (!b->d_x[i]) D2D_CHECK(b->ctx->alloc(&b->d_x[i], (size_t)b->ntot * 8));
        t.x[i] = b->d_x[i];
    }
    if (parts && !b->fuse[prec]) {
        *parts = HvParts{};
        parts = nullptr;
    }
    if (parts) {
        t.w2 = b->d_w2;
        for (int i = 0; i < 3; ++i) parts->x[i] = t.x[i];
        parts->central = t.w2;
    }
    t.persist = b->persist[prec];
    return hv_launch(t, prec, shape, *wl, v, w, s);
}

struct BatchHv : HvOps {
    d2d_batch* b;
    explicit BatchHv(d2d_batch* x) : b(x) {}
    d2d_status hv(int prec, const void* v, void* w, hipStream_t s) override { return batch_hv(b, prec, v, w, s); }
    d2d_status hv_fused(int prec, const void* v, void* w, hipStream_t s, HvParts* parts) override {
        return batch_hv(b, prec, v, w, s, parts);
    }
    d2d_status prepare(int prec) override {
        int shape = 0;
        const WorkList* wl = nullptr;
        D2D_CHECK(batch_work(b, prec, &shape, &wl));
        for (int i = 0; i < split_parts(b->split[prec]); ++i)
            if (!b->d_x[i]) D2D_CHECK(b->ctx->alloc(&b->d_x[i], (size_t)b->ntot * 8));
        return D2D_OK;
    }
    d2d_status set_active(const std::vector<int>& a, bool* rebuilt) override {
        if (rebuilt) *rebuilt = false;
        if (a == b->active) return D2D_OK;
        b->active = a;
        std::vector<int> shapes;
        for (auto& kv : b->work) shapes.push_back(kv.first);
        for (int sh : shapes) D2D_CHECK(build_work(b, sh));
        D2D_CHECK(build_tiles(b));
        if (rebuilt) *rebuilt = true;
        return D2D_OK;
    }
    bool has(int prec) override { return (b->prec_mask & (1u << prec)) && b->HL[prec]; }
    void count(int prec, int64_t n) override { b->hv_count[prec] += n; }
    int64_t counter(int prec) override { return b->hv_count[prec]; }
    uint64_t fingerprint() override {
        return config_fingerprint(b->tile_sel, b->split, b->fuse, b->xcd, b->dense, b->persist, b->d_x, b->d_w2, b->builds);
    }
};

}  // namespace

d2d_batch::~d2d_batch() {
    free_lanczos_work(ctx, lz);
    const size_t np = pairs.size();
    dfree(ctx, d_sec, np);
    for (int p = 0; p < D2D_NPREC; ++p) {
        if (HL[p]) ctx->free(HL[p], hl_bytes[p]);
        if (HR[p]) ctx->free(HR[p], hr_bytes[p]);
    }
    dfree(ctx, d_cterms, cterms.size());
    dfree(ctx, d_cunits, (size_t)cap_cunits);
    dfree(ctx, d_ptiles, (size_t)cap_ptiles);
    dfree(ctx, d_vp, (size_t)vp_len * vparts);
    dfree(ctx, d_vt, (size_t)vt_len * vparts);
    for (auto& kv : work) free_work(ctx, kv.second);
    for (auto& x : d_x)
        if (x) ctx->free(x, (size_t)ntot * 8);
    if (d_w2) ctx->free(d_w2, (size_t)ntot * 8);
    if (stage_v) ctx->free(stage_v, (size_t)ntot * 8);
    if (stage_w) ctx->free(stage_w, (size_t)ntot * 8);
}

extern "C" d2d_status d2d_batch_create(d2d_ctx* ctx, d2d_sb* const* sbs, int n, d2d_batch** out) {
    if (!ctx || !sbs || !out || n < 1) {
        set_error("d2d_batch_create: bad argument");
        return D2D_EINVAL;
    }
    *out = nullptr;
    auto b = std::make_unique<d2d_batch>();
    b->ctx = ctx;
    b->prec_mask = (1u << D2D_NPREC) - 1u;
    for (int i = 0; i < n; ++i) {
        if (!sbs[i] || sbs[i]->ctx != ctx) {
            set_error("d2d_batch_create: superblock %d is NULL or of another context", i);
            return D2D_EINVAL;
        }
        b->sbs.push_back(sbs[i]);
        b->prec_mask &= sbs[i]->prec_mask;
    }
    // concatenation offsets
    int64_t voff = 0, hl = 0, hr = 0, h16 = 0, r16 = 0, vp = 0, vt = 0, rb = 0, cb = 0;
    std::vector<int> pbase(n);
    for (int i = 0; i < n; ++i) {
        const d2d_sb* s = sbs[i];
        pbase[i] = (int)b->pairs.size();
        for (size_t j = 0; j < s->pairs.size(); ++j) {
            SectorDev q = s->pairs[j];
            b->nz.L.push_back(s->nzL[j].data());
            b->nz.R.push_back(s->nzR[j].data());
            b->nz.rowL.push_back(s->nzRowL[j].data());
            b->nz.colR.push_back(s->nzColR[j].data());
            b->nz.runsL.push_back(&s->runsL[j]);
            b->nz.runsR.push_back(&s->runsR[j]);
            q.off += voff;
            q.hl_off += hl;
            q.hr_off += hr;
            q.row_base += rb;
            q.col_base += cb;
            q.hl16_off += h16;
            q.hr16_off += r16;
            q.vp_off += vp;
            q.vt_off += vt;
            b->pairs.push_back(q);
            b->pair_prob.push_back(i);
        }
        b->voff.push_back(voff);
        b->len.push_back(s->N);
        b->max_dl = std::max(b->max_dl, s->max_dl);
        b->max_dr = std::max(b->max_dr, s->max_dr);
        voff += s->N;
        hl += s->hl_len;
        hr += s->hr_len;
        h16 += s->hl16_len;
        r16 += s->hr16_len;
        vp += s->vp_len;
        vt += s->vt_len;
        rb += s->Drows;
        cb += s->Dcols;
    }
    b->ntot = voff;
    b->vp_len = vp;
    b->vt_len = vt;
    D2D_CHECK(dupload(ctx, b->pairs, &b->d_sec));
    // operators: device-to-device concatenation
    // (BF16x3: every problem's hi parts, then every problem's lo parts)
    const size_t esz[D2D_NPREC] = {8, 4, 2, 2};
    b->h16_len = h16;
    b->r16_len = r16;
    for (int p = 0; p < D2D_NPREC; ++p) {
        if (!(b->prec_mask & (1u << p))) continue;
        const bool b16 = p == D2D_BF16 || p == D2D_BF16X3;
        const int parts = p == D2D_BF16X3 ? 2 : 1;
        b->hl_bytes[p] = (size_t)(b16 ? h16 : hl) * esz[p] * parts;
        b->hr_bytes[p] = (size_t)(b16 ? r16 : hr) * esz[p] * parts;
        D2D_CHECK(ctx->alloc(&b->HL[p], b->hl_bytes[p]));
        D2D_CHECK(ctx->alloc(&b->HR[p], b->hr_bytes[p]));
        for (int part = 0; part < parts; ++part) {
            size_t ol = (size_t)part * (b16 ? h16 : hl) * esz[p], orr = (size_t)part * (b16 ? r16 : hr) * esz[p];
            for (int i = 0; i < n; ++i) {
                const d2d_sb* s = sbs[i];
                const size_t bl = (size_t)(b16 ? s->hl16_len : s->hl_len) * esz[p];
                const size_t br = (size_t)(b16 ? s->hr16_len : s->hr_len) * esz[p];
                D2D_HIP(hipMemcpy((char*)b->HL[p] + ol, (const char*)s->HL[p] + part * bl, bl,
                                  hipMemcpyDeviceToDevice));
                D2D_HIP(hipMemcpy((char*)b->HR[p] + orr, (const char*)s->HR[p] + part * br, br,
                                  hipMemcpyDeviceToDevice));
                ol += bl;
                orr += br;
            }
        }
    }
    if (b->prec_mask & ((1u << D2D_BF16) | (1u << D2D_BF16X3))) {
        b->vparts = (b->prec_mask & (1u << D2D_BF16X3)) ? 2 : 1;
        D2D_CHECK(ctx->alloc((void**)&b->d_vp, (size_t)vp * 2 * b->vparts));
        D2D_CHECK(ctx->alloc((void**)&b->d_vt, (size_t)vt * 2 * b->vparts));
        D2D_HIP(hipMemset(b->d_vp, 0, (size_t)vp * 2 * b->vparts));
        D2D_HIP(hipMemset(b->d_vt, 0, (size_t)vt * 2 * b->vparts));
    }
    // central units and terms of every problem, rebased
    for (int i = 0; i < n; ++i) {
        const d2d_sb* s = sbs[i];
        const int tbase = (int)b->cterms.size();
        for (CentralTerm t : s->h_cterms) {
            t.base += b->voff[i];
            b->cterms.push_back(t);
        }
        for (CentralUnit u : s->h_cunits) {
            u.off += b->voff[i];
            u.tofs += tbase;
            u.p += pbase[i];
            b->cunits.push_back(u);
        }
    }
    D2D_CHECK(dupload(ctx, b->cterms, &b->d_cterms));
    b->active.assign(n, 1);
    // every sector small: the GEMM is latency-bound, split its two K-loops
    const int split = std::max(b->max_dl, b->max_dr) <= 768 ? 1 : 0;
    for (int p = 0; p < D2D_NPREC; ++p) b->split[p] = split;
    D2D_CHECK(ctx->alloc(&b->d_w2, (size_t)b->ntot * 8));
    D2D_CHECK(build_tiles(b.get()));
    D2D_CHECK(ctx->alloc(&b->stage_v, (size_t)b->ntot * 8));
    D2D_CHECK(ctx->alloc(&b->stage_w, (size_t)b->ntot * 8));
    ctx->children++;
    *out = b.release();
    return D2D_OK;
}

extern "C" d2d_status d2d_batch_destroy(d2d_batch* b) {
    if (!b) return D2D_OK;
    d2d_ctx* c = b->ctx;
    (void)hipStreamSynchronize(c->stream);
    delete b;
    c->children--;
    return D2D_OK;
}

extern "C" d2d_status d2d_batch_hv(d2d_batch* b, int prec, const void* const* v, void* const* w) {
    if (!b || !v || !w || prec < 0 || prec >= D2D_NPREC) {
        set_error("d2d_batch_hv: bad argument");
        return D2D_EINVAL;
    }
    const int n = (int)b->sbs.size();
    const size_t in_sz = prec == D2D_FP64 ? 8 : (prec == D2D_BF16 ? 2 : 4);
    const size_t out_sz = prec == D2D_FP64 ? 8 : 4;
    hipStream_t s = b->ctx->stream;
    std::vector<int> all(n, 1);
    BatchHv ops(b);
    bool rebuilt = false;
    D2D_CHECK(ops.set_active(all, &rebuilt));
    for (int i = 0; i < n; ++i) {
        if (!v[i] || !w[i]) {
            set_error("d2d_batch_hv: NULL vector of problem %d", i);
            return D2D_EINVAL;
        }
        D2D_HIP(hipMemcpyAsync((char*)b->stage_v + b->voff[i] * in_sz, v[i], (size_t)b->len[i] * in_sz,
                               hipMemcpyDeviceToDevice, s));
    }
    D2D_CHECK(batch_hv(b, prec, b->stage_v, b->stage_w, s));
    b->hv_count[prec]++;
    for (int i = 0; i < n; ++i)
        D2D_HIP(hipMemcpyAsync(w[i], (char*)b->stage_w + b->voff[i] * out_sz, (size_t)b->len[i] * out_sz,
                               hipMemcpyDeviceToDevice, s));
    return D2D_OK;
}

extern "C" d2d_status d2d_batch_lanczos(d2d_batch* b, const d2d_lanczos_opts* opts, const double* const* v0,
                                        double* energies, double* const* psi, d2d_lanczos_stats* per_problem) {
    if (!b || !opts || !energies) {
        set_error("d2d_batch_lanczos: NULL argument");
        return D2D_EINVAL;
    }
    D2D_CHECK(check_lanczos_opts(opts));
    if (!(b->prec_mask & (1u << opts->prec))) {
        set_error("d2d_batch_lanczos: precision %d not kept by every superblock", opts->prec);
        return D2D_EINVAL;
    }
    BatchHv ops(b);
    return run_lanczos(b->ctx, b->lz, ops, opts, b->len, v0, energies, psi, per_problem);
}

extern "C" d2d_status d2d_batch_set_tile(d2d_batch* b, int prec, int tile) {
    if (!b || prec < 0 || prec >= D2D_NPREC) {
        set_error("d2d_batch_set_tile: bad argument");
        return D2D_EINVAL;
    }
    TileSel t;
    if (!decode_tile(prec, tile, &t)) {
        set_error("d2d_batch_set_tile: tile %d is not a shape of precision %d", tile, prec);
        return D2D_EINVAL;
    }
    b->tile_sel[prec] = t.shape;
    b->split[prec] = tile < 0 ? (std::max(b->max_dl, b->max_dr) <= 768 ? 1 : 0) : t.split;
    b->fuse[prec] = t.fuse;
    b->xcd[prec] = t.xcd;
    b->dense[prec] = t.dense;
    b->persist[prec] = t.persist;
    return D2D_OK;
}

namespace {
uint64_t batch_key(const d2d_batch* b, int prec) {
    uint64_t h = 0x9e3779b97f4a7c15ull ^ (uint64_t)prec;
    auto mix = [&](uint64_t v) {
        h ^= v;
        h *= 1099511628211ull;
    };
    mix(b->sbs.size());
    for (const auto& p : b->pairs) {
        mix((uint64_t)p.dL);
        mix((uint64_t)p.dR);
    }
    return h;
}
}  // namespace

extern "C" d2d_status d2d_batch_autotune(d2d_batch* b, int prec, int reps, int* best_tile, double* best_ms) {
    if (!b || !best_tile || !best_ms || prec < 0 || prec >= D2D_NPREC || reps < 1 || reps > 10000) {
        set_error("d2d_batch_autotune: bad argument");
        return D2D_EINVAL;
    }
    if (!(b->prec_mask & (1u << prec)) || !b->HL[prec]) {
        set_error("d2d_batch_autotune: precision %d not kept by every superblock", prec);
        return D2D_EINVAL;
    }
    auto apply = [&](const TileSel& c) {
        b->tile_sel[prec] = c.shape;
        b->split[prec] = c.split;
        b->fuse[prec] = c.fuse;
        b->xcd[prec] = c.xcd;
        b->dense[prec] = c.dense;
        b->persist[prec] = c.persist;
    };
    const uint64_t key = batch_key(b, prec);
    TileSel sel;
    if (tune_cache_lookup(key, prec, &sel, best_tile, best_ms)) {
        apply(sel);
        return D2D_OK;
    }
    hipStream_t s = b->ctx->stream;
    const TileSel saved{b->tile_sel[prec], b->split[prec], b->fuse[prec], b->xcd[prec], b->dense[prec],
                        b->persist[prec]};
    // every problem active, as at the start of a solve
    BatchHv ops(b);
    D2D_CHECK(ops.set_active(std::vector<int>(b->sbs.size(), 1), nullptr));
    if (launch_fill(b->stage_v, prec, b->ntot, 0.5, s) != hipSuccess) {
        set_error("d2d_batch_autotune: HIP setup failed");
        return D2D_EDEVICE;
    }
    double bms = 0;
    const d2d_status st = tune_configs(s, prec, reps, [&](const TileSel& c) {
        apply(c);
        HvParts parts{};
        D2D_CHECK(batch_hv(b, prec, b->stage_v, b->stage_w, s, c.fuse ? &parts : nullptr));
        if (!c.fuse) return D2D_OK;
        // a fused product leaves its parts to the consumer: charge reading them
        const void* pp[4] = {parts.x[0], parts.x[1], parts.x[2], parts.central};
        D2D_HIP(launch_read_parts(pp, prec, b->ntot, b->stage_w, s));
        return D2D_OK;
    }, &sel, &bms);
    if (st != D2D_OK) {
        apply(saved);
    } else {
        apply(sel);
        *best_tile = encode_tile(sel);
        *best_ms = bms;
        tune_cache_store(key, *best_tile, bms);
    }
    // keep only the work lists still selected (set_active rebuilds every list held)
    std::vector<int> keys;
    for (int p = 0; p < D2D_NPREC; ++p)
        if (b->HL[p]) keys.push_back(work_key(batch_shape(b, p), b->split[p], b->xcd[p], b->dense[p]));
    for (auto it = b->work.begin(); it != b->work.end();) {
        if (std::find(keys.begin(), keys.end(), it->first) == keys.end()) {
            free_work(b->ctx, it->second);
            it = b->work.erase(it);
        } else {
            ++it;
        }
    }
    return st;
}

extern "C" d2d_status d2d_batch_gemm_flops(d2d_batch* b, int prec, double* flops) {
    if (!b || !flops || prec < 0 || prec >= D2D_NPREC) {
        set_error("d2d_batch_gemm_flops: bad argument");
        return D2D_EINVAL;
    }
    if (!(b->prec_mask & (1u << prec)) || !b->HL[prec]) {
        set_error("d2d_batch_gemm_flops: precision %d not kept by every superblock", prec);
        return D2D_EINVAL;
    }
    // the figure is for every problem of the batch
    BatchHv ops(b);
    D2D_CHECK(ops.set_active(std::vector<int>(b->sbs.size(), 1), nullptr));
    int shape = 0;
    const WorkList* wl = nullptr;
    D2D_CHECK(batch_work(b, prec, &shape, &wl));
    *flops = wl->flops;
    return D2D_OK;
}
