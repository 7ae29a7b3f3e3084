// Host-only checks of the library's host logic, built with AddressSanitizer
// and UndefinedBehaviorSanitizer on the host side (no device code runs):
//   1. tile configuration codes: decode / encode round trip, rejected codes;
//   2. work lists (make_work) for every tile shape, split level, XCD order and
//      dense / skipping step lists, on random ragged sectors with random zero
//      patterns and run boundaries: the items are emulated on the host as the
//      grouped GEMM runs them (each item stores its tile into its slot) and
//      the sum of the slots must equal H_l V + V H_r^T, with every element of
//      every slot written exactly once and no listed K step out of range;
//   3. block import / export round trip and the import's rejection of
//      inconsistent descriptors, on a context object that never touches a GPU;
//   4. the autotuner cache reader on a malformed file.
// Exit status 0 when every check passes; failures are printed.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "host.h"

using namespace d2d;

static int failures = 0;
static bool mutate = false;   // --mutate: drop one K step from every list (the checks must fail)
#define CHECK(c, ...)                                  \
    do {                                               \
        if (!(c)) {                                    \
            ++failures;                                \
            if (failures < 20) {                       \
                std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
                std::printf(__VA_ARGS__);              \
                std::printf("\n");                     \
            }                                          \
        }                                              \
    } while (0)

// ---------------------------------------------------------------- 1. tile codes
static void check_tile_codes() {
    const int flags[] = {0, D2D_TILE_SPLIT, D2D_TILE_SPLIT4, D2D_TILE_FUSED, D2D_TILE_XCD, D2D_TILE_DENSE,
                         D2D_TILE_ASYM, D2D_TILE_PERSIST};
    int ok = 0;
    for (int prec = 0; prec < D2D_NPREC; ++prec)
        for (int sh = -1; sh <= tile_shape_count(); ++sh)
            for (int m = 0; m < 256; ++m) {
                int f = 0;
                for (int b = 0; b < 8; ++b)
                    if (m & (1 << b)) f |= flags[b];
                const int tile = sh < 0 ? -1 : (sh | f);
                if (sh < 0 && m) continue;
                TileSel t;
                const bool valid = decode_tile(prec, tile, &t);
                if (!valid) continue;
                ++ok;
                CHECK(tile < 0 || encode_tile(t) == tile, "encode(decode(%d)) = %d", tile, encode_tile(t));
                CHECK(tile < 0 || tile_shape(t.shape).prec == prec, "shape %d not of precision %d", t.shape, prec);
                CHECK(!(t.persist && t.xcd), "persistent with XCD order accepted");
                CHECK(t.split != 3 || asym_partner(t.shape) >= 0, "asymmetric split without a partner");
            }
    CHECK(ok > 100, "only %d valid codes", ok);
    TileSel t;
    CHECK(!decode_tile(D2D_FP32, tile_shape_count(), &t), "shape past the table accepted");
    CHECK(!decode_tile(D2D_FP32, 4 | (1 << 30), &t), "unknown flag accepted");
    CHECK(!decode_tile(D2D_FP64, 4, &t), "FP32 shape accepted for FP64");
}

// ---------------------------------------------------------------- 2. work lists
struct Sector {
    int dL, dR;
    std::vector<double> HL, HRt, V;   // column-major: HL dL x dL, HRt dR x dR (stored H_r^T), V dL x dR
    std::vector<uint8_t> L, R, rowL, colR;
    std::vector<int> runsL, runsR;
};

static void pattern(std::mt19937_64& g, int d, double density, std::vector<double>& a) {
    std::uniform_real_distribution<double> u(0.0, 1.0), x(-1.0, 1.0);
    a.assign((size_t)d * d, 0.0);
    // zero or nonzero in 16-column blocks and single entries, so that whole cells vanish
    for (int j = 0; j < d; ++j)
        for (int i = 0; i < d; ++i)
            if (u(g) < density && ((i / 16 + j / 16) % 3 != 1 || u(g) < 0.1)) a[i + (size_t)j * d] = x(g);
}

static void masks(const std::vector<double>& a, int d, bool by_row, std::vector<uint8_t>& cells,
                  std::vector<uint8_t>& lines) {
    const int c = (d + NZ_CELL - 1) / NZ_CELL;
    cells.assign((size_t)c * c, 0);
    lines.assign((size_t)d * c, 0);
    for (int j = 0; j < d; ++j)
        for (int i = 0; i < d; ++i)
            if (a[i + (size_t)j * d] != 0.0) {
                cells[(size_t)(j / NZ_CELL) * c + i / NZ_CELL] = 1;
                if (by_row) lines[(size_t)i * c + j / NZ_CELL] = 1;
                else lines[(size_t)j * c + i / NZ_CELL] = 1;
            }
}

static std::vector<int> random_runs(std::mt19937_64& g, int d) {
    std::vector<int> r{0};
    std::uniform_int_distribution<int> len(1, 90);
    while (r.back() < d) r.push_back(std::min(d, r.back() + len(g)));
    return r;
}

// the grouped GEMM's semantics on the host: each item stores its tile (the
// sum over its K steps of its phases) into its slot
static void emulate(const std::vector<Sector>& secs, const std::vector<SectorDev>& pairs, const WorkHost& h,
                    const TileShape& ts0, const TileShape* ts1, int nslots, const std::vector<double>& ref,
                    const std::vector<double>& mag, const char* what) {
    std::vector<std::vector<double>> out(nslots);
    std::vector<std::vector<int>> wrote(nslots);
    size_t N = 0;
    for (auto& s : secs) N += (size_t)s.dL * s.dR;
    for (int k = 0; k < nslots; ++k) {
        out[k].assign(N, 0.0);
        wrote[k].assign(N, 0);
    }
    for (size_t n = 0; n < h.items.size(); ++n) {
        const WorkItem& wi = h.items[n];
        if (wi.p < 0) continue;
        CHECK(wi.p < (int)secs.size(), "%s: item %zu of pair %d", what, n, wi.p);
        if (wi.p >= (int)secs.size()) continue;
        const TileShape& ts = (h.n0 >= 0 && (int)n >= h.n0) ? *ts1 : ts0;
        const Sector& s = secs[wi.p];
        const SectorDev& sd = pairs[wi.p];
        const int ph = wi.part & 3, slot = (wi.part >> 2) & 3;
        const int ph_lo = ph == 2 ? 1 : 0, ph_hi = ph == 1 ? 1 : 2;
        const bool al = (wi.part & ITEM_ALIGNED) != 0;
        const int row0 = al && ph_lo == 0 ? wi.tm : wi.tm * ts.BM, col0 = al && ph_lo == 1 ? wi.tn : wi.tn * ts.BN;
        const int rlim = al && ph_lo == 0 ? row0 + wi.kn[1] : std::min(s.dL, row0 + ts.BM);
        const int clim = al && ph_lo == 1 ? col0 + wi.kn[0] : std::min(s.dR, col0 + ts.BN);
        CHECK(slot < nslots, "%s: slot %d of %d", what, slot, nslots);
        CHECK(row0 >= 0 && rlim <= s.dL && row0 < rlim && col0 >= 0 && clim <= s.dR && col0 < clim,
              "%s: tile rows [%d,%d) cols [%d,%d) outside %dx%d", what, row0, rlim, col0, clim, s.dL, s.dR);
        if (slot >= nslots || row0 < 0 || rlim > s.dL || col0 < 0 || clim > s.dR) continue;
        const bool b16 = ts.prec == D2D_BF16 || ts.prec == D2D_BF16X3;
        for (int c = col0; c < clim; ++c)
            for (int r = row0; r < rlim; ++r) {
                double acc = 0.0;
                for (int phase = ph_lo; phase < ph_hi; ++phase) {
                    const int K = phase == 0 ? s.dL : s.dR;
                    const int KP = b16 ? (phase == 0 ? sd.dLp : sd.dRp) : K;
                    const int ko = phase == 0 ? wi.ks[0] : wi.ks[1], kn = phase == 0 ? wi.kn[0] : wi.kn[1];
                    CHECK(ko >= 0 && kn >= 0 && (size_t)(ko + kn) <= h.ksteps.size(), "%s: steps [%d,+%d) of %zu",
                          what, ko, kn, h.ksteps.size());
                    if (ko < 0 || kn < 0 || (size_t)(ko + kn) > h.ksteps.size()) continue;
                    for (int q = 0; q < kn; ++q) {
                        const int k0 = h.ksteps[ko + q];
                        CHECK(k0 >= 0 && k0 < KP && k0 % ts.BK == 0, "%s: step %d (K %d, BK %d)", what, k0, KP, ts.BK);
                        for (int k = k0; k < std::min(k0 + ts.BK, K); ++k)
                            acc += phase == 0 ? s.HL[r + (size_t)k * s.dL] * s.V[k + (size_t)c * s.dL]
                                              : s.V[r + (size_t)k * s.dL] * s.HRt[k + (size_t)c * s.dR];
                    }
                }
                const size_t e = sd.off + r + (size_t)c * s.dL;
                out[slot][e] = acc;
                wrote[slot][e]++;
            }
    }
    size_t off = 0;
    for (size_t p = 0; p < secs.size(); ++p) {
        const Sector& s = secs[p];
        for (int c = 0; c < s.dR; ++c)
            for (int r = 0; r < s.dL; ++r) {
                const size_t e = off + r + (size_t)c * s.dL;
                double sum = 0.0;
                for (int k = 0; k < nslots; ++k) {
                    CHECK(wrote[k][e] == 1, "%s: pair %zu element (%d,%d) slot %d written %d times", what, p, r, c,
                          k, wrote[k][e]);
                    sum += out[k][e];
                }
                CHECK(std::fabs(sum - ref[e]) <= 1e-12 * (mag[e] + 1e-300), "%s: pair %zu (%d,%d) %.17g vs %.17g",
                      what, p, r, c, sum, ref[e]);
            }
        off += (size_t)s.dL * s.dR;
    }
}

// H_l V + V H_r^T of every sector (packed), and the sum of the terms' magnitudes
static void reference(const std::vector<Sector>& secs, std::vector<double>& ref, std::vector<double>& mag) {
    ref.clear();
    mag.clear();
    for (const Sector& s : secs)
        for (int c = 0; c < s.dR; ++c)
            for (int r = 0; r < s.dL; ++r) {
                double x = 0.0, a = 0.0;
                for (int k = 0; k < s.dL; ++k) {
                    x += s.HL[r + (size_t)k * s.dL] * s.V[k + (size_t)c * s.dL];
                    a += std::fabs(s.HL[r + (size_t)k * s.dL] * s.V[k + (size_t)c * s.dL]);
                }
                for (int k = 0; k < s.dR; ++k) {
                    x += s.V[r + (size_t)k * s.dL] * s.HRt[k + (size_t)c * s.dR];
                    a += std::fabs(s.V[r + (size_t)k * s.dL] * s.HRt[k + (size_t)c * s.dR]);
                }
                ref.push_back(x);
                mag.push_back(a);
            }
}

static void check_work_lists() {
    std::mt19937_64 g(20070159);
    // ragged sectors: a 1-row and a 2-column one, one taller than the widest
    // tile, one spanning several tiles both ways, one of exactly one 64 tile
    const int dims[5][2] = {{1, 21}, {70, 2}, {300, 9}, {97, 131}, {64, 64}};
    const int nsec = 5;
    std::vector<Sector> secs(nsec);
    std::vector<SectorDev> pairs(nsec);
    int64_t off = 0, hl = 0, hr = 0;
    for (int p = 0; p < nsec; ++p) {
        Sector& s = secs[p];
        s.dL = dims[p][0];
        s.dR = dims[p][1];
        pattern(g, s.dL, 0.35, s.HL);
        pattern(g, s.dR, 0.35, s.HRt);
        std::uniform_real_distribution<double> x(-1.0, 1.0);
        s.V.resize((size_t)s.dL * s.dR);
        for (auto& v : s.V) v = x(g);
        masks(s.HL, s.dL, true, s.L, s.rowL);
        masks(s.HRt, s.dR, false, s.R, s.colR);
        s.runsL = random_runs(g, s.dL);
        s.runsR = random_runs(g, s.dR);
        SectorDev& sd = pairs[p];
        sd = SectorDev{};
        sd.dL = s.dL;
        sd.dR = s.dR;
        sd.off = off;
        sd.hl_off = hl;
        sd.hr_off = hr;
        sd.dLp = (s.dL + 7) / 8 * 8;
        sd.dRp = (s.dR + 7) / 8 * 8;
        off += (int64_t)s.dL * s.dR;
        hl += (int64_t)s.dL * s.dL;
        hr += (int64_t)s.dR * s.dR;
    }
    NzCells nz;
    for (auto& s : secs) {
        nz.L.push_back(s.L.data());
        nz.R.push_back(s.R.data());
        nz.rowL.push_back(s.rowL.data());
        nz.colR.push_back(s.colR.data());
        nz.runsL.push_back(&s.runsL);
        nz.runsR.push_back(&s.runsR);
    }
    std::vector<int> keep(nsec, 1);
    std::vector<double> ref, mag;
    reference(secs, ref, mag);
    int lists = 0;
    for (int sh = 0; sh < tile_shape_count(); ++sh)
        for (int split = 0; split <= 3; ++split)
            for (int xcd = 0; xcd <= 1; ++xcd)
                for (int dense = 0; dense <= 1; ++dense) {
                    const int partner = asym_partner(sh);
                    if (split == 3 && partner < 0) continue;
                    const TileShape& ts = tile_shape(sh);
                    const TileShape* ts1 = split == 3 ? &tile_shape(partner) : nullptr;
                    WorkHost h;
                    // as the library calls it: the asymmetric split keeps the runs
                    // and the row-exact masks even when it runs every step
                    make_work(pairs, &keep, ts, split, xcd, (dense && split != 3) ? nullptr : &nz, h, ts1,
                              dense && split == 3);
                    if (mutate)
                        for (auto& wi : h.items)
                            if (wi.p >= 0 && wi.kn[0] > 0 && (wi.part & 3) != 2) {
                                wi.kn[0]--;
                                break;
                            }
                    char what[96];
                    std::snprintf(what, sizeof what, "shape %d split %d xcd %d dense %d", sh, split, xcd, dense);
                    emulate(secs, pairs, h, ts, ts1, split_parts(split) + 1, ref, mag, what);
                    ++lists;
                }
    CHECK(lists > 300, "only %d lists", lists);
    // a subset of the pairs (a batch with finished problems): items of kept pairs only
    keep[1] = keep[3] = 0;
    WorkHost h;
    make_work(pairs, &keep, tile_shape(4), 1, 1, &nz, h);
    for (auto& wi : h.items) CHECK(wi.p < 0 || keep[wi.p], "item of a pair left out");
}

// ---------------------------------------------------------------- 3. blocks
struct Exported {
    std::vector<int64_t> qn, dim, key, blk, off;
    std::vector<double> H, data;
    int64_t sizes[5] = {0, 0, 0, 0, 0};
};

static bool export_block(const d2d_block* b, Exported& e) {
    if (d2d_block_export(b, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, e.sizes) != D2D_OK)
        return false;
    e.qn.assign(2 * e.sizes[0] + 1, 0);
    e.dim.assign(e.sizes[0] + 1, 0);
    e.H.assign(e.sizes[1] + 1, 0.0);
    e.key.assign(3 * e.sizes[2] + 1, 0);
    e.blk.assign(3 * e.sizes[3] + 1, 0);
    e.off.assign(e.sizes[3] + 1, 0);
    e.data.assign(e.sizes[4] + 1, 0.0);
    // a capacity one short is refused with nothing written
    int64_t small[5] = {e.sizes[0], e.sizes[1] - 1, e.sizes[2], e.sizes[3], e.sizes[4]};
    CHECK(d2d_block_export(b, e.qn.data(), e.dim.data(), e.H.data(), e.key.data(), e.blk.data(), e.off.data(),
                           e.data.data(), small) == D2D_EINVAL, "export into a short buffer accepted");
    return d2d_block_export(b, e.qn.data(), e.dim.data(), e.H.data(), e.key.data(), e.blk.data(), e.off.data(),
                            e.data.data(), e.sizes) == D2D_OK;
}

static d2d_block_desc desc_of(const Exported& e, int side, int ncols) {
    d2d_block_desc d{};
    d.side = side;
    d.ncols = ncols;
    d.nsec = (int)e.sizes[0];
    d.sec_qn = e.qn.data();
    d.sec_dim = e.dim.data();
    d.H = e.H.data();
    d.nops = (int)e.sizes[2];
    d.op_key = e.key.data();
    d.nblk = (int)e.sizes[3];
    d.op_blk = e.blk.data();
    d.op_off = e.off.data();
    d.op_data = e.data.data();
    d.op_data_len = e.sizes[4];
    d.H_len = e.sizes[1];
    return d;
}

static void check_blocks() {
    d2d_ctx ctx;   // host-side bookkeeping only: block objects live on the host
    const d2d_model models[2] = {{D2D_HEISENBERG, 2, 1.0, 0.0, 1.0}, {D2D_HUBBARD, 2, 1.0, 4.0, 0.0}};
    for (const d2d_model& model : models)
        for (int side = 0; side < 2; ++side) {
            d2d_block* ex = nullptr;
            const int ncols = model.kind == D2D_HUBBARD ? 1 : 2;
            CHECK(d2d_block_exact(&ctx, &model, ncols, side, &ex) == D2D_OK && ex, "exact block: %s",
                  d2d_last_error());
            if (!ex) continue;
            Exported a, b;
            CHECK(export_block(ex, a), "export: %s", d2d_last_error());
            d2d_block_desc d = desc_of(a, side, ncols);
            d2d_block* im = nullptr;
            CHECK(d2d_block_import(&ctx, &model, &d, &im) == D2D_OK && im, "import: %s", d2d_last_error());
            if (im) {
                CHECK(export_block(im, b), "re-export: %s", d2d_last_error());
                CHECK(a.qn == b.qn && a.dim == b.dim && a.H == b.H && a.key == b.key && a.blk == b.blk &&
                          a.off == b.off && a.data == b.data,
                      "round trip differs");
                d2d_block_destroy(im);
            }
            // inconsistent descriptors are refused (and leave nothing behind)
            d2d_block* bad = nullptr;
            d2d_block_desc d1 = d;
            d1.op_data_len = d.op_data_len - 1;
            CHECK(d2d_block_import(&ctx, &model, &d1, &bad) != D2D_OK && !bad, "short op_data accepted");
            d1 = d;
            d1.H_len = d.H_len - 1;
            CHECK(d2d_block_import(&ctx, &model, &d1, &bad) != D2D_OK && !bad, "short H accepted");
            std::vector<int64_t> dim2 = a.dim;
            dim2[0] += 1;
            d1 = d;
            d1.sec_dim = dim2.data();
            CHECK(d2d_block_import(&ctx, &model, &d1, &bad) != D2D_OK && !bad, "sector size off by one accepted");
            if (a.sizes[3] > 0) {
                std::vector<int64_t> blk2 = a.blk;
                blk2[1] = a.sizes[0];   // a sector index past the last
                d1 = d;
                d1.op_blk = blk2.data();
                CHECK(d2d_block_import(&ctx, &model, &d1, &bad) != D2D_OK && !bad, "sector index past the end accepted");
                std::vector<int64_t> off2 = a.off;
                off2[0] = a.sizes[4];   // a block starting at the end of op_data
                d1 = d;
                d1.op_off = off2.data();
                CHECK(d2d_block_import(&ctx, &model, &d1, &bad) != D2D_OK && !bad, "offset past op_data accepted");
            }
            if (a.sizes[0] > 1) {
                std::vector<int64_t> qn2 = a.qn;
                std::swap(qn2[0], qn2[2]);   // sectors out of order
                std::swap(qn2[1], qn2[3]);
                d1 = d;
                d1.sec_qn = qn2.data();
                CHECK(d2d_block_import(&ctx, &model, &d1, &bad) != D2D_OK && !bad, "unsorted sectors accepted");
            }
            d2d_block_destroy(ex);
        }
    CHECK(ctx.children == 0, "children %d", ctx.children);
}

// ---------------------------------------------------------------- 4. tune cache
static void check_tune_cache() {
    char path[] = "/tmp/d2d_tune_cache_XXXXXX";
    const int fd = mkstemp(path);
    CHECK(fd >= 0, "mkstemp");
    if (fd < 0) return;
    FILE* f = fdopen(fd, "w");
    std::fprintf(f, "zz not a line\n12ab 4 0.5\n%llx %d 1.25\n", 0x1234abcdULL, 4 | D2D_TILE_SPLIT);
    std::fclose(f);
    setenv("D2D_TUNE_CACHE", path, 1);
    TileSel sel;
    int tile = 0;
    double ms = 0;
    // the reader stops at the malformed first line: nothing found, nothing read past it
    CHECK(!tune_cache_lookup(0x1234abcdULL, D2D_FP32, &sel, &tile, &ms), "malformed cache line accepted");
    tune_cache_store(0x77ULL, 4, 0.25);
    unsetenv("D2D_TUNE_CACHE");
    std::remove(path);
}

int main(int argc, char** argv) {
    mutate = argc > 1 && std::string(argv[1]) == "--mutate";
    check_tile_codes();
    check_work_lists();
    check_blocks();
    check_tune_cache();
    if (failures) {
        std::printf("%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
