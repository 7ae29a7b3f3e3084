// Errors, context, dense host matrices, columns and blocks of libd2d.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <numeric>

#include "host.h"

namespace d2d {

uint64_t new_block_id() {
    static std::atomic<uint64_t> next{1};
    return next.fetch_add(1);
}

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}

// ---------------------------------------------------------------- dense helpers
Mat mat_transpose(const Mat& x) {
    Mat y(x.cols, x.rows);
    for (int j = 0; j < x.cols; ++j)
        for (int i = 0; i < x.rows; ++i) y(j, i) = x(i, j);
    return y;
}

Mat mat_mul(const Mat& x, const Mat& y) {
    Mat z(x.rows, y.cols);
    for (int j = 0; j < y.cols; ++j)
        for (int k = 0; k < x.cols; ++k) {
            const double b = y(k, j);
            if (b == 0.0) continue;
            for (int i = 0; i < x.rows; ++i) z(i, j) += x(i, k) * b;
        }
    return z;
}

Mat mat_add(const Mat& x, const Mat& y, double cy) {
    Mat z = x;
    for (size_t i = 0; i < z.a.size(); ++i) z.a[i] += cy * y.a[i];
    return z;
}

// kron(slow, fast): index (i_slow * fast.rows + i_fast)
Mat mat_kron(const Mat& s, const Mat& f) {
    Mat z(s.rows * f.rows, s.cols * f.cols);
    for (int sj = 0; sj < s.cols; ++sj)
        for (int si = 0; si < s.rows; ++si) {
            const double v = s(si, sj);
            if (v == 0.0) continue;
            for (int fj = 0; fj < f.cols; ++fj)
                for (int fi = 0; fi < f.rows; ++fi) z(si * f.rows + fi, sj * f.cols + fj) = v * f(fi, fj);
        }
    return z;
}

Mat mat_identity(int n) {
    Mat z(n, n);
    for (int i = 0; i < n; ++i) z(i, i) = 1.0;
    return z;
}

Mat mat_scale_rows(const Mat& x, const std::vector<double>& d) {
    Mat z = x;
    for (int j = 0; j < x.cols; ++j)
        for (int i = 0; i < x.rows; ++i) z(i, j) *= d[i];
    return z;
}

Mat mat_scale_cols(const Mat& x, const std::vector<double>& d) {
    Mat z = x;
    for (int j = 0; j < x.cols; ++j)
        for (int i = 0; i < x.rows; ++i) z(i, j) *= d[j];
    return z;
}

// ---------------------------------------------------------------- columns
const Mat& Column::op(const OpKey& k) const {
    for (size_t i = 0; i < keys.size(); ++i)
        if (keys[i] == k) return ops[i];
    static Mat empty;
    return empty;
}

static int popc(uint64_t x) { return __builtin_popcountll(x); }

std::vector<OpKey> edge_keys(const d2d_model& model) {
    std::vector<OpKey> k;
    if (model.kind == D2D_HUBBARD) {
        for (int y = 0; y < model.legs; ++y)
            for (int s = 0; s < 2; ++s) k.push_back({0, y, s});
    } else {
        for (int y = 0; y < model.legs; ++y) k.push_back({1, y, 0});
        for (int y = 0; y < model.legs; ++y) k.push_back({2, y, 0});
    }
    std::sort(k.begin(), k.end());
    return k;
}

// Hubbard: mode j = 2y + sigma is bit j; a basis state is the product of
// creators in increasing mode order on the vacuum, so c_j carries
// (-1)^(number of occupied modes below j).  Heisenberg: bit y = spin up.
Column make_column(const d2d_model& model) {
    Column c;
    const int L = model.legs;
    if (model.kind == D2D_HUBBARD) {
        c.n = 1 << (2 * L);
        c.qn.resize(c.n);
        c.parity.resize(c.n);
        for (int b = 0; b < c.n; ++b) {
            int64_t up = 0, dn = 0;
            for (int y = 0; y < L; ++y) {
                up += (b >> (2 * y)) & 1;
                dn += (b >> (2 * y + 1)) & 1;
            }
            c.qn[b] = {up, dn};
            c.parity[b] = ((up + dn) & 1) ? -1.0 : 1.0;
        }
        c.keys = edge_keys(model);
        for (const auto& k : c.keys) {
            const int j = (int)(2 * k[1] + k[2]);
            Mat a(c.n, c.n);
            for (int b = 0; b < c.n; ++b) {
                if (!((b >> j) & 1)) continue;
                const double sign = (popc((uint64_t)b & ((1ull << j) - 1)) & 1) ? -1.0 : 1.0;
                a(b ^ (1 << j), b) = sign;
            }
            c.ops.push_back(a);
        }
        c.H = Mat(c.n, c.n);
        for (int y = 0; y + 1 < L; ++y)
            for (int s = 0; s < 2; ++s) {
                const Mat& a = c.op({0, y, s});
                const Mat& b = c.op({0, y + 1, s});
                Mat hop = mat_add(mat_mul(mat_transpose(a), b), mat_mul(mat_transpose(b), a));
                c.H = mat_add(c.H, hop, -model.t);
            }
        for (int b = 0; b < c.n; ++b) {
            int dbl = 0;
            for (int y = 0; y < L; ++y) dbl += ((b >> (2 * y)) & 1) & ((b >> (2 * y + 1)) & 1);
            c.H(b, b) += model.U * dbl;
        }
    } else {
        c.n = 1 << L;
        c.qn.resize(c.n);
        c.parity.assign(c.n, 1.0);
        for (int b = 0; b < c.n; ++b) c.qn[b] = {popc((uint64_t)b), 0};
        c.keys = edge_keys(model);
        for (const auto& k : c.keys) {
            const int y = (int)k[1];
            Mat a(c.n, c.n);
            for (int b = 0; b < c.n; ++b) {
                if (k[0] == 1) a(b, b) = ((b >> y) & 1) ? 0.5 : -0.5;
                else if (!((b >> y) & 1)) a(b | (1 << y), b) = 1.0;
            }
            c.ops.push_back(a);
        }
        c.H = Mat(c.n, c.n);
        for (int y = 0; y + 1 < L; ++y) {
            const Mat& z1 = c.op({1, y, 0});
            const Mat& z2 = c.op({1, y + 1, 0});
            const Mat& p1 = c.op({2, y, 0});
            const Mat& p2 = c.op({2, y + 1, 0});
            Mat t = mat_mul(z1, z2);
            Mat flip = mat_add(mat_mul(p1, mat_transpose(p2)), mat_mul(mat_transpose(p1), p2));
            t = mat_add(t, flip, 0.5);
            c.H = mat_add(c.H, t, model.J);
        }
    }
    return c;
}

static const Mat& find_op(const std::vector<OpKey>& keys, const std::vector<Mat>& ops, const OpKey& k) {
    for (size_t i = 0; i < keys.size(); ++i)
        if (keys[i] == k) return ops[i];
    static Mat empty;
    return empty;
}

// Hubbard: c_x^dag c_y = (c_x^dag P_X) (x) c_y and c_y^dag c_x = (P_X c_x) (x) c_y^dag, coefficient -t.
// Heisenberg: J [S^z S^z + (S^+ S^- + S^- S^+)/2].
// The column Hamiltonian's off-diagonal part (the terms between the
// column's own sites: rung hops, rung spin flips) as matrices with at most
// one nonzero per row.  They act on one column and leave the other and both
// blocks alone, so the product applies them as the central term's gathers
// (scaled copies of rectangles of V) instead of as diagonal lines inside the
// dense sector operators, where every such line fills whole 16 x 16 cells
// of the K-loop.
std::vector<Mat> offdiagonal_pieces(const Mat& h) {
    const int n = h.rows;
    std::vector<std::vector<std::pair<int, double>>> rows(n);
    size_t pieces = 0;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j)
            if (i != j && h(i, j) != 0.0) rows[i].push_back({j, h(i, j)});
        pieces = std::max(pieces, rows[i].size());
    }
    std::vector<Mat> out(pieces, Mat(n, n));
    for (int i = 0; i < n; ++i)
        for (size_t t = 0; t < rows[i].size(); ++t) out[t](i, rows[i][t].first) = rows[i][t].second;
    return out;
}

std::vector<BondTerm> bond_terms(const d2d_model& model, const std::vector<OpKey>& kx, const std::vector<Mat>& ox,
                                 const std::vector<double>& px, const std::vector<OpKey>& ky,
                                 const std::vector<Mat>& oy) {
    std::vector<BondTerm> t;
    if (model.kind == D2D_HUBBARD) {
        for (int y = 0; y < model.legs; ++y)
            for (int s = 0; s < 2; ++s) {
                const Mat& cx = find_op(kx, ox, {0, y, s});
                const Mat& cy = find_op(ky, oy, {0, y, s});
                t.push_back({-model.t, mat_scale_cols(mat_transpose(cx), px), cy});
                t.push_back({-model.t, mat_scale_rows(cx, px), mat_transpose(cy)});
            }
    } else {
        for (int y = 0; y < model.legs; ++y) {
            const Mat& zx = find_op(kx, ox, {1, y, 0});
            const Mat& zy = find_op(ky, oy, {1, y, 0});
            const Mat& sx = find_op(kx, ox, {2, y, 0});
            const Mat& sy = find_op(ky, oy, {2, y, 0});
            t.push_back({model.J, zx, zy});
            t.push_back({0.5 * model.J, sx, mat_transpose(sy)});
            t.push_back({0.5 * model.J, mat_transpose(sx), sy});
        }
    }
    return t;
}

}  // namespace d2d

using namespace d2d;

// ---------------------------------------------------------------- context
d2d_status d2d_ctx::alloc(void** p, size_t nbytes) {
    *p = nullptr;
    if (nbytes == 0) return D2D_OK;
    if (mem_cap && bytes + nbytes > mem_cap) {
        set_error("context memory cap of %zu bytes exceeded (%zu in use, %zu requested)", mem_cap, bytes, nbytes);
        return D2D_ENOMEM;
    }
    hipError_t e = hipMalloc(p, nbytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        set_error("hipMalloc(%zu) failed: %s", nbytes, hipGetErrorString(e));
        return D2D_ENOMEM;
    }
    bytes += nbytes;
    return D2D_OK;
}

void d2d_ctx::free(void* p, size_t nbytes) {
    if (!p) return;
    (void)hipFree(p);
    bytes -= nbytes;
}

extern "C" const char* d2d_last_error(void) { return g_err.c_str(); }

extern "C" const char* d2d_version(void) { return "libd2d 0.1 (gfx950)"; }

extern "C" d2d_status d2d_ctx_create(int device, void* hip_stream, size_t mem_cap, d2d_ctx** out) {
    if (!out) {
        set_error("d2d_ctx_create: out is NULL");
        return D2D_EINVAL;
    }
    *out = nullptr;
    int count = 0;
    D2D_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) {
        set_error("d2d_ctx_create: device %d out of range (%d devices)", device, count);
        return D2D_EINVAL;
    }
    D2D_HIP(hipSetDevice(device));
    auto* c = new d2d_ctx();
    c->device = device;
    c->mem_cap = mem_cap;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete c;
            set_error("hipStreamCreate failed: %s", hipGetErrorString(e));
            return D2D_EDEVICE;
        }
        c->own_stream = true;
    }
    *out = c;
    return D2D_OK;
}

extern "C" d2d_status d2d_ctx_destroy(d2d_ctx* ctx) {
    if (!ctx) return D2D_OK;
    if (ctx->children > 0) {
        set_error("d2d_ctx_destroy: %d live objects still use this context", ctx->children);
        return D2D_ESTATE;
    }
    // work the context queued (asynchronous products, copies) ends before the
    // context does: nothing of it may run on into the runtime's teardown
    const hipError_t e = hipStreamSynchronize(ctx->stream);
    free_eig_lanes(ctx);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    if (e != hipSuccess) {
        set_error("d2d_ctx_destroy: work queued on the context's stream failed: %s", hipGetErrorString(e));
        return D2D_EDEVICE;
    }
    return D2D_OK;
}

extern "C" d2d_status d2d_ctx_bytes(const d2d_ctx* ctx, size_t* bytes) {
    if (!ctx || !bytes) {
        set_error("d2d_ctx_bytes: NULL argument");
        return D2D_EINVAL;
    }
    *bytes = ctx->bytes;
    return D2D_OK;
}

// ---------------------------------------------------------------- blocks
std::vector<double> d2d_block::parity() const {
    std::vector<double> p(m);
    for (int i = 0; i < m; ++i) p[i] = ((qn[i].first + qn[i].second) & 1) ? -1.0 : 1.0;
    return p;
}

static d2d_status check_model(const d2d_model* model) {
    if (!model) {
        set_error("model is NULL");
        return D2D_EINVAL;
    }
    if (model->kind == D2D_HUBBARD) {
        if (model->legs < 1 || model->legs > 4) {
            set_error("Hubbard legs must be 1..4 (got %d)", model->legs);
            return D2D_EINVAL;
        }
    } else if (model->kind == D2D_HEISENBERG) {
        if (model->legs < 1 || model->legs > 8) {
            set_error("Heisenberg legs must be 1..8 (got %d)", model->legs);
            return D2D_EINVAL;
        }
    } else {
        set_error("unknown model kind %d", model->kind);
        return D2D_EINVAL;
    }
    if (!std::isfinite(model->t) || !std::isfinite(model->U) || !std::isfinite(model->J)) {
        set_error("model parameters must be finite");
        return D2D_EINVAL;
    }
    return D2D_OK;
}

// quantum-number change of an edge operator: annihilator lowers n_sigma, S^+ raises n_up
static QN op_shift(const OpKey& k) {
    if (k[0] == 0) return k[2] == 0 ? QN{-1, 0} : QN{0, -1};
    if (k[0] == 1) return {0, 0};
    return {1, 0};
}

static void finish_sectors(d2d_block* b) {
    b->sec_qn.clear();
    b->sec_dim.clear();
    b->sec_start.clear();
    for (int i = 0; i < b->m; ++i) {
        if (i == 0 || b->qn[i] != b->qn[i - 1]) {
            b->sec_qn.push_back(b->qn[i]);
            b->sec_dim.push_back(0);
            b->sec_start.push_back(i);
        }
        b->sec_dim.back()++;
    }
}

extern "C" d2d_status d2d_block_import(d2d_ctx* ctx, const d2d_model* model, const d2d_block_desc* d,
                                       d2d_block** out) {
    if (!ctx || !d || !out) {
        set_error("d2d_block_import: NULL argument");
        return D2D_EINVAL;
    }
    *out = nullptr;
    D2D_CHECK(check_model(model));
    if (d->side != 0 && d->side != 1) {
        set_error("block side must be 0 or 1");
        return D2D_EINVAL;
    }
    if (d->nsec < 1 || !d->sec_qn || !d->sec_dim || !d->H) {
        set_error("block needs at least one sector and its Hamiltonian");
        return D2D_EINVAL;
    }
    int64_t m = 0;
    for (int s = 0; s < d->nsec; ++s) {
        if (d->sec_dim[s] < 1) {
            set_error("sector %d has dimension %lld", s, (long long)d->sec_dim[s]);
            return D2D_EINVAL;
        }
        if (s > 0) {
            QN a{d->sec_qn[2 * (s - 1)], d->sec_qn[2 * (s - 1) + 1]}, b{d->sec_qn[2 * s], d->sec_qn[2 * s + 1]};
            if (!(a < b)) {
                set_error("sector quantum numbers must be strictly ascending (sector %d)", s);
                return D2D_EINVAL;
            }
        }
        if (model->kind == D2D_HEISENBERG && d->sec_qn[2 * s + 1] != 0) {
            set_error("Heisenberg sectors must have n_dn = 0");
            return D2D_EINVAL;
        }
        m += d->sec_dim[s];
    }
    if (m > 16384) {
        set_error("block of %lld states exceeds the supported 16384", (long long)m);
        return D2D_EINVAL;
    }
    int64_t hlen = 0;
    for (int s = 0; s < d->nsec; ++s) hlen += d->sec_dim[s] * d->sec_dim[s];
    if (d->H_len != hlen) {
        set_error("H holds %lld doubles, the sectors' blocks need %lld", (long long)d->H_len, (long long)hlen);
        return D2D_EINVAL;
    }
    auto b = std::make_unique<d2d_block>();
    b->ctx = ctx;
    b->id = new_block_id();
    b->model = *model;
    b->side = d->side;
    b->ncols = d->ncols;
    b->m = (int)m;
    for (int s = 0; s < d->nsec; ++s)
        for (int64_t i = 0; i < d->sec_dim[s]; ++i) b->qn.push_back({d->sec_qn[2 * s], d->sec_qn[2 * s + 1]});
    finish_sectors(b.get());
    b->H = Mat((int)m, (int)m);
    int64_t off = 0;
    for (int s = 0; s < d->nsec; ++s) {
        const int dd = (int)d->sec_dim[s];
        const int st = (int)b->sec_start[s];
        for (int j = 0; j < dd; ++j)
            for (int i = 0; i < dd; ++i) {
                const double v = d->H[off + (int64_t)j * dd + i];
                if (!std::isfinite(v)) {
                    set_error("block Hamiltonian has a non-finite entry");
                    return D2D_EINVAL;
                }
                b->H(st + i, st + j) = v;
            }
        off += (int64_t)dd * dd;
    }
    // edge operators
    const std::vector<OpKey> need = edge_keys(*model);
    if (d->nops < 0 || (d->nops > 0 && !d->op_key) || d->nblk < 0 ||
        (d->nblk > 0 && (!d->op_blk || !d->op_off || !d->op_data))) {
        set_error("bad edge operator arrays");
        return D2D_EINVAL;
    }
    std::vector<OpKey> keys;
    for (int o = 0; o < d->nops; ++o) keys.push_back({d->op_key[3 * o], d->op_key[3 * o + 1], d->op_key[3 * o + 2]});
    b->keys = need;
    b->ops.assign(need.size(), Mat((int)m, (int)m));
    std::vector<int> slot(keys.size(), -1);
    for (size_t o = 0; o < keys.size(); ++o)
        for (size_t q = 0; q < need.size(); ++q)
            if (keys[o] == need[q]) slot[o] = (int)q;
    for (const auto& k : need)
        if (std::find(keys.begin(), keys.end(), k) == keys.end()) {
            set_error("block lacks edge operator (%lld,%lld,%lld) of this model", (long long)k[0], (long long)k[1],
                      (long long)k[2]);
            return D2D_EINVAL;
        }
    for (int bl = 0; bl < d->nblk; ++bl) {
        const int64_t oi = d->op_blk[3 * bl], sf = d->op_blk[3 * bl + 1], st = d->op_blk[3 * bl + 2];
        if (oi < 0 || oi >= d->nops || sf < 0 || sf >= d->nsec || st < 0 || st >= d->nsec) {
            set_error("edge operator block %d out of range", bl);
            return D2D_EINVAL;
        }
        const int64_t df = d->sec_dim[sf], dt = d->sec_dim[st], o = d->op_off[bl];
        if (o < 0 || o + df * dt > d->op_data_len) {
            set_error("edge operator block %d overruns op_data", bl);
            return D2D_EINVAL;
        }
        if (slot[oi] < 0) continue;   // operator not used by this model
        const QN sh = op_shift(keys[oi]);
        const QN qf = b->sec_qn[sf], qt = b->sec_qn[st];
        if (qt.first - qf.first != sh.first || qt.second - qf.second != sh.second) {
            set_error("edge operator block %d connects sectors that the operator cannot connect", bl);
            return D2D_EINVAL;
        }
        Mat& M = b->ops[slot[oi]];
        for (int64_t j = 0; j < df; ++j)
            for (int64_t i = 0; i < dt; ++i) {
                const double v = d->op_data[o + j * dt + i];
                if (!std::isfinite(v)) {
                    set_error("edge operator has a non-finite entry");
                    return D2D_EINVAL;
                }
                M((int)(b->sec_start[st] + i), (int)(b->sec_start[sf] + j)) = v;
            }
    }
    ctx->children++;
    *out = b.release();
    return D2D_OK;
}

// Sort a freshly grown block by quantum number (stable) and record its sectors.
static void sort_block(d2d_block* b) {
    std::vector<int> order(b->m);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->qn[x] < b->qn[y]; });
    auto perm = [&](const Mat& x) {
        Mat y(b->m, b->m);
        for (int j = 0; j < b->m; ++j)
            for (int i = 0; i < b->m; ++i) y(i, j) = x(order[i], order[j]);
        return y;
    };
    b->H = perm(b->H);
    for (auto& o : b->ops) o = perm(o);
    std::vector<QN> q(b->m);
    for (int i = 0; i < b->m; ++i) q[i] = b->qn[order[i]];
    b->qn = q;
    finish_sectors(b);
}

extern "C" d2d_status d2d_block_exact(d2d_ctx* ctx, const d2d_model* model, int ncols, int side, d2d_block** out) {
    if (!ctx || !out) {
        set_error("d2d_block_exact: NULL argument");
        return D2D_EINVAL;
    }
    *out = nullptr;
    D2D_CHECK(check_model(model));
    if (side != 0 && side != 1) {
        set_error("side must be 0 or 1");
        return D2D_EINVAL;
    }
    const Column col = make_column(*model);
    double m = 1;
    for (int i = 0; i < ncols; ++i) m *= col.n;
    if (ncols < 1 || m > 4096) {
        set_error("exact block of %d columns has %g states (1..4096 supported)", ncols, m);
        return D2D_EINVAL;
    }
    auto b = std::make_unique<d2d_block>();
    b->ctx = ctx;
    b->id = new_block_id();
    b->model = *model;
    b->side = side;
    b->ncols = 1;
    b->m = col.n;
    b->qn = col.qn;
    b->H = col.H;
    b->keys = col.keys;
    b->ops = col.ops;
    sort_block(b.get());
    for (int c = 1; c < ncols; ++c) {
        const int mo = b->m, n = col.n;
        const Mat Im = mat_identity(mo), In = mat_identity(n);
        Mat H;
        std::vector<Mat> ops;
        std::vector<QN> qn((size_t)mo * n);
        if (side == 0) {
            // L' = L (x) column on index i_col*m + i_L
            H = mat_add(mat_kron(In, b->H), mat_kron(col.H, Im));
            for (auto& t : bond_terms(*model, b->keys, b->ops, b->parity(), col.keys, col.ops))
                H = mat_add(H, mat_kron(t.B, t.A), t.coef);
            const std::vector<double> pl = b->parity();
            Mat P(mo, mo);
            for (int i = 0; i < mo; ++i) P(i, i) = model->kind == D2D_HUBBARD ? pl[i] : 1.0;
            for (size_t o = 0; o < col.keys.size(); ++o) ops.push_back(mat_kron(col.ops[o], P));
        } else {
            // R' = column (x) R on index i_col*m + i_R; the new column's modes come first
            H = mat_add(mat_kron(col.H, Im), mat_kron(In, b->H));
            for (auto& t : bond_terms(*model, col.keys, col.ops, col.parity, b->keys, b->ops))
                H = mat_add(H, mat_kron(t.A, t.B), t.coef);
            for (size_t o = 0; o < col.keys.size(); ++o) ops.push_back(mat_kron(col.ops[o], Im));
        }
        for (int a = 0; a < n; ++a)
            for (int i = 0; i < mo; ++i)
                qn[(size_t)a * mo + i] = {col.qn[a].first + b->qn[i].first, col.qn[a].second + b->qn[i].second};
        b->m = mo * n;
        b->H = H;
        b->ops = ops;
        b->keys = col.keys;
        b->qn = qn;
        b->ncols = c + 1;
        sort_block(b.get());
    }
    ctx->children++;
    *out = b.release();
    return D2D_OK;
}

extern "C" d2d_status d2d_block_dims(const d2d_block* b, int* m, int* nsec) {
    if (!b || !m || !nsec) {
        set_error("d2d_block_dims: NULL argument");
        return D2D_EINVAL;
    }
    *m = b->m;
    *nsec = (int)b->sec_qn.size();
    return D2D_OK;
}

extern "C" d2d_status d2d_block_export(const d2d_block* b, int64_t* sec_qn, int64_t* sec_dim, double* H,
                                       int64_t* op_key, int64_t* op_blk, int64_t* op_off, double* op_data,
                                       int64_t sizes[5]) {
    if (!b || !sizes) {
        set_error("d2d_block_export: NULL argument");
        return D2D_EINVAL;
    }
    const int ns = (int)b->sec_qn.size();
    int64_t hlen = 0;
    for (int s = 0; s < ns; ++s) hlen += b->sec_dim[s] * b->sec_dim[s];
    // nonzero operator blocks
    struct Blk { int o, sf, st; };
    std::vector<Blk> blks;
    int64_t dlen = 0;
    for (size_t o = 0; o < b->ops.size(); ++o)
        for (int sf = 0; sf < ns; ++sf)
            for (int st = 0; st < ns; ++st) {
                bool nz = false;
                for (int64_t j = 0; j < b->sec_dim[sf] && !nz; ++j)
                    for (int64_t i = 0; i < b->sec_dim[st] && !nz; ++i)
                        nz = b->ops[o]((int)(b->sec_start[st] + i), (int)(b->sec_start[sf] + j)) != 0.0;
                if (nz) {
                    blks.push_back({(int)o, sf, st});
                    dlen += b->sec_dim[sf] * b->sec_dim[st];
                }
            }
    const int64_t need[5] = {ns, hlen, (int64_t)b->ops.size(), (int64_t)blks.size(), dlen};
    if (!H) {
        for (int i = 0; i < 5; ++i) sizes[i] = need[i];
        return D2D_OK;
    }
    for (int i = 0; i < 5; ++i)
        if (sizes[i] < need[i]) {
            set_error("d2d_block_export: buffer %d holds %lld, needs %lld", i, (long long)sizes[i], (long long)need[i]);
            return D2D_EINVAL;
        }
    if (!sec_qn || !sec_dim || !op_key || !op_blk || !op_off || !op_data) {
        set_error("d2d_block_export: NULL buffer");
        return D2D_EINVAL;
    }
    int64_t off = 0;
    for (int s = 0; s < ns; ++s) {
        sec_qn[2 * s] = b->sec_qn[s].first;
        sec_qn[2 * s + 1] = b->sec_qn[s].second;
        sec_dim[s] = b->sec_dim[s];
        const int64_t dd = b->sec_dim[s], st = b->sec_start[s];
        for (int64_t j = 0; j < dd; ++j)
            for (int64_t i = 0; i < dd; ++i) H[off + j * dd + i] = b->H((int)(st + i), (int)(st + j));
        off += dd * dd;
    }
    for (size_t o = 0; o < b->keys.size(); ++o)
        for (int c = 0; c < 3; ++c) op_key[3 * o + c] = b->keys[o][c];
    off = 0;
    for (size_t q = 0; q < blks.size(); ++q) {
        const Blk& x = blks[q];
        op_blk[3 * q] = x.o;
        op_blk[3 * q + 1] = x.sf;
        op_blk[3 * q + 2] = x.st;
        op_off[q] = off;
        const int64_t df = b->sec_dim[x.sf], dt = b->sec_dim[x.st];
        for (int64_t j = 0; j < df; ++j)
            for (int64_t i = 0; i < dt; ++i)
                op_data[off + j * dt + i] = b->ops[x.o]((int)(b->sec_start[x.st] + i), (int)(b->sec_start[x.sf] + j));
        off += df * dt;
    }
    for (int i = 0; i < 5; ++i) sizes[i] = need[i];
    return D2D_OK;
}

extern "C" d2d_status d2d_block_destroy(d2d_block* b) {
    if (!b) return D2D_OK;
    if (b->ctx) b->ctx->children--;
    delete b;
    return D2D_OK;
}
