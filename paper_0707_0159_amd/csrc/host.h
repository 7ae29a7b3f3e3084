// Host-side objects of libd2d (not part of the ABI).
#pragma once

#include <functional>
#include <map>
#include <memory>
#include <utility>

#include "internal.h"

namespace d2d {

typedef std::pair<int64_t, int64_t> QN;

// Dense column-major FP64 matrix on the host.
struct Mat {
    int rows = 0, cols = 0;
    std::vector<double> a;
    Mat() = default;
    Mat(int r, int c) : rows(r), cols(c), a((size_t)r * c, 0.0) {}
    double& operator()(int i, int j) { return a[(size_t)j * rows + i]; }
    double operator()(int i, int j) const { return a[(size_t)j * rows + i]; }
};

Mat mat_transpose(const Mat& x);
Mat mat_mul(const Mat& x, const Mat& y);
Mat mat_add(const Mat& x, const Mat& y, double cy = 1.0);
Mat mat_kron(const Mat& slow, const Mat& fast);
Mat mat_identity(int n);
Mat mat_scale_rows(const Mat& x, const std::vector<double>& d);   // diag(d) x
Mat mat_scale_cols(const Mat& x, const std::vector<double>& d);   // x diag(d)

// Operator name: (kind, leg, spin); kind 0 annihilator, 1 S^z, 2 S^+.
typedef std::array<int64_t, 3> OpKey;

// One column (rung of `legs` sites) in the occupation basis.
struct Column {
    int n = 0;
    std::vector<QN> qn;
    std::vector<double> parity;
    Mat H;
    std::vector<OpKey> keys;
    std::vector<Mat> ops;
    const Mat& op(const OpKey& k) const;
};
Column make_column(const d2d_model& m);
// the off-diagonal part of a column operator as matrices with at most one
// nonzero per row (their sum is the operator minus its diagonal)
std::vector<Mat> offdiagonal_pieces(const Mat& h);

// A bond term coef * (A on the part whose modes come first) (x) (B on the other).
struct BondTerm {
    double coef;
    Mat A, B;
};
// Leg bonds between part X (earlier modes; ops_x, parity px) and part Y.
std::vector<BondTerm> bond_terms(const d2d_model& model, const std::vector<OpKey>& keys_x,
                                 const std::vector<Mat>& ops_x, const std::vector<double>& px,
                                 const std::vector<OpKey>& keys_y, const std::vector<Mat>& ops_y);
std::vector<OpKey> edge_keys(const d2d_model& model);

}  // namespace d2d

// streams of the density-matrix eigensolver (created on first use)
struct EigLanes;
constexpr int EIG_LANES = 4;

struct d2d_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t mem_cap = 0;
    size_t bytes = 0;
    int children = 0;
    EigLanes* eig = nullptr;
    d2d_status alloc(void** p, size_t bytes);
    void free(void* p, size_t bytes);
};
void free_eig_lanes(d2d_ctx* ctx);

namespace d2d {
// One sector of a block's transformation: the enlarged half's basis states
// `rows` (half indices: column state * m_parent + parent state) onto the
// block's states col0 .. col0 + ncols - 1, dense column-major rows x ncols.
struct USector {
    std::vector<int32_t> rows;
    int col0 = 0, ncols = 0;
    std::vector<double> v;
};
// a fresh block id (never 0)
uint64_t new_block_id();
}  // namespace d2d

struct d2d_block {
    d2d_ctx* ctx = nullptr;
    d2d_model model{};
    int side = 0, ncols = 0, m = 0;
    // Lineage for the wavefunction transformation: the block was made from
    // the enlarged half (parent block + one column) by the transformation U;
    // parent 0 and no U for imported and exact blocks.
    uint64_t id = 0, parent = 0;
    int64_t u_dim = 0;                    // dimension of that enlarged half (0: no transformation)
    std::vector<d2d::USector> U;
    std::vector<d2d::QN> qn;           // per state, sorted
    std::vector<d2d::QN> sec_qn;
    std::vector<int64_t> sec_dim, sec_start;
    d2d::Mat H;
    std::vector<d2d::OpKey> keys;
    std::vector<d2d::Mat> ops;
    std::vector<double> parity() const;
};

// Workspace of a restarted Lanczos over a set of problems (vectors concatenated).
struct LanczosWork {
    int kmax = 0, nprob = 0, NB = 0;
    int64_t ntot = 0;
    std::vector<int64_t> seg_off, seg_len;
    int64_t ldq = 0;             // basis vector stride: ntot rounded up to 64 elements
    int64_t max_seg = 0;         // longest block segment of the step kernels
    double* Q = nullptr;         // (kmax+1) x ldq doubles (or as many FP32 / BF16 elements)
    double* X = nullptr;
    double* W = nullptr;
    float* wlo = nullptr;
    float* vlo = nullptr;        // FP32 input (BF16 uses it as uint16 storage)
    double* partial = nullptr;   // 2 x 34 x NB
    double* scal = nullptr;      // nprob x S_LEN
    double* res = nullptr;       // 2 x nprob
    double* res_host = nullptr;  // pinned copy of res
    d2d::LzSeg* bt = nullptr;
    std::vector<d2d::LzSeg> h_bt;   // host copy (its act flags follow the active set)
    int2* prange = nullptr;
    int* active = nullptr;
    // captured restarts, two per precision: index 2 prec + 0 for the full
    // cycle, 2 prec + 1 for a shortened one
    hipGraphExec_t exec[2 * D2D_NPREC] = {};
    hipGraph_t graph[2 * D2D_NPREC] = {};
    uint64_t graph_key[2 * D2D_NPREC] = {};   // what the capture was made for (see restart)
};

namespace d2d {
// Device tables of one grouped Hv launch sequence (one superblock or a batch).
struct HvTables {
    const SectorDev* sec;
    int npairs;
    void* x[3];               // partial outputs of split K-loops (ntot doubles each; null = unused)
    void* w2;                 // central-term output of a fused launch (ntot doubles; null = unfused)
    const void* HL[D2D_NPREC];
    const void* HR[D2D_NPREC];
    int64_t lo[4];            // BF16x3: elements from the hi to the lo parts of HL, HR, VP, VT
    const CentralUnit* cunits;   // central-term launch table
    int n_cunits;
    const CentralTerm* cterms;
    const int4* ptiles;
    int n_ptiles;
    bf16_t* vp;
    bf16_t* vt;
    int persist;              // persistent grouped launch (the work list's counters)
};
// Zero pattern of the sector operators in cells of NZ_CELL x NZ_CELL: for
// pair p, L[p] has ceil(dL/NZ_CELL)^2 bytes for the stored H_l (column-major,
// cell (i, j) at j * ceil(dL/NZ_CELL) + i, nonzero when any element is), R[p]
// likewise for the stored H_r^T.  Null pointers: treat as dense.
constexpr int NZ_CELL = 16;
struct NzCells {
    std::vector<const uint8_t*> L, R;
    // Row-exact patterns for the asymmetric split: rowL[p][r * cL + j] != 0
    // when row r of H_l[q_L] has a nonzero in columns [16 j, 16 j + 16);
    // colR[p][c * cR + j] likewise for column c of the stored H_r^T (rows
    // [16 j, 16 j + 16)); runsL[p] / runsR[p]: start of every run of rows
    // (columns) with one column state, then d_L (d_R).  Empty: not known.
    std::vector<const uint8_t*> rowL, colR;
    std::vector<const std::vector<int>*> runsL, runsR;
};
// A work list on the host: items, their K-step table, the flops it executes.
struct WorkHost {
    std::vector<WorkItem> items;
    std::vector<int32_t> ksteps;
    double flops = 0;
    int n0 = -1;   // asymmetric split: items [0, n0) in the lead shape, the rest in its partner
};
// A work list on the device.
struct WorkList {
    WorkItem* items = nullptr;
    int32_t* ksteps = nullptr;
    int n = 0, nsteps = 0;
    size_t cap_items = 0, cap_steps = 0;
    double flops = 0;   // GEMM flops of one launch over the list
    int n0 = -1;        // asymmetric split: items of the lead shape (the rest: its partner)
    int* ctr = nullptr; // persistent launches: two counters per launch (next item, groups done), zero between launches
};
// stages of one Hv launch sequence (a whole product is all three)
constexpr int HV_PACK = 1, HV_GEMM = 2, HV_CENTRAL = 4, HV_ALL = 7;
// pack (BF16) + grouped GEMM + central term, the stages selected
d2d_status hv_launch(const HvTables& t, int prec, int shape, const WorkList& wl, const void* v, void* w,
                     hipStream_t s, int stages = HV_ALL);

// Output of a fused Hv left in parts: the product is
// (((w + x0) + x1) + x2) + central, added in that order by the consumer (the
// x present depend on how the K-loops are split; central null when unfused).
struct HvParts {
    const void* x[3];
    const void* central;
};

// Hv of a set of problems on concatenated vectors (one superblock or a batch).
struct HvOps {
    virtual ~HvOps() = default;
    virtual d2d_status hv(int prec, const void* v, void* w, hipStream_t s) = 0;   // no counting
    // one launch for GEMMs and central term; the result stays in parts
    virtual d2d_status hv_fused(int prec, const void* v, void* w, hipStream_t s, HvParts* parts) = 0;
    virtual d2d_status prepare(int prec) = 0;                                      // before graph capture
    virtual d2d_status set_active(const std::vector<int>& active, bool* rebuilt) = 0;
    virtual bool has(int prec) = 0;
    virtual void count(int prec, int64_t n) = 0;
    virtual int64_t counter(int prec) = 0;
    // fingerprint of everything a captured launch sequence depends on beyond
    // the Lanczos workspace: launch configuration per precision, partial-output
    // buffers, work-list builds; a captured restart is replayed only while it holds
    virtual uint64_t fingerprint() = 0;
};
// FNV-1a over 64-bit words (launch-configuration fingerprints)
inline uint64_t fnv_mix(uint64_t h, uint64_t x) {
    for (int i = 0; i < 8; ++i) {
        h ^= (x >> (8 * i)) & 0xffu;
        h *= 0x100000001b3ull;
    }
    return h;
}
inline uint64_t config_fingerprint(const int* tile, const int* split, const int* fuse, const int* xcd,
                                   const int* dense, const int* persist, void* const* parts, const void* w2,
                                   uint64_t builds) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (int p = 0; p < D2D_NPREC; ++p) {
        h = fnv_mix(h, (uint64_t)(int64_t)tile[p]);
        h = fnv_mix(h, (uint64_t)split[p]);
        h = fnv_mix(h, (uint64_t)fuse[p]);
        h = fnv_mix(h, (uint64_t)xcd[p]);
        h = fnv_mix(h, (uint64_t)dense[p]);
        h = fnv_mix(h, (uint64_t)persist[p]);
    }
    for (int i = 0; i < 3; ++i) h = fnv_mix(h, (uint64_t)(uintptr_t)parts[i]);
    h = fnv_mix(h, (uint64_t)(uintptr_t)w2);
    return fnv_mix(h, builds);
}
}  // namespace d2d

struct d2d_sb {
    d2d_ctx* ctx = nullptr;
    d2d_model model{};
    int m = 0, n = 0;
    int64_t Q[2] = {0, 0};
    unsigned prec_mask = 0;
    std::vector<d2d::QN> qn1, qn4;     // block-state quantum numbers (block 1, block 4)
    int ncols1 = 0, ncols4 = 0;
    // the blocks' lineage and transformations (copies; see d2d_block)
    uint64_t id1 = 0, parent1 = 0, id4 = 0, parent4 = 0;
    int64_t u_dim1 = 0, u_dim4 = 0;
    std::vector<d2d::USector> U1, U4;
    // sector pairs
    std::vector<d2d::QN> pair_q;
    std::vector<d2d::SectorDev> pairs;
    std::vector<std::vector<int32_t>> rowsL, colsR;   // half indices per pair
    int64_t N = 0, Drows = 0, Dcols = 0;
    int max_dl = 0, max_dr = 0;
    int64_t hl_len = 0, hr_len = 0;
    double flops_exec = 0, flops_nnz = 0, flops_central = 0;
    // device tables
    d2d::SectorDev* d_sec = nullptr;
    void* HL[D2D_NPREC] = {nullptr, nullptr, nullptr, nullptr};
    void* HR[D2D_NPREC] = {nullptr, nullptr, nullptr, nullptr};
    int K = 0;                               // central bond terms
    int64_t max_elems = 0;
    // central term: work units and terms of every rectangle (host copies build batches)
    std::vector<d2d::CentralUnit> h_cunits;
    std::vector<d2d::CentralTerm> h_cterms;
    d2d::CentralUnit* d_cunits = nullptr;
    d2d::CentralTerm* d_cterms = nullptr;
    int32_t* d_rowsL = nullptr;              // [Drows] left half index of every packed row
    int32_t* d_colsR = nullptr;              // [Dcols] right half index of every packed column
    // BF16 operands and per-Hv padded copies of the input vector
    int64_t hl16_len = 0, hr16_len = 0, vp_len = 0, vt_len = 0;
    d2d::bf16_t* d_vp = nullptr;
    d2d::bf16_t* d_vt = nullptr;
    int vparts = 1;                    // 2 when VP / VT also hold BF16x3 lo parts
    int4* d_ptiles = nullptr;          // pack launch table (pair, 64-row tile, 64-column tile)
    int n_ptiles = 0;
    // work lists per tile shape
    std::map<int, d2d::WorkList> work;             // key: shape | split << 16 | xcd << 18 | dense << 19
    std::vector<std::vector<uint8_t>> nzL, nzR;    // zero pattern of each pair's operators (NzCells)
    std::vector<std::vector<uint8_t>> nzRowL, nzColR;   // row-exact patterns (NzCells::rowL, colR)
    std::vector<std::vector<int>> runsL, runsR;         // run starts (NzCells::runsL, runsR)
    int tile_sel[D2D_NPREC] = {-1, -1, -1, -1};   // shape index, or -1 = by size
    int split[D2D_NPREC] = {0, 0, 0, 0};          // 0 none, 1 two K-loops apart, 2 each K-loop halved too
    int fuse[D2D_NPREC] = {0, 1, 1, 1};           // inner Lanczos steps: central term inside the GEMM launch
    int xcd[D2D_NPREC] = {0, 0, 0, 0};            // XCD-aware work order
    int dense[D2D_NPREC] = {0, 0, 0, 0};          // 1: run every K step (no skipping of zero operator tiles)
    int persist[D2D_NPREC] = {0, 0, 0, 0};        // 1: persistent grouped launch (work items from a counter)
    void* d_x[3] = {nullptr, nullptr, nullptr};   // split-K partial outputs, N doubles each, on demand
    void* d_w2 = nullptr;               // N doubles, central-term part of fused launches
    int64_t hv_count[D2D_NPREC] = {0, 0, 0, 0};
    LanczosWork* lz = nullptr;          // owned; freed by free_lanczos
    ~d2d_sb();
};

namespace d2d {
d2d_status sb_hv(d2d_sb* sb, int prec, const void* v, void* w, hipStream_t s);
d2d_status sb_hv_nocount(d2d_sb* sb, int prec, const void* v, void* w, hipStream_t s);
void free_lanczos_work(d2d_ctx* c, LanczosWork*& lw);
d2d_status ensure_lanczos_work(d2d_ctx* c, LanczosWork*& lw, const std::vector<int64_t>& len, int kmax);
d2d_status check_lanczos_opts(const d2d_lanczos_opts* o);
d2d_status run_lanczos(d2d_ctx* ctx, LanczosWork*& lw, HvOps& hv, const d2d_lanczos_opts* opts,
                       const std::vector<int64_t>& len, const double* const* v0, double* energies,
                       double* const* psi, d2d_lanczos_stats* stats);
// Hv of a superblock; with parts non-null the launch is fused and the result
// is left in parts (see HvParts), else w holds the whole product.
d2d_status sb_hv_parts(d2d_sb* sb, int prec, const void* v, void* w, hipStream_t s, int stages = HV_ALL,
                       HvParts* parts = nullptr);
// partial outputs of a split level (and the central part) allocated on demand
d2d_status sb_ensure_parts(d2d_sb* sb, int split, bool central);
int sb_auto_tile(const d2d_sb* sb, int prec);
// a launch configuration: shape index (-1 = by size), K-loop split level, central
// term fused into the GEMM launch, XCD-aware order
struct TileSel {
    int shape = -1, split = 0, fuse = 0, xcd = 0, dense = 0, persist = 0;
};
// d2d_sb_set_tile's tile argument (shape | D2D_TILE_* flags, or -1) for precision
// prec; false when it names no shape of that precision or unknown flags
bool decode_tile(int prec, int tile, TileSel* out);
int encode_tile(const TileSel& t);
// Autotuner core: for every shape of precision prec x split level x fused x XCD
// order, run(c) once to warm up and reps times between HIP events on s; the
// fastest configuration and its average milliseconds per run.
d2d_status tune_configs(hipStream_t s, int prec, int reps, const std::function<d2d_status(const TileSel&)>& run,
                        TileSel* best, double* best_ms);
// D2D_TUNE_CACHE file (lines "key tile ms"): the first valid entry for key
bool tune_cache_lookup(uint64_t key, int prec, TileSel* sel, int* tile, double* ms);
void tune_cache_store(uint64_t key, int tile, double ms);
// work list of a launch configuration (built on first use)
d2d_status sb_work(d2d_sb* sb, int shape, int split, int xcd, int dense, const WorkList** wl);
// upload a host work list into wl (reusing its buffers when large enough)
d2d_status upload_work(d2d_ctx* ctx, const WorkHost& h, WorkList& wl);
void free_work(d2d_ctx* ctx, WorkList& wl);
// number of partial outputs of a split level (0 none, 1 two K-loops, 2 halves,
// 3 two K-loops in asymmetric tiles): 0, 1, 3, 1
inline int split_parts(int split) { return split == 0 ? 0 : (split == 2 ? 3 : 1); }
// work items of the pairs with keep[p] != 0 for a tile shape; split level 0:
// one item per output tile, 1: one per K-loop, 2: one per half K-loop
// xcd: the XCD-aware order (rectangles of each pair's tiles per XCD, interleaved, padded with p = -1)
// nz: zero pattern of the operators (K steps whose operator tile is zero are
// left out), or null for every step
// split 3: the V H_r^T items in shape ts1 (the partner of ts), after the H_l V
// items; with run boundaries in nz the items are run-aligned (see make_work);
// all_steps: every K step (the zero pattern then only places the runs)
void make_work(const std::vector<SectorDev>& pairs, const std::vector<int>* keep, const TileShape& ts, int split, int xcd,
               const NzCells* nz, WorkHost& out, const TileShape* ts1 = nullptr, bool all_steps = false);
void free_lanczos(d2d_sb* sb);
}  // namespace d2d
