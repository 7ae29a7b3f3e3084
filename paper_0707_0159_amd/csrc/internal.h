// Internal declarations of libd2d (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "d2d.h"

namespace d2d {

void set_error(const char* fmt, ...);

#define D2D_HIP(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            d2d::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),       \
                           __FILE__, __LINE__);                                         \
            return D2D_EDEVICE;                                                         \
        }                                                                               \
    } while (0)

#define D2D_CHECK(st)                          \
    do {                                       \
        d2d_status s_ = (st);                  \
        if (s_ != D2D_OK) return s_;           \
    } while (0)

typedef uint16_t bf16_t;   // bfloat16 bits

// ---------------------------------------------------------------- device tables
// One sector pair (q_L, Q - q_L) of the packed vector.
struct SectorDev {
    int32_t dL, dR;
    int64_t off;        // packed offset of the d_L x d_R block
    int64_t hl_off;     // offset of H_l[q_L] (d_L x d_L, column-major)
    int64_t hr_off;     // offset of H_r[Q - q_L] (d_R x d_R)
    int64_t row_base;   // first global row slot of this pair
    int64_t col_base;   // first global column slot
    // BF16 operands, K-major with leading dimensions padded to a multiple of 8
    int32_t dLp, dRp;   // padded d_L, d_R
    int64_t hl16_off;   // H_l row-major: dL rows of dLp (sum dLp*dL)
    int64_t hr16_off;   // H_r^T column-major: dR columns of dRp (sum dRp*dR)
    int64_t vp_off;     // V column-major, ld dLp (sum dLp*dR)
    int64_t vt_off;     // V^T column-major, ld dRp (sum dRp*dL)
};

// One output tile of the grouped GEMM: pair, tile row, tile column.
// part: bits 0-1 K-loops (0 both, 1 H_l V only, 2 V H_r^T only); bits 2-3
// output slot (0 W, s partial X[s-1]); bit 4 one half of the K-loop only,
// bit 5 which half; bit 6 (ITEM_ALIGNED) a run-aligned item of one K-loop:
// an H_l V item covers rows [tm, tm + kn[1]) (tm a row, not a tile index),
// a V H_r^T item columns [tn, tn + kn[0]); the unused K-loop's count holds
// the extent.
// ks[f], kn[f]: the K steps of K-loop f (0: H_l V, 1: V H_r^T) are the kn[f]
// step starts (multiples of BK, ascending) at ks[f] in the work list's step
// table: every step whose operator tile (the item's rows or columns x the
// step's BK columns of H_l or H_r) holds a nonzero, or every step.
struct WorkItem {
    int32_t p, tm, tn, part;
    int32_t ks[2], kn[2];
};
constexpr int ITEM_ALIGNED = 64;

// Tile shapes built into the library.
struct TileShape {
    int prec, BM, BN, BK;
    int PF = 1;   // K steps whose loads are in flight during a step's MFMAs
};
int tile_shape_count();
const TileShape& tile_shape(int i);
// the shape of the V H_r^T items when shape i leads an asymmetric split (the
// next entry of the table, i's transpose), or -1
int asym_partner(int i);

// ---------------------------------------------------------------- launchers
// Central term W += sum_k c_k A_k V B_k^T.  Every A_k (column 2) and B_k
// (column 3) has at most one nonzero per row, so on the rectangle of a pair
// block where the column-2 state i2 and the column-3 state i3 are fixed (a
// run of block-1 rows x a run of block-4 columns) each term is one scalar
// times the rectangle of a source pair block of the same shape.  The launch
// table lists, per rectangle, its terms (those with a nonzero coefficient;
// the terms that map the rectangle onto itself, such as S^z S^z, merged into
// one), and cuts the rectangle into work units of one wave.
// Unit: rows [ru, ru+nr) x columns [cu, cu+nc) of a rectangle whose element
// (r, c) is W[off + r + c * ldw]; its terms are terms[tofs .. tofs+nt).
struct CentralUnit {
    int64_t off;
    int32_t ldw;
    int32_t ru, nr, cu, nc;
    int32_t tofs, nt;
    int32_t p;        // sector pair (host bookkeeping)
};
// Term: coefficient times the source rectangle, element (r, c) at V[base + r + c * ld].
struct CentralTerm {
    int64_t base;
    int32_t ld, pad;
    double c64;
    float c32, pad2;
};
struct CentralArgs {
    const CentralUnit* units;  // [nunits]
    int nunits;
    const CentralTerm* terms;
    const void* V;
    void* W;
    const void* X[3];          // split-K partial outputs added into W first, in order (nullable)
};
// elements of a unit per lane (a unit has at most 64 * CENTRAL_CS elements)
constexpr int CENTRAL_CS = 8;
hipError_t launch_central(int prec, const CentralArgs& a, hipStream_t s);

// packed <-> full space (dir 0: dst packed from full src; dir 1: dst full from packed src)
hipError_t launch_full_pack(const SectorDev* sec, int npairs, int64_t max_elems, const int32_t* rows,
                            const int32_t* cols, int64_t D, int dir, const double* src, double* dst, hipStream_t s);

// Grouped GEMM W = H_l V + V H_r^T over a work list; split work items write
// their share of the K-loops to the partial outputs X (the product is
// ((W + X0) + X1) + X2, added by the central term).  With fuse set, the same
// launch also evaluates the central term into fuse->W (a separate output: the
// consumer adds the GEMM parts in order and then fuse->W).
struct HvGemmArgs {
    const WorkItem* work;
    int nwork;
    const int32_t* ksteps;     // K-step table of the work list
    const SectorDev* sec;
    const void* HL;
    const void* HR;
    const void* V;
    void* W;
    void* X[3];                // partial outputs of split work items (slot s -> X[s-1]; nullable)
    const CentralArgs* fuse;   // nullable
    int64_t lo[4];             // BF16x3: element offsets of the lo parts of HL, HR, VP, VT
    int* ctr;                  // non-null: persistent launch with these counters (next item, groups done),
                               // zero on entry and left zero by the launch
};
hipError_t launch_hv_gemm(int shape, const HvGemmArgs& a, hipStream_t s);
// BF16: HvGemmArgs.V is the padded copy VP, VT its padded transpose.
hipError_t launch_hv_gemm_bf16(int shape, const HvGemmArgs& a, const void* VT, hipStream_t s);
// VP / VT of a packed BF16 vector (padding stays as it was: zero).
hipError_t launch_pack_bf16(const int4* tiles, int ntiles, const SectorDev* sec, const bf16_t* v, bf16_t* vp,
                            bf16_t* vt, hipStream_t s);
// BF16 operator copies from the FP64 masters: HL (column-major dL x dL) ->
// row-major padded; HRt (column-major H_r^T) -> padded; two-step RNE rounding.
hipError_t launch_op_bf16(const int64_t* src_off, const int64_t* dst_off, const int32_t* d, const int32_t* dp,
                          int nsec, int transpose, int lo, const double* src, bf16_t* dst, int64_t max_d2,
                          hipStream_t s);
// BF16x3 copies (hi and lo parts) of a packed FP32 vector
hipError_t launch_pack_bf16x3(const int4* tiles, int ntiles, const SectorDev* sec, const float* v, bf16_t* vp,
                              bf16_t* vt, int64_t lo_vp, int64_t lo_vt, hipStream_t s);



// Assembly of dense half Hamiltonian sectors on the device:
// out[s](r,c) = d(a,a') F0(b,b') + S0(a,a') d(b,b') + sum_t coef_t S_t(a,a') F_t(b,b')
// with half index h = a*m + b (a: column state, b: block state).
struct AssembleArgs {
    int nsec;
    const int64_t* rows_off;   // [nsec+1] into rows
    const int32_t* rows;       // half indices
    const int64_t* out_off;    // [nsec]
    int m, n, T;
    const double* F0;          // m x m
    const double* S0;          // n x n
    const double* S;           // T x n x n
    const double* F;           // T x m x m
    const double* coef;        // T
    double* out;
    int64_t max_d2;
    int transpose;             // 1: store the transposed block
};
hipError_t launch_assemble(const AssembleArgs& a, hipStream_t s);

hipError_t launch_cast_f64_f32(const double* x, float* y, int64_t n, hipStream_t s);
hipError_t launch_cast_f64_bf16(const double* x, bf16_t* y, int64_t n, hipStream_t s);
hipError_t launch_cast_f32_bf16(const float* x, bf16_t* y, int64_t n, hipStream_t s);
hipError_t launch_fill(void* x, int prec, int64_t n, double v, hipStream_t s);
// reads the (nullable) parts[0..4) of a fused product (FP64 for FP64, else FP32)
hipError_t launch_read_parts(const void* const* parts, int prec, int64_t n, void* sink, hipStream_t s);

// ---------------------------------------------------------------- Lanczos kernels

// ------------------------------------------------------------------ Lanczos sets
// Scalar layout per problem (doubles), at scal + prob * S_LEN.
constexpr int S_ALPHA = 0, S_BETA = 130, S_THETA = 524, S_Y = 528, S_LEN = 660;

// Block of a segmented kernel: problem, its block range [pb0, pb1), chunk [lo, hi).
struct LzSeg {
    int prob, pb0, pb1;
    int act;     // the problem is still iterating (kept equal to the active flags)
    int64_t lo, hi;
};

// A set of problems whose vectors are concatenated (offsets in the block table).
struct LzSet {
    int nprob;
    int NB;                 // blocks of the segmented kernels
    int64_t ntot;           // total vector length (leading dimension of Q)
    const LzSeg* bt;        // [NB]
    const int2* prange;     // [nprob] block range of each problem
    const int* active;      // [nprob] 1 while the problem iterates
    double* partial;        // two partial-sum buffers of 33 x NB
    double* partial2;
    double* scal;           // [nprob * S_LEN]
    double* res;            // [3 nprob] (theta, rho) of the last residual per problem, then the
                            // Ritz residual estimate of the last inner Lanczos per problem
};

// Lanczos step i (nq = i+1 <= 32): c1 = Q^T w (w upcast from w32 first if
// upcast), w -= Q c1, c2 = Q^T w, alpha_i = c1[i] + c2[i],
// beta_{i+1} = sqrt(|w|^2 - |c2|^2), and if qnext != null:
// qnext = (w - [need2] Q c2) / beta_{i+1}, lo = cast(qnext).  The basis Q
// (and qnext) has qbytes per element: FP64 (8), FP32 (4) or BF16 (2; the
// narrow ones with upcast only); the arithmetic is FP64 either way.
struct LzStepArgs {
    const LzSeg* bt;
    const void* Q;
    int64_t ldq;
    int nq, i;
    bool upcast;
    int qbytes;
    bool coop;              // the Gram step as one cooperative kernel (caller checked lz_coop_fits
                            // and that no segment exceeds lz_coop_segment_max)
    bool gram;              // two-kernel Gram form of the step (nq <= 4)
    const float* w32;
    double* w;
    // parts of a fused Hv: the product is (((w32 or w) + P0) + P1) + P2 + P3
    // in the Hv's own precision (FP32 when upcast, else FP64); each nullable
    const void* wpart[4];
    double* partial;
    double* partial2;
    int NB;
    double* scal;
    void* qnext;
    void* lo;
    int lo_prec;
};
int lz_step_blocks(int64_t n);
// the one-kernel Gram step: elements of a block's segment it can hold, and
// whether a grid of NB blocks of its kernel fits the device at once
int lz_coop_segment_max();
bool lz_coop_fits(int NB, bool upcast, int qbytes);
// x[i] = N(0,1) sample i of the SplitMix64 stream seeded with seed (Box-Muller)
hipError_t launch_seeded_normal(double* x, int64_t n, uint64_t seed, hipStream_t s);
hipError_t launch_lz_step(const LzStepArgs& a, hipStream_t s);
// theta = x.w, w -= theta x, rho = |w|; alpha_0 = theta, beta_1 = rho, res = (theta, rho)
hipError_t launch_lz_residual(const LzSet& z, const double* x, double* w, hipStream_t s);
// x = (y_0 x + sum_{j>=1} y_j Q[j]) / |.| per problem (Q: qbytes per element, vectors ldq apart)
hipError_t launch_lz_ritz(const LzSet& z, const void* Q, int qbytes, int64_t ldq, int k, double* x,
                          hipStream_t s);
// x = v / |v| per problem
hipError_t launch_lz_normalize_into(const LzSet& z, const double* v, double* x, hipStream_t s);
// res[2p] = |v_p|^2
hipError_t launch_lz_norms(const LzSet& z, const double* v, hipStream_t s);
// Q[0] = x, Q[1] = w / beta_1 (qbytes per element, ldq apart), lo = cast(Q[1])
hipError_t launch_lz_first(const LzSet& z, const double* x, const double* w, void* Q, int qbytes, int64_t ldq,
                           void* lo, int lo_prec, hipStream_t s);
// lowest eigenpair of each problem's k x k tridiagonal (theta at S_THETA+1, y at S_Y)
hipError_t launch_lz_tridiag(const LzSet& z, int k, hipStream_t s);

// Column densities (kernels_dmrg.hip): per column 2 and 3, DENS_SLOTS - 1
// occupation-bit sums and the total weight of psi^2; gx blocks per pair, sums
// in partial[(p * gx + x) * 2 * DENS_SLOTS + slot]
constexpr int DENS_SLOTS = 9;
hipError_t launch_col_dens(const SectorDev* sec, int npairs, int gx, const int32_t* rowsL, const int32_t* colsR, int m,
                           int nbits, const double* psi, double* partial, hipStream_t s);

// Grouped FP64 GEMM on the matrix cores: C = op(A) op(B), column-major, one
// 64 x 64 tile per work-group; tiles[i] = (problem, tile row, tile column, 0)
struct GemmProb {
    const double* A;
    const double* B;
    double* C;
    int M, N, K, lda, ldb, ldc;
    int ta, tb;   // 1: the operand is used transposed
};
hipError_t launch_gemm_f64(const GemmProb* probs, const int4* tiles, int ntiles, hipStream_t s);
// kept density-matrix eigenvectors: sel[j] = (rows, source column, offsets index, 0),
// offs[2i] source matrix offset in Z, offs[2i+1] destination of the column in U
hipError_t launch_pick_columns(const int4* sel, int ncols, const int64_t* offs, const double* Z, double* U,
                               hipStream_t s);
// G = O U_from row gathers: ent[e] = (rows, columns, offsets index, U_from leading dim)
hipError_t launch_gather_rows(const int4* ent, int nent, int64_t maxn, const int64_t* offs, const int32_t* src,
                              const double* val, const double* U, double* G, hipStream_t s);

}  // namespace d2d
