/*
 * d2d.h -- C ABI of libd2d, the MI355X (gfx950) superblock Hamiltonian-vector
 * product of the direct two-dimensional DMRG and the Lanczos ground-state
 * solve built on it.
 *
 * The method (Yamada, Okumura, Machida, "Direct Extension of DMRG toward
 * 2-Dimensional Quantum Lattice Systems"): a superblock of four blocks, left
 * to right block 1 (m states, index i1), column 2 (n states, i2), column 3
 * (n states, i3) and block 4 (m states, i4), Fig. 2.  Its Hamiltonian splits
 * as in Eq. (1) into H_l on (i1,i2), H_r on (i3,i4) and H_c on (i2,i3).  The
 * superblock vector, reshaped into the matrix V with row (i2-1)m+i1 and
 * column (i3-1)m+i4, turns Hv into H_l V + V H_r^T + (central term), the
 * matrix form given right after Eq. (1).  The central term is applied as
 * sum_k A_k V B_k^T with A_k acting on column 2 and B_k on column 3 (the same
 * operator as the paper's H_c V_c).  Every term is split into quantum-number
 * sectors: (N_up, N_dn) for the Hubbard model, N_up (i.e. S_z) for the
 * Heisenberg model.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns a d2d_status; nothing aborts or throws across the ABI.
 *   d2d_last_error() returns a thread-local message for the last failure.
 * - "host" pointers are read during the call only and copied when kept.
 *   "device" pointers must point to memory of the context's device; they are
 *   borrowed for the duration of the call and work is ordered on the
 *   context's stream.  The library keeps no caller pointer after a return.
 * - Every *_create has a matching *_destroy owned by the caller.  Objects may
 *   be destroyed in any order except that a context must outlive everything
 *   made from it; d2d_ctx_destroy() with live children returns D2D_ESTATE and
 *   destroys nothing.
 * - Quantum numbers are int64 pairs (n_up, n_dn); for the Heisenberg model
 *   n_dn is 0 and n_up counts up spins.
 *
 * Packed superblock-vector layout (used by d2d_hv, d2d_lanczos, ...)
 * -----------------------------------------------------------------
 * For a target total quantum number Q the vector is block sparse: nonzero only
 * where q(i1)+q(i2) = q_L and q(i3)+q(i4) = Q - q_L.  The packed vector lists
 * the sector pairs in ascending q_L (lexicographic (n_up, n_dn)), each pair as
 * a dense d_L x d_R column-major block.  Rows are the left-half states with
 * quantum number q_L in ascending i2*m + i1 (i2 slow, i1 fast); columns are the
 * right-half states with Q - q_L in ascending i3*m + i4 (i3 slow, i4 fast).
 * This is the paper's element ((i2-1)m+i1, (i3-1)m+i4) of V restricted to the
 * sector.  Block states are ordered by quantum number (each sector a
 * contiguous range), column states by their occupation bits.
 */
#ifndef D2D_H
#define D2D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int d2d_status;
#define D2D_OK       0
#define D2D_EINVAL  -1   /* bad argument: null pointer, size, empty target, a
                            non-finite block entry or model parameter, a zero
                            or non-finite Lanczos start vector               */
#define D2D_ENOMEM  -2   /* device allocation failed or context memory cap hit */
#define D2D_EDEVICE -3   /* HIP runtime error                                  */
#define D2D_ENOCONV -4   /* Lanczos did not reach the tolerance                */
#define D2D_ESTATE  -5   /* object in the wrong state (live children, ...)     */

/* Precision of one Hv.  Inputs v: double / float / bfloat16 (uint16 bits) /
 * float; output w: double for D2D_FP64, float otherwise.  Products accumulate
 * in the output precision (FP32 accumulation for BF16 inputs).  D2D_BF16X3
 * splits every FP32 operand x into bf16 parts hi = bf16(x), lo = bf16(x - hi)
 * and forms hi*hi + hi*lo + lo*hi on the BF16 matrix cores (the dropped lo*lo
 * is about 2^-16 of a product): near-FP32 accuracy at BF16 matrix-core rate. */
#define D2D_FP64 0
#define D2D_FP32 1
#define D2D_BF16 2
#define D2D_BF16X3 3
#define D2D_NPREC 4

#define D2D_HEISENBERG 0
#define D2D_HUBBARD    1

typedef struct d2d_ctx d2d_ctx;
typedef struct d2d_block d2d_block;
typedef struct d2d_sb d2d_sb;
typedef struct d2d_batch d2d_batch;

/* Model of the ladder.  Hubbard: -t on every nearest-neighbour bond, +U n_up
 * n_dn on every site.  Heisenberg: J (S^z S^z + (S^+S^- + S^-S^+)/2) on every
 * bond (J_z = J_xy, as in the paper's spin model).  legs = sites per column. */
typedef struct {
    int kind;          /* D2D_HEISENBERG or D2D_HUBBARD */
    int legs;          /* 1..4 for Hubbard (column dim 4^legs), 1..8 Heisenberg */
    double t, U, J;
} d2d_model;

/* Last error message of the calling thread ("" if none). */
const char* d2d_last_error(void);

/* Version string of the library. */
const char* d2d_version(void);

/* ------------------------------------------------------------------ context
 * device     HIP device ordinal.
 * hip_stream hipStream_t to order all work on (NULL = the null stream).
 * mem_cap    upper bound in bytes on what the context allocates (0 = none);
 *            an allocation beyond it fails with D2D_ENOMEM. */
d2d_status d2d_ctx_create(int device, void* hip_stream, size_t mem_cap, d2d_ctx** out);
d2d_status d2d_ctx_destroy(d2d_ctx* ctx);
/* Bytes currently allocated by the context. */
d2d_status d2d_ctx_bytes(const d2d_ctx* ctx, size_t* bytes);

/* ------------------------------------------------------------------- blocks
 * A block (Fig. 1a: block 1 or block 4) of m states, all host FP64 arrays,
 * copied by d2d_block_import.  Layout:
 *   sec_qn[2*nsec], sec_dim[nsec]: sectors in ascending (n_up, n_dn).
 *   H: block Hamiltonian, per sector one dense column-major d x d block.
 *   op_key[3*nops]: edge-column operators that enter bonds with the next
 *     column: (0, y, sigma) annihilator c_{y,sigma} with the Jordan-Wigner
 *     string over the block's own earlier modes folded in (mode order: columns
 *     left to right, inside a column leg by leg, up before down);
 *     (1, y, 0) S^z_y; (2, y, 0) S^+_y.
 *   op_blk[3*nblk] = (op index, sector from, sector to), op_off[nblk] offsets
 *     into op_data of dense column-major d_to x d_from blocks.
 *   side: 0 = left block (block 1, edge = rightmost column), 1 = right block
 *     (block 4, edge = leftmost column). */
typedef struct {
    int side;
    int ncols;
    int nsec;
    const int64_t* sec_qn;
    const int64_t* sec_dim;
    const double* H;
    int nops;
    const int64_t* op_key;
    int nblk;
    const int64_t* op_blk;
    const int64_t* op_off;
    const double* op_data;
    int64_t op_data_len;   /* number of doubles in op_data (bounds check) */
    int64_t H_len;         /* number of doubles in H: the sum of sec_dim[s]^2 (bounds check) */
} d2d_block_desc;

d2d_status d2d_block_import(d2d_ctx* ctx, const d2d_model* model, const d2d_block_desc* desc,
                            d2d_block** out);
/* Exact block of ncols columns grown by Kronecker products (Fig. 1a), no
 * truncation: m = (column dim)^ncols.  side as in d2d_block_desc. */
d2d_status d2d_block_exact(d2d_ctx* ctx, const d2d_model* model, int ncols, int side,
                           d2d_block** out);
/* Number of states and sectors of a block. */
d2d_status d2d_block_dims(const d2d_block* b, int* m, int* nsec);
/* Copy a block out in the d2d_block_desc layout (host buffers owned by the
 * caller; sec_qn holds 2 entries per sector, op_key 3 per operator, op_blk 3
 * per nonzero operator block).  sizes[5] = (number of sectors, length of H,
 * number of operators, number of nonzero operator blocks, length of
 * op_data).  With H == NULL the call only writes the needed sizes into sizes
 * (size query); otherwise sizes holds the capacities of the caller's
 * buffers, and a capacity below the need returns D2D_EINVAL with nothing
 * written. */
d2d_status d2d_block_export(const d2d_block* b, int64_t* sec_qn, int64_t* sec_dim, double* H,
                            int64_t* op_key, int64_t* op_blk, int64_t* op_off, double* op_data,
                            int64_t sizes[5] /* out: nsec, H len, nops, nblk, op_data len */);
d2d_status d2d_block_destroy(d2d_block* b);

/* --------------------------------------------------------------- superblock
 * Superblock block1 (x) column (x) column (x) block4 restricted to the target
 * quantum number target_q[2] (Eq. (1)).  Both blocks must be of the model
 * given and of equal size m (the index maps of the paper assume it).  The
 * superblock copies what it needs; the blocks may be destroyed afterwards.
 * prec_mask: bits (1<<D2D_FP64 | 1<<D2D_FP32 | 1<<D2D_BF16 | 1<<D2D_BF16X3) of
 * the precisions whose operator copies are kept on the device.  Fails with D2D_EINVAL when
 * the target space is empty. */
d2d_status d2d_sb_create(d2d_ctx* ctx, const d2d_block* b1, const d2d_block* b4,
                         const d2d_model* model, const int64_t target_q[2], unsigned prec_mask,
                         d2d_sb** out);
d2d_status d2d_sb_destroy(d2d_sb* sb);

typedef struct {
    int64_t n;              /* packed vector length N_sb                         */
    int32_t npairs;         /* sector pairs                                      */
    int32_t m, ncol;        /* block and column dimension                        */
    int32_t nterms;         /* central terms K                                   */
    int32_t max_dl, max_dr; /* largest sector dimensions                        */
    double flops_exec;      /* dense-sector flops of one Hv: sum 2dL^2dR+2dLdR^2 */
    double flops_nnz;       /* same with the nonzeros of H_l, H_r sectors        */
    double flops_central;   /* 2 x nonzero central gathers                       */
    double bytes_min_fp64;  /* minimal HBM bytes of one FP64 Hv                  */
    double bytes_min_fp32;  /* same, FP32 operators and vectors                  */
    double bytes_min_bf16;  /* same, BF16 operators and inputs, FP32 output      */
    int64_t op_entries;     /* sum dL^2 + sum dR^2                               */
    double bytes_min_bf16x3; /* same, hi and lo BF16 operators, FP32 input/output */
} d2d_sb_info_t;

d2d_status d2d_sb_info(const d2d_sb* sb, d2d_sb_info_t* info);
/* Sector table in packed order: qL[2*npairs], dL[npairs], dR[npairs],
 * offset[npairs] (host buffers of npairs entries). */
d2d_status d2d_sb_sectors(const d2d_sb* sb, int64_t* qL, int64_t* dL, int64_t* dR, int64_t* offset);

/* Conversion between the packed sector layout (length n) and the full
 * superblock space of Eq. (1) (length D^2, D = m*ncol), whose element
 * (i1, i2, i3, i4) (block 1, column 2, column 3, block 4 states) sits at
 * (i2*m + i1) + D*(i3*m + i4), i.e. the superblock vector in the paper's
 * index order, or the column-major D x D matrix V.  Device FP64 buffers,
 * asynchronous on the context stream.  d2d_pack keeps the target-sector
 * elements of full; d2d_unpack writes every element of full (zero outside the
 * target sector).  Buffers must not overlap. */
d2d_status d2d_pack(d2d_sb* sb, const double* full, double* packed);
d2d_status d2d_unpack(d2d_sb* sb, const double* packed, double* full);

/* --------------------------------------------------------------------- Hv
 * w = H v in the packed layout, on the context stream, asynchronous.
 * prec D2D_FP64: v, w double.  D2D_FP32: v float, w float.  D2D_BF16: v
 * bfloat16 (uint16 storage), w float.  v and w must not overlap.  The entries
 * of v are not inspected (the call does not wait for the device): non-finite
 * entries give non-finite products, as in a BLAS routine. */
d2d_status d2d_hv(d2d_sb* sb, int prec, const void* v, void* w);

/* Hv for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * product as d2d_hv, bit for bit (same kernels, same launch configuration),
 * with the partial outputs of split K-loops (see D2D_TILE_SPLIT) in a
 * file-scope device array of D2D_NOALLOC_SCRATCH_BYTES that every GPU the
 * library runs on holds until the process ends, instead of buffers the
 * superblock allocates on first use.  The call allocates nothing and does not
 * wait for the device.  Requirements:
 *   - the grouped-GEMM work list of prec's current launch configuration is
 *     built: d2d_sb_create builds the default configuration's, d2d_sb_set_tile
 *     and d2d_sb_autotune the one they select; otherwise D2D_ESTATE;
 *   - (partial outputs of the split level: 0, 1 or 3) x n x (8 bytes for
 *     D2D_FP64, else 4) <= D2D_NOALLOC_SCRATCH_BYTES; otherwise D2D_EINVAL.
 * Arguments and errors otherwise as d2d_hv.  All calls on one GPU share the
 * array, whose contents stay from the last call (every element a call reads
 * it writes first): calls that overlap on one GPU (several streams or
 * threads) race. */
#define D2D_NOALLOC_SCRATCH_BYTES (64u << 20)
d2d_status d2d_hv_noalloc(d2d_sb* sb, int prec, const void* v, void* w);

/* Kernel timing of Hv on the context stream: after one product, `reps`
 * grouped-GEMM launches back to back and then `reps` central-term launches
 * back to back, each group between two HIP events; returns the average
 * duration in milliseconds of one grouped-GEMM launch (ms_gemm; for BF16 the
 * pack kernel that precedes it is not included) and of one central-term
 * launch (ms_central).  A last product leaves w = H v.  Synchronous. */
d2d_status d2d_hv_profile(d2d_sb* sb, int prec, const void* v, void* w, int reps, double* ms_gemm,
                          double* ms_central);

/* Number of Hv launches the superblock has issued per precision (counters). */
d2d_status d2d_hv_count(const d2d_sb* sb, int64_t counts[D2D_NPREC]);

/* Tile shape of the grouped-GEMM launch used for one precision: index into
 * the library's table of tile shapes (see d2d_tile_shapes), or -1 to let the
 * library choose by problem size.  OR-ing D2D_TILE_SPLIT runs the two K-loops
 * of every output tile (H_l V and V H_r^T) as separate work items into two
 * partial outputs, which the central-term launch adds (shorter critical path
 * for small, latency-bound sectors); D2D_TILE_SPLIT4 also halves each K-loop
 * (four work items and four partial outputs per tile, added in a fixed order,
 * so results stay deterministic).  D2D_TILE_XCD orders the work items so that
 * each of the 8 XCDs (work-groups go to them round-robin, each has its own L2)
 * works on one rectangle of every sector's tiles, cutting L2 misses on large
 * sectors.  OR-ing D2D_TILE_FUSED makes the inner
 * Lanczos steps evaluate the central term inside the grouped-GEMM launch (its
 * tiles as extra blocks after the GEMM work items, into an output of its own
 * that the first vector kernel of the step adds: same result bit for bit, one
 * launch less, the central term overlapping the GEMM's tail); d2d_hv always
 * returns the whole product.  Without a call (or after tile -1) FP32 and BF16
 * are fused, FP64 is not.  A K-loop leaves out every K step whose operator
 * tile (the output tile's rows of H_l[q_L], or its columns of H_r[q_R], times
 * the step's BK columns) is zero: the sector operators are block sparse (a
 * row run of column state i2 couples only to the runs of the column states
 * that the column's Hamiltonian and bond operators reach), and a left-out
 * step would add exact zeros.  D2D_TILE_DENSE runs every step instead (the
 * same result bit for bit, except with D2D_TILE_SPLIT4, whose halves are cut
 * in the list of steps run).  Returns D2D_EINVAL for an index out of range,
 * a shape not built for that precision or an unknown flag. */
#define D2D_TILE_SPLIT (1 << 16)
#define D2D_TILE_FUSED (1 << 17)
#define D2D_TILE_SPLIT4 (1 << 18)
#define D2D_TILE_XCD (1 << 19)
#define D2D_TILE_DENSE (1 << 20)
/* D2D_TILE_ASYM: the two K-loops as separate work items in two launches,
 * each in a tile that is narrow along the dimension its K-step list depends
 * on and wide along the other: H_l V items in the shape given (e.g. 64 rows x
 * 256 columns: the step list follows the 64 rows of H_l, the 256 columns
 * share it), V H_r^T items in the next shape of the table, its transpose
 * (256 x 64).  Valid only for shapes whose next entry is their transpose;
 * one partial output, added as with D2D_TILE_SPLIT. */
#define D2D_TILE_ASYM (1 << 21)
/* D2D_TILE_PERSIST: a persistent grouped launch.  The grid holds only the
 * work-groups the device runs at once (occupancy per compute unit times the
 * compute units); each takes work items, longest K-loop first, from a device
 * counter kept with the work list until none is left, and the last to finish
 * clears the counter, so consecutive launches (and launches replayed from a
 * captured graph) need no reset.  The same items and the same arithmetic per
 * item as the plain launch: the result is identical bit for bit.  Launches
 * of one superblock (or batch) on streams that overlap share the counter and
 * must not run at the same time.  Not with D2D_TILE_XCD (an XCD order steers
 * work-groups by index, which a persistent launch does not use). */
#define D2D_TILE_PERSIST (1 << 22)
d2d_status d2d_sb_set_tile(d2d_sb* sb, int prec, int tile);
/* Floating-point operations of one grouped-GEMM launch of precision prec
 * under the superblock's current launch configuration: 2 per multiply-add
 * over the K steps run, output tiles and steps clipped to the sector blocks
 * (with D2D_TILE_DENSE this is sb_info's flops_exec).  Builds the work list
 * if needed. */
d2d_status d2d_sb_gemm_flops(d2d_sb* sb, int prec, double* flops);
/* Autotuner: times every grouped-GEMM tile shape of precision prec on this
 * superblock, unsplit, with D2D_TILE_SPLIT and with D2D_TILE_SPLIT4, each with
 * and without D2D_TILE_FUSED and D2D_TILE_XCD (reps launches each, on internal scratch vectors, HIP events
 * on the context stream), selects the fastest for later d2d_hv / d2d_lanczos
 * calls and returns it (shape index OR-ed with the flags) and its average
 * milliseconds.  If the environment variable D2D_TUNE_CACHE names a file,
 * results are looked up there first (key: precision and the list of sector
 * dimensions) and appended after a measurement.  Synchronous. */
d2d_status d2d_sb_autotune(d2d_sb* sb, int prec, int reps, int* best_tile, double* best_ms);

/* Number of tile shapes and, if desc != NULL, for each shape i: desc[5*i..] =
 * (precision, BM, BN, BK, prefetch depth: K steps whose loads are in flight
 * while a step's MFMAs run). */
d2d_status d2d_tile_shapes(int* count, int* desc);

/* ------------------------------------------------------------------ Lanczos
 * Ground state of the superblock in its target sector by FP64
 * residual-corrected restarted Lanczos:
 *   restart j: w = H_64 x_j, theta_j = x_j.w, r = w - theta_j x_j,
 *   rho_j = |r|; stop if converged; else an inner Lanczos started from x_j
 *   (alpha_0 = theta_j, beta_1 = rho_j, q_1 = r/rho_j) runs k_in - 1 more
 *   steps (fewer in a cycle fitted to the residual bar, see fixed_cycles)
 *   with Hv in precision prec_j, reorthogonalisation by classical
 *   Gram-Schmidt twice in FP64 (against all basis vectors, or the last
 *   reorth_window ones), the tridiagonal lowest eigenpair on the device, and
 *   x_{j+1} = y_0 x_j + sum_{i>=1} y_i q_i.
 * All recurrences, dot products, the tridiagonal solve and the Ritz vector
 * are FP64 arithmetic on the device; the host reads (theta_j, rho_j) once per
 * restart.  Below FP64 the basis q_0..q_{k-1} is stored in the products'
 * input precision (see basis): x_j enters x_{j+1} in FP64, so the storage
 * rounding only touches the correction sum_{i>=1} y_i q_i, which shrinks with
 * the residual.
 * Precision schedule: start in opts.prec; the precision is raised (BF16 ->
 * BF16X3 when kept -> FP32 -> FP64) after a restart with rho_{j+1} > escalate
 * * rho_j whose shortfall is the low-precision products' doing: theta_{j+1} >
 * theta_j (1e-13 relative; exact arithmetic never raises it) or rho_{j+1} > 4
 * beta_k |y_k| (the true FP64 residual well above the one the Krylov
 * recurrence predicts).  Slow convergence of the Krylov space itself keeps
 * the precision.  In a batch, a problem that meets the condition waits
 * while the others go on converging at the current precision; when none is
 * left, the waiting problems continue one precision higher (for one
 * superblock this is plain escalation).  k_in (k_in_bf16 for BF16 cycles)
 * is capped at the smallest problem dimension.
 * Convergence: rho_j <= tol_res * |theta_j|, or, when tol_rel_e > 0, two
 * successive FP64 Rayleigh quotients with |theta_j - theta_{j-1}| <=
 * tol_rel_e * |theta_j|.
 * v0: device FP64 start vector of length n (need not be normalised), or NULL
 * for a seeded N(0,1) vector: element i is the Box-Muller normal
 * sqrt(-2 ln u1) cos(2 pi u2) of u1, u2 from outputs 2i and 2i+1 of the
 * SplitMix64 stream (Steele, Lea and Flood 2014) seeded with opts.seed (a
 * batch adds the problem index to the seed).
 * energy: host out, the last theta.  psi: device out (nullable), the unit
 * Ritz vector.  Returns D2D_ENOCONV (with energy/psi/stats filled) when
 * max_restarts is reached. */
typedef struct {
    int prec;            /* Hv precision of the inner steps                    */
    int k_in;            /* Krylov dimension per restart (2..128; 2..32 with
                            full reorthogonalisation)                         */
    int max_restarts;
    double tol_res;      /* relative residual |r|/|theta|                      */
    double escalate;     /* precision raise threshold on rho_{j+1}/rho_j        */
    int use_graph;       /* 1: capture each restart (its cycle and the FP64
                            residual) in a hipGraph and replay it; 0: launch
                            the kernels directly.  Captures are kept with the
                            superblock's (batch's) Lanczos workspace and
                            replayed by later calls while the cycle length,
                            the options they depend on and the launch
                            configuration hold (see graph_captures)         */
    int reorth_window;   /* 0: reorthogonalise against every basis vector (full);
                            w in 2..32: only against the last w vectors (the FP64
                            restarts keep the fixed point exact either way)   */
    int separate_central; /* 0: inner-step Hv is one launch where the tile choice
                            says so (D2D_TILE_FUSED); 1: the central term always
                            as a launch of its own.  Same result bit for bit  */
    double tol_rel_e;    /* energy-change stop (0: off)                         */
    uint64_t seed;       /* seed of the start vector when v0 is NULL            */
    int plain_cgs2;      /* 0: with a window of 2..4 each step is two kernels: the
                            second Gram-Schmidt pass and the norm follow from the
                            first pass's sums and the window's Gram matrix;
                            1: always two explicit passes (three kernels)     */
    int basis;           /* storage of the inner basis: 0: the products' input
                            precision (FP64; FP32 for FP32 and BF16x3; BF16
                            for BF16), so a basis vector is the Hv input
                            itself; 1: FP64 at every precision; 2: FP32
                            below FP64 (BF16 products read a BF16 copy)      */
    int k_in_bf16;       /* Krylov dimension of BF16 inner cycles (0: k_in);
                            limits as k_in.  A BF16 cycle gains little past
                            the point where the BF16 products' error stops
                            it, so it may be shorter than the others        */
    int fixed_cycles;    /* 0: a cycle stops early when the problems' previous
                            cycle reduced the residual at a rate that meets
                            tol_res in fewer steps (1.25 x those steps + 4);
                            1: every cycle has k_in (k_in_bf16) vectors     */
    int one_kernel_step; /* 0: a step runs as its two kernels; 1: with a
                            window of 2..4 and direct launches, a step runs as
                            one cooperative kernel (sums, grid barrier, update
                            from registers) where every block's share fits its
                            registers and the grid fits the device.  Same
                            result bit for bit; slower on MI355X, where the
                            cooperative launch and its grid barrier cost more
                            than the launch and the re-read of the window
                            they save                                       */
} d2d_lanczos_opts;

#define D2D_LOG_MAX 256
typedef struct {
    int restarts;
    int64_t hv_count[D2D_NPREC]; /* Hv applications to this problem per
                                    precision (in a batch: the grouped launches
                                    that included it)                          */
    double residual;          /* last rho                                      */
    double seconds;           /* wall time of the call                         */
    int nlog;                 /* entries in the per-restart log                */
    double log_t[D2D_LOG_MAX];      /* seconds since the call started           */
    double log_theta[D2D_LOG_MAX];
    double log_rho[D2D_LOG_MAX];
    int log_prec[D2D_LOG_MAX];      /* precision of the inner Lanczos that
                                       produced this entry (opts.prec first)   */
    double log_pred[D2D_LOG_MAX];   /* residual the previous inner Lanczos
                                       predicted for its Ritz vector
                                       (beta_k |y_k|; 0 for the first entry)     */
    int graph_captures;       /* restarts captured as hipGraphs in this call
                                 (use_graph: a capture made by an earlier call
                                 on the same superblock or batch is replayed
                                 while the cycle length, options and launch
                                 configuration it was made for hold)          */
    int64_t coop_steps;       /* inner steps run as the one cooperative kernel
                                 (one_kernel_step)                             */
} d2d_lanczos_stats;

d2d_status d2d_lanczos(d2d_sb* sb, const d2d_lanczos_opts* opts, const double* v0, double* energy,
                       double* psi, d2d_lanczos_stats* stats);

/* ----------------------------------------------------------- density matrix
 * Reduced density matrix of one half of the packed state psi (device, FP64,
 * unit norm): side 0 -> rho_L[q_L] = V[q] V[q]^T (block 1 (x) column 2),
 * side 1 -> rho_R[q_R] = V[q]^T V[q] (column 3 (x) block 4); the paper's
 * density-matrix formation.  Each sector is diagonalised (density-matrix
 * diagonalisation) and the m_keep eigenvectors of largest weight are kept
 * (ties: sector ascending, index ascending); the enlarged half's operators are
 * projected onto them, giving the block of the next, one column longer,
 * superblock.  trunc_err (host out) = 1 - kept weight.  spectrum (host,
 * nullable) receives all eigenvalues in descending order; spectrum_len (in:
 * capacity, out: count). */
d2d_status d2d_density_matrix(d2d_sb* sb, const double* psi, int side, int m_keep,
                              d2d_block** new_block, double* trunc_err, double* spectrum,
                              int64_t* spectrum_len);
/* d2d_density_matrix with the wall time of its three phases in ms[3] (host
 * out, milliseconds, the stream synchronised at each boundary), the paper's
 * split of the step after the exact diagonalisation: ms[0] density-matrix
 * formation (rho of every sector, one grouped FP64 matrix-core launch),
 * ms[1] density-matrix diagonalisation (every sector's eigenpairs, the
 * selection of the kept states), ms[2] renormalisation (kept eigenvectors,
 * H' = U^T H U and the new edge operators on the device, the new block's
 * host copy).  D2D_EINVAL when ms is NULL. */
d2d_status d2d_density_matrix_timed(d2d_sb* sb, const double* psi, int side, int m_keep,
                                    d2d_block** new_block, double* trunc_err, double* spectrum,
                                    int64_t* spectrum_len, double ms[3]);

/* Both halves of one state at once, as in a step of the infinite-system
 * algorithm (Fig. 1a: blocks 1 and 4 both grow by a column): the results of
 * d2d_density_matrix for side 0 (*new_left, trunc_err[0]) and side 1
 * (*new_right, trunc_err[1]), bit for bit, with the two halves' sectors
 * diagonalised together on the context's eigensolver streams, so that the
 * two halves' longest eigensolves overlap.  ms (host, nullable) receives the
 * wall times of the three phases over both halves (formation,
 * diagonalisation with the selections, renormalisation).  On failure no
 * block is returned. */
d2d_status d2d_density_matrix_both(d2d_sb* sb, const double* psi, int m_keep, d2d_block** new_left,
                                   d2d_block** new_right, double trunc_err[2], double ms[3]);

/* Wavefunction transformation: the initial guess of the next superblock of
 * a finite-system sweep (the sweeps whose energies Fig. 3 follows).  A block
 * returned by d2d_density_matrix remembers the enlarged half it was made
 * from (its parent block plus one column) and its transformation U, the
 * kept density-matrix eigenvectors in that half's basis.  Moving the
 * superblock one column right (direction 0), `to`'s block 1 is the new block
 * made from `from`'s left half, and `from`'s block 4 was made from `to`'s
 * right half:
 *   psi_to[(i3, j1), (j3, j4)] = sum over i1, i2, i4 of
 *       U1[(i2, i1), j1] psi_from[(i2, i1), (i3, i4)] U4[(j3, j4), i4]
 * with U1 the transformation of to's block 1 and U4 that of from's block 4
 * (indices as in the packed layout: column state, then block state).
 * Direction 1 (moving left) is the mirror image: to's block 4 was made from
 * from's right half, from's block 1 from to's left half.  psi_from and
 * psi_to are packed device FP64 vectors of the two superblocks (lengths
 * their N); the result is the projection of psi_from onto the kept states,
 * not normalised.  Computed on the device (full-space form, grouped FP64
 * GEMMs).  D2D_EINVAL when the superblocks' blocks are not one step apart in
 * that direction (imported and exact blocks carry no transformation).
 * Synchronous. */
d2d_status d2d_wavefunction_transform(d2d_sb* from, const double* psi_from, d2d_sb* to, double* psi_to,
                                      int direction);

/* -------------------------------------------------------------- observables
 * Site densities <n_{y,sigma}> of a packed superblock state psi (device,
 * FP64, unit norm) on the superblock's two explicit columns: the inputs of
 * the hole density h(x,y) = 1 - <n_up + n_dn> and the staggered spin density
 * s(x,y) = <n_up - n_dn> of the paper's stripe analysis (Eqs. (2) and (3);
 * S(x) of Eq. (4) is the largest |s(x,y)| over the legs).  Column 2 is the
 * lattice column right of block 1, column 3 the next one.  The density
 * operators of a column are diagonal in its occupation basis, so
 * <n_{y,sigma}> = sum over packed elements of psi^2 times the occupation of
 * mode (y, sigma) in the element's column state.  Spin model: n_up = 1/2 +
 * S^z, n_dn = 1/2 - S^z.  out (host, 4 * legs doubles):
 * out[(c * legs + y) * 2 + sigma], c = 0 column 2, 1 column 3; sigma 0 up,
 * 1 down.  Deterministic (partial sums added in a fixed order); synchronous. */
d2d_status d2d_column_densities(d2d_sb* sb, const double* psi, double* out);

/* -------------------------------------------------------------------- batch
 * Many independent superblocks advanced together: one grouped launch per
 * Lanczos step covers every sector tile of every problem.  The superblocks
 * are borrowed and must outlive the batch. */
d2d_status d2d_batch_create(d2d_ctx* ctx, d2d_sb* const* sbs, int n, d2d_batch** out);
d2d_status d2d_batch_destroy(d2d_batch* b);
/* One batched Hv: v[i], w[i] device pointers of problem i (precision prec). */
d2d_status d2d_batch_hv(d2d_batch* b, int prec, const void* const* v, void* const* w);
/* Launch configuration of the batch's grouped launches in precision prec, as
 * d2d_sb_set_tile for one superblock (shape index OR-ed with the D2D_TILE_*
 * flags).  tile -1 restores the default: shape by the largest sector
 * dimension, K-loops split when every sector dimension is at most 768, central
 * term fused except in FP64, plain order.  The superblocks' own settings are
 * not used by, nor changed by, the batch.  D2D_EINVAL for a shape not built
 * for prec or unknown flags. */
d2d_status d2d_batch_set_tile(d2d_batch* b, int prec, int tile);
/* Autotuner of the batch, as d2d_sb_autotune: every shape of prec x split
 * level x fused x XCD order timed over reps batched Hv with all problems
 * active (on the batch's staging vectors, HIP events on the context stream);
 * the fastest is kept for later d2d_batch_hv / d2d_batch_lanczos calls and
 * returned (best_tile as for d2d_batch_set_tile, best_ms its average
 * milliseconds per batched Hv).  D2D_TUNE_CACHE is consulted and appended as
 * for a superblock (key: precision, problem count and every sector
 * dimension).  Synchronous.  On an error the previous configuration stays. */
d2d_status d2d_batch_autotune(d2d_batch* b, int prec, int reps, int* best_tile, double* best_ms);
/* As d2d_sb_gemm_flops, for one batched grouped-GEMM launch over every
 * problem of the batch. */
d2d_status d2d_batch_gemm_flops(d2d_batch* b, int prec, double* flops);
/* Batched restarted Lanczos; v0[i] device start vectors (array or entries
 * nullable: seeded as for d2d_lanczos with seed opts.seed + i); energies host out
 * [n]; psi[i] device out (nullable array or entries); per_problem (nullable)
 * stats [n].  Converged problems leave the launch at the next restart. */
d2d_status d2d_batch_lanczos(d2d_batch* b, const d2d_lanczos_opts* opts, const double* const* v0,
                             double* energies, double* const* psi, d2d_lanczos_stats* per_problem);

#ifdef __cplusplus
}
#endif

#endif /* D2D_H */
