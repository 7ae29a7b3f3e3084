// Kernels of the DMRG step around the exact diagonalisation for gfx950: the
// local densities of Eqs. (2)-(4) on the superblock's explicit columns, and
// the density-matrix step (grouped FP64 matrix-core GEMM for rho, H' = U^T H U
// and the new edge operators; kept-eigenvector gather; operator row gather).
#include <algorithm>

#include "internal.h"

namespace d2d {

// Column densities: for every packed element (r, c) of pair p, w = psi^2 goes
// to the occupation slots of its column-2 state a2 = rowsL[row_base + r] / m
// and column-3 state a3 = colsR[col_base + c] / m.  Slots per column: bit k of
// the state (k < nbits: Hubbard mode 2y + sigma, spin model up spin y), then
// the total weight.  Block (x, p) writes its sums to partial[(p * gx + x) *
// 2 * DENS_SLOTS + slot]; the host adds them in that order.
__global__ void __launch_bounds__(256)
k_col_dens(const SectorDev* __restrict__ sec, const int32_t* __restrict__ rowsL, const int32_t* __restrict__ colsR,
           int m, int nbits, const double* __restrict__ psi, double* __restrict__ partial) {
    constexpr int S = 2 * DENS_SLOTS;
    const SectorDev s = sec[blockIdx.y];
    const int64_t n = (int64_t)s.dL * s.dR;
    double acc[S];
#pragma unroll
    for (int k = 0; k < S; ++k) acc[k] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e % s.dL), c = (int)(e / s.dL);
        const double x = psi[s.off + e];
        const double w = x * x;
        const int a2 = rowsL[s.row_base + r] / m, a3 = colsR[s.col_base + c] / m;
#pragma unroll
        for (int k = 0; k < DENS_SLOTS - 1; ++k) {
            if (k < nbits) {
                acc[k] += ((a2 >> k) & 1) ? w : 0.0;
                acc[DENS_SLOTS + k] += ((a3 >> k) & 1) ? w : 0.0;
            }
        }
        acc[DENS_SLOTS - 1] += w;
        acc[S - 1] += w;
    }
    __shared__ double sh[256 / 64][S];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < S; ++k) {
        double v = acc[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if (lane == 0) sh[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < S) {
        double t = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sh[q][threadIdx.x];
        partial[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * S + threadIdx.x] = t;
    }
}

hipError_t launch_col_dens(const SectorDev* sec, int npairs, int gx, const int32_t* rowsL, const int32_t* colsR, int m,
                           int nbits, const double* psi, double* partial, hipStream_t st) {
    if (npairs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_col_dens, dim3(gx, npairs), dim3(256), 0, st, sec, rowsL, colsR, m, nbits, psi, partial);
    return hipGetLastError();
}

}  // namespace d2d

namespace d2d {

// ------------------------------------------------------------------ grouped FP64 GEMM
// C_i = op(A_i) op(B_i) for a list of problems (column-major, op = identity
// or transpose), one 64 x 64 output tile per work-group, on the FP64 matrix
// instruction v_mfma_f64_16x16x4: lane l holds Aop[l%16][l/16] and
// Bop[l/16][l%16]; value v of lane l is D[4v + l/16][l%16].  The tile's B
// fragment is fed as the instruction's A operand and the A fragment as its
// B operand, so D = (A B)^T and a lane's four results run down one column of
// the column-major C (the same arrangement as the Hv kernels).  Per K step of
// 16 the A tile (64 x 16) and the B tile (16 x 64) go through LDS; each
// operand is loaded along its contiguous direction (rows of an
// untransposed column-major operand, K of a transposed one), with elements
// outside the problem read as zero.
typedef double f64x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256)
k_gemm_f64(const GemmProb* __restrict__ probs, const int4* __restrict__ tiles) {
    constexpr int BM = 64, BN = 64, BK = 16, NT = 256;
    __shared__ double As[BK][BM + 1];
    __shared__ double Bs[BN][BK + 1];
    const int4 ti = tiles[blockIdx.x];
    const GemmProb P = probs[ti.x];
    const int row0 = ti.y * BM, col0 = ti.z * BN;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1;   // 2 x 2 waves of 32 x 32
    f64x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < P.K; k0 += BK) {
        // A tile: BM x BK = 1024 elements, 4 per thread
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = t + NT * e;
            int r, k;
            if (!P.ta) { r = idx % BM; k = idx / BM; }     // contiguous along rows
            else { k = idx % BK; r = idx / BK; }           // contiguous along K
            const int gr = row0 + r, gk = k0 + k;
            double x = 0.0;
            if (gr < P.M && gk < P.K) x = P.ta ? P.A[gk + (int64_t)gr * P.lda] : P.A[gr + (int64_t)gk * P.lda];
            As[k][r] = x;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = t + NT * e;
            int c, k;
            if (!P.tb) { k = idx % BK; c = idx / BK; }     // contiguous along K
            else { c = idx % BN; k = idx / BN; }           // contiguous along columns
            const int gc = col0 + c, gk = k0 + k;
            double x = 0.0;
            if (gc < P.N && gk < P.K) x = P.tb ? P.B[gc + (int64_t)gk * P.ldb] : P.B[gk + (int64_t)gc * P.ldb];
            Bs[c][k] = x;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            double a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[kk + lane / 16][wm * 32 + i * 16 + lane % 16];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[wn * 32 + j * 16 + lane % 16][kk + lane / 16];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[j], a[i], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int r = row0 + wm * 32 + i * 16 + lane % 16;
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = col0 + wn * 32 + j * 16 + 4 * v + lane / 16;
                if (r < P.M && c < P.N) P.C[r + (int64_t)c * P.ldc] = acc[i][j][v];
            }
    }
}

hipError_t launch_gemm_f64(const GemmProb* probs, const int4* tiles, int ntiles, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gemm_f64, dim3(ntiles), dim3(256), 0, st, probs, tiles);
    return hipGetLastError();
}

// ------------------------------------------------------------------ kept eigenvectors
// U columns from the eigenvector matrices of the density-matrix sectors:
// column j of problem entry sel[j] = (source matrix offset, its leading
// dimension = rows d, source column, destination offset), sign fixed so that
// the entry of largest modulus (the first such entry on ties) is positive.
// One wave per column.
__global__ void __launch_bounds__(64)
k_pick_columns(const int4* __restrict__ sel, const int64_t* __restrict__ offs, const double* __restrict__ Z,
               double* __restrict__ U) {
    const int4 s = sel[blockIdx.x];     // x: rows d, y: source column, z: index into offs (src, dst)
    const int64_t src = offs[2 * s.z] + (int64_t)s.y * s.x, dst = offs[2 * s.z + 1];
    const int lane = threadIdx.x;
    double best = 0.0;
    int bi = s.x;
    for (int r = lane; r < s.x; r += 64) {
        const double v = fabs(Z[src + r]);
        if (v > best) { best = v; bi = r; }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const double sg = (bi < s.x && Z[src + bi] < 0.0) ? -1.0 : 1.0;
    for (int r = lane; r < s.x; r += 64) U[dst + r] = sg * Z[src + r];
}

hipError_t launch_pick_columns(const int4* sel, int ncols, const int64_t* offs, const double* Z, double* U,
                               hipStream_t st) {
    if (ncols == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pick_columns, dim3(ncols), dim3(64), 0, st, sel, offs, Z, U);
    return hipGetLastError();
}

// ------------------------------------------------------------------ edge operators
// G = O U_from for an edge-column operator with at most one nonzero per row:
// row r of G (d_to rows, cnt columns) is val[r] times row src[r] of U_from
// (zero where src[r] < 0).  grid.y = one (operator, target sector) entry of
// the table; entry e: x = rows, y = columns, z = index of its offsets
// (row map, U_from, G) in offs[3 z ..].
__global__ void __launch_bounds__(256)
k_gather_rows(const int4* __restrict__ ent, const int64_t* __restrict__ offs, const int32_t* __restrict__ src,
              const double* __restrict__ val, const double* __restrict__ U, double* __restrict__ G) {
    const int4 e = ent[blockIdx.y];
    const int64_t mo = offs[3 * e.z], uo = offs[3 * e.z + 1], go = offs[3 * e.z + 2];
    const int64_t n = (int64_t)e.x * e.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i % e.x), j = (int)(i / e.x);
        const int sr = src[mo + r];
        G[go + i] = sr >= 0 ? val[mo + r] * U[uo + sr + (int64_t)j * e.w] : 0.0;
    }
}

hipError_t launch_gather_rows(const int4* ent, int nent, int64_t maxn, const int64_t* offs, const int32_t* src,
                              const double* val, const double* U, double* G, hipStream_t st) {
    if (nent == 0) return hipSuccess;
    int gx = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (maxn + 255) / 256));
    hipLaunchKernelGGL(k_gather_rows, dim3(gx, nent), dim3(256), 0, st, ent, offs, src, val, U, G);
    return hipGetLastError();
}

}  // namespace d2d
