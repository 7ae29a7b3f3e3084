// Lanczos vector kernels (FP64 arithmetic on a basis stored in FP64, FP32 or
// BF16) and the tridiagonal eigensolver for gfx950.
//
// Scalars (alpha, beta, projection coefficients, norms) stay in device memory
// so that a Lanczos inner loop runs without any host round trip.
#include <hip/hip_cooperative_groups.h>

#include "internal.h"

// Multiply-adds are fused only where one expression writes them (a += b * c),
// never across statements: the fused and the two-kernel forms of a step then
// round alike, whatever the scheduler does with their registers.
#pragma clang fp contract(on)

namespace d2d {

static constexpr int LZ_THREADS = 256;

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}


__device__ inline uint16_t f32_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

static int ew_grid(int64_t n) {
    int64_t g = (n + LZ_THREADS - 1) / LZ_THREADS;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

// ------------------------------------------------------------------ tridiagonal
// Lowest eigenpair of the symmetric tridiagonal T (diagonal alpha[0..k-1],
// off-diagonal beta[1..k-1]), k <= 128, one wave:
//  - eigenvalue: Sturm-sequence multisection.  The count of eigenvalues below
//    x is the number of sign changes of the leading principal minors
//    p_i = (a_i - x) p_{i-1} - b_i^2 p_{i-2} (p_0 = 1): two multiply-adds
//    per step and no division (one wave issues every instruction, so the
//    instruction count is the cost); a zero minor counts as a change (as a
//    zero pivot taken as slightly negative would); rescaled when large (a
//    tiny pivot is always followed by a large one, so the minors do not
//    underflow).  The 64 lanes split the bracket into 65 pieces per round.
//  - eigenvector: twisted factorization (T - theta I = N_r D_r N_r^T, Dhillon
//    and Parlett): the forward pivots D+ (lane 0) and backward pivots D-
//    (lane 1) run in parallel; the twist index r minimises
//    |D+_i + D-_i - (a_i - theta)|; from y_r = 1 the components below r
//    (lane 0) and above r (lane 1) follow from the pivots, then the vector
//    is normalised with y[0] >= 0.
__device__ inline double sturm_pivot(double d) {
    // a zero pivot is replaced by a tiny negative one (the count treats it as below)
    return d == 0.0 ? -1e-290 : d;
}

__device__ void tridiag_body(const double* __restrict__ alpha, const double* __restrict__ beta, int k,
                             double* __restrict__ theta_out, double* __restrict__ y_out,
                             double* __restrict__ pred_out) {
    __shared__ double a[128], b[128], b2[128], dp[128], dm[128], y[128];
    __shared__ double lo_s, hi_s, scale_s;
    __shared__ int r_s;
    const int l = threadIdx.x;
    for (int i = l; i < k; i += 64) {
        a[i] = alpha[i];
        b[i] = i > 0 ? beta[i] : 0.0;
        b2[i] = b[i] * b[i];
    }
    __syncthreads();
    if (l == 0) {
        double lo = a[0], hi = a[0];
        for (int i = 0; i < k; ++i) {
            const double r = (i > 0 ? fabs(b[i]) : 0.0) + (i + 1 < k ? fabs(b[i + 1]) : 0.0);
            lo = fmin(lo, a[i] - r);
            hi = fmax(hi, a[i] + r);
        }
        const double pad = 1e-12 * fmax(1.0, fmax(fabs(lo), fabs(hi)));
        lo_s = lo - pad;
        hi_s = hi + pad;
    }
    __syncthreads();
    constexpr int P = 1;                     // points per lane
    constexpr double NP1 = 64.0 * P + 1.0;   // pieces per round
    double plo = 0.0, phi = 0.0;
    for (int it = 0; it < 40; ++it) {
        const double lo = lo_s, hi = hi_s;
        if (hi - lo <= 4.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)) || hi <= lo) break;
        // a bracket of a few ulps can stop shrinking (the points round onto its ends)
        if (it > 0 && lo == plo && hi == phi) break;
        plo = lo;
        phi = hi;
        double x[P], pm[P], pc[P];
        int c[P];
#pragma unroll
        for (int u = 0; u < P; ++u) {
            x[u] = lo + (hi - lo) * (double)(P * l + u + 1) / NP1;
            pm[u] = 1.0;
            pc[u] = sturm_pivot(a[0] - x[u]);
            c[u] = pc[u] < 0.0 ? 1 : 0;
        }
        for (int i = 1; i < k; ++i) {
            const double ai = a[i], bi2 = b2[i];
#pragma unroll
            for (int u = 0; u < P; ++u) {
                double pn = (ai - x[u]) * pc[u] - bi2 * pm[u];
                if (pn == 0.0) pn = pc[u] < 0.0 ? 1e-290 : -1e-290;
                c[u] += (pn < 0.0) != (pc[u] < 0.0) ? 1 : 0;
                pm[u] = pc[u];
                pc[u] = pn;
                if (fabs(pn) > 1e150) {
                    pm[u] *= 1e-150;
                    pc[u] *= 1e-150;
                }
            }
        }
        // smallest point index (over the wave) with at least one eigenvalue below it
        int q = 1 << 30;
#pragma unroll
        for (int u = P - 1; u >= 0; --u)
            if (c[u] >= 1) q = P * l + u;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) q = min(q, __shfl_xor(q, o, 64));
        __syncthreads();
        if (l == 0) {
            if (q >= (1 << 30)) {
                lo_s = lo + (hi - lo) * (NP1 - 1.0) / NP1;
            } else {
                hi_s = lo + (hi - lo) * (double)(q + 1) / NP1;
                if (q > 0) lo_s = lo + (hi - lo) * (double)q / NP1;
            }
        }
        __syncthreads();
    }
    const double th = 0.5 * (lo_s + hi_s);
    if (l == 0) theta_out[0] = th;
    // twisted factorization: pivots from both ends in parallel
    if (l == 0) {
        double d = sturm_pivot(a[0] - th);
        dp[0] = d;
        for (int i = 1; i < k; ++i) {
            d = sturm_pivot((a[i] - th) - b2[i] / d);
            dp[i] = d;
        }
    } else if (l == 1) {
        double d = sturm_pivot(a[k - 1] - th);
        dm[k - 1] = d;
        for (int i = k - 2; i >= 0; --i) {
            d = sturm_pivot((a[i] - th) - b2[i + 1] / d);
            dm[i] = d;
        }
    }
    __syncthreads();
    {
        // twist index: argmin |gamma_i|, ties to the smallest i
        double best = 1e308;
        int bi = 0;
        for (int i = l; i < k; i += 64) {
            const double g = fabs(dp[i] + dm[i] - (a[i] - th));
            if (g < best) {
                best = g;
                bi = i;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(best, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (ob < best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        if (l == 0) r_s = bi;
    }
    __syncthreads();
    const int r = r_s;
    if (l == 0) {
        double v = 1.0;
        y[r] = 1.0;
        for (int i = r - 1; i >= 0; --i) {
            v = -b[i + 1] * v / dp[i];
            y[i] = v;
        }
    } else if (l == 1) {
        double v = 1.0;
        for (int i = r + 1; i < k; ++i) {
            v = -b[i] * v / dm[i];
            y[i] = v;
        }
    }
    __syncthreads();
    // normalise: scale by the largest modulus first (the recurrences can grow large)
    double mx = 0.0;
    for (int i = l; i < k; i += 64) mx = fmax(mx, fabs(y[i]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    double ss = 0.0;
    for (int i = l; i < k; i += 64) {
        const double t = y[i] / mx;
        ss += t * t;
    }
    ss = wave_sum(ss);
    if (l == 0) scale_s = (y[0] < 0.0 ? -1.0 : 1.0) / (mx * sqrt(ss));   // lane 0 holds the sum
    __syncthreads();
    for (int i = l; i < k; i += 64) y_out[i] = y[i] * scale_s;
    // residual norm of the Ritz vector by the recurrence: beta_k |y_{k-1}|
    if (l == 0) *pred_out = fabs(beta[k] * y[k - 1] * scale_s);
}

}  // namespace d2d

// ====================================================================== segmented step kernels
// Kernels of the restarted Lanczos for a set of problems at once (one problem
// is the case of one segment).  The vectors of all problems are concatenated;
// a block table maps every block to one problem and to a contiguous chunk of
// that problem's segment.  Global sums are per problem: every block writes
// per-block partial sums, and a kernel that needs a sum produced by the
// previous kernel adds the partials of its problem's blocks itself (every
// block redundantly, in block order), so no separate reduction launches and
// no inter-block fences are needed: the kernel boundary orders the partials
// before their use, and the sums are deterministic.
// Scalars live per problem at scal + prob * S_LEN (layout in lz_layout.h).
namespace d2d {

static constexpr int LZ_STEP_NB = 1024;

// About 2048 elements per block: with the U-way unrolled element loops below a
// block covers its segment in one or two rounds of loads, so a step kernel
// costs about one memory latency on mid-sized problems and is bandwidth-bound
// on large ones.
int lz_step_blocks(int64_t n) {
    int64_t nb = (n + 2047) / 2048;
    if (nb > LZ_STEP_NB) nb = LZ_STEP_NB;
    if (nb < 1) nb = 1;
    return (int)nb;
}

// out_sh[j] = sum_{b in [b0,b1)} partial[j*NB + b], j < rows (shared result).
// Always inlined: as a call it made every caller reserve the registers of its
// unrolled loads (246, two waves per SIMD).
// A problem has at most LZ_STEP_NB blocks, so a lane adds at most
// LZ_STEP_NB / 64 partials of a row; all of them are loaded at once (index
// clamped into the problem's range, the extra values masked afterwards), so
// the sum costs one memory latency, not one per partial.
// When the problem has at most 512 blocks, a wave loads the partials of up to
// four of its rows together (8 per lane and row) before adding any.
__device__ __attribute__((always_inline)) inline void reduce_rows(const double* __restrict__ partial, int rows,
                                                                  int NB, int b0, int b1, double* out_sh) {
    constexpr int R = LZ_STEP_NB / 64;
    constexpr int NW = LZ_THREADS / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (b1 - b0 <= 512) {
        constexpr int L = 8, MR = 4;
        for (int j0 = wv; j0 < rows; j0 += NW * MR) {
            double v[MR][L];
#pragma unroll
            for (int r = 0; r < MR; ++r) {
                const int j = j0 + NW * r;
#pragma unroll
                for (int q = 0; q < L; ++q) {
                    const int b = b0 + lane + 64 * q;
                    v[r][q] = j < rows ? partial[(int64_t)j * NB + (b < b1 ? b : b0)] : 0.0;
                }
            }
#pragma unroll
            for (int r = 0; r < MR; ++r) {
                const int j = j0 + NW * r;
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < L; ++q)
                    if (b0 + lane + 64 * q < b1) s += v[r][q];
                s = wave_sum(s);
                if (lane == 0 && j < rows) out_sh[j] = s;
            }
        }
        __syncthreads();
        return;
    }
    for (int j = wv; j < rows; j += NW) {
        double v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int b = b0 + lane + 64 * q;
            v[q] = partial[(int64_t)j * NB + (b < b1 ? b : b0)];
        }
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < R; ++q)
            if (b0 + lane + 64 * q < b1) s += v[q];
        s = wave_sum(s);
        if (lane == 0) out_sh[j] = s;
    }
    __syncthreads();
}

// Per-block sums of acc[0..rows) (rows <= R) written to partial[j*NB + b].
template <int R>
__device__ inline void write_partials(const double (&acc)[R], int rows, double* __restrict__ partial, int NB,
                                      int b) {
    __shared__ double sh[LZ_THREADS / 64][R];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (j < rows) {
            const double t = wave_sum(acc[j]);
            if (lane == 0) sh[wv][j] = t;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < rows) {
        double t = 0.0;
        for (int w = 0; w < LZ_THREADS / 64; ++w) t += sh[w][threadIdx.x];
        partial[(int64_t)threadIdx.x * NB + b] = t;
    }
}

// Elements a thread keeps in flight per round in the step kernels (bounded
// so that the U x NQ loaded values stay in registers).
template <int NQ>
struct StepUnroll {
    static constexpr int U = NQ <= 4 ? 4 : (NQ <= 8 ? 2 : 1);
};

struct HvPartPtrs {
    const void* p[4];
};

// The next Hv's input copy of a basis vector: FP32 (FP32 and BF16x3 products)
// or BF16 (round to nearest even); lo_prec -1 writes nothing (the product
// reads the basis vector itself).
__device__ inline void store_lo(void* __restrict__ lo, int lo_prec, int64_t e, double q) {
    if (lo_prec == D2D_FP32 || lo_prec == D2D_BF16X3) ((float*)lo)[e] = (float)q;
    else if (lo_prec == D2D_BF16) ((uint16_t*)lo)[e] = f32_bf16_rne((float)q);
}

// A basis element stored in BF16 (the bits; FP64 -> FP32 -> BF16, each to
// nearest even, as every BF16 copy here).
struct bf16q {
    uint16_t b;
};
__device__ inline double q_to_f64(double x) { return x; }
__device__ inline double q_to_f64(float x) { return (double)x; }
__device__ inline double q_to_f64(bf16q x) { return (double)__uint_as_float((uint32_t)x.b << 16); }
template <typename TQ>
__device__ inline TQ q_from_f64(double q);
template <>
__device__ inline double q_from_f64<double>(double q) { return q; }
template <>
__device__ inline float q_from_f64<float>(double q) { return (float)q; }
template <>
__device__ inline bf16q q_from_f64<bf16q>(double q) { return bf16q{f32_bf16_rne((float)q)}; }

// Step kernel 1: w = (((w + P0) + P1) + P2) + P3 in the Hv's precision (the
// parts of a split or fused Hv, each nullable), upcast from FP32 when UPCAST,
// stored as FP64 when it changed; partials of c1 = Q[0..nq)^T w.
template <int NQ, bool UPCAST, typename TQ>
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_dots(const LzSeg* __restrict__ bt, const TQ* __restrict__ Q,
          int64_t ldq, int nq, const double* w64in, const float* __restrict__ w32, const HvPartPtrs P,
          double* w64out, double* __restrict__ partial, int NB) {
    const bool any = P.p[0] || P.p[1] || P.p[2] || P.p[3];
    constexpr int U = StepUnroll<NQ>::U;
    const LzSeg sg = bt[blockIdx.x];
    if (!sg.act) return;
    double acc[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j) acc[j] = 0.0;
    const int64_t st = blockDim.x;
    using TW = typename std::conditional<UPCAST, float, double>::type;
    const TW* win = UPCAST ? (const TW*)w32 : (const TW*)w64in;
    for (int64_t e0 = sg.lo + threadIdx.x; e0 < sg.hi; e0 += U * st) {
        // loads at an index clamped into the segment, issued together; the
        // lanes past the end are masked afterwards
        double x[U], q[U][NQ];
        TQ qr[U][NQ];
        TW wv[U], pv[4][U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = e0 + u * st;
            const int64_t ec = e < sg.hi ? e : sg.lo;
            wv[u] = win[ec];
#pragma unroll
            for (int i = 0; i < 4; ++i) pv[i][u] = P.p[i] ? ((const TW*)P.p[i])[ec] : TW(0);
#pragma unroll
            for (int j = 0; j < NQ; ++j) qr[u][j] = Q[(j < nq ? j : nq - 1) * ldq + ec];
        }
        // every window load is issued before any is waited for (rows past nq
        // re-read row nq-1 and are zeroed here)
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < NQ; ++j) q[u][j] = j < nq ? q_to_f64(qr[u][j]) : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = e0 + u * st < sg.hi;
            TW f = wv[u];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (P.p[i]) f = f + pv[i][u];
            x[u] = ok ? (double)f : 0.0;
#pragma unroll
            for (int j = 0; j < NQ; ++j) q[u][j] = ok ? q[u][j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (UPCAST || any) {
                const int64_t e = e0 + u * st;
                if (e < sg.hi) w64out[e] = x[u];
            }
#pragma unroll
            for (int j = 0; j < NQ; ++j) acc[j] += q[u][j] * x[u];
        }
    }
    write_partials<NQ>(acc, nq, partial, NB, blockIdx.x);
}

// Step kernel 2: c1 from partial_in; w <- w - Q c1; partials of c2 = Q^T w
// (rows 0..nq-1) and |w|^2 (row nq) into partial_out; alpha_i = c1[i].
template <int NQ, typename TQ>
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_update_dots(const LzSeg* __restrict__ bt, const TQ* __restrict__ Q,
                 int64_t ldq, int nq, const double* __restrict__ partial_in, double* __restrict__ w,
                 double* __restrict__ partial_out, int NB, double* __restrict__ scal, int i) {
    const LzSeg sg = bt[blockIdx.x];
    if (!sg.act) return;
    __shared__ double cs[NQ];
    if ((int)threadIdx.x < NQ) cs[threadIdx.x] = 0.0;
    __syncthreads();
    reduce_rows(partial_in, nq, NB, sg.pb0, sg.pb1, cs);
    if ((int)blockIdx.x == sg.pb0 && threadIdx.x == 0) scal[(int64_t)sg.prob * S_LEN + S_ALPHA + i] = cs[nq - 1];
    constexpr int U = StepUnroll<NQ>::U;
    double acc[NQ + 1];
#pragma unroll
    for (int j = 0; j <= NQ; ++j) acc[j] = 0.0;
    const int64_t st = blockDim.x;
    for (int64_t e0 = sg.lo + threadIdx.x; e0 < sg.hi; e0 += U * st) {
        double x[U], q[U][NQ];
        TQ qr[U][NQ];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = e0 + u * st;
            const int64_t ec = e < sg.hi ? e : sg.lo;
            x[u] = w[ec];
#pragma unroll
            for (int j = 0; j < NQ; ++j) qr[u][j] = Q[(j < nq ? j : nq - 1) * ldq + ec];
        }
        // every window load is issued before any is waited for (rows past nq
        // re-read row nq-1 and are zeroed here)
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < NQ; ++j) q[u][j] = j < nq ? q_to_f64(qr[u][j]) : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (e0 + u * st >= sg.hi) {
                x[u] = 0.0;
#pragma unroll
                for (int j = 0; j < NQ; ++j) q[u][j] = 0.0;
            }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int j = 0; j < NQ; ++j) x[u] -= cs[j] * q[u][j];
            const int64_t e = e0 + u * st;
            if (e < sg.hi) w[e] = x[u];
#pragma unroll
            for (int j = 0; j < NQ; ++j) acc[j] += q[u][j] * x[u];
            acc[NQ] += x[u] * x[u];
        }
    }
    // rows 0..nq-1: projections; row nq: |w|^2
    __shared__ double sh[LZ_THREADS / 64][NQ + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
        if (j < nq) {
            const double t = wave_sum(acc[j]);
            if (lane == 0) sh[wv][j] = t;
        }
    }
    {
        const double t = wave_sum(acc[NQ]);
        if (lane == 0) sh[wv][nq] = t;
    }
    __syncthreads();
    if ((int)threadIdx.x <= nq) {
        double t = 0.0;
        for (int ww = 0; ww < LZ_THREADS / 64; ++ww) t += sh[ww][threadIdx.x];
        partial_out[(int64_t)threadIdx.x * NB + blockIdx.x] = t;
    }
}

// Step kernel 3: c2 and |w|^2 from partial_in; beta = sqrt(|w|^2 - |c2|^2);
// q_next = (w - [need2] Q c2) / beta with need2 = |c2| > 1e-13 |w|;
// lo = cast(q_next); the problem's first block writes alpha_i += c2[i], beta_{i+1}.
template <int NQ, typename TQ>
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_next(const LzSeg* __restrict__ bt, const TQ* __restrict__ Q,
          int64_t ldq, int nq, const double* __restrict__ partial_in, int NB, const double* __restrict__ w,
          TQ* __restrict__ qnext, void* __restrict__ lo, int lo_prec, double* __restrict__ scal, int i) {
    const LzSeg sg = bt[blockIdx.x];
    if (!sg.act) return;
    __shared__ double cs[NQ + 1];
    reduce_rows(partial_in, nq + 1, NB, sg.pb0, sg.pb1, cs);
    double s2 = 0.0;
    for (int j = 0; j < nq; ++j) s2 += cs[j] * cs[j];
    const double w2 = cs[nq];
    const double b2 = w2 - s2;
    const double bb = sqrt(b2 > 0.0 ? b2 : 0.0);
    const bool corr = sqrt(s2) > 1e-13 * sqrt(w2 > 0.0 ? w2 : 0.0);
    if ((int)blockIdx.x == sg.pb0 && threadIdx.x == 0) {
        double* sc = scal + (int64_t)sg.prob * S_LEN;
        sc[S_ALPHA + i] += cs[nq - 1];
        sc[S_BETA + i + 1] = bb;
    }
    if (!qnext) return;
    const double inv = bb > 0.0 ? 1.0 / bb : 0.0;
    const int64_t st = blockDim.x;
    for (int64_t e0 = sg.lo + threadIdx.x; e0 < sg.hi; e0 += 4 * st) {
        // loads at an index clamped into the segment, issued together
        double x[4], q[4][NQ];
        TQ qr[4][NQ];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t e = e0 + u * st;
            const int64_t ec = e < sg.hi ? e : sg.lo;
            x[u] = w[ec];
#pragma unroll
            for (int j = 0; j < NQ; ++j) qr[u][j] = Q[(j < nq ? j : nq - 1) * ldq + ec];
        }
        // every window load is issued before any is waited for (rows past nq
        // re-read row nq-1 and are zeroed here)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int j = 0; j < NQ; ++j) q[u][j] = (corr && j < nq) ? q_to_f64(qr[u][j]) : 0.0;
        if (corr)
#pragma unroll
            for (int j = 0; j < NQ; ++j)
                if (j < nq)   // cs[nq] holds |w|^2, and entries past it are not written
#pragma unroll
                    for (int u = 0; u < 4; ++u) x[u] -= cs[j] * q[u][j];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t e = e0 + u * st;
            if (e >= sg.hi) break;
            const double q = x[u] * inv;
            qnext[e] = q_from_f64<TQ>(q);
            store_lo(lo, lo_prec, e, q);
        }
    }
}

// ---- Gram form of the step for a short window (nq <= 4): two kernels.
// The second classical Gram-Schmidt pass and the norm follow from the first
// pass's sums and the window's Gram matrix G = Q^T Q, gathered in the same
// read of the window: c2 = c1 - G c1, d = c1 + c2, and
// |w - Q d|^2 = |w|^2 - 2 d.c1 + d^T G d.  Partial rows (fixed layout):
// c1 in 0..NQ-1, |w|^2 in NQ, G_jl (j <= l) from NQ+1 on.
// Elements a thread keeps in flight per round in the Gram kernels (8 ran no
// faster and cost the first kernel a wave of occupancy).
static constexpr int GRAM_U = 4;

template <int NQ>
struct GramLayout {
    static constexpr int NG = NQ * (NQ + 1) / 2;
    static constexpr int ROWS = NQ + 1 + NG;
    __host__ __device__ static constexpr int g(int j, int l) { return NQ + 1 + j * NQ - j * (j - 1) / 2 + (l - j); }
};

// First kernel of the Gram form: w = (((w + P0) + P1) + P2) + P3 in the Hv's
// precision, stored back in place (in that precision: the FP32 sum is what
// the second kernel upcasts) when there are parts; partials of c1 = Q^T w,
// |w|^2 and the window's Gram matrix.
template <int NQ, bool UPCAST, typename TQ>
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_dots_gram(const LzSeg* __restrict__ bt, const TQ* __restrict__ Q, int64_t ldq, int nq,
               typename std::conditional<UPCAST, float, double>::type* wio, const HvPartPtrs P,
               double* __restrict__ partial, int NB) {
    using GL = GramLayout<NQ>;
    constexpr int U = GRAM_U;
    const LzSeg sg = bt[blockIdx.x];
    if (!sg.act) return;
    const bool any = P.p[0] || P.p[1] || P.p[2] || P.p[3];
    double acc[GL::ROWS];
#pragma unroll
    for (int j = 0; j < GL::ROWS; ++j) acc[j] = 0.0;
    const int64_t st = blockDim.x;
    using TW = typename std::conditional<UPCAST, float, double>::type;
    const TW* win = wio;
    for (int64_t e0 = sg.lo + threadIdx.x; e0 < sg.hi; e0 += U * st) {
        double x[U], q[U][NQ];
        TQ qr[U][NQ];
        TW wv[U], pv[4][U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = e0 + u * st;
            const int64_t ec = e < sg.hi ? e : sg.lo;
            wv[u] = win[ec];
#pragma unroll
            for (int i = 0; i < 4; ++i) pv[i][u] = P.p[i] ? ((const TW*)P.p[i])[ec] : TW(0);
#pragma unroll
            for (int j = 0; j < NQ; ++j) qr[u][j] = Q[(j < nq ? j : nq - 1) * ldq + ec];
        }
        // every window load is issued before any is waited for (rows past nq
        // re-read row nq-1 and are zeroed here)
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < NQ; ++j) q[u][j] = j < nq ? q_to_f64(qr[u][j]) : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = e0 + u * st;
            const bool ok = e < sg.hi;
            TW f = wv[u];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (P.p[i]) f = f + pv[i][u];
            x[u] = ok ? (double)f : 0.0;
            if (any && ok) wio[e] = f;
#pragma unroll
            for (int j = 0; j < NQ; ++j) q[u][j] = ok ? q[u][j] : 0.0;
#pragma unroll
            for (int j = 0; j < NQ; ++j) acc[j] += q[u][j] * x[u];
            acc[NQ] += x[u] * x[u];
#pragma unroll
            for (int j = 0; j < NQ; ++j)
#pragma unroll
                for (int l = j; l < NQ; ++l) acc[GL::g(j, l)] += q[u][j] * q[u][l];
        }
    }
    write_partials<GL::ROWS>(acc, GL::ROWS, partial, NB, blockIdx.x);
}

// d = c1 + (c1 - G c1) and beta = sqrt(|w|^2 - 2 d.c1 + d^T G d) from the
// block's copy cs of the summed rows.
template <int NQ>
__device__ __attribute__((always_inline)) inline void gram_coeffs(const double* cs, int nq, double (&d)[NQ],
                                                                  double& bb) {
    using GL = GramLayout<NQ>;
    double c1[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j) c1[j] = j < nq ? cs[j] : 0.0;
    auto gram = [&](int j, int l) { return j <= l ? cs[GL::g(j, l)] : cs[GL::g(l, j)]; };
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
        double gc = 0.0;
#pragma unroll
        for (int l = 0; l < NQ; ++l) gc += gram(j, l) * c1[l];
        d[j] = j < nq ? c1[j] + (c1[j] - gc) : 0.0;
    }
    double dc = 0.0, dgd = 0.0;
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
        dc += d[j] * c1[j];
        double gd = 0.0;
#pragma unroll
        for (int l = 0; l < NQ; ++l) gd += gram(j, l) * d[l];
        dgd += d[j] * gd;
    }
    const double b2 = cs[NQ] - 2.0 * dc + dgd;
    bb = sqrt(b2 > 0.0 ? b2 : 0.0);
}

// Second kernel: d, alpha_i = d[nq-1], beta = |w - Q d| from the sums;
// q_next = (w - Q d) / beta and its low-precision copy.
template <int NQ, bool UPCAST, typename TQ>
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_update_gram(const LzSeg* __restrict__ bt, const TQ* __restrict__ Q, int64_t ldq, int nq,
                 const double* __restrict__ partial_in, int NB,
                 const typename std::conditional<UPCAST, float, double>::type* __restrict__ w,
                 TQ* __restrict__ qnext, void* __restrict__ lo, int lo_prec, double* __restrict__ scal, int i) {
    using GL = GramLayout<NQ>;
    const LzSeg sg = bt[blockIdx.x];
    if (!sg.act) return;
    __shared__ double cs[GL::ROWS];
    reduce_rows(partial_in, GL::ROWS, NB, sg.pb0, sg.pb1, cs);
    double d[NQ], bb;
    gram_coeffs<NQ>(cs, nq, d, bb);
    if ((int)blockIdx.x == sg.pb0 && threadIdx.x == 0) {
        double* sc = scal + (int64_t)sg.prob * S_LEN;
        sc[S_ALPHA + i] = d[nq - 1];
        sc[S_BETA + i + 1] = bb;
    }
    if (!qnext) return;
    constexpr int U = GRAM_U;
    const double inv = bb > 0.0 ? 1.0 / bb : 0.0;
    const int64_t st = blockDim.x;
    for (int64_t e0 = sg.lo + threadIdx.x; e0 < sg.hi; e0 += U * st) {
        double x[U], q[U][NQ];
        TQ qr[U][NQ];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = e0 + u * st;
            const int64_t ec = e < sg.hi ? e : sg.lo;
            x[u] = (double)w[ec];
#pragma unroll
            for (int j = 0; j < NQ; ++j) qr[u][j] = Q[(j < nq ? j : nq - 1) * ldq + ec];
        }
        // every window load is issued before any is waited for (rows past nq
        // re-read row nq-1 and are zeroed here)
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < NQ; ++j) q[u][j] = j < nq ? q_to_f64(qr[u][j]) : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = e0 + u * st;
            if (e >= sg.hi) break;
#pragma unroll
            for (int j = 0; j < NQ; ++j) x[u] -= d[j] * q[u][j];
            const double qv = x[u] * inv;
            qnext[e] = q_from_f64<TQ>(qv);
            store_lo(lo, lo_prec, e, qv);
        }
    }
}

// One-kernel Gram step for segments a block covers in COOP_ROUNDS rounds of
// GRAM_U elements per thread: the first kernel's sums, a grid barrier, then
// the second kernel's update from the product and window values still held in
// registers (neither is read twice, and one launch is saved).  Launched
// cooperatively only (every block of the grid resident at once), and every
// block, active or not, reaches the barrier exactly once.  The arithmetic and
// its order are the two kernels', so the result is the same bit for bit.
static constexpr int COOP_ROUNDS = 2;

template <int NQ, bool UPCAST, typename TQ>
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_step_gram_coop(const LzSeg* __restrict__ bt, const TQ* __restrict__ Q, int64_t ldq, int nq,
                    const typename std::conditional<UPCAST, float, double>::type* __restrict__ win,
                    const HvPartPtrs P, double* __restrict__ partial, int NB, TQ* __restrict__ qnext,
                    void* __restrict__ lo, int lo_prec, double* __restrict__ scal, int i) {
    using GL = GramLayout<NQ>;
    using TW = typename std::conditional<UPCAST, float, double>::type;
    constexpr int U = GRAM_U, RR = COOP_ROUNDS;
    const LzSeg sg = bt[blockIdx.x];
    const bool act = sg.act != 0;
    const int64_t st = blockDim.x;
    double x[RR][U], q[RR][U][NQ];
    if (act) {
        double acc[GL::ROWS];
#pragma unroll
        for (int j = 0; j < GL::ROWS; ++j) acc[j] = 0.0;
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const int64_t e0 = sg.lo + threadIdx.x + (int64_t)r * U * st;
            TQ qr[U][NQ];
            TW wv[U], pv[4][U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t e = e0 + u * st;
                const int64_t ec = e < sg.hi ? e : sg.lo;
                wv[u] = win[ec];
#pragma unroll
                for (int k = 0; k < 4; ++k) pv[k][u] = P.p[k] ? ((const TW*)P.p[k])[ec] : TW(0);
#pragma unroll
                for (int j = 0; j < NQ; ++j) qr[u][j] = Q[(j < nq ? j : nq - 1) * ldq + ec];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int j = 0; j < NQ; ++j) q[r][u][j] = j < nq ? q_to_f64(qr[u][j]) : 0.0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool ok = e0 + u * st < sg.hi;
                TW f = wv[u];
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (P.p[k]) f = f + pv[k][u];
                x[r][u] = ok ? (double)f : 0.0;
#pragma unroll
                for (int j = 0; j < NQ; ++j) q[r][u][j] = ok ? q[r][u][j] : 0.0;
            }
            // a lane whose round starts past the segment adds nothing (as the
            // two-kernel loop, which ends before that round)
            if (e0 < sg.hi) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int j = 0; j < NQ; ++j) acc[j] += q[r][u][j] * x[r][u];
                    acc[NQ] += x[r][u] * x[r][u];
#pragma unroll
                    for (int j = 0; j < NQ; ++j)
#pragma unroll
                        for (int l = j; l < NQ; ++l) acc[GL::g(j, l)] += q[r][u][j] * q[r][u][l];
                }
            }
        }
        write_partials<GL::ROWS>(acc, GL::ROWS, partial, NB, blockIdx.x);
    }
    __threadfence();
    cooperative_groups::this_grid().sync();
    if (!act) return;
    __shared__ double cs[GL::ROWS];
    reduce_rows(partial, GL::ROWS, NB, sg.pb0, sg.pb1, cs);
    double d[NQ], bb;
    gram_coeffs<NQ>(cs, nq, d, bb);
    if ((int)blockIdx.x == sg.pb0 && threadIdx.x == 0) {
        double* sc = scal + (int64_t)sg.prob * S_LEN;
        sc[S_ALPHA + i] = d[nq - 1];
        sc[S_BETA + i + 1] = bb;
    }
    if (!qnext) return;
    const double inv = bb > 0.0 ? 1.0 / bb : 0.0;
#pragma unroll
    for (int r = 0; r < RR; ++r) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = sg.lo + threadIdx.x + (int64_t)r * U * st + u * st;
            if (e >= sg.hi) continue;
            double xv = x[r][u];
#pragma unroll
            for (int j = 0; j < NQ; ++j) xv -= d[j] * q[r][u][j];
            const double qv = xv * inv;
            qnext[e] = q_from_f64<TQ>(qv);
            store_lo(lo, lo_prec, e, qv);
        }
    }
}

// Elements of a segment the one-kernel step can hold (per block).
int lz_coop_segment_max() { return COOP_ROUNDS * GRAM_U * LZ_THREADS; }

template <bool UPCAST, typename TQ>
static bool coop_fits_t(int NB) {
    int dev = 0, cus = 0, per = 0, coop = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return false;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_lz_step_gram_coop<4, UPCAST, TQ>, LZ_THREADS, 0) !=
        hipSuccess)
        return false;
    return (int64_t)per * cus >= NB;
}

bool lz_coop_fits(int NB, bool upcast, int qbytes) {
    if (!upcast) return qbytes == 8 && coop_fits_t<false, double>(NB);
    if (qbytes == 8) return coop_fits_t<true, double>(NB);
    if (qbytes == 4) return coop_fits_t<true, float>(NB);
    if (qbytes == 2) return coop_fits_t<true, bf16q>(NB);
    return false;
}

template <typename TQ>
static hipError_t lz_step_gram_coop(const LzStepArgs& a, hipStream_t s) {
    HvPartPtrs P;
    for (int k = 0; k < 4; ++k) P.p[k] = a.wpart[k];
    const TQ* Q = (const TQ*)a.Q;
    TQ* qn = (TQ*)a.qnext;
    int64_t ldq = a.ldq;
    int nq = a.nq, NB = a.NB, lp = a.lo ? a.lo_prec : -1, i = a.i;
    double* partial = a.partial;
    void* lo = a.lo;
    double* scal = a.scal;
    const LzSeg* bt = a.bt;
    if (a.upcast) {
        const float* win = a.w32;
        void* args[] = {&bt, &Q, &ldq, &nq, &win, &P, &partial, &NB, &qn, &lo, &lp, &scal, &i};
        return hipLaunchCooperativeKernel((const void*)k_lz_step_gram_coop<4, true, TQ>, dim3(NB), dim3(LZ_THREADS),
                                          args, 0, s);
    }
    const double* win = a.w;
    void* args[] = {&bt, &Q, &ldq, &nq, &win, &P, &partial, &NB, &qn, &lo, &lp, &scal, &i};
    return hipLaunchCooperativeKernel((const void*)k_lz_step_gram_coop<4, false, TQ>, dim3(NB), dim3(LZ_THREADS),
                                      args, 0, s);
}

template <typename TQ>
static hipError_t lz_step_gram(const LzStepArgs& a, hipStream_t s) {
    constexpr int NQ = 4;
    const int NB = a.NB;
    const TQ* Q = (const TQ*)a.Q;
    TQ* qn = (TQ*)a.qnext;
    const int lp = a.lo ? a.lo_prec : -1;
    HvPartPtrs P;
    for (int i = 0; i < 4; ++i) P.p[i] = a.wpart[i];
    // the low-precision product's sum stays in its FP32 buffer (the upcast is exact)
    if (a.upcast) {
        hipLaunchKernelGGL((k_lz_dots_gram<NQ, true, TQ>), dim3(NB), dim3(LZ_THREADS), 0, s, a.bt, Q, a.ldq, a.nq,
                           (float*)a.w32, P, a.partial, NB);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_lz_update_gram<NQ, true, TQ>), dim3(NB), dim3(LZ_THREADS), 0, s, a.bt, Q, a.ldq,
                           a.nq, a.partial, NB, (const float*)a.w32, qn, a.lo, lp, a.scal, a.i);
    } else {
        hipLaunchKernelGGL((k_lz_dots_gram<NQ, false, TQ>), dim3(NB), dim3(LZ_THREADS), 0, s, a.bt, Q, a.ldq,
                           a.nq, a.w, P, a.partial, NB);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_lz_update_gram<NQ, false, TQ>), dim3(NB), dim3(LZ_THREADS), 0, s, a.bt, Q, a.ldq,
                           a.nq, a.partial, NB, (const double*)a.w, qn, a.lo, lp, a.scal, a.i);
    }
    return hipGetLastError();
}

template <int NQ, typename TQ>
static hipError_t lz_step_nq(const LzStepArgs& a, hipStream_t s) {
    const int NB = a.NB;
    const TQ* Q = (const TQ*)a.Q;
    HvPartPtrs P;
    for (int i = 0; i < 4; ++i) P.p[i] = a.wpart[i];
    if (a.upcast)
        hipLaunchKernelGGL((k_lz_dots<NQ, true, TQ>), dim3(NB), dim3(LZ_THREADS), 0, s, a.bt, Q, a.ldq, a.nq,
                           (const double*)nullptr, a.w32, P, a.w, a.partial, NB);
    else
        hipLaunchKernelGGL((k_lz_dots<NQ, false, TQ>), dim3(NB), dim3(LZ_THREADS), 0, s, a.bt, Q, a.ldq,
                           a.nq, a.w, (const float*)nullptr, P, a.w, a.partial, NB);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_lz_update_dots<NQ, TQ>), dim3(NB), dim3(LZ_THREADS), 0, s, a.bt, Q, a.ldq, a.nq,
                       a.partial, a.w, a.partial2, NB, a.scal, a.i);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_lz_next<NQ, TQ>), dim3(NB), dim3(LZ_THREADS), 0, s, a.bt, Q, a.ldq, a.nq,
                       a.partial2, NB, a.w, (TQ*)a.qnext, a.lo, a.lo ? a.lo_prec : -1, a.scal, a.i);
    return hipGetLastError();
}

template <typename TQ>
static hipError_t lz_step(const LzStepArgs& a, hipStream_t s) {
    if (a.gram && a.nq <= 4 && a.coop) return lz_step_gram_coop<TQ>(a, s);
    if (a.gram && a.nq <= 4) return lz_step_gram<TQ>(a, s);
    if (a.nq <= 4) return lz_step_nq<4, TQ>(a, s);
    if (a.nq <= 8) return lz_step_nq<8, TQ>(a, s);
    if (a.nq <= 16) return lz_step_nq<16, TQ>(a, s);
    if (a.nq <= 32) return lz_step_nq<32, TQ>(a, s);
    return hipErrorInvalidValue;
}

hipError_t launch_lz_step(const LzStepArgs& a, hipStream_t s) {
    // a narrow basis only with a low-precision product (the FP64 recurrence keeps an FP64 basis)
    if (a.qbytes != 8 && !a.upcast) return hipErrorInvalidValue;
    if (a.qbytes == 8) return lz_step<double>(a, s);
    if (a.qbytes == 4) return lz_step<float>(a, s);
    if (a.qbytes == 2) return lz_step<bf16q>(a, s);
    return hipErrorInvalidValue;
}

// partials of x.w (row 0)
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_dot1(const LzSeg* __restrict__ bt, const double* __restrict__ x,
          const double* __restrict__ w, double* __restrict__ partial, int NB) {
    const LzSeg sg = bt[blockIdx.x];
    if (!sg.act) return;
    double acc[1] = {0.0};
    for (int64_t e = sg.lo + threadIdx.x; e < sg.hi; e += blockDim.x) acc[0] += x[e] * w[e];
    write_partials<1>(acc, 1, partial, NB, blockIdx.x);
}

// theta from partial_in; w <- w - theta x; partials of |w|^2
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_resid(const LzSeg* __restrict__ bt, const double* __restrict__ x,
           const double* __restrict__ partial_in, double* __restrict__ w, double* __restrict__ partial_out, int NB) {
    const LzSeg sg = bt[blockIdx.x];
    if (!sg.act) return;
    __shared__ double th[1];
    reduce_rows(partial_in, 1, NB, sg.pb0, sg.pb1, th);
    const double t = th[0];
    double acc[1] = {0.0};
    for (int64_t e = sg.lo + threadIdx.x; e < sg.hi; e += blockDim.x) {
        const double r = w[e] - t * x[e];
        w[e] = r;
        acc[0] += r * r;
    }
    write_partials<1>(acc, 1, partial_out, NB, blockIdx.x);
}

// one block per problem: alpha_0 = theta, beta_1 = rho, res[2p..2p+1] = (theta, rho)
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_restart_finish(const int2* __restrict__ prange, const int* __restrict__ active,
                    const double* __restrict__ p_theta, const double* __restrict__ p_rho, int NB,
                    double* __restrict__ scal, double* __restrict__ res) {
    const int p = blockIdx.x;
    if (!active[p]) return;
    const int2 r = prange[p];
    __shared__ double v[2];
    reduce_rows(p_theta, 1, NB, r.x, r.y, v);
    reduce_rows(p_rho, 1, NB, r.x, r.y, v + 1);
    if (threadIdx.x == 0) {
        const double rho = sqrt(v[1] > 0.0 ? v[1] : 0.0);
        double* sc = scal + (int64_t)p * S_LEN;
        sc[S_ALPHA] = v[0];
        sc[S_BETA + 1] = rho;
        res[2 * p] = v[0];
        res[2 * p + 1] = rho;
    }
}

hipError_t launch_lz_residual(const LzSet& z, const double* x, double* w, hipStream_t s) {
    hipLaunchKernelGGL(k_lz_dot1, dim3(z.NB), dim3(LZ_THREADS), 0, s, z.bt, x, w, z.partial, z.NB);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lz_resid, dim3(z.NB), dim3(LZ_THREADS), 0, s, z.bt, x, z.partial, w, z.partial2,
                       z.NB);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lz_restart_finish, dim3(z.nprob), dim3(LZ_THREADS), 0, s, z.prange, z.active, z.partial,
                       z.partial2, z.NB, z.scal, z.res);
    return hipGetLastError();
}

// x = y_0 x + sum_{j>=1} y_j Q[j] (y of the problem; Q[0] is x itself, or
// its FP32 copy in an FP32 basis, so x enters in FP64 either way), in place;
// partials of |x|^2
template <typename TQ>
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_ritz(const LzSeg* __restrict__ bt, const TQ* __restrict__ Q, int64_t ldq,
          int k, const double* __restrict__ scal, double* __restrict__ x, double* __restrict__ partial, int NB) {
    const LzSeg sg = bt[blockIdx.x];
    if (!sg.act) return;
    __shared__ double ys[128];
    const double* y = scal + (int64_t)sg.prob * S_LEN + S_Y;
    for (int j = threadIdx.x; j < k && j < 128; j += blockDim.x) ys[j] = y[j];
    __syncthreads();
    double acc[1] = {0.0};
    for (int64_t e = sg.lo + threadIdx.x; e < sg.hi; e += blockDim.x) {
        double v = ys[0] * x[e];
        for (int j = 1; j < k; ++j) v += ys[j] * q_to_f64(Q[j * ldq + e]);
        x[e] = v;
        acc[0] += v * v;
    }
    write_partials<1>(acc, 1, partial, NB, blockIdx.x);
}

// dst = src / |src| per problem (|src|^2 from the partials of its blocks)
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_normalize(const LzSeg* __restrict__ bt, const double* __restrict__ partial,
               int NB, const double* __restrict__ src, double* __restrict__ dst) {
    const LzSeg sg = bt[blockIdx.x];
    if (!sg.act) return;
    __shared__ double v[1];
    reduce_rows(partial, 1, NB, sg.pb0, sg.pb1, v);
    const double inv = v[0] > 0.0 ? 1.0 / sqrt(v[0]) : 0.0;
    for (int64_t e = sg.lo + threadIdx.x; e < sg.hi; e += blockDim.x) dst[e] = src[e] * inv;
}

hipError_t launch_lz_ritz(const LzSet& z, const void* Q, int qbytes, int64_t ldq, int k, double* x,
                          hipStream_t s) {
    if (k > 128) return hipErrorInvalidValue;
    if (qbytes == 2)
        hipLaunchKernelGGL(k_lz_ritz<bf16q>, dim3(z.NB), dim3(LZ_THREADS), 0, s, z.bt, (const bf16q*)Q, ldq, k,
                           z.scal, x, z.partial, z.NB);
    else if (qbytes == 4)
        hipLaunchKernelGGL(k_lz_ritz<float>, dim3(z.NB), dim3(LZ_THREADS), 0, s, z.bt, (const float*)Q, ldq, k,
                           z.scal, x, z.partial, z.NB);
    else if (qbytes == 8)
        hipLaunchKernelGGL(k_lz_ritz<double>, dim3(z.NB), dim3(LZ_THREADS), 0, s, z.bt, (const double*)Q, ldq,
                           k, z.scal, x, z.partial, z.NB);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lz_normalize, dim3(z.NB), dim3(LZ_THREADS), 0, s, z.bt, z.partial, z.NB,
                       (const double*)x, x);
    return hipGetLastError();
}

// x = v / |v| per problem (start vectors)
hipError_t launch_lz_normalize_into(const LzSet& z, const double* v, double* x, hipStream_t s) {
    hipLaunchKernelGGL(k_lz_dot1, dim3(z.NB), dim3(LZ_THREADS), 0, s, z.bt, v, v, z.partial, z.NB);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lz_normalize, dim3(z.NB), dim3(LZ_THREADS), 0, s, z.bt, z.partial, z.NB, v, x);
    return hipGetLastError();
}

// squared norms per problem into res[2p] (start-vector check)
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_norms(const int2* __restrict__ prange, const double* __restrict__ partial, int NB, double* __restrict__ res) {
    __shared__ double v[1];
    const int2 r = prange[blockIdx.x];
    reduce_rows(partial, 1, NB, r.x, r.y, v);
    if (threadIdx.x == 0) res[2 * blockIdx.x] = v[0];
}

hipError_t launch_lz_norms(const LzSet& z, const double* v, hipStream_t s) {
    hipLaunchKernelGGL(k_lz_dot1, dim3(z.NB), dim3(LZ_THREADS), 0, s, z.bt, v, v, z.partial, z.NB);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lz_norms, dim3(z.nprob), dim3(LZ_THREADS), 0, s, z.prange, z.partial, z.NB, z.res);
    return hipGetLastError();
}

// Q[0] = x, Q[1] = r / beta_1 of each problem (rounded to the basis type);
// lo = cast(Q[1])
template <typename TQ>
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_first(const LzSeg* __restrict__ bt, const double* __restrict__ x, const double* __restrict__ w,
           const double* __restrict__ scal, TQ* __restrict__ q0, TQ* __restrict__ q1, void* __restrict__ lo,
           int lo_prec) {
    const LzSeg sg = bt[blockIdx.x];
    if (!sg.act) return;
    const double b = scal[(int64_t)sg.prob * S_LEN + S_BETA + 1];
    const double inv = b > 0.0 ? 1.0 / b : 0.0;
    for (int64_t e = sg.lo + threadIdx.x; e < sg.hi; e += blockDim.x) {
        const double q = w[e] * inv;
        q0[e] = q_from_f64<TQ>(x[e]);
        q1[e] = q_from_f64<TQ>(q);
        store_lo(lo, lo_prec, e, q);
    }
}

// Seeded start vector.  SplitMix64 (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", 2014) is counter-based: output c of the
// stream seeded with s is mix(s + (c + 1) * 0x9E3779B97F4A7C15).  Element i
// takes outputs 2i and 2i+1 as u1, u2 in (0, 1) (53-bit mantissas, offset by
// half an ulp) and the Box-Muller normal sqrt(-2 ln u1) cos(2 pi u2).
__device__ inline uint64_t splitmix64_out(uint64_t seed, uint64_t c) {
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void __launch_bounds__(LZ_THREADS) k_seeded_normal(double* __restrict__ x, int64_t n, uint64_t seed) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double u1 = ((double)(splitmix64_out(seed, 2 * (uint64_t)i) >> 11) + 0.5) * 0x1.0p-53;
        const double u2 = ((double)(splitmix64_out(seed, 2 * (uint64_t)i + 1) >> 11) + 0.5) * 0x1.0p-53;
        x[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    }
}

hipError_t launch_seeded_normal(double* x, int64_t n, uint64_t seed, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_seeded_normal, dim3(ew_grid(n)), dim3(LZ_THREADS), 0, s, x, n, seed);
    return hipGetLastError();
}

hipError_t launch_lz_first(const LzSet& z, const double* x, const double* w, void* Q, int qbytes, int64_t ldq,
                           void* lo, int lo_prec, hipStream_t s) {
    const int lp = lo ? lo_prec : -1;
    if (qbytes == 2)
        hipLaunchKernelGGL(k_lz_first<bf16q>, dim3(z.NB), dim3(LZ_THREADS), 0, s, z.bt, x, w, z.scal, (bf16q*)Q,
                           (bf16q*)Q + ldq, lo, lp);
    else if (qbytes == 4)
        hipLaunchKernelGGL(k_lz_first<float>, dim3(z.NB), dim3(LZ_THREADS), 0, s, z.bt, x, w, z.scal, (float*)Q,
                           (float*)Q + ldq, lo, lp);
    else if (qbytes == 8)
        hipLaunchKernelGGL(k_lz_first<double>, dim3(z.NB), dim3(LZ_THREADS), 0, s, z.bt, x, w, z.scal, (double*)Q,
                           (double*)Q + ldq, lo, lp);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// tridiagonal eigenpairs, one block per problem; the recurrence's residual
// estimate of the Ritz vector at res[2 nprob + p]
__global__ void __launch_bounds__(64)
k_lz_tridiag(const int* __restrict__ active, int k, double* __restrict__ scal, double* __restrict__ res) {
    if (!active[blockIdx.x]) return;
    double* sc = scal + (int64_t)blockIdx.x * S_LEN;
    tridiag_body(sc + S_ALPHA, sc + S_BETA, k, sc + S_THETA + 1, sc + S_Y, res + 2 * gridDim.x + blockIdx.x);
}

hipError_t launch_lz_tridiag(const LzSet& z, int k, hipStream_t s) {
    if (k < 1 || k > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_lz_tridiag, dim3(z.nprob), dim3(64), 0, s, z.active, k, z.scal, z.res);
    return hipGetLastError();
}

}  // namespace d2d
