// FP64 Lanczos vector kernels and the tridiagonal eigensolver for gfx950.
//
// All reductions are two-stage and deterministic: a fixed grid of NB blocks
// writes per-block partial sums, a second kernel adds them in a fixed order.
// Scalars (alpha, beta, projection coefficients, norms) stay in device memory
// so that a Lanczos inner loop runs without any host round trip.
#include "internal.h"

namespace d2d {

static constexpr int LZ_THREADS = 256;
static constexpr int LZ_MAXNB = 1024;
static constexpr int DOT_GROUP = 8;     // vectors per block in the multi-dot kernels

int lz_nblocks(int64_t n) {
    int64_t nb = (n + LZ_THREADS * 4 - 1) / (LZ_THREADS * 4);
    if (nb > LZ_MAXNB) nb = LZ_MAXNB;
    if (nb < 1) nb = 1;
    return (int)nb;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Sum over the block; result valid in thread 0.
__device__ inline double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    __syncthreads();
    return r;
}

// Contiguous chunk of [0, n) owned by block b of nb.
__device__ inline void chunk(int64_t n, int b, int nb, int64_t* lo, int64_t* hi) {
    const int64_t per = (n + nb - 1) / nb;
    *lo = (int64_t)b * per;
    *hi = *lo + per < n ? *lo + per : n;
    if (*lo > n) *lo = n;
}

// partial[j*NB + b] = sum_{e in chunk b} Q[j][e] * w[e]; blockIdx.y = group of DOT_GROUP vectors.
template <bool UPCAST>
__global__ void __launch_bounds__(LZ_THREADS)
k_dots(const double* __restrict__ Q, int64_t ldq, int nq, const double* __restrict__ w64in,
       const float* __restrict__ w32, double* __restrict__ w64out, int64_t n, double* __restrict__ partial) {
    __shared__ double sh[LZ_THREADS / 64];
    const int nb = gridDim.x, b = blockIdx.x;
    const int j0 = blockIdx.y * DOT_GROUP;
    int64_t lo, hi;
    chunk(n, b, nb, &lo, &hi);
    double acc[DOT_GROUP];
#pragma unroll
    for (int j = 0; j < DOT_GROUP; ++j) acc[j] = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
        double x;
        if constexpr (UPCAST) {
            x = (double)w32[e];
            if (blockIdx.y == 0) w64out[e] = x;
        } else {
            x = w64in[e];
        }
#pragma unroll
        for (int j = 0; j < DOT_GROUP; ++j)
            if (j0 + j < nq) acc[j] += Q[(j0 + j) * ldq + e] * x;
    }
#pragma unroll
    for (int j = 0; j < DOT_GROUP; ++j) {
        if (j0 + j >= nq) break;
        const double s = block_sum(acc[j], sh);
        if (threadIdx.x == 0) partial[(int64_t)(j0 + j) * nb + b] = s;
    }
}

hipError_t launch_dots_f64(const double* Q, int64_t ldq, int nq, const double* w, int64_t n, double* partial,
                           hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    dim3 grid(lz_nblocks(n), (nq + DOT_GROUP - 1) / DOT_GROUP);
    hipLaunchKernelGGL((k_dots<false>), grid, dim3(LZ_THREADS), 0, s, Q, ldq, nq, w, (const float*)nullptr,
                       (double*)nullptr, n, partial);
    return hipGetLastError();
}

hipError_t launch_upcast_dots(const double* Q, int64_t ldq, int nq, const float* w32, double* w64, int64_t n,
                              double* partial, hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    dim3 grid(lz_nblocks(n), (nq + DOT_GROUP - 1) / DOT_GROUP);
    hipLaunchKernelGGL((k_dots<true>), grid, dim3(LZ_THREADS), 0, s, Q, ldq, nq, (const double*)nullptr, w32, w64,
                       n, partial);
    return hipGetLastError();
}

__global__ void __launch_bounds__(LZ_THREADS)
k_reduce(const double* __restrict__ partial, int nb, double* __restrict__ out) {
    __shared__ double sh[LZ_THREADS / 64];
    const int j = blockIdx.x;
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) v += partial[(int64_t)j * nb + b];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) out[j] = v;
}

hipError_t launch_reduce(const double* partial, int nq, int nb, double* out, hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3(nq), dim3(LZ_THREADS), 0, s, partial, nb, out);
    return hipGetLastError();
}

// w -= sum_j c[j] Q[j]; optional partial |w|^2.
__global__ void __launch_bounds__(LZ_THREADS)
k_update(const double* __restrict__ Q, int64_t ldq, int nq, const double* __restrict__ c, double* __restrict__ w,
         int64_t n, double* __restrict__ partial) {
    __shared__ double sh[LZ_THREADS / 64];
    __shared__ double cs[128];
    for (int j = threadIdx.x; j < nq && j < 128; j += blockDim.x) cs[j] = c[j];
    __syncthreads();
    const int nb = gridDim.x, b = blockIdx.x;
    int64_t lo, hi;
    chunk(n, b, nb, &lo, &hi);
    double nrm = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
        double x = w[e];
        for (int j = 0; j < nq; ++j) x -= cs[j] * Q[j * ldq + e];
        w[e] = x;
        nrm += x * x;
    }
    if (partial) {
        const double s = block_sum(nrm, sh);
        if (threadIdx.x == 0) partial[b] = s;
    }
}

hipError_t launch_update(const double* Q, int64_t ldq, int nq, const double* c, double* w, int64_t n,
                         double* partial_norm, hipStream_t s) {
    if (nq > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_update, dim3(lz_nblocks(n)), dim3(LZ_THREADS), 0, s, Q, ldq, nq, c, w, n, partial_norm);
    return hipGetLastError();
}

// alpha[i] = c1[i] + c2[i]; beta[i+1] = sqrt(nrm2)
__global__ void k_step_scalars(int i, const double* c1, const double* c2, const double* nrm2, double* alpha,
                               double* beta, double* flags) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        alpha[i] = c1[i] + c2[i];
        const double b = sqrt(nrm2[0] > 0.0 ? nrm2[0] : 0.0);
        beta[i + 1] = b;
        if (flags && !(b > 0.0)) flags[0] = 1.0;   // breakdown marker
    }
}

hipError_t launch_step_scalars(int i, const double* c1, const double* c2, const double* nrm2, double* alpha,
                               double* beta, double* flags, hipStream_t s) {
    hipLaunchKernelGGL(k_step_scalars, dim3(1), dim3(64), 0, s, i, c1, c2, nrm2, alpha, beta, flags);
    return hipGetLastError();
}

__device__ inline uint16_t f32_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// qnext = w / beta; lo = cast(qnext).  A zero beta (breakdown) writes zeros.
__global__ void __launch_bounds__(LZ_THREADS)
k_scale_store(const double* __restrict__ w, const double* __restrict__ beta, double* __restrict__ qnext,
              void* __restrict__ lo, int lo_prec, int64_t n) {
    const double b = beta[0];
    const double inv = b > 0.0 ? 1.0 / b : 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const double q = w[e] * inv;
        qnext[e] = q;
        if (lo_prec == D2D_FP32) ((float*)lo)[e] = (float)q;
        else if (lo_prec == D2D_BF16) ((uint16_t*)lo)[e] = f32_bf16_rne((float)q);
    }
}

static int ew_grid(int64_t n) {
    int64_t g = (n + LZ_THREADS - 1) / LZ_THREADS;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_scale_store(const double* w, const double* beta_ip1, double* qnext, void* lo, int lo_prec,
                              int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_store, dim3(ew_grid(n)), dim3(LZ_THREADS), 0, s, w, beta_ip1, qnext, lo,
                       lo ? lo_prec : -1, n);
    return hipGetLastError();
}

// x = sum_j y[j] Q[j]; partial |x|^2
__global__ void __launch_bounds__(LZ_THREADS)
k_ritz(const double* __restrict__ Q, int64_t ldq, int k, const double* __restrict__ y, double* __restrict__ x,
       int64_t n, double* __restrict__ partial) {
    __shared__ double sh[LZ_THREADS / 64];
    __shared__ double ys[128];
    for (int j = threadIdx.x; j < k && j < 128; j += blockDim.x) ys[j] = y[j];
    __syncthreads();
    const int nb = gridDim.x, b = blockIdx.x;
    int64_t lo, hi;
    chunk(n, b, nb, &lo, &hi);
    double nrm = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
        double v = 0.0;
        for (int j = 0; j < k; ++j) v += ys[j] * Q[j * ldq + e];
        x[e] = v;
        nrm += v * v;
    }
    const double s = block_sum(nrm, sh);
    if (threadIdx.x == 0) partial[b] = s;
}

hipError_t launch_ritz(const double* Q, int64_t ldq, int k, const double* y, double* x, int64_t n,
                       double* partial_norm, hipStream_t s) {
    if (k > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ritz, dim3(lz_nblocks(n)), dim3(LZ_THREADS), 0, s, Q, ldq, k, y, x, n, partial_norm);
    return hipGetLastError();
}

__global__ void __launch_bounds__(LZ_THREADS)
k_normalize(double* __restrict__ x, const double* __restrict__ nrm2, int64_t n) {
    const double v = nrm2[0];
    const double inv = v > 0.0 ? 1.0 / sqrt(v) : 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        x[e] *= inv;
}

hipError_t launch_normalize(double* x, const double* nrm2, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_normalize, dim3(ew_grid(n)), dim3(LZ_THREADS), 0, s, x, nrm2, n);
    return hipGetLastError();
}

__global__ void __launch_bounds__(LZ_THREADS)
k_scale_copy(const double* __restrict__ x, const double* __restrict__ nrm2, double* __restrict__ y, int64_t n) {
    const double v = nrm2[0];
    const double inv = v > 0.0 ? 1.0 / sqrt(v) : 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = x[e] * inv;
}

hipError_t launch_scale_copy(const double* x, const double* nrm2, double* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_copy, dim3(ew_grid(n)), dim3(LZ_THREADS), 0, s, x, nrm2, y, n);
    return hipGetLastError();
}

__global__ void __launch_bounds__(LZ_THREADS)
k_copy(const double* __restrict__ x, double* __restrict__ y, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = x[e];
}

hipError_t launch_copy_f64(const double* x, double* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_copy, dim3(ew_grid(n)), dim3(LZ_THREADS), 0, s, x, y, n);
    return hipGetLastError();
}

// r = w - theta x in place in w; partial |r|^2
__global__ void __launch_bounds__(LZ_THREADS)
k_residual(const double* __restrict__ x, const double* __restrict__ theta, double* __restrict__ w, int64_t n,
           double* __restrict__ partial) {
    __shared__ double sh[LZ_THREADS / 64];
    const double th = theta[0];
    const int nb = gridDim.x, b = blockIdx.x;
    int64_t lo, hi;
    chunk(n, b, nb, &lo, &hi);
    double nrm = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
        const double r = w[e] - th * x[e];
        w[e] = r;
        nrm += r * r;
    }
    const double s = block_sum(nrm, sh);
    if (threadIdx.x == 0) partial[b] = s;
}

hipError_t launch_residual(const double* x, const double* theta, double* w, int64_t n, double* partial_norm,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_residual, dim3(lz_nblocks(n)), dim3(LZ_THREADS), 0, s, x, theta, w, n, partial_norm);
    return hipGetLastError();
}

__global__ void k_restart_scalars(const double* theta, const double* nrm2, double* alpha, double* beta, double* res) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double th = theta[0];
        const double rho = sqrt(nrm2[0] > 0.0 ? nrm2[0] : 0.0);
        alpha[0] = th;
        beta[1] = rho;
        res[0] = th;
        res[1] = rho;
    }
}

hipError_t launch_restart_scalars(const double* theta, const double* nrm2, double* alpha, double* beta,
                                  double* res, hipStream_t s) {
    hipLaunchKernelGGL(k_restart_scalars, dim3(1), dim3(64), 0, s, theta, nrm2, alpha, beta, res);
    return hipGetLastError();
}

// ------------------------------------------------------------------ tridiagonal
// Lowest eigenpair of the symmetric tridiagonal T (diagonal alpha[0..k-1],
// off-diagonal beta[1..k-1]), one wave:
//  - eigenvalue: Sturm-sequence bisection, each round splitting the bracket
//    into 65 pieces evaluated by the 64 lanes (count of eigenvalues below x);
//  - eigenvector: two steps of inverse iteration with (T - theta I), solved by
//    Gaussian elimination with partial pivoting on lane 0 (k <= 128).
__device__ int sturm_count(const double* a, const double* b, int k, double x) {
    // number of eigenvalues < x
    int cnt = 0;
    double d = a[0] - x;
    const double tiny = 1e-300;
    if (d == 0.0) d = -tiny;
    if (d < 0.0) ++cnt;
    for (int i = 1; i < k; ++i) {
        d = (a[i] - x) - b[i] * b[i] / d;
        if (d == 0.0) d = -tiny;
        if (d < 0.0) ++cnt;
    }
    return cnt;
}

__global__ void __launch_bounds__(64)
k_tridiag(const double* __restrict__ alpha, const double* __restrict__ beta, int k, double* __restrict__ theta_out,
          double* __restrict__ y, double* __restrict__ work) {
    __shared__ double a[128], b[128];
    __shared__ double lo_s, hi_s;
    const int l = threadIdx.x;
    for (int i = l; i < k; i += 64) {
        a[i] = alpha[i];
        b[i] = i > 0 ? beta[i] : 0.0;
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
    for (int it = 0; it < 40; ++it) {
        const double lo = lo_s, hi = hi_s;
        if (hi - lo <= 4.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)) || hi <= lo) break;
        const double x = lo + (hi - lo) * (double)(l + 1) / 65.0;
        const int c = sturm_count(a, b, k, x);
        // first lane whose point has at least one eigenvalue below it
        const unsigned long long mask = __ballot(c >= 1);
        __syncthreads();
        if (l == 0) {
            if (mask == 0ull) {
                lo_s = lo + (hi - lo) * 64.0 / 65.0;
            } else {
                const int f = __ffsll((long long)mask) - 1;
                hi_s = lo + (hi - lo) * (double)(f + 1) / 65.0;
                if (f > 0) lo_s = lo + (hi - lo) * (double)f / 65.0;
            }
        }
        __syncthreads();
    }
    if (l == 0) {
        const double th = 0.5 * (lo_s + hi_s);
        theta_out[0] = th;
        // inverse iteration: (T - th I) z = y, Gaussian elimination with partial pivoting.
        // work: dl[k], d[k], du[k], du2[k], z[k]
        double* dl = work;
        double* d = work + 128;
        double* du = work + 256;
        double* du2 = work + 384;
        int* piv = (int*)(work + 512);
        const double eps = 2.220446049250313e-16 * fmax(1.0, fabs(th));
        for (int i = 0; i < k; ++i) {
            d[i] = a[i] - th;
            du[i] = i + 1 < k ? b[i + 1] : 0.0;
            dl[i] = i + 1 < k ? b[i + 1] : 0.0;
            du2[i] = 0.0;
        }
        // LU with partial pivoting (LAPACK dgttrf scheme)
        for (int i = 0; i < k - 1; ++i) {
            if (fabs(d[i]) >= fabs(dl[i])) {
                piv[i] = i;
                const double piv_v = d[i] != 0.0 ? d[i] : eps;
                d[i] = piv_v;
                const double f = dl[i] / piv_v;
                dl[i] = f;
                d[i + 1] -= f * du[i];
                du2[i] = 0.0;
            } else {
                piv[i] = i + 1;
                const double f = d[i] / dl[i];
                d[i] = dl[i];
                dl[i] = f;
                const double tmp = du[i];
                du[i] = d[i + 1];
                d[i + 1] = tmp - f * d[i + 1];
                if (i + 1 < k - 1) {
                    du2[i] = du[i + 1];
                    du[i + 1] = -f * du[i + 1];
                }
            }
        }
        if (d[k - 1] == 0.0) d[k - 1] = eps;
        for (int i = 0; i < k; ++i) y[i] = 1.0 / sqrt((double)k);
        for (int rep = 0; rep < 3; ++rep) {
            // solve L U z = y (forward with pivots, then back substitution)
            for (int i = 0; i < k - 1; ++i) {
                if (piv[i] == i) {
                    y[i + 1] -= dl[i] * y[i];
                } else {
                    const double t = y[i];
                    y[i] = y[i + 1];
                    y[i + 1] = t - dl[i] * y[i];
                }
            }
            y[k - 1] /= d[k - 1];
            if (k > 1) y[k - 2] = (y[k - 2] - du[k - 2] * y[k - 1]) / d[k - 2];
            for (int i = k - 3; i >= 0; --i) y[i] = (y[i] - du[i] * y[i + 1] - du2[i] * y[i + 2]) / d[i];
            double nrm = 0.0;
            for (int i = 0; i < k; ++i) nrm += y[i] * y[i];
            nrm = sqrt(nrm);
            for (int i = 0; i < k; ++i) y[i] /= nrm;
        }
        if (y[0] < 0.0)
            for (int i = 0; i < k; ++i) y[i] = -y[i];
    }
}

hipError_t launch_tridiag(const double* alpha, const double* beta, int k, double* theta, double* y, double* work,
                          hipStream_t s) {
    if (k < 1 || k > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(64), 0, s, alpha, beta, k, theta, y, work);
    return hipGetLastError();
}

// ------------------------------------------------------------------ density matrix helpers
// rho = V V^T (side 0, dL x dL) or V^T V (side 1, dR x dR); V column-major dL x dR.
__global__ void k_syrk(const double* __restrict__ V, int dL, int dR, int side, double* __restrict__ rho) {
    const int d = side == 0 ? dL : dR;
    const int64_t dd = (int64_t)d * d;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < dd; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % d), j = (int)(e / d);
        double s = 0.0;
        if (side == 0)
            for (int c = 0; c < dR; ++c) s += V[i + (int64_t)c * dL] * V[j + (int64_t)c * dL];
        else
            for (int r = 0; r < dL; ++r) s += V[r + (int64_t)i * dL] * V[r + (int64_t)j * dL];
        rho[e] = s;
    }
}

hipError_t launch_syrk_f64(const double* V, int dL, int dR, int side, double* rho, hipStream_t s) {
    const int d = side == 0 ? dL : dR;
    hipLaunchKernelGGL(k_syrk, dim3(ew_grid((int64_t)d * d)), dim3(LZ_THREADS), 0, s, V, dL, dR, side, rho);
    return hipGetLastError();
}

// C (M x N) = op(A) (M x K) * B (K x N), column-major; op(A) = A or A^T.
__global__ void k_gemm_nn(const double* __restrict__ A, int lda, const double* __restrict__ B, int ldb,
                          double* __restrict__ C, int ldc, int M, int N, int K, int transA) {
    const int64_t mn = (int64_t)M * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < mn; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % M), j = (int)(e / M);
        double s = 0.0;
        if (transA)
            for (int k = 0; k < K; ++k) s += A[k + (int64_t)i * lda] * B[k + (int64_t)j * ldb];
        else
            for (int k = 0; k < K; ++k) s += A[i + (int64_t)k * lda] * B[k + (int64_t)j * ldb];
        C[i + (int64_t)j * ldc] = s;
    }
}

hipError_t launch_gemm_nn_f64(const double* A, int lda, const double* B, int ldb, double* C, int ldc, int M, int N,
                              int K, int transA, hipStream_t s) {
    if ((int64_t)M * N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gemm_nn, dim3(ew_grid((int64_t)M * N)), dim3(LZ_THREADS), 0, s, A, lda, B, ldb, C, ldc, M,
                       N, K, transA);
    return hipGetLastError();
}

}  // namespace d2d

// ====================================================================== fused step
// Kernels of one Lanczos step with full reorthogonalisation.  A kernel that
// needs a global sum produced by the previous kernel adds that kernel's
// per-block partial sums itself (every block redundantly, in a fixed order),
// so no separate reduction launches and no inter-block fences are needed: the
// kernel boundary orders the partial sums before their use.  The number of
// blocks of these kernels is capped at LZ_STEP_NB to bound that re-reading.
namespace d2d {

static constexpr int LZ_STEP_NB = 256;

int lz_step_blocks(int64_t n) {
    int64_t nb = (n + 1023) / 1024;
    if (nb > LZ_STEP_NB) nb = LZ_STEP_NB;
    if (nb < 1) nb = 1;
    return (int)nb;
}

// out_sh[j] = sum_b partial[j*nb + b] for j < rows (shared memory result).
__device__ inline void reduce_rows(const double* __restrict__ partial, int rows, int nb, double* out_sh) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int j = wv; j < rows; j += LZ_THREADS / 64) {
        double s = 0.0;
        for (int b = lane; b < nb; b += 64) s += partial[(int64_t)j * nb + b];
        s = wave_sum(s);
        if (lane == 0) out_sh[j] = s;
    }
    __syncthreads();
}

// Per-block sums of acc[0..rows) (rows <= R) written to partial[j*nb + b].
template <int R>
__device__ inline void write_partials(const double (&acc)[R], int rows, double* __restrict__ partial, int nb,
                                      int b) {
    __shared__ double sh[LZ_THREADS / 64][R];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (j < rows) {
            const double s = wave_sum(acc[j]);
            if (lane == 0) sh[wv][j] = s;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < rows) {
        double s = 0.0;
        for (int w = 0; w < LZ_THREADS / 64; ++w) s += sh[w][threadIdx.x];
        partial[(int64_t)threadIdx.x * nb + b] = s;
    }
}

// Step kernel 1: partials of c1 = Q[0..nq)^T w (w upcast from FP32 first when UPCAST).
template <int NQ, bool UPCAST>
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_dots(const double* __restrict__ Q, int64_t ldq, int nq, const double* __restrict__ w64in,
          const float* __restrict__ w32, double* __restrict__ w64out, int64_t n, double* __restrict__ partial) {
    const int nb = gridDim.x, b = blockIdx.x;
    int64_t lo, hi;
    chunk(n, b, nb, &lo, &hi);
    double acc[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j) acc[j] = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
        double x;
        if constexpr (UPCAST) {
            x = (double)w32[e];
            w64out[e] = x;
        } else {
            x = w64in[e];
        }
        double q[NQ];
#pragma unroll
        for (int j = 0; j < NQ; ++j) q[j] = j < nq ? Q[j * ldq + e] : 0.0;
#pragma unroll
        for (int j = 0; j < NQ; ++j) acc[j] += q[j] * x;
    }
    write_partials<NQ>(acc, nq, partial, nb, b);
}

// Step kernel 2: c1 from partial_in; w <- w - Q c1; partials of c2 = Q^T w
// (rows 0..nq-1) and |w|^2 (row nq) into partial_out; alpha[i] = c1[i].
template <int NQ>
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_update_dots(const double* __restrict__ Q, int64_t ldq, int nq, const double* __restrict__ partial_in,
                 int nb_in, double* __restrict__ w, int64_t n, double* __restrict__ partial_out,
                 double* __restrict__ alpha, int i) {
    __shared__ double cs[NQ];
    if ((int)threadIdx.x < NQ) cs[threadIdx.x] = 0.0;
    __syncthreads();
    reduce_rows(partial_in, nq, nb_in, cs);
    if (blockIdx.x == 0 && threadIdx.x == 0) alpha[i] = cs[i];
    const int nb = gridDim.x, b = blockIdx.x;
    int64_t lo, hi;
    chunk(n, b, nb, &lo, &hi);
    double acc[NQ + 1];
#pragma unroll
    for (int j = 0; j <= NQ; ++j) acc[j] = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
        double q[NQ];
        double x = w[e];
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            q[j] = j < nq ? Q[j * ldq + e] : 0.0;
            x -= cs[j] * q[j];
        }
        w[e] = x;
#pragma unroll
        for (int j = 0; j < NQ; ++j) acc[j] += q[j] * x;
        acc[NQ] += x * x;
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
        partial_out[(int64_t)threadIdx.x * nb + b] = t;
    }
}

// Step kernel 3: c2 and |w|^2 from partial_in; beta = sqrt(|w|^2 - |c2|^2);
// q_next = (w - [need2] Q c2) / beta with need2 = |c2| > 1e-13 |w|;
// lo = cast(q_next); block 0 writes alpha[i] += c2[i], beta[i+1].
template <int NQ>
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_next(const double* __restrict__ Q, int64_t ldq, int nq, const double* __restrict__ partial_in, int nb_in,
          const double* __restrict__ w, double* __restrict__ qnext, void* __restrict__ lo, int lo_prec, int64_t n,
          double* __restrict__ alpha, double* __restrict__ beta, int i) {
    __shared__ double cs[NQ + 1];
    reduce_rows(partial_in, nq + 1, nb_in, cs);
    double s2 = 0.0;
    for (int j = 0; j < nq; ++j) s2 += cs[j] * cs[j];
    const double w2 = cs[nq];
    const double b2 = w2 - s2;
    const double bb = sqrt(b2 > 0.0 ? b2 : 0.0);
    const bool corr = sqrt(s2) > 1e-13 * sqrt(w2 > 0.0 ? w2 : 0.0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        alpha[i] += cs[i];
        beta[i + 1] = bb;
    }
    if (!qnext) return;
    const double inv = bb > 0.0 ? 1.0 / bb : 0.0;
    // four independent elements per thread and iteration (memory-level parallelism)
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e0 < n; e0 += 4 * stride) {
        double x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t e = e0 + u * stride;
            x[u] = e < n ? w[e] : 0.0;
        }
        if (corr)
            for (int j = 0; j < nq; ++j)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t e = e0 + u * stride;
                    if (e < n) x[u] -= cs[j] * Q[j * ldq + e];
                }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t e = e0 + u * stride;
            if (e >= n) break;
            const double q = x[u] * inv;
            qnext[e] = q;
            if (lo_prec == D2D_FP32) ((float*)lo)[e] = (float)q;
            else if (lo_prec == D2D_BF16) ((uint16_t*)lo)[e] = f32_bf16_rne((float)q);
        }
    }
}

template <int NQ>
static hipError_t lz_step_nq(const LzStepArgs& a, hipStream_t s) {
    const int nb = lz_step_blocks(a.n);
    double* p1 = a.partial;
    double* p2 = a.partial2;
    if (a.upcast)
        hipLaunchKernelGGL((k_lz_dots<NQ, true>), dim3(nb), dim3(LZ_THREADS), 0, s, a.Q, a.n, a.nq,
                           (const double*)nullptr, a.w32, a.w, a.n, p1);
    else
        hipLaunchKernelGGL((k_lz_dots<NQ, false>), dim3(nb), dim3(LZ_THREADS), 0, s, a.Q, a.n, a.nq, a.w,
                           (const float*)nullptr, (double*)nullptr, a.n, p1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_lz_update_dots<NQ>), dim3(nb), dim3(LZ_THREADS), 0, s, a.Q, a.n, a.nq, p1, nb, a.w, a.n,
                       p2, a.alpha, a.i);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int gn = a.qnext ? nb : 1;
    hipLaunchKernelGGL((k_lz_next<NQ>), dim3(gn), dim3(LZ_THREADS), 0, s, a.Q, a.n, a.nq, p2, nb, a.w, a.qnext,
                       a.lo, a.lo ? a.lo_prec : -1, a.n, a.alpha, a.beta, a.i);
    return hipGetLastError();
}

hipError_t launch_lz_step(const LzStepArgs& a, hipStream_t s) {
    if (a.nq <= 8) return lz_step_nq<8>(a, s);
    if (a.nq <= 16) return lz_step_nq<16>(a, s);
    if (a.nq <= 32) return lz_step_nq<32>(a, s);
    return hipErrorInvalidValue;
}

// Residual of the restart: partials of theta = x.w; then r = w - theta x with
// partials of |r|^2; then one block finishes alpha[0] = theta, beta[1] = rho
// and res = (theta, rho).
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_theta(const double* __restrict__ x, const double* __restrict__ w, int64_t n, double* __restrict__ partial) {
    double acc[1] = {0.0};
    const int nb = gridDim.x, b = blockIdx.x;
    int64_t lo, hi;
    chunk(n, b, nb, &lo, &hi);
    for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) acc[0] += x[e] * w[e];
    write_partials<1>(acc, 1, partial, nb, b);
}

__global__ void __launch_bounds__(LZ_THREADS)
k_lz_resid(const double* __restrict__ x, const double* __restrict__ partial_in, int nb_in, double* __restrict__ w,
           int64_t n, double* __restrict__ partial_out) {
    __shared__ double th[1];
    reduce_rows(partial_in, 1, nb_in, th);
    const double t = th[0];
    double acc[1] = {0.0};
    const int nb = gridDim.x, b = blockIdx.x;
    int64_t lo, hi;
    chunk(n, b, nb, &lo, &hi);
    for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
        const double r = w[e] - t * x[e];
        w[e] = r;
        acc[0] += r * r;
    }
    write_partials<1>(acc, 1, partial_out, nb, b);
}

__global__ void __launch_bounds__(LZ_THREADS)
k_lz_restart_finish(const double* __restrict__ p_theta, const double* __restrict__ p_rho, int nb,
                    double* __restrict__ alpha, double* __restrict__ beta, double* __restrict__ res) {
    __shared__ double v[2];
    reduce_rows(p_theta, 1, nb, v);
    reduce_rows(p_rho, 1, nb, v + 1);
    if (threadIdx.x == 0) {
        const double rho = sqrt(v[1] > 0.0 ? v[1] : 0.0);
        alpha[0] = v[0];
        beta[1] = rho;
        res[0] = v[0];
        res[1] = rho;
    }
}

hipError_t launch_lz_residual(const double* x, double* w, int64_t n, double* partial, double* partial2,
                              double* alpha, double* beta, double* res, hipStream_t s) {
    const int nb = lz_step_blocks(n);
    hipLaunchKernelGGL(k_lz_theta, dim3(nb), dim3(LZ_THREADS), 0, s, x, w, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lz_resid, dim3(nb), dim3(LZ_THREADS), 0, s, x, partial, nb, w, n, partial2);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lz_restart_finish, dim3(1), dim3(LZ_THREADS), 0, s, partial, partial2, nb, alpha, beta, res);
    return hipGetLastError();
}

// x = Q y with partials of |x|^2; then x /= |x|.
__global__ void __launch_bounds__(LZ_THREADS)
k_lz_ritz(const double* __restrict__ Q, int64_t ldq, int k, const double* __restrict__ y, double* __restrict__ x,
          int64_t n, double* __restrict__ partial) {
    __shared__ double ys[128];
    for (int j = threadIdx.x; j < k && j < 128; j += blockDim.x) ys[j] = y[j];
    __syncthreads();
    double acc[1] = {0.0};
    const int nb = gridDim.x, b = blockIdx.x;
    int64_t lo, hi;
    chunk(n, b, nb, &lo, &hi);
    for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
        double v = 0.0;
        for (int j = 0; j < k; ++j) v += ys[j] * Q[j * ldq + e];
        x[e] = v;
        acc[0] += v * v;
    }
    write_partials<1>(acc, 1, partial, nb, b);
}

__global__ void __launch_bounds__(LZ_THREADS)
k_lz_normalize(double* __restrict__ x, const double* __restrict__ partial, int nb, int64_t n) {
    __shared__ double v[1];
    reduce_rows(partial, 1, nb, v);
    const double inv = v[0] > 0.0 ? 1.0 / sqrt(v[0]) : 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        x[e] *= inv;
}

hipError_t launch_lz_ritz(const double* Q, int64_t ldq, int k, const double* y, double* x, int64_t n,
                          double* partial, hipStream_t s) {
    if (k > 128) return hipErrorInvalidValue;
    const int nb = lz_step_blocks(n);
    hipLaunchKernelGGL(k_lz_ritz, dim3(nb), dim3(LZ_THREADS), 0, s, Q, ldq, k, y, x, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lz_normalize, dim3(nb), dim3(LZ_THREADS), 0, s, x, partial, nb, n);
    return hipGetLastError();
}

}  // namespace d2d
