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
