// Small dense kernels of the preconditioner: inverses of triangular diagonal
// blocks (the blocked solves with R^T and with the Cholesky factor use them
// so that every off-diagonal step is an MFMA GEMM), the Cholesky of one
// diagonal block of the Gram (the factorization that replaces the explicit
// inverse Y = X^{-1} of eq. inversion), and helpers.
#include "rt_common.h"

namespace rt {

namespace {

constexpr int NBMAX = 64;

constexpr int LDP = NBMAX + 1;  // padded LDS row stride

// X = L^{-1} for the NBMAX x NBMAX lower-triangular L in LDS (row stride LDP).
// Columns are independent: four lanes own column j = tid/4 and split the dot
// products of the forward substitution
//   X[i][j] = -(sum_{j<=k<i} L[i][k] X[k][j]) / L[i][i],  X[j][j] = 1/L[j][j],
// so no block barrier is needed inside.
__device__ void lower_inverse_lds(const double *L, double *X)
{
    const int j = threadIdx.x >> 2, q = threadIdx.x & 3;
    for (int i = 0; i < NBMAX; ++i) {
        double s = 0.0;
        if (i > j)
            for (int k = j + q; k < i; k += 4) s += L[i * LDP + k] * X[k * LDP + j];
        s += __shfl_xor(s, 1, 64);
        s += __shfl_xor(s, 2, 64);
        if (q == 0) {
            const double d = L[i * LDP + i];
            X[i * LDP + j] = (i > j) ? -s / d : ((i == j) ? 1.0 / d : 0.0);
        }
        // the four lanes of a column are in one wave: they see each other's
        // LDS writes after a wave-level barrier
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void tri_diag_inv_kernel(const double *T, int64_t t_i, int64_t t_j, int m, int nb,
                                                           double *Dinv)
{
    __shared__ double L[NBMAX * LDP];
    __shared__ double X[NBMAX * LDP];
    const int b = blockIdx.x;
    const int base = b * nb, nbb = min(nb, m - base);
    for (int e = threadIdx.x; e < NBMAX * NBMAX; e += blockDim.x) {
        const int i = e / NBMAX, j = e % NBMAX;
        double v;
        if (i < nbb && j < nbb) v = (j <= i) ? T[(int64_t)(base + i) * t_i + (int64_t)(base + j) * t_j] : 0.0;
        else v = (i == j) ? 1.0 : 0.0;
        L[i * LDP + j] = v;
    }
    __syncthreads();
    lower_inverse_lds(L, X);
    double *out = Dinv + (int64_t)b * nb * nb;
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) out[e] = X[(e / nb) * LDP + (e % nb)];
}

// Cholesky of one NBMAX x NBMAX diagonal block (right-looking).  Four lanes
// own row i = tid/4 and split its columns by c mod 4.
__global__ __launch_bounds__(256) void chol_diag_kernel(const double *Xg, int64_t ldx, int m, int nb, int b, double *Lg,
                                                        int64_t ldl, double *Dinv, int *err)
{
    __shared__ double A[NBMAX * LDP];
    __shared__ double X[NBMAX * LDP];
    __shared__ int bad;
    const int base = b * nb, nbb = min(nb, m - base);
    for (int e = threadIdx.x; e < NBMAX * NBMAX; e += blockDim.x) {
        const int i = e / NBMAX, j = e % NBMAX;
        double v;
        if (i < nbb && j < nbb) v = (j <= i) ? Xg[(int64_t)(base + i) * ldx + base + j] : 0.0;
        else v = (i == j) ? 1.0 : 0.0;
        A[i * LDP + j] = v;
    }
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    __shared__ double colj[NBMAX];
    __shared__ double diag[NBMAX];
    const int i = threadIdx.x >> 2, q = threadIdx.x & 3;
    for (int j = 0; j < NBMAX; ++j) {
        const double d = A[j * LDP + j];
        if (!(d > 0.0) || !isfinite(d)) {
            if (threadIdx.x == 0) bad = 1;
            break;
        }
        const double ljj = __builtin_sqrt(d);
        // column j of L into its own vector, so the update below reads it
        // without any dependence on the stores into A.  The diagonal entry is
        // kept aside (every thread has just read A[j][j]) and stored after
        // the loop.
        if (q == 0 && i >= j) {
            const double lij = (i == j) ? ljj : A[i * LDP + j] / ljj;
            colj[i] = lij;
            if (i == j) diag[j] = ljj;
            else A[i * LDP + j] = lij;
        }
        __syncthreads();
        if (i > j) {
            const double lij = colj[i];
            const int c0 = j + 1 + ((q - (j + 1)) & 3);
#pragma unroll
            for (int r = 0; r < NBMAX / 4; ++r) {
                const int c = c0 + 4 * r;
                if (c <= i) A[i * LDP + c] -= lij * colj[c];
            }
        }
        __syncthreads();
    }
    __syncthreads();
    if (bad) {
        if (threadIdx.x == 0) atomicExch(err, 1);
        return;
    }
    if (threadIdx.x < NBMAX) A[threadIdx.x * LDP + threadIdx.x] = diag[threadIdx.x];
    for (int e = threadIdx.x; e < NBMAX * NBMAX; e += blockDim.x) {
        const int r = e / NBMAX, c = e % NBMAX;
        if (c > r) A[r * LDP + c] = 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nbb * nbb; e += blockDim.x) {
        const int r = e / nbb, c = e % nbb;
        Lg[(int64_t)(base + r) * ldl + base + c] = A[r * LDP + c];
    }
    lower_inverse_lds(A, X);
    double *out = Dinv + (int64_t)b * nb * nb;
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) out[e] = X[(e / nb) * LDP + (e % nb)];
}

__global__ void set_matrix_kernel(double *X, int64_t ld, int m, int n, int ident)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * n) return;
    const int i = (int)(e / n), j = (int)(e % n);
    X[(int64_t)i * ld + j] = (ident && i == j) ? 1.0 : 0.0;
}

__global__ void zero_triangle_kernel(double *X, int64_t ld, int m, int upper)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * m) return;
    const int i = (int)(e / m), j = (int)(e % m);
    if ((upper && j > i) || (!upper && j < i)) X[(int64_t)i * ld + j] = 0.0;
}

__global__ void rdiag_kernel(const double *R, int64_t ldr, int m, double *out)
{
    __shared__ double smin[256], smax[256];
    double lo = INFINITY, hi = 0.0;
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const double d = fabs(R[(int64_t)i * ldr + i]);
        lo = (d < lo || d != d) ? d : lo;
        hi = (d > hi || d != d) ? d : hi;
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double a = smin[threadIdx.x + s], c = smax[threadIdx.x + s];
            if (a < smin[threadIdx.x] || a != a) smin[threadIdx.x] = a;
            if (c > smax[threadIdx.x] || c != c) smax[threadIdx.x] = c;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = fabs(R[0]);
        out[1] = fabs(R[(int64_t)(m - 1) * ldr + (m - 1)]);
        out[2] = smin[0];
        out[3] = smax[0];
    }
}

// out[0] = T'^T and out[1] = T' (row-major m x m each) for T' = T Pi:
// column piv[c] of T' is column c of T.
__global__ void form_tp_kernel(const double *T, const int32_t *piv, int m, double *out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * m) return;
    const int r = (int)(e / m), c = (int)(e % m);
    const double v = T[e];
    const int pc = piv[c];
    out[(int64_t)pc * m + r] = v;
    out[(int64_t)m * m + (int64_t)r * m + pc] = v;
}

}  // namespace

hipError_t form_tp_f64(const double *T, const int32_t *piv, int m, double *out, hipStream_t stream)
{
    const int64_t total = (int64_t)m * m;
    hipLaunchKernelGGL(form_tp_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, T, piv, m, out);
    return hipGetLastError();
}

hipError_t tri_diag_inv_f64(const double *T, int64_t t_i, int64_t t_j, int m, int nb, double *Dinv, hipStream_t stream)
{
    if (nb != NBMAX) return hipErrorInvalidValue;
    const int nblk = (m + nb - 1) / nb;
    hipLaunchKernelGGL(tri_diag_inv_kernel, dim3(nblk), dim3(256), 0, stream, T, t_i, t_j, m, nb, Dinv);
    return hipGetLastError();
}

hipError_t chol_diag_f64(const double *X, int64_t ldx, int m, int nb, int b, double *L, int64_t ldl, double *Dinv,
                         int *err, hipStream_t stream)
{
    if (nb != NBMAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(256), 0, stream, X, ldx, m, nb, b, L, ldl, Dinv, err);
    return hipGetLastError();
}

hipError_t set_matrix_f64(double *X, int64_t ld, int m, int n, int ident, hipStream_t stream)
{
    const int64_t total = (int64_t)m * n;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(set_matrix_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, X, ld, m, n,
                       ident);
    return hipGetLastError();
}

hipError_t zero_triangle_f64(double *X, int64_t ld, int m, int upper, hipStream_t stream)
{
    const int64_t total = (int64_t)m * m;
    hipLaunchKernelGGL(zero_triangle_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, X, ld, m,
                       upper);
    return hipGetLastError();
}

hipError_t rdiag_ends_f64(const double *R, int64_t ldr, int m, double *out, hipStream_t stream)
{
    hipLaunchKernelGGL(rdiag_kernel, dim3(1), dim3(256), 0, stream, R, ldr, m, out);
    return hipGetLastError();
}

}  // namespace rt
