// The classical scheme the paper compares against (Sec. 1, eq.
// basic_identity; Sec. 5, the s_pre and s_pro columns): z = b - A^*
// (A A^*)^{-1} A b evaluated directly, with the Gram A A^* formed on MFMA and
// factored by a Householder pivoted QR (A A^*) Pi = Q R whose reflectors are
// kept.  Per right-hand side c = A b this kernel forms
//   x = Pi R^{-1} Q^T c,   Q^T c = H_{m-1} ... H_1 H_0 c,
// the solution of (A A^*) x = A b by the factorization.  It is the normal-
// equations baseline: its error grows like u cond(A)^2 (the paper's
// epsilon_norm), against u cond(A) for the preconditioned method.
//
// One workgroup per right-hand side; the vector lives in LDS.  Reflector j
// (V[j m + i] for i >= j, v_j = 1) is applied with one block reduction, then
// the back substitution with the row-major upper-triangular R runs column
// by column (y_j = c_j / R_jj, then c_i -= R_ij y_j for i < j).
#include "rt_common.h"

namespace rt {

namespace {

constexpr int QS_THREADS = 256;
constexpr int QS_WAVES = QS_THREADS / 64;

__device__ __forceinline__ double block_sum(double v, double *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();  // red[] free from the previous use
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < QS_WAVES; ++w) s += red[w];
    return s;
}

__global__ __launch_bounds__(QS_THREADS) void qr_solve_kernel(int m, const double *__restrict__ V,
                                                               const double *__restrict__ tau,
                                                               const double *__restrict__ R,
                                                               const int32_t *__restrict__ piv,
                                                               const double *__restrict__ C, int64_t ldc,
                                                               double *__restrict__ X, int64_t ldx)
{
    extern __shared__ double c[];
    __shared__ double red[QS_WAVES];
    const int col = blockIdx.x, tid = threadIdx.x;
    const double *cc = C + (int64_t)col * ldc;
    for (int i = tid; i < m; i += QS_THREADS) c[i] = cc[i];
    __syncthreads();
    // Q^T c: reflectors in factorization order
    for (int j = 0; j < m; ++j) {
        const double *v = V + (int64_t)j * m;
        double part = 0.0;
        for (int i = j + tid; i < m; i += QS_THREADS) part += v[i] * c[i];
        const double s = tau[j] * block_sum(part, red);
        for (int i = j + tid; i < m; i += QS_THREADS) c[i] -= s * v[i];
        __syncthreads();
    }
    // R y = Q^T c, column-oriented back substitution
    for (int j = m - 1; j >= 0; --j) {
        const double yj = c[j] / R[(int64_t)j * m + j];
        __syncthreads();
        if (tid == 0) c[j] = yj;
        for (int i = tid; i < j; i += QS_THREADS) c[i] -= R[(int64_t)i * m + j] * yj;
        __syncthreads();
    }
    // x = Pi y: entry k of y belongs to column piv[k] of A A^*
    double *xc = X + (int64_t)col * ldx;
    for (int k = tid; k < m; k += QS_THREADS) xc[piv[k]] = c[k];
}

}  // namespace

hipError_t qr_solve_f64(int m, const double *V, const double *tau, const double *R, const int32_t *piv,
                        const double *C, int64_t ldc, double *X, int64_t ldx, int k, hipStream_t stream)
{
    if (k <= 0 || m <= 0) return hipSuccess;
    hipLaunchKernelGGL(qr_solve_kernel, dim3((unsigned)k), dim3(QS_THREADS), (size_t)m * sizeof(double), stream, m, V,
                       tau, R, piv, C, ldc, X, ldx);
    return hipGetLastError();
}

}  // namespace rt
