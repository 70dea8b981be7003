// Conjugate gradients on the well-conditioned normal matrix W W^T, W =
// P^{-1}A, for the iterative variant of the method (Sec. 1: a
// preconditioned iterative approach is also feasible; Remark 4.3).  The
// caller forms the products q = W W^T pp; these kernels do the per-column
// scalar work of CG for k independent right-hand sides (column-major m x k
// blocks, leading dimension m), one workgroup per column:
//   cg_init:  r = t, pp = t, u = 0, gamma = r.r
//   cg_step:  alpha = gamma / (pp.q), u += alpha pp, r -= alpha q,
//             gamma' = r.r, pp = r + (gamma' / gamma) pp, gamma = gamma'
// A zero gamma or pp.q (an exactly converged column) leaves that column
// unchanged.
#include "rt_common.h"

namespace rt {

namespace {

constexpr int CG_T = 256;

__device__ __forceinline__ double cg_block_sum(double v, double *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < CG_T / 64; ++w) s += red[w];
    return s;
}

__global__ __launch_bounds__(CG_T) void cg_init_kernel(int m, const double *t, double *u, double *r, double *pp,
                                                       double *gamma)
{
    __shared__ double red[CG_T / 64];
    const int64_t off = (int64_t)blockIdx.x * m;
    double g = 0.0;
    for (int i = threadIdx.x; i < m; i += CG_T) {
        const double v = t[off + i];
        r[off + i] = v;
        pp[off + i] = v;
        u[off + i] = 0.0;
        g += v * v;
    }
    g = cg_block_sum(g, red);
    if (threadIdx.x == 0) gamma[blockIdx.x] = g;
}

__global__ __launch_bounds__(CG_T) void cg_step_kernel(int m, double *u, double *r, double *pp, const double *q,
                                                       double *gamma)
{
    __shared__ double red[CG_T / 64];
    const int64_t off = (int64_t)blockIdx.x * m;
    const double g = gamma[blockIdx.x];
    double d = 0.0;
    for (int i = threadIdx.x; i < m; i += CG_T) d += pp[off + i] * q[off + i];
    d = cg_block_sum(d, red);
    const double alpha = (d > 0.0 && g > 0.0) ? g / d : 0.0;
    double gn = 0.0;
    for (int i = threadIdx.x; i < m; i += CG_T) {
        u[off + i] += alpha * pp[off + i];
        const double ri = r[off + i] - alpha * q[off + i];
        r[off + i] = ri;
        gn += ri * ri;
    }
    gn = cg_block_sum(gn, red);
    const double beta = g > 0.0 ? gn / g : 0.0;
    for (int i = threadIdx.x; i < m; i += CG_T) pp[off + i] = r[off + i] + beta * pp[off + i];
    if (threadIdx.x == 0) gamma[blockIdx.x] = gn;
}

}  // namespace

hipError_t cg_init_f64(int m, int k, const double *t, double *u, double *r, double *pp, double *gamma,
                       hipStream_t stream)
{
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(cg_init_kernel, dim3((unsigned)k), dim3(CG_T), 0, stream, m, t, u, r, pp, gamma);
    return hipGetLastError();
}

hipError_t cg_step_f64(int m, int k, double *u, double *r, double *pp, const double *q, double *gamma,
                       hipStream_t stream)
{
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(cg_step_kernel, dim3((unsigned)k), dim3(CG_T), 0, stream, m, u, r, pp, q, gamma);
    return hipGetLastError();
}

}  // namespace rt
