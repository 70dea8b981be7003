// Column-pivoted Householder QR of the sketch, S^T = Q R Pi (Sec. 4,
// eq. QR_decomp), Businger-Golub pivoting: at step k the pivot is the
// remaining column with the largest trailing 2-norm (ties: lowest index).
//
// One cooperative launch.  Block g owns columns j = g, g + G, g + 2G, ... of
// S^T and keeps them resident in LDS for the whole factorization.  Each step:
//   1. every block posts its best candidate (trailing norm^2, column);
//   2. grid barrier;
//   3. every block reads the G candidates and agrees on the pivot p;
//   4. p's owner forms the reflector H = I - tau v v^T (v[k] = 1,
//      beta = -sign(alpha) |x|), writes v, tau, the new column of R and
//      piv[k], then raises a flag; the other blocks wait for the flag;
//   5. every block applies H to its remaining columns and, in the same
//      pass, accumulates the trailing norms for the next step.
// The norms are recomputed exactly every step (no downdating).  Every wait is
// bounded: a block that spins too long records an error and returns, so the
// grid always drains.
#include "rt_common.h"

namespace rt {

namespace {

constexpr int QR_THREADS = 256;
constexpr int QR_MAXCOL = 16;  // columns per block
constexpr long SPIN_LIMIT = 1L << 20;

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum `n` per-thread values across the block; result in out[0..n) (LDS) for
// all threads after return.
__device__ void block_sums(double *vals, int n, double *scratch, double *out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c = 0; c < n; ++c) {
        const double s = wave_sum(vals[c]);
        if (lane == 0) scratch[wave * QR_MAXCOL + c] = s;
    }
    __syncthreads();
    if (threadIdx.x < n) {
        double s = 0.0;
        for (int w = 0; w < QR_THREADS / 64; ++w) s += scratch[w * QR_MAXCOL + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

__global__ __launch_bounds__(QR_THREADS) void qrcp_kernel(const double *S, int64_t lds, int rows, int cols,
                                                          double *R, int32_t *piv, QrcpWork w, int G, int ncol_max)
{
    extern __shared__ double smem[];
    double *colbuf = smem;                          // ncol_max x rows
    double *v = smem + (int64_t)ncol_max * rows;    // rows
    __shared__ double scratch[(QR_THREADS / 64) * QR_MAXCOL];
    __shared__ double nrm[QR_MAXCOL];
    __shared__ double dots[QR_MAXCOL];
    __shared__ int done[QR_MAXCOL];
    __shared__ int s_p, s_abort;
    __shared__ double s_pn, s_tau;

    const int g = blockIdx.x, tid = threadIdx.x;
    int ncol = 0;
    while (ncol < ncol_max && g + G * ncol < cols) ++ncol;

    for (int c = 0; c < ncol; ++c) {
        const double *src = S + (int64_t)(g + G * c) * lds;
        for (int i = tid; i < rows; i += QR_THREADS) colbuf[(int64_t)c * rows + i] = src[i];
    }
    if (tid < QR_MAXCOL) done[tid] = 0;
    if (tid == 0) s_abort = 0;
    double part[QR_MAXCOL];
    for (int c = 0; c < QR_MAXCOL; ++c) part[c] = 0.0;
    __syncthreads();
    for (int c = 0; c < ncol; ++c)
        for (int i = tid; i < rows; i += QR_THREADS) {
            const double x = colbuf[(int64_t)c * rows + i];
            part[c] += x * x;
        }
    block_sums(part, ncol, scratch, nrm);

    for (int k = 0; k < cols; ++k) {
        const int buf = k & 1;
        // 1. post the local candidate
        if (tid == 0) {
            double bn = -1.0;
            int bj = -1;
            for (int c = 0; c < ncol; ++c)
                if (!done[c] && nrm[c] > bn) { bn = nrm[c]; bj = g + G * c; }
            w.slots[(buf * G + g) * 2 + 0] = bn;
            w.slots[(buf * G + g) * 2 + 1] = (double)bj;
            // 2. grid barrier (arrival counter is monotonic across steps)
            __hip_atomic_fetch_add(w.counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned target = (unsigned)(k + 1) * (unsigned)G;
            long spins = 0;
            while (__hip_atomic_load(w.counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > SPIN_LIMIT || __hip_atomic_load(w.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    __hip_atomic_store(w.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    s_abort = 1;
                    break;
                }
            }
        }
        __syncthreads();
        if (s_abort) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        // 3. agree on the pivot (wave 0 scans the G candidates)
        if (tid < 64) {
            double bn = -2.0;
            int bj = 0x7fffffff;
            for (int q = tid; q < G; q += 64) {
                const double n = w.slots[(buf * G + q) * 2 + 0];
                const int j = (int)w.slots[(buf * G + q) * 2 + 1];
                if (j >= 0 && (n > bn || (n == bn && j < bj))) { bn = n; bj = j; }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double on = __shfl_xor(bn, o, 64);
                const int oj = __shfl_xor(bj, o, 64);
                if (on > bn || (on == bn && oj < bj)) { bn = on; bj = oj; }
            }
            if (tid == 0) { s_p = bj; s_pn = bn; }
        }
        __syncthreads();
        const int p = s_p;
        if (p < 0 || p >= cols) {
            // no finite candidate anywhere (NaN input): every block sees the
            // same candidates, so every block leaves here together
            if (tid == 0 && g == 0) __hip_atomic_store(w.err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        if (p % G == g) {
            // 4. owner: reflector from the trailing part of column p
            const int c = p / G;
            double *x = colbuf + (int64_t)c * rows;
            const double alpha = x[k];
            const double xnorm = __builtin_sqrt(s_pn);
            double beta, tau, inv;
            if (xnorm == 0.0) { beta = 0.0; tau = 0.0; inv = 0.0; }
            else {
                beta = alpha >= 0.0 ? -xnorm : xnorm;
                tau = (beta - alpha) / beta;
                inv = 1.0 / (alpha - beta);
            }
            double *vg = w.vbuf + (int64_t)buf * rows;
            for (int i = k + tid; i < rows; i += QR_THREADS) {
                const double vi = (i == k) ? 1.0 : x[i] * inv;
                v[i] = vi;
                vg[i] = vi;
            }
            for (int i = tid; i < k; i += QR_THREADS) R[(int64_t)i * cols + k] = x[i];
            if (tid == 0) {
                R[(int64_t)k * cols + k] = beta;
                piv[k] = p;
                w.scal[buf * 4 + 0] = tau;
                s_tau = tau;
                done[c] = 1;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (tid == 0) __hip_atomic_store(w.flag, (unsigned)(k + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (tid == 0) {
                long spins = 0;
                while (__hip_atomic_load(w.flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)(k + 1)) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > SPIN_LIMIT || __hip_atomic_load(w.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        __hip_atomic_store(w.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        s_abort = 1;
                        break;
                    }
                }
            }
            __syncthreads();
            if (s_abort) return;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const double *vg = w.vbuf + (int64_t)buf * rows;
            for (int i = k + tid; i < rows; i += QR_THREADS) v[i] = vg[i];
            if (tid == 0) s_tau = w.scal[buf * 4 + 0];
        }
        __syncthreads();
        // 5. apply H_k to the remaining owned columns; accumulate next norms
        const double tau = s_tau;
        for (int c = 0; c < QR_MAXCOL; ++c) part[c] = 0.0;
        for (int c = 0; c < ncol; ++c) {
            if (done[c]) continue;
            const double *x = colbuf + (int64_t)c * rows;
            for (int i = k + tid; i < rows; i += QR_THREADS) part[c] += v[i] * x[i];
        }
        block_sums(part, ncol, scratch, dots);
        for (int c = 0; c < QR_MAXCOL; ++c) part[c] = 0.0;
        for (int c = 0; c < ncol; ++c) {
            if (done[c]) continue;
            double *x = colbuf + (int64_t)c * rows;
            const double f = tau * dots[c];
            for (int i = k + tid; i < rows; i += QR_THREADS) {
                const double nx = x[i] - f * v[i];
                x[i] = nx;
                if (i > k) part[c] += nx * nx;
            }
        }
        block_sums(part, ncol, scratch, nrm);
    }
}

__global__ void zero_u32_kernel(unsigned *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

}  // namespace

int qrcp_max_blocks(int rows, int cols, int cu_count, size_t lds_max)
{
    // smallest column count per block that fits LDS, then as many blocks as
    // there are compute units (one resident block per CU at most).
    for (int ncol = 1; ncol <= QR_MAXCOL; ++ncol) {
        const size_t need = ((size_t)ncol + 1) * (size_t)rows * sizeof(double) + 4096;
        if (need > lds_max) return -1;
        const int G = (cols + ncol - 1) / ncol;
        if (G <= cu_count) return G;
    }
    return -1;
}

hipError_t zero_u32(unsigned *p, int n, hipStream_t stream)
{
    hipLaunchKernelGGL(zero_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t qrcp_f64(const double *S, int64_t lds, int rows, int cols, double *R, int32_t *piv, const QrcpWork &w,
                    int blocks, size_t lds_bytes_max, hipStream_t stream)
{
    const int G = blocks;
    const int ncol_max = (cols + G - 1) / G;
    if (ncol_max > QR_MAXCOL) return hipErrorInvalidValue;
    const size_t shmem = ((size_t)ncol_max + 1) * (size_t)rows * sizeof(double);
    if (shmem > lds_bytes_max) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)qrcp_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)shmem);
    if (e != hipSuccess) return e;
    // counter, flag and err live in one 4-word block
    e = zero_u32(w.counter, 4, stream);
    if (e != hipSuccess) return e;
    QrcpWork wk = w;
    int rows_ = rows, cols_ = cols, G_ = G, ncm = ncol_max;
    int64_t lds_ = lds;
    void *args[] = {(void *)&S, (void *)&lds_, (void *)&rows_, (void *)&cols_, (void *)&R, (void *)&piv,
                    (void *)&wk, (void *)&G_, (void *)&ncm};
    return hipLaunchCooperativeKernel((const void *)qrcp_kernel, dim3(G), dim3(QR_THREADS), args, (unsigned)shmem,
                                      stream);
}

}  // namespace rt
