// Column-pivoted Householder QR of the sketch, S^T = Q R Pi (Sec. 4,
// eq. QR_decomp), Businger-Golub pivoting: at step k the pivot is the
// remaining column with the largest trailing 2-norm (ties: lowest index).
//
// One cooperative launch.  Block g owns columns j = g, g + G, g + 2G, ... of
// the input and keeps them for the whole factorization in LDS (or, for
// sketches too tall for LDS, in a private slice of global memory).  Each step
// costs ONE grid barrier:
//   1. every block posts its best remaining column (trailing norm^2, index,
//      and the trailing part of the column itself) to a double-buffered slot;
//   2. grid barrier;
//   3. every block reads the G candidates, agrees on the pivot p (largest
//      norm, lowest index) and rebuilds the reflector H = I - tau v v^T
//      (v[k] = 1, beta = -sign(alpha)|x|) from p's posted column;
//   4. p's owner writes the new column of R and piv[k];
//   5. every block applies H to its remaining columns and, in the same pass,
//      accumulates the trailing norms for the next step.
// Norms are recomputed exactly every step (no downdating).  Every wait is
// bounded: a block that spins too long records an error and returns, so the
// grid always drains.
#include <algorithm>

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

// Sum over each group of TPC consecutive lanes; every lane of the group gets
// the result.  Groups wider than a wave combine the wave sums through LDS
// (`scratch`, one slot per wave) with two block barriers.
template <int TPC>
__device__ __forceinline__ double group_sum(double v, double *scratch)
{
    if constexpr (TPC <= 64) {
#pragma unroll
        for (int o = TPC / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        return v;
    } else {
        v = wave_sum(v);
        const int wave = threadIdx.x >> 6, w0 = (wave * 64 / TPC) * (TPC / 64);
        if ((threadIdx.x & 63) == 0) scratch[wave] = v;
        __syncthreads();
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < TPC / 64; ++w) s += scratch[w0 + w];
        __syncthreads();
        return s;
    }
}

__device__ __forceinline__ bool spin_until(unsigned *addr, unsigned target, int *err)
{
    long spins = 0;
    // relaxed polling (no cache invalidation per poll); the caller issues one
    // acquire fence after the wait
    while (__hip_atomic_load(addr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > SPIN_LIMIT || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    return true;
}

// GCOLS: the block's columns live in global memory (w.cols + g*NC*rows,
// private to the block) instead of LDS, for sketches too tall for LDS.
template <int NC, bool GCOLS>
__global__ __launch_bounds__(QR_THREADS) void qrcp_kernel(const double *S, int64_t lds, int rows, int cols,
                                                          double *R, int32_t *piv, QrcpWork w, int G)
{
    extern __shared__ double smem[];
    double *colbuf = GCOLS ? w.cols + (int64_t)blockIdx.x * NC * rows : smem;  // NC x rows
    double *v = GCOLS ? smem : smem + (int64_t)NC * rows;                       // rows
    __shared__ double scratch[(QR_THREADS / 64) * QR_MAXCOL];
    __shared__ double nrm[QR_MAXCOL];
    __shared__ int done[QR_MAXCOL];
    __shared__ int s_p, s_abort, s_best;
    __shared__ double s_pn;

    const int g = blockIdx.x, tid = threadIdx.x;
    int ncol = 0;
    while (ncol < NC && g + G * ncol < cols) ++ncol;
    // candidate slots: header (norm^2, column) and the column's values
    double *hdr = w.slots;                 // 2 x G x 2
    double *cand = w.vbuf;                 // 2 x G x rows

    for (int c = 0; c < ncol; ++c) {
        const double *src = S + (int64_t)(g + G * c) * lds;
        for (int i = tid; i < rows; i += QR_THREADS) colbuf[(int64_t)c * rows + i] = src[i];
    }
    if (tid < QR_MAXCOL) done[tid] = (tid < ncol) ? 0 : 1;
    if (tid == 0) s_abort = 0;
    __syncthreads();
    // each column is owned by a group of TPC = 256/NC consecutive lanes
    constexpr int TPC = QR_THREADS / NC;
    const int mc = tid / TPC, mq = tid % TPC;
    const bool mine = mc < ncol;
    {
        double part = 0.0;
        if (mine)
            for (int i = mq; i < rows; i += TPC) {
                const double x = colbuf[(int64_t)mc * rows + i];
                part += x * x;
            }
        part = group_sum<TPC>(part, scratch);
        if (mine && mq == 0) nrm[mc] = part;
        __syncthreads();
    }

    for (int k = 0; k < cols; ++k) {
        const int buf = k & 1;
        // 1. post the local candidate
        if (tid == 0) {
            double bn = -1.0;
            int bc = -1;
            for (int c = 0; c < ncol; ++c)
                if (!done[c] && nrm[c] > bn) { bn = nrm[c]; bc = c; }
            s_best = bc;
            hdr[(buf * G + g) * 2 + 0] = bn;
            hdr[(buf * G + g) * 2 + 1] = bc >= 0 ? (double)(g + G * bc) : -1.0;
        }
        __syncthreads();
        if (s_best >= 0) {
            const double *x = colbuf + (int64_t)s_best * rows;
            double *dst = cand + ((int64_t)buf * G + g) * rows;
            for (int i = k + tid; i < rows; i += QR_THREADS) dst[i] = x[i];
        }
        // every wave's stores are complete before the barrier; one agent-scope
        // release (L2 write-back) per block then publishes them
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        // 2. grid barrier (arrival counter is monotonic across steps)
        if (tid == 0) {
            __hip_atomic_fetch_add(w.counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            if (!spin_until(w.counter, (unsigned)(k + 1) * (unsigned)G, w.err)) s_abort = 1;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (s_abort) return;
        // 3. agree on the pivot (wave 0 scans the G candidates)
        if (tid < 64) {
            double bn = -2.0;
            int bj = 0x7fffffff;
            for (int q = tid; q < G; q += 64) {
                const double n = hdr[(buf * G + q) * 2 + 0];
                const int j = (int)hdr[(buf * G + q) * 2 + 1];
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
        const double *xp = cand + ((int64_t)buf * G + (p % G)) * rows;
        const double alpha = xp[k];
        const double xnorm = __builtin_sqrt(s_pn);
        double beta, tau, inv;
        if (xnorm == 0.0) { beta = 0.0; tau = 0.0; inv = 0.0; }
        else {
            beta = alpha >= 0.0 ? -xnorm : xnorm;
            tau = (beta - alpha) / beta;
            inv = 1.0 / (alpha - beta);
        }
        for (int i = k + tid; i < rows; i += QR_THREADS) v[i] = (i == k) ? 1.0 : xp[i] * inv;
        // 4. owner: column k of R and piv[k]
        if (p % G == g) {
            const int c = p / G;
            const double *x = colbuf + (int64_t)c * rows;
            for (int i = tid; i < k; i += QR_THREADS) R[(int64_t)i * cols + k] = x[i];
            if (tid == 0) {
                R[(int64_t)k * cols + k] = beta;
                piv[k] = p;
                done[c] = 1;
            }
        }
        __syncthreads();
        // 5. apply H_k to the remaining owned columns; accumulate next norms
        {
            const bool act = mine && !done[mc];
            double *x = colbuf + (int64_t)mc * rows;
            const int i0 = k + ((mq - k % TPC + TPC) % TPC);
            double dot = 0.0;
            if (act)
                for (int i = i0; i < rows; i += TPC) dot += v[i] * x[i];
            dot = group_sum<TPC>(dot, scratch);
            double nn = 0.0;
            if (act) {
                const double f = tau * dot;
                for (int i = i0; i < rows; i += TPC) {
                    const double nx = x[i] - f * v[i];
                    x[i] = nx;
                    if (i > k) nn += nx * nx;
                }
            }
            nn = group_sum<TPC>(nn, scratch);
            if (act && mq == 0) nrm[mc] = nn;
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Register-resident form (the default): 512 threads, block g keeps its NC
// columns in registers, thread t owning rows t, t + 512, ..., so that each
// thread reads the reflector's entries for its rows once and applies them to
// all NC columns; dot products and trailing norms are block reductions.  The
// pivot column is read straight from its owner's posted copy.
constexpr int RQ_T = 512;
constexpr int RQ_W = RQ_T / 64;

template <int NC>
__device__ __forceinline__ void block_sums(double (&v)[NC], double (*red)[NC], double *out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = wave_sum(v[c]);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NC; ++c) red[wave][c] = v[c];
    __syncthreads();
    if (threadIdx.x < NC) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < RQ_W; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

template <int NC, int RPT>
__global__ __launch_bounds__(RQ_T) void qrcp_reg_kernel(const double *S, int64_t lds, int rows, int cols, double *R,
                                                        int32_t *piv, QrcpWork w, int G)
{
    __shared__ double red[RQ_W][NC];
    __shared__ double s_dot[NC], nrm[NC];
    __shared__ int done[NC];
    __shared__ int s_p, s_abort, s_best;
    __shared__ double s_pn;
    const int g = blockIdx.x, tid = threadIdx.x;
    int ncol = 0;
    while (ncol < NC && g + G * ncol < cols) ++ncol;
    double *hdr = w.slots;  // 2 x G x 2: candidate (norm^2, column)
    double *cand = w.vbuf;  // 2 x G x rows: candidate columns

    double x[NC][RPT];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = tid + RQ_T * r;
            x[c][r] = (c < ncol && i < rows) ? S[(int64_t)(g + G * c) * lds + i] : 0.0;
        }
    if (tid < NC) done[tid] = (tid < ncol) ? 0 : 1;
    if (tid == 0) s_abort = 0;
    {
        double part[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            part[c] = 0.0;
#pragma unroll
            for (int r = 0; r < RPT; ++r) part[c] += x[c][r] * x[c][r];
        }
        block_sums<NC>(part, red, nrm);
    }

    for (int k = 0; k < cols; ++k) {
        const int buf = k & 1;
        // 1. post the local candidate (header and rows >= k of its column)
        if (tid == 0) {
            double bn = -1.0;
            int bc = -1;
            for (int c = 0; c < ncol; ++c)
                if (!done[c] && nrm[c] > bn) { bn = nrm[c]; bc = c; }
            s_best = bc;
            hdr[(buf * G + g) * 2 + 0] = bn;
            hdr[(buf * G + g) * 2 + 1] = bc >= 0 ? (double)(g + G * bc) : -1.0;
        }
        __syncthreads();
        const int best = s_best;
        if (best >= 0) {
            double *dst = cand + ((int64_t)buf * G + g) * rows;
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = tid + RQ_T * r;
                double val = 0.0;
#pragma unroll
                for (int c = 0; c < NC; ++c) val = (c == best) ? x[c][r] : val;
                if (i >= k && i < rows) dst[i] = val;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        // 2. grid barrier (arrival counter is monotonic across steps)
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(w.counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!spin_until(w.counter, (unsigned)(k + 1) * (unsigned)G, w.err)) s_abort = 1;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (s_abort) return;
        // 3. agree on the pivot (wave 0 scans the G candidates)
        if (tid < 64) {
            double bn = -2.0;
            int bj = 0x7fffffff;
            for (int q = tid; q < G; q += 64) {
                const double n = hdr[(buf * G + q) * 2 + 0];
                const int j = (int)hdr[(buf * G + q) * 2 + 1];
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
            if (tid == 0 && g == 0) __hip_atomic_store(w.err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        // 4. reflector entries for this thread's rows, from the posted column
        const double *xp = cand + ((int64_t)buf * G + (p % G)) * rows;
        const double alpha = xp[k];
        const double xnorm = __builtin_sqrt(s_pn);
        double beta, tau, inv;
        if (xnorm == 0.0) { beta = 0.0; tau = 0.0; inv = 0.0; }
        else {
            beta = alpha >= 0.0 ? -xnorm : xnorm;
            tau = (beta - alpha) / beta;
            inv = 1.0 / (alpha - beta);
        }
        double v[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = tid + RQ_T * r;
            v[r] = (i == k) ? 1.0 : ((i > k && i < rows) ? xp[i] * inv : 0.0);
        }
        // 5. owner: column k of R and piv[k]
        if (p % G == g) {
            const int c = p / G;
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = tid + RQ_T * r;
                double val = 0.0;
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) val = (cc == c) ? x[cc][r] : val;
                if (i < k) R[(int64_t)i * cols + k] = val;
            }
            if (tid == 0) {
                R[(int64_t)k * cols + k] = beta;
                piv[k] = p;
                done[c] = 1;
            }
        }
        // 6. dot products v . x_c (block sums), then the update and the next
        //    trailing norms
        {
            double d[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                d[c] = 0.0;
#pragma unroll
                for (int r = 0; r < RPT; ++r) d[c] += v[r] * x[c][r];
            }
            block_sums<NC>(d, red, s_dot);
        }
        {
            double nn[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const bool act = !done[c];
                const double f = act ? tau * s_dot[c] : 0.0;
                nn[c] = 0.0;
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int i = tid + RQ_T * r;
                    const double nx = x[c][r] - f * v[r];
                    x[c][r] = nx;
                    if (i > k) nn[c] += nx * nx;
                }
            }
            block_sums<NC>(nn, red, nrm);
        }
    }
}

template <int NC, int RPT>
hipError_t launch_reg(const double *S, int64_t lds, int rows, int cols, double *R, int32_t *piv, const QrcpWork &w,
                      int G, hipStream_t stream)
{
    QrcpWork wk = w;
    int rows_ = rows, cols_ = cols, G_ = G;
    int64_t lds_ = lds;
    void *args[] = {(void *)&S, (void *)&lds_, (void *)&rows_, (void *)&cols_, (void *)&R, (void *)&piv,
                    (void *)&wk, (void *)&G_};
    return hipLaunchCooperativeKernel((const void *)qrcp_reg_kernel<NC, RPT>, dim3(G), dim3(RQ_T), args, 0, stream);
}

__global__ void zero_u32_kernel(unsigned *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

template <int NC, bool GCOLS>
hipError_t launch_qrcp(const double *S, int64_t lds, int rows, int cols, double *R, int32_t *piv, const QrcpWork &w,
                       int G, size_t shmem, hipStream_t stream)
{
    hipError_t e = hipFuncSetAttribute((const void *)qrcp_kernel<NC, GCOLS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
    QrcpWork wk = w;
    int rows_ = rows, cols_ = cols, G_ = G;
    int64_t lds_ = lds;
    void *args[] = {(void *)&S, (void *)&lds_, (void *)&rows_, (void *)&cols_, (void *)&R, (void *)&piv,
                    (void *)&wk, (void *)&G_};
    return hipLaunchCooperativeKernel((const void *)qrcp_kernel<NC, GCOLS>, dim3(G), dim3(QR_THREADS), args,
                                      (unsigned)shmem, stream);
}

}  // namespace

int qrcp_max_blocks(int rows, int cols, int cu_count, size_t lds_max, int *global_cols)
{
    // fewest blocks (one barrier participant each) whose columns fit in LDS,
    // at most one block per compute unit; otherwise 16 columns per block held
    // in global memory
    *global_cols = 0;
    for (int ncol = QR_MAXCOL; ncol >= 1; ncol >>= 1) {
        const size_t need = ((size_t)ncol + 1) * (size_t)rows * sizeof(double) + 4096;
        if (need > lds_max) continue;
        const int G = (cols + ncol - 1) / ncol;
        if (G <= cu_count) return G;
        break;
    }
    if ((size_t)rows * sizeof(double) + 4096 > lds_max) return -1;
    *global_cols = 1;
    const int G = (cols + QR_MAXCOL - 1) / QR_MAXCOL;
    return G <= cu_count ? G : -1;
}

// Register form: rows per thread RPT = 1, 2, 4, 8 or 16 (rows <= 8192) and
// NC columns per block with NC * RPT <= 64, NC aimed at about 64 blocks.
bool qrcp_reg_shape(int rows, int cols, int cu_count, int *nc_out, int *rpt_out, int *g_out)
{
    int rpt = 1;
    while (rpt * RQ_T < rows) rpt <<= 1;
    if (rpt > 16) return false;
    const int cap = rpt == 1 ? 32 : (rpt == 2 ? 16 : 64 / rpt);
    int want = (cols + 63) / 64, nc = 4;
    while (nc < want && nc < cap) nc <<= 1;
    if (nc > cap) nc = cap;
    const int G = (cols + nc - 1) / nc;
    if (G > cu_count) return false;
    *nc_out = nc;
    *rpt_out = rpt;
    *g_out = G;
    return true;
}

hipError_t qrcp_reg_f64(const double *S, int64_t lds, int rows, int cols, double *R, int32_t *piv, const QrcpWork &w,
                        int cu_count, hipStream_t stream)
{
    int nc, rpt, G;
    if (!qrcp_reg_shape(rows, cols, cu_count, &nc, &rpt, &G)) return hipErrorInvalidValue;
    hipError_t e = zero_u32(w.counter, 4, stream);
    if (e != hipSuccess) return e;
#define RQ_CASE(NC_, RPT_) \
    if (nc == NC_ && rpt == RPT_) return launch_reg<NC_, RPT_>(S, lds, rows, cols, R, piv, w, G, stream);
    RQ_CASE(4, 1) RQ_CASE(8, 1) RQ_CASE(16, 1) RQ_CASE(32, 1)
    RQ_CASE(4, 2) RQ_CASE(8, 2) RQ_CASE(16, 2)
    RQ_CASE(4, 4) RQ_CASE(8, 4) RQ_CASE(16, 4)
    RQ_CASE(4, 8) RQ_CASE(8, 8)
    RQ_CASE(4, 16)
#undef RQ_CASE
    return hipErrorInvalidValue;
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
    const int need_cols = (cols + G - 1) / G;
    int nc = 1;
    while (nc < need_cols) nc <<= 1;
    if (nc > QR_MAXCOL) return hipErrorInvalidValue;
    const bool gcols = w.cols != nullptr;
    const size_t shmem = ((size_t)(gcols ? 0 : nc) + 1) * (size_t)rows * sizeof(double);
    if (shmem + 4096 > lds_bytes_max) return hipErrorInvalidValue;
    hipError_t e = zero_u32(w.counter, 4, stream);  // counter, flag, err
    if (e != hipSuccess) return e;
    // the global-memory column slices are laid out for QR_MAXCOL columns per block
    if (gcols) return launch_qrcp<QR_MAXCOL, true>(S, lds, rows, cols, R, piv, w, G, shmem, stream);
    switch (nc) {
    case 1: return launch_qrcp<1, false>(S, lds, rows, cols, R, piv, w, G, shmem, stream);
    case 2: return launch_qrcp<2, false>(S, lds, rows, cols, R, piv, w, G, shmem, stream);
    case 4: return launch_qrcp<4, false>(S, lds, rows, cols, R, piv, w, G, shmem, stream);
    case 8: return launch_qrcp<8, false>(S, lds, rows, cols, R, piv, w, G, shmem, stream);
    default: return launch_qrcp<16, false>(S, lds, rows, cols, R, piv, w, G, shmem, stream);
    }
}

}  // namespace rt
