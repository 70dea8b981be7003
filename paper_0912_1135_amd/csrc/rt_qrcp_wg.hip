// Column-pivoted Householder QR (Businger-Golub, Sec. 4 eq. QR_decomp) of
// one matrix per workgroup: no grid-wide synchronization at all, so a single
// launch factors a whole batch of uneven problems concurrently, one per
// compute unit.  Used on the small triangular factor R0 of the sketch (the
// second stage of the two-stage pivoted QR: S^T = Q0 R0, then R0 Pi = Q1 R,
// so S^T Pi = (Q0 Q1) R with the same pivots in exact arithmetic).
//
// The matrix (column-major, overwritten) stays in global memory and is
// streamed through L2 at each step; pivot bookkeeping (trailing norms,
// column order) and the reflector live in LDS.  Per step k:
//   1. argmax of the trailing norms over the remaining positions (ties: the
//      lowest original column index), swap it to position k;
//   2. reflector H = I - tau v v^T with v[k] = 1, beta = -sign(alpha)|x|,
//      built from the pivot column; column k of R and piv[k] written;
//   3. every remaining column gets H applied and its trailing norm
//      recomputed exactly (no downdating).  Waves take four columns at a time
//      so that many loads are in flight.
#include "rt_common.h"

namespace rt {

namespace {

constexpr int WG_THREADS = 1024;
constexpr int WG_WAVES = WG_THREADS / 64;
constexpr int WG_COLS = 4;     // columns per wave per round
constexpr int WG_CH = 8;       // rows per lane per chunk (512-row chunks)
constexpr int WG_MAXR = 4096;  // rows
constexpr int WG_MAXC = 2048;  // columns

__device__ __forceinline__ double wave_sum64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(WG_THREADS) void qrcp_wg_kernel(const QrcpWgArgs *args)
{
    const QrcpWgArgs a = args[blockIdx.x];
    const int rows = a.rows, cols = a.cols;
    if (rows <= 0 || cols <= 0) return;
    __shared__ double v[WG_MAXR];
    __shared__ double nrm[WG_MAXC];
    __shared__ int cidx[WG_MAXC];
    __shared__ double red_n[WG_WAVES];
    __shared__ int red_c[WG_WAVES], red_q[WG_WAVES];
    __shared__ int s_q, s_fail;
    __shared__ double s_tau;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double *M = a.M;
    const int64_t ldm = a.ldm;

    // initial norms: one wave per column
    for (int j = wave; j < cols; j += WG_WAVES) {
        const double *x = M + (int64_t)j * ldm;
        double s = 0.0;
        for (int i = lane; i < rows; i += 64) s += x[i] * x[i];
        s = wave_sum64(s);
        if (lane == 0) {
            nrm[j] = s;
            cidx[j] = j;
        }
    }
    if (tid == 0) s_fail = 0;
    __syncthreads();

    const int steps = min(rows, cols);
    for (int k = 0; k < steps; ++k) {
        // 1. pivot: largest trailing norm, lowest original index on ties
        double bn = -1.0;
        int bc = 0x7fffffff, bq = -1;
        for (int q = k + tid; q < cols; q += WG_THREADS) {
            const double n = nrm[q];
            const int c = cidx[q];
            if (n > bn || (n == bn && c < bc)) { bn = n; bc = c; bq = q; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double on = __shfl_xor(bn, o, 64);
            const int oc = __shfl_xor(bc, o, 64), oq = __shfl_xor(bq, o, 64);
            if (on > bn || (on == bn && oc < bc)) { bn = on; bc = oc; bq = oq; }
        }
        if (lane == 0) { red_n[wave] = bn; red_c[wave] = bc; red_q[wave] = bq; }
        __syncthreads();
        if (tid == 0) {
            double n0 = -1.0;
            int c0 = 0x7fffffff, q0 = -1;
            for (int w = 0; w < WG_WAVES; ++w)
                if (red_q[w] >= 0 && (red_n[w] > n0 || (red_n[w] == n0 && red_c[w] < c0))) {
                    n0 = red_n[w]; c0 = red_c[w]; q0 = red_q[w];
                }
            if (q0 < 0) s_fail = 1;  // only NaN norms left
            else if (q0 != k) {
                const double tn = nrm[k]; nrm[k] = nrm[q0]; nrm[q0] = tn;
                const int tc = cidx[k]; cidx[k] = cidx[q0]; cidx[q0] = tc;
            }
            s_q = q0;
        }
        __syncthreads();
        if (s_fail) {
            if (tid == 0) atomicExch(a.err, 2);
            return;
        }
        // 2. reflector from the pivot column
        const int c = cidx[k];
        const double *x = M + (int64_t)c * ldm;
        const double alpha = x[k];
        const double xnorm = __builtin_sqrt(nrm[k]);
        double beta, tau, inv;
        if (xnorm == 0.0) { beta = 0.0; tau = 0.0; inv = 0.0; }
        else {
            beta = alpha >= 0.0 ? -xnorm : xnorm;
            tau = (beta - alpha) / beta;
            inv = 1.0 / (alpha - beta);
        }
        for (int i = k + tid; i < rows; i += WG_THREADS) v[i] = (i == k) ? 1.0 : x[i] * inv;
        for (int i = tid; i < k; i += WG_THREADS) a.R[(int64_t)i * cols + k] = x[i];
        if (tid == 0) {
            a.R[(int64_t)k * cols + k] = beta;
            a.piv[k] = c;
            s_tau = tau;
        }
        __syncthreads();
        // 3. apply H to the remaining columns, four per wave per round
        const double t = s_tau;
        const int rem = cols - (k + 1);
        const int nrows = rows - k;
        for (int base = wave * WG_COLS; base < rem; base += WG_WAVES * WG_COLS) {
            double *y[WG_COLS];
            bool ok[WG_COLS];
#pragma unroll
            for (int j = 0; j < WG_COLS; ++j) {
                ok[j] = base + j < rem;
                y[j] = M + (int64_t)cidx[ok[j] ? k + 1 + base + j : k] * ldm + k;
            }
            if (nrows <= 64 * WG_CH) {
                // whole trailing column in registers: one read, one write
                double val[WG_COLS][WG_CH];
                double dot[WG_COLS];
#pragma unroll
                for (int j = 0; j < WG_COLS; ++j) {
                    dot[j] = 0.0;
#pragma unroll
                    for (int r = 0; r < WG_CH; ++r) {
                        const int i = lane + 64 * r;
                        val[j][r] = (ok[j] && i < nrows) ? y[j][i] : 0.0;
                    }
                }
#pragma unroll
                for (int r = 0; r < WG_CH; ++r) {
                    const int i = lane + 64 * r;
                    const double vi = i < nrows ? v[k + i] : 0.0;
#pragma unroll
                    for (int j = 0; j < WG_COLS; ++j) dot[j] += vi * val[j][r];
                }
#pragma unroll
                for (int j = 0; j < WG_COLS; ++j) dot[j] = wave_sum64(dot[j]);
                double nn[WG_COLS];
#pragma unroll
                for (int j = 0; j < WG_COLS; ++j) nn[j] = 0.0;
#pragma unroll
                for (int r = 0; r < WG_CH; ++r) {
                    const int i = lane + 64 * r;
                    if (i < nrows) {
                        const double vi = v[k + i];
#pragma unroll
                        for (int j = 0; j < WG_COLS; ++j) {
                            const double nv = val[j][r] - t * dot[j] * vi;
                            if (ok[j]) y[j][i] = nv;
                            if (i > 0) nn[j] += nv * nv;
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < WG_COLS; ++j) {
                    nn[j] = wave_sum64(nn[j]);
                    if (lane == 0 && ok[j]) nrm[k + 1 + base + j] = nn[j];
                }
            } else {
                // tall columns: dot pass, then update pass
                double dot[WG_COLS];
#pragma unroll
                for (int j = 0; j < WG_COLS; ++j) dot[j] = 0.0;
                for (int i = lane; i < nrows; i += 64) {
                    const double vi = v[k + i];
#pragma unroll
                    for (int j = 0; j < WG_COLS; ++j)
                        if (ok[j]) dot[j] += vi * y[j][i];
                }
#pragma unroll
                for (int j = 0; j < WG_COLS; ++j) dot[j] = wave_sum64(dot[j]);
                double nn[WG_COLS];
#pragma unroll
                for (int j = 0; j < WG_COLS; ++j) nn[j] = 0.0;
                for (int i = lane; i < nrows; i += 64) {
                    const double vi = v[k + i];
#pragma unroll
                    for (int j = 0; j < WG_COLS; ++j)
                        if (ok[j]) {
                            const double nv = y[j][i] - t * dot[j] * vi;
                            y[j][i] = nv;
                            if (i > 0) nn[j] += nv * nv;
                        }
                }
#pragma unroll
                for (int j = 0; j < WG_COLS; ++j) {
                    nn[j] = wave_sum64(nn[j]);
                    if (lane == 0 && ok[j]) nrm[k + 1 + base + j] = nn[j];
                }
            }
        }
        __syncthreads();
    }
    // columns past min(rows, cols) (cols > rows) keep their remaining rows as R's
    for (int q = steps; q < cols; ++q) {
        const double *xq = M + (int64_t)cidx[q] * ldm;
        for (int i = tid; i < rows; i += WG_THREADS) a.R[(int64_t)i * cols + q] = xq[i];
        if (tid == 0) a.piv[q] = cidx[q];
    }
}

}  // namespace

hipError_t qrcp_wg_f64(const QrcpWgArgs *d_args, int count, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(qrcp_wg_kernel, dim3(count), dim3(WG_THREADS), 0, stream, d_args);
    return hipGetLastError();
}

int qrcp_wg_max_rows() { return WG_MAXR; }
int qrcp_wg_max_cols() { return WG_MAXC; }

}  // namespace rt
