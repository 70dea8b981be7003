// Column-pivoted Householder QR of the sketch, S^T = Q R Pi (Sec. 4,
// eq. QR_decomp), Businger-Golub pivoting: at step k the pivot is the
// remaining column with the largest trailing 2-norm (ties: lowest index).
//
// One cooperative launch.  Block g owns columns j = g, g + G, g + 2G, ... of
// the input and keeps them for the whole factorization in registers (or in
// LDS, or, for sketches too tall for LDS, in a private slice of global
// memory).  Each step costs ONE exchange between the blocks:
//   1. every block posts its best remaining column (trailing norm^2, index,
//      and the trailing part of the column itself) to a double-buffered slot;
//   2. the blocks meet: in the register form each block tags its own slot
//      with the step once its posts have completed, and every block polls the
//      G tags (loads issued together); the LDS forms count arrivals on one
//      counter instead;
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
constexpr int QR_TAG_SLOTS = 4;  // header tags per lane of the polling wave: the register form takes G <= 256

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
    // relaxed device-scope polling (no cache maintenance per poll); the error
    // word is looked at only every 256 polls so that a poll is one load
    while (__hip_atomic_load(addr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        ++spins;
        if (spins > SPIN_LIMIT ||
            ((spins & 255) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
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
        const bool keep_v = w.V && p % G == g;
        for (int i = k + tid; i < rows; i += QR_THREADS) {
            const double vi = (i == k) ? 1.0 : xp[i] * inv;
            v[i] = vi;
            if (keep_v) w.V[(int64_t)k * rows + i] = vi;
        }
        if (keep_v && tid == 0) w.tau[k] = tau;
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
// Register-resident form (the default): TT = 256 or 512 threads, block g keeps its NC
// columns in registers, thread t owning rows t, t + TT, ..., so that each
// thread reads the reflector's entries for its rows once and applies them to
// all NC columns.  A step is a chain of dependent latencies (post, barrier,
// candidate headers, pivot column), so everything between them is kept short:
//   - the column sums (dot products, trailing norms) transpose the columns
//     across lanes while adding them (DPP quad permutes, row mirror and
//     rotation), with one LDS exchange per block;
//   - the pivot choice and the broadcast of sums stay in registers;
//   - posted data (headers and candidate columns) is written and read with
//     device-scope accesses, which are coherent across the L2 slices of the
//     XCDs without flushing or invalidating them; a block announces its
//     arrival only after its posting stores have completed.
// Threads per block: 256 or 512 (template parameter TT, TW = TT / 64 waves).


__device__ __forceinline__ double u64_to_d(unsigned lo, unsigned hi)
{
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// DPP move of a double (two 32-bit lane moves); lanes of rows outside
// ROW_MASK receive 0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_d(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROW_MASK, 0xF, false);
    return u64_to_d((unsigned)lo, (unsigned)hi);
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ double readlane_d(double v, int lane)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return u64_to_d((unsigned)lo, (unsigned)hi);
}

constexpr int DPP_QUAD_XOR1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int DPP_ROW_MIRROR = 0x140;
constexpr int DPP_ROW_HALF_MIRROR = 0x141;

// Candidate order: larger norm^2 first, then the lower column index.  Every
// candidate carries a norm >= -1 (never NaN), so the order is total.
__device__ __forceinline__ bool cand_better(double n2, int c2, double n, int c)
{
    return n2 > n || (n2 == n && c2 < c);
}

template <int CTRL>
__device__ __forceinline__ void amax_step(double &n, int &c)
{
    const double n2 = dpp_d<CTRL>(n);
    const int c2 = dpp_i<CTRL>(c);
    if (cand_better(n2, c2, n, c)) { n = n2; c = c2; }
}

// Best candidate of the wave, returned uniformly.
__device__ __forceinline__ void wave_best(double &n, int &c)
{
    amax_step<DPP_QUAD_XOR1>(n, c);
    amax_step<DPP_QUAD_XOR2>(n, c);
    amax_step<DPP_ROW_HALF_MIRROR>(n, c);
    amax_step<DPP_ROW_MIRROR>(n, c);
    double bn = readlane_d(n, 0);
    int bc = __builtin_amdgcn_readlane(c, 0);
#pragma unroll
    for (int r = 1; r < 4; ++r) {
        const double n2 = readlane_d(n, 16 * r);
        const int c2 = __builtin_amdgcn_readlane(c, 16 * r);
        if (cand_better(n2, c2, bn, bc)) { bn = n2; bc = c2; }
    }
    n = bn;
    c = bc;
}

__device__ __forceinline__ void st_dev(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until this thread's outstanding memory operations (the posting
// stores) have completed.
__device__ __forceinline__ void wait_mem()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

constexpr int DPP_ROW_ROR8 = 0x128;  // row_ror:8, i.e. lane i <-> i ^ 8 within a row

// One level of the transposing reduction: the partner differs from this lane
// in bit BIT.  With N > 1 values the lane keeps the half selected by that bit
// and adds the partner's copy of the same half (the partner sends the half it
// does not keep); with one value left it adds the partner's, and only the lane
// with the bit clear remains the representative of the duplicate pair.
template <int CTRL, int BIT, int N, int NC>
__device__ __forceinline__ void red_level(double (&v)[NC], int lane, int &off, bool &rep)
{
    const bool kb = (lane >> BIT) & 1;
    if constexpr (N > 1) {
        constexpr int H = N / 2;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const double mine = kb ? v[j + H] : v[j];
            const double other = kb ? v[j] : v[j + H];
            v[j] = mine + dpp_d<CTRL>(other);
        }
        if (kb) off += H;
    } else {
        v[0] += dpp_d<CTRL>(v[0]);
        if (kb) rep = false;
    }
}

// Block-wide column sums of the per-thread partials p[0..NC) (NC a power of
// two).  Inside each 16-lane row the NC values are transposed while being
// added: four DPP levels (partners i <-> 7-i within 8 lanes, i <-> i^2,
// i <-> i^1, i <-> i^8) halve the values per lane while any remain, so a lane
// ends with the row sums of max(1, NC/16) consecutive columns starting at
// `off` (set by its lane bits).  The representatives write these row sums to
// LDS (red: 4 TW x NC, one row per wave and lane row, columns contiguous so
// that the lanes reading them hit distinct banks); after one block barrier
// lane c of every wave adds column c's 4 TW partials in a fixed order.
// Returns that sum in lane c (0 for c >= NC), identical in every wave.
template <int NC, int TW>
__device__ __forceinline__ double block_col_sums(const double (&p)[NC], double (*red)[NC])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = p[c];
    int off = 0;
    bool rep = true;
    red_level<DPP_ROW_HALF_MIRROR, 2, NC, NC>(v, lane, off, rep);
    red_level<DPP_QUAD_XOR2, 1, (NC > 2 ? NC / 2 : 1), NC>(v, lane, off, rep);
    red_level<DPP_QUAD_XOR1, 0, (NC > 4 ? NC / 4 : 1), NC>(v, lane, off, rep);
    red_level<DPP_ROW_ROR8, 3, (NC > 8 ? NC / 8 : 1), NC>(v, lane, off, rep);
    constexpr int NF = NC > 16 ? NC / 16 : 1;
    if (rep)
#pragma unroll
        for (int j = 0; j < NF; ++j) red[wave * 4 + (lane >> 4)][off + j] = v[j];
    __syncthreads();
    double s = 0.0;
    if (lane < NC) {
        double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 4 * TW; ++q) a[q & 3] += red[q][lane];
        s = (a[0] + a[1]) + (a[2] + a[3]);
    }
    return s;
}

// Local candidate from lane c's trailing norm^2 s: the largest norm among the
// block's remaining columns (lowest local index on ties); -1 when none is
// left (or only NaN norms are).
template <int NC>
__device__ __forceinline__ void local_best(double s, int ncol, unsigned done, double &bn, int &bc)
{
    const int lane = threadIdx.x & 63;
    const bool ok = lane < ncol && !((done >> lane) & 1u) && s >= 0.0;
    double n = ok ? s : -1.0;
    int c = ok ? lane : 0x7fffffff;
    wave_best(n, c);
    bn = n;
    bc = n >= 0.0 ? c : -1;
}

// Block g of the G blocks that factor one matrix: the whole factorization
// with the G blocks' only contact through the workspace w.
template <int NC, int RPT, int TT>
__device__ __forceinline__ void reg_qr_body(const double *S, int64_t lds, int rows, int cols, double *R, int32_t *piv,
                                            const QrcpWork &w, int G, int g)
{
    static_assert(NC <= 32 && (NC & (NC - 1)) == 0, "done mask, lane-per-column sums, power of two");
    constexpr int TW = TT / 64;
    __shared__ double red[2][4 * TW][NC];
    __shared__ double s_pn;
    __shared__ int s_p, s_abort;
    const int tid = threadIdx.x, lane = tid & 63;
    int ncol = 0;
    while (ncol < NC && g + G * ncol < cols) ++ncol;
    double *hdr = w.slots;  // 2 x G x 2: candidate norm^2, tagged column (zeroed before the launch)
    double *cand = w.vbuf;  // 2 x G x rows: candidate columns

    double x[NC][RPT];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = tid + TT * r;
            x[c][r] = (c < ncol && i < rows) ? S[(int64_t)(g + G * c) * lds + i] : 0.0;
        }
    if (tid == 0) s_abort = 0;
    unsigned done = 0;  // bit c: local column c retired (uniform)
    double bn;
    int bc;
    {
        double part[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            part[c] = 0.0;
#pragma unroll
            for (int r = 0; r < RPT; ++r) part[c] += x[c][r] * x[c][r];
        }
        local_best<NC>(block_col_sums<NC, TW>(part, red[1]), ncol, done, bn, bc);
    }

    for (int k = 0; k < cols; ++k) {
        const int buf = k & 1;
        // 1. post the local candidate: header, and rows >= k of its column
        if (bc >= 0) {
            double *dst = cand + ((int64_t)buf * G + g) * rows;
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = tid + TT * r;
                double val = 0.0;
#pragma unroll
                for (int c = 0; c < NC; ++c) val = (c == bc) ? x[c][r] : val;
                if (i >= k && i < rows) st_dev(dst + i, val);
            }
        }
        if (tid == 0) st_dev(hdr + (buf * G + g) * 2 + 0, bn);
        wait_mem();
        __syncthreads();
        // 2. arrival and pivot in one exchange: each block tags its own header
        // word (step + 1 in the high half, its candidate column + 1 in the
        // low half) once its posts have completed; wave 0 polls all G tags
        // with the loads issued together (no shared counter, no serialized
        // atomics), then reads the norms and picks the pivot
        if (tid < 64) {
            unsigned long long *tw = reinterpret_cast<unsigned long long *>(hdr);
            const unsigned want = (unsigned)(k + 1);
            if (tid == 0)
                __hip_atomic_store(tw + (buf * G + g) * 2 + 1,
                                   ((unsigned long long)want << 32) | (unsigned)(bc >= 0 ? g + G * bc + 1 : 0),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            unsigned long long tv[QR_TAG_SLOTS];
            long spins = 0;
            for (;;) {
#pragma unroll
                for (int u = 0; u < QR_TAG_SLOTS; ++u) {
                    const int q = lane + 64 * u;
                    tv[u] = q < G ? __hip_atomic_load(tw + (buf * G + q) * 2 + 1, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT)
                                  : ((unsigned long long)want << 32);
                }
                bool mine = true;
#pragma unroll
                for (int u = 0; u < QR_TAG_SLOTS; ++u) mine = mine && (unsigned)(tv[u] >> 32) == want;
                if (__all(mine)) break;
                __builtin_amdgcn_s_sleep(1);
                if (++spins > SPIN_LIMIT) {
                    if (tid == 0) {
                        __hip_atomic_store(w.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        s_abort = 1;
                    }
                    break;
                }
            }
            double qn[QR_TAG_SLOTS];
#pragma unroll
            for (int u = 0; u < QR_TAG_SLOTS; ++u) {
                const int q = lane + 64 * u;
                qn[u] = q < G ? ld_dev(hdr + (buf * G + q) * 2 + 0) : -2.0;
            }
            double n = -2.0;
            int j = 0x7fffffff;
#pragma unroll
            for (int u = 0; u < QR_TAG_SLOTS; ++u) {
                const int qj = (int)(unsigned)(tv[u] & 0xffffffffull) - 1;
                if (lane + 64 * u < G && qj >= 0 && cand_better(qn[u], qj, n, j)) { n = qn[u]; j = qj; }
            }
            wave_best(n, j);
            if (tid == 0) {
                s_p = n >= 0.0 ? j : -1;
                s_pn = n;
            }
        }
        __syncthreads();
        if (s_abort) return;
        const int p = s_p;
        if (p < 0 || p >= cols) {
            if (tid == 0 && g == 0) __hip_atomic_store(w.err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        // 4. reflector entries for this thread's rows, from the posted column
        const double *xp = cand + ((int64_t)buf * G + (p % G)) * rows;
        const double alpha = ld_dev(xp + k);
        double v[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = tid + TT * r;
            v[r] = (i > k && i < rows) ? ld_dev(xp + i) : 0.0;
        }
        const double xnorm = __builtin_sqrt(s_pn);
        double beta, tau, inv;
        if (xnorm == 0.0) { beta = 0.0; tau = 0.0; inv = 0.0; }
        else {
            beta = alpha >= 0.0 ? -xnorm : xnorm;
            tau = (beta - alpha) / beta;
            inv = 1.0 / (alpha - beta);
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) v[r] = (tid + TT * r == k) ? 1.0 : v[r] * inv;
        // 5. owner: column k of R and piv[k]
        if (p % G == g) {
            const int c = p / G;
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = tid + TT * r;
                double val = 0.0;
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) val = (cc == c) ? x[cc][r] : val;
                if (i < k) R[(int64_t)i * cols + k] = val;
            }
            if (tid == 0) {
                R[(int64_t)k * cols + k] = beta;
                piv[k] = p;
            }
            if (w.V) {
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int i = tid + TT * r;
                    if (i >= k && i < rows) w.V[(int64_t)k * rows + i] = v[r];
                }
                if (tid == 0) w.tau[k] = tau;
            }
            done |= 1u << c;
        }
        // 6. dot products v . x_c, then the update and the next trailing norms
        double d[NC];
        {
            double part[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                part[c] = 0.0;
#pragma unroll
                for (int r = 0; r < RPT; ++r) part[c] += v[r] * x[c][r];
            }
            const double s = block_col_sums<NC, TW>(part, red[0]);
#pragma unroll
            for (int c = 0; c < NC; ++c) d[c] = readlane_d(s, c);
        }
        {
            double nn[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double f = ((done >> c) & 1u) ? 0.0 : tau * d[c];
                nn[c] = 0.0;
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int i = tid + TT * r;
                    const double nx = x[c][r] - f * v[r];
                    x[c][r] = nx;
                    if (i > k) nn[c] += nx * nx;
                }
            }
            local_best<NC>(block_col_sums<NC, TW>(nn, red[1]), ncol, done, bn, bc);
        }
    }
}

template <int NC, int RPT, int TT>
__global__ __launch_bounds__(TT) void qrcp_reg_kernel(const double *S, int64_t lds, int rows, int cols, double *R,
                                                        int32_t *piv, QrcpWork w, int G)
{
    reg_qr_body<NC, RPT, TT>(S, lds, rows, cols, R, piv, w, G, blockIdx.x);
}

// Grouped form: member blockIdx.y is factored by blocks x < its G (the grid is
// as wide as the largest member's group; the rest leave at once).  Each
// member synchronizes only its own group, through its own workspace.
template <int NC, int RPT, int TT>
__global__ __launch_bounds__(TT) void qrcp_grp_kernel(const QrcpGrpArgs *args)
{
    const QrcpGrpArgs a = args[blockIdx.y];
    if ((int)blockIdx.x >= a.G || a.rows <= 0 || a.cols <= 0) return;
    reg_qr_body<NC, RPT, TT>(a.S, a.lds, a.rows, a.cols, a.R, a.piv, a.w, a.G, blockIdx.x);
}

template <int NC, int RPT, int TT>
hipError_t launch_reg(const double *S, int64_t lds, int rows, int cols, double *R, int32_t *piv, const QrcpWork &w,
                      int G, hipStream_t stream)
{
    QrcpWork wk = w;
    int rows_ = rows, cols_ = cols, G_ = G;
    int64_t lds_ = lds;
    void *args[] = {(void *)&S, (void *)&lds_, (void *)&rows_, (void *)&cols_, (void *)&R, (void *)&piv,
                    (void *)&wk, (void *)&G_};
    return hipLaunchCooperativeKernel((const void *)qrcp_reg_kernel<NC, RPT, TT>, dim3(G), dim3(TT), args, 0,
                                      stream);
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

// Register form: 256 threads per block with RPT = 1, 2, 4, 8 or 16 rows per
// thread (rows <= 4096; 512 threads with 16 rows each up to 8192), and NC
// columns per block (a power of two, NC * RPT <= 64 for registers; 32 only
// for one row per thread).  Measured on the tagged exchange, whose cost
// barely grows with the block count: fewer waves per block and less work
// per block per step win, so 256 threads and the fewest columns per block
// whose block count G fits the device (one block per compute unit) and the
// polling wave (G <= 256).  At 2048 x 2048: 8 columns, 256 blocks, 6.4 us
// per step, against 7.8 us with 16 columns and 128 blocks.
static bool reg_geometry(int rows, int *rpt_out, int *tt_out, int *cap_out)
{
    int tt = 256, rpt = 1;
    while (rpt * tt < rows) rpt <<= 1;
    if (rpt > 16) {
        tt = 512;
        rpt = 1;
        while (rpt * tt < rows) rpt <<= 1;
        if (rpt > 16) return false;
    }
    *rpt_out = rpt;
    *tt_out = tt;
    *cap_out = rpt == 1 ? 32 : (rpt == 2 ? 16 : 64 / rpt);
    return true;
}

bool qrcp_reg_shape(int rows, int cols, int cu_count, int *nc_out, int *rpt_out, int *g_out, int *tt_out)
{
    int rpt, tt, cap;
    if (!reg_geometry(rows, &rpt, &tt, &cap)) return false;
    const int gmax = std::min(cu_count, 64 * QR_TAG_SLOTS);
    int nc = 4;
    while (nc < cap && (cols + nc - 1) / nc > gmax) nc <<= 1;
    const int G = (cols + nc - 1) / nc;
    if (G > gmax) return false;
    *nc_out = nc;
    *rpt_out = rpt;
    *g_out = G;
    *tt_out = tt;
    return true;
}

hipError_t qrcp_reg_f64(const double *S, int64_t lds, int rows, int cols, double *R, int32_t *piv, const QrcpWork &w,
                        int cu_count, hipStream_t stream)
{
    int nc, rpt, G, tt;
    if (!qrcp_reg_shape(rows, cols, cu_count, &nc, &rpt, &G, &tt)) return hipErrorInvalidValue;
    hipError_t e = zero_u32(w.counter, 4, stream);  // counter, flag, err
    if (e == hipSuccess) e = zero_u32(reinterpret_cast<unsigned *>(w.slots), 8 * G, stream);  // header tags
    if (e != hipSuccess) return e;
#define RQ_CASE(NC_, RPT_)                                                                                        \
    if (nc == NC_ && rpt == RPT_)                                                                                 \
        return tt == 256 ? launch_reg<NC_, RPT_, 256>(S, lds, rows, cols, R, piv, w, G, stream)                   \
                         : launch_reg<NC_, RPT_, 512>(S, lds, rows, cols, R, piv, w, G, stream);
    RQ_CASE(4, 1) RQ_CASE(8, 1) RQ_CASE(16, 1) RQ_CASE(32, 1)
    RQ_CASE(4, 2) RQ_CASE(8, 2) RQ_CASE(16, 2)
    RQ_CASE(4, 4) RQ_CASE(8, 4) RQ_CASE(16, 4)
    RQ_CASE(4, 8) RQ_CASE(8, 8)
    RQ_CASE(4, 16)
#undef RQ_CASE
    return hipErrorInvalidValue;
}

static __global__ void grp_zero_kernel(const QrcpGrpArgs *args)
{
    const QrcpGrpArgs a = args[blockIdx.x];
    for (int i = threadIdx.x; i < 4 * a.G; i += blockDim.x) reinterpret_cast<unsigned long long *>(a.w.slots)[i] = 0ull;
}

// The grouped form's kernel for a (columns per block, rows per thread,
// threads) shape; null when there is none.
static const void *grp_kernel_for(int nc, int rpt, int tt)
{
#define RG_CASE(NC_, RPT_)                                                                                        \
    if (nc == NC_ && rpt == RPT_)                                                                                 \
        return tt == 256 ? (const void *)qrcp_grp_kernel<NC_, RPT_, 256>                                          \
                         : (const void *)qrcp_grp_kernel<NC_, RPT_, 512>;
    RG_CASE(4, 1) RG_CASE(8, 1) RG_CASE(16, 1) RG_CASE(32, 1)
    RG_CASE(4, 2) RG_CASE(8, 2) RG_CASE(16, 2)
    RG_CASE(4, 4) RG_CASE(8, 4) RG_CASE(16, 4)
    RG_CASE(4, 8) RG_CASE(8, 8)
    RG_CASE(4, 16)
#undef RG_CASE
    return nullptr;
}

bool qrcp_grp_shape(int max_rows, int max_cols, int cu_count, QrcpGrpShape *sh)
{
    // the widest blocks: the fewest blocks per member, so that the most
    // members run at once
    int rpt, tt, nc;
    if (!reg_geometry(max_rows, &rpt, &tt, &nc)) return false;
    const int g = (max_cols + nc - 1) / nc;
    if (g > std::min(cu_count, 64 * QR_TAG_SLOTS)) return false;
    const void *fn = grp_kernel_for(nc, rpt, tt);
    if (!fn) return false;
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, tt, 0) != hipSuccess || per < 1) return false;
    sh->nc = nc;
    sh->rpt = rpt;
    sh->threads = tt;
    sh->gmax = g;
    // members whose groups are resident together (a group's blocks wait on
    // each other, so a launch never holds more than the device keeps resident)
    sh->per_launch = std::max(1, per * cu_count / g);
    return true;
}

hipError_t qrcp_grp_f64(const QrcpGrpArgs *d_args, int count, const QrcpGrpShape &sh, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    if (count > sh.per_launch) return hipErrorInvalidValue;
    const void *fn = grp_kernel_for(sh.nc, sh.rpt, sh.threads);
    if (!fn) return hipErrorInvalidValue;
    // every member's header tags start from zero (a kernel, so that graph replays clear them too)
    hipLaunchKernelGGL(grp_zero_kernel, dim3(count), dim3(256), 0, stream, d_args);
    const QrcpGrpArgs *a = d_args;
    void *args[] = {(void *)&a};
    return hipLaunchKernel(fn, dim3(sh.gmax, count), dim3(sh.threads), args, 0, stream);
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
