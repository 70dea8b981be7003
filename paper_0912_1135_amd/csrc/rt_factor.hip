// Small dense kernels of the preconditioner: inverses of triangular diagonal
// blocks (the blocked solves with R^T and with the Cholesky factor use them
// so that every off-diagonal step is an MFMA GEMM), the Cholesky of one
// diagonal block of the Gram (the factorization that replaces the explicit
// inverse Y = X^{-1} of eq. inversion), and helpers.
#include <algorithm>

#include "rt_common.h"

namespace rt {

namespace {

constexpr int NBMAX = 64;
constexpr int LDP = NBMAX + 1;                  // padded LDS row stride
constexpr int DT = 256;                         // threads of the diagonal-block kernels
constexpr int NTRI = NBMAX * (NBMAX + 1) / 2;   // entries of a 64 x 64 lower triangle
constexpr int NE = (NTRI + DT - 1) / DT;        // entries owned per thread

// Thread t owns the lower-triangle entries e = t + DT*s (row-wise order
// e = i(i+1)/2 + c, c <= i) and keeps them in registers; slots past the
// triangle get row -1 and never match.
__device__ __forceinline__ void tri_slots(int *ri, int *ci)
{
#pragma unroll
    for (int s = 0; s < NE; ++s) {
        const int e = threadIdx.x + DT * s;
        int i = (int)((__builtin_sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while ((i + 1) * (i + 2) / 2 <= e) ++i;
        while (i * (i + 1) / 2 > e) --i;
        ri[s] = e < NTRI ? i : -1;
        ci[s] = e < NTRI ? e - i * (i + 1) / 2 : NBMAX;
    }
}

// X = L^{-1} for the lower-triangular L in LDS (row stride LDP), written to
// X (row stride LDP; may not alias L).  Column j of X solves L x = e_j by
// forward substitution, x_i = (delta_ij - sum_{c<i} L_ic x_c) / L_ii for
// i = 0..63 in turn, and the 64 columns are independent: four lanes of one
// wave share a column (lanes 4j..4j+3), each summing the terms c = q mod 4
// before two shuffles add the four parts, so no block barrier is needed
// between rows (a wave's LDS accesses complete in order).  Rows above j come
// out as exact zeros.  The reciprocals 1 / L_ii are formed once.
__device__ void lower_inverse_block(const double *L, double *X)
{
    static_assert(DT == 4 * NBMAX, "four lanes per column of the block");
    __shared__ double invd[NBMAX];
    for (int e = threadIdx.x; e < NBMAX * NBMAX; e += DT) X[(e / NBMAX) * LDP + (e % NBMAX)] = 0.0;
    if (threadIdx.x < NBMAX) invd[threadIdx.x] = 1.0 / L[threadIdx.x * LDP + threadIdx.x];
    __syncthreads();
    const int j = threadIdx.x >> 2, q = threadIdx.x & 3;
    for (int i = 0; i < NBMAX; ++i) {
        const double *li = L + i * LDP;
        double sq = 0.0;
        for (int c0 = 0; c0 < i; c0 += 4) {
            const int c = c0 + q;
            const double t = li[c < i ? c : 0] * X[(c < i ? c : 0) * LDP + j];
            sq += c < i ? t : 0.0;
        }
        sq += __shfl_xor(sq, 1, 64);
        sq += __shfl_xor(sq, 2, 64);
        const double xi = ((i == j ? 1.0 : 0.0) - sq) * invd[i];
        if (q == 0) X[i * LDP + j] = xi;
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
}

__device__ __forceinline__ void tri_diag_inv_body(const double *T, int64_t t_i, int64_t t_j, int m, int nb,
                                                  double *Dinv, int b)
{
    if (b * nb >= m) return;  // whole block (grouped launches)
    __shared__ double L[NBMAX * LDP];
    __shared__ double X[NBMAX * LDP];
    const int base = b * nb, nbb = min(nb, m - base);
    for (int e = threadIdx.x; e < NBMAX * NBMAX; e += DT) {
        const int i = e / NBMAX, j = e % NBMAX;
        double v;
        if (i < nbb && j < nbb) v = (j <= i) ? T[(int64_t)(base + i) * t_i + (int64_t)(base + j) * t_j] : 0.0;
        else v = (i == j) ? 1.0 : 0.0;
        L[i * LDP + j] = v;
    }
    __syncthreads();
    lower_inverse_block(L, X);
    double *out = Dinv + (int64_t)b * nb * nb;
    for (int e = threadIdx.x; e < nb * nb; e += DT) out[e] = X[(e / nb) * LDP + (e % nb)];
}

__global__ __launch_bounds__(DT) void tri_diag_inv_kernel(const double *T, int64_t t_i, int64_t t_j, int m, int nb,
                                                          double *Dinv)
{
    tri_diag_inv_body(T, t_i, t_j, m, nb, Dinv, blockIdx.x);
}

__global__ __launch_bounds__(DT) void tri_diag_inv_grouped(const TriInvGroupArgs *gs, int nb)
{
    const TriInvGroupArgs g = gs[blockIdx.y];
    tri_diag_inv_body(g.T, g.t_i, g.t_j, g.m, nb, g.Dinv, blockIdx.x);
}

// Cholesky of one 64 x 64 diagonal block (right-looking) and the inverse of
// its factor, by one wave.  A non-positive or non-finite pivot sets *err
// (the outputs are then garbage).
__device__ __forceinline__ double lane_value(double v, int src)
{
    const unsigned long long bits = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)bits, src);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(bits >> 32), src);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// One wave: lane i keeps row i of the block (a[c], c <= i) in registers.
// Step j: the pivot d = A[j][j] is read from lane j, every lane finalizes its
// entry of column j (L[j][j] = sqrt(d), L[i][j] = A[i][j] / sqrt(d) below),
// publishes it in LDS, and updates its row, A[i][c] -= L[i][j] L[c][j] for
// c > j.  Then L goes to LDS and lane i solves L x = e_i for column i of
// X = L^{-1}.  A wave's LDS accesses complete in order, so no barrier is
// needed between the steps.
__device__ __forceinline__ void chol_diag_body(const double *Xg, int64_t ldx, int m, int nb, int b, double *Lg,
                                               int64_t ldl, double *Dinv, int *err)
{
    if (b * nb >= m) return;  // whole block (grouped launches)
    __shared__ double pub[NBMAX];
    __shared__ double Ls[NBMAX * LDP];
    const int i = threadIdx.x;
    const int base = b * nb, nbb = min(nb, m - base);
    double a[NBMAX];
#pragma unroll
    for (int c = 0; c < NBMAX; ++c) {
        double v = (i == c) ? 1.0 : 0.0;
        if (i < nbb && c < nbb && c <= i) v = Xg[(int64_t)(base + i) * ldx + base + c];
        a[c] = v;
    }
    bool bad = false;
#pragma unroll
    for (int j = 0; j < NBMAX; ++j) {
        const double d = lane_value(a[j], j);
        bad |= !(d > 0.0 && d < INFINITY);
        const double ljj = __builtin_sqrt(d);
        const double lij = (i == j) ? ljj : (i > j ? a[j] / ljj : 0.0);
        a[j] = lij;
        pub[i] = lij;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int c = j + 1; c < NBMAX; ++c) a[c] -= lij * pub[c];
        __builtin_amdgcn_wave_barrier();
    }
    if (i < nbb)
        for (int c = 0; c < nbb; ++c) Lg[(int64_t)(base + i) * ldl + base + c] = c <= i ? a[c] : 0.0;
    // X = L^{-1} by forward substitution, lane i solving for column i of X:
    // x[r] = (delta_ri - sum_{p<r} L[r][p] x[p]) / L[r][r], with L read from
    // LDS (the same address in every lane)
#pragma unroll
    for (int c = 0; c < NBMAX; ++c) Ls[i * LDP + c] = c <= i ? a[c] : 0.0;
    __builtin_amdgcn_wave_barrier();
    double x[NBMAX];
#pragma unroll
    for (int r = 0; r < NBMAX; ++r) {
        double t = (r == i) ? 1.0 : 0.0;
#pragma unroll
        for (int p = 0; p < r; ++p) t -= Ls[r * LDP + p] * x[p];
        x[r] = t / Ls[r * LDP + r];
    }
    double *out = Dinv + (int64_t)b * nb * nb;
    if (i < nb)
        for (int r = 0; r < nb; ++r) out[(int64_t)r * nb + i] = x[r];
    if (bad && i == 0) atomicExch(err, 1);
}

__global__ __launch_bounds__(NBMAX) void chol_diag_kernel(const double *Xg, int64_t ldx, int m, int nb, int b,
                                                          double *Lg, int64_t ldl, double *Dinv, int *err)
{
    chol_diag_body(Xg, ldx, m, nb, b, Lg, ldl, Dinv, err);
}

__global__ __launch_bounds__(NBMAX) void chol_diag_grouped(const CholGroupArgs *gs, int nb, int b)
{
    const CholGroupArgs g = gs[blockIdx.x];
    chol_diag_body(g.X, g.ldx, g.m, nb, b, g.L, g.ldl, g.Dinv, g.err);
}

__device__ __forceinline__ void shift_diag_body(double *G, int64_t ld, int m, double c)
{
    __shared__ double red[256];
    double t = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) t += G[(int64_t)i * ld + i];
    red[threadIdx.x] = t;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double sh = c * red[0];
    for (int i = threadIdx.x; i < m; i += 256) G[(int64_t)i * ld + i] += sh;
}

__global__ void shift_diag_kernel(double *G, int64_t ld, int m, double c) { shift_diag_body(G, ld, m, c); }

// piv[i] = i: the pivot vector is valid (in range) even when a pivoted QR
// stops early on non-finite input, so later gathers through it stay in bounds.
__global__ void iota_grouped(const MatGroupArgs *gs)
{
    const MatGroupArgs g = gs[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < g.m) const_cast<int32_t *>(g.piv)[i] = i;
}

__global__ void iota_kernel(int32_t *piv, int m)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) piv[i] = i;
}

__global__ void shift_diag_grouped(const MatGroupArgs *gs)
{
    const MatGroupArgs g = gs[blockIdx.x];
    shift_diag_body(g.X, g.ld, g.m, g.c);
}

__device__ __forceinline__ void set_matrix_body(double *X, int64_t ld, int m, int n, int ident, int64_t e)
{
    if (e >= (int64_t)m * n) return;
    const int i = (int)(e / n), j = (int)(e % n);
    X[(int64_t)i * ld + j] = (ident && i == j) ? 1.0 : 0.0;
}

__global__ void set_matrix_kernel(double *X, int64_t ld, int m, int n, int ident)
{
    set_matrix_body(X, ld, m, n, ident, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void set_matrix_grouped(const MatGroupArgs *gs, int ident)
{
    const MatGroupArgs g = gs[blockIdx.y];
    set_matrix_body(g.X, g.ld, g.m, g.n, ident, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void zero_triangle_kernel(double *X, int64_t ld, int m, int upper)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * m) return;
    const int i = (int)(e / m), j = (int)(e % m);
    if ((upper && j > i) || (!upper && j < i)) X[(int64_t)i * ld + j] = 0.0;
}

__device__ __forceinline__ void rdiag_body(const double *R, int64_t ldr, int m, double *out)
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

__global__ void rdiag_kernel(const double *R, int64_t ldr, int m, double *out) { rdiag_body(R, ldr, m, out); }

__global__ void rdiag_grouped(const MatGroupArgs *gs)
{
    const MatGroupArgs g = gs[blockIdx.x];
    rdiag_body(g.X, g.ld, g.m, g.out);
}

// out[0] = T'^T and out[1] = T' (row-major m x m each) for T' = T Pi:
// column piv[c] of T' is column c of T.
__device__ __forceinline__ void form_tp_body(const double *T, const int32_t *piv, int m, double *out, int64_t e)
{
    if (e >= (int64_t)m * m) return;
    const int r = (int)(e / m), c = (int)(e % m);
    const double v = T[e];
    const int pc = piv[c];
    out[(int64_t)pc * m + r] = v;
    out[(int64_t)m * m + (int64_t)r * m + pc] = v;
}

__global__ void form_tp_kernel(const double *T, const int32_t *piv, int m, double *out)
{
    form_tp_body(T, piv, m, out, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void form_tp_grouped(const MatGroupArgs *gs)
{
    const MatGroupArgs g = gs[blockIdx.y];
    form_tp_body(g.X, g.piv, g.m, g.out, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}


// X's diagonal 64-blocks from the inverted blocks Dinv (nb x nb row-major
// each, block b at Dinv + b nb^2); the rest of X is left as it is.
__global__ void place_diag_blocks_kernel(const double *Dinv, int m, int nb, double *X, int64_t ldx)
{
    const int b = blockIdx.y, base = b * nb, nbb = min(nb, m - base);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nbb * nbb; e += gridDim.x * blockDim.x) {
        const int i = e / nbb, j = e % nbb;
        X[(int64_t)(base + i) * ldx + base + j] = Dinv[(int64_t)b * nb * nb + (int64_t)i * nb + j];
    }
}

// ---------------------------------------------------------------------------
// Newton-Schulz inverse of the Gram.  One wave per row for the norms; the
// affine reduction also yields the Frobenius norm of (out - I) in block
// partials, combined in a fixed order.

// 16 rows per block, 4 per wave: the row maxima meet in LDS and one thread
// per block posts them, so the two slots see two atomics per block rather
// than two per row.
constexpr int NSN_ROWS_PER_WAVE = 4;

__global__ __launch_bounds__(256) void ns_norms_kernel(const double *X, int m, unsigned long long *slots)
{
    __shared__ double wmax[2][4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r0 = (blockIdx.x * 4 + w) * NSN_ROWS_PER_WAVE;
    double rs = 0.0, dg = 0.0;  // largest absolute row sum and positive diagonal entry of this wave
    for (int r = 0; r < NSN_ROWS_PER_WAVE; ++r) {
        const int row = r0 + r;
        if (row >= m) break;  // uniform across the wave
        const double *x = X + (int64_t)row * m;
        double s = 0.0;
        for (int j = lane; j < m; j += 64) s += fabs(x[j]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        // fmax drops a NaN operand: keep NaN row sums by comparing as below
        rs = (s > rs || s != s) ? s : rs;
        const double d = x[row];
        dg = d > dg ? d : dg;
    }
    if (lane == 0) {
        wmax[0][w] = rs;
        wmax[1][w] = dg;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = wmax[0][0], b = wmax[1][0];
        for (int v = 1; v < 4; ++v) {
            a = (wmax[0][v] > a || wmax[0][v] != wmax[0][v]) ? wmax[0][v] : a;
            b = wmax[1][v] > b ? wmax[1][v] : b;
        }
        // non-negative doubles order like their bit patterns (NaN above all)
        atomicMax(slots + 0, (unsigned long long)__double_as_longlong(a));
        atomicMax(slots + 1, (unsigned long long)__double_as_longlong(b));
    }
}

__global__ void ns_start_kernel(const double *X, int m, const unsigned long long *slots, double *Y)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * m) return;
    const double a = 1.0 / __longlong_as_double((long long)slots[0]);
    const int i = (int)(e / m), j = (int)(e % m);
    Y[e] = (i == j ? 2.0 * a : 0.0) - a * a * X[e];
}

__global__ __launch_bounds__(256) void reduce_affine_kernel(const double *part, int64_t stride, int splits, int m,
                                                            double *out, double scale, double diag, double *bsum)
{
    __shared__ double red[4];
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double q = 0.0;
    if (e < (int64_t)m * m) {
        double s = 0.0;
        for (int p = 0; p < splits; ++p) s += part[p * stride + e];
        const double id = ((int)(e / m) == (int)(e % m)) ? 1.0 : 0.0;
        const double v = scale * s + diag * id;
        out[e] = v;
        q = (v - id) * (v - id);
    }
    if (!bsum) return;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void sum_blocks_sqrt_kernel(const double *bsum, int nb, double *out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += bsum[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = __builtin_sqrt(red[0]);
}

// ------------------------------------------------------------------------
// Blocked right-looking Cholesky G = L L^T in one cooperative launch.
//
// The lower triangle of 64 x 64 tiles is numbered column by column,
// t(i, j) = j nb - j (j - 1) / 2 + (i - j), and block b owns the tiles with
// t = b mod (grid size) for the whole factorization (a sub-diagonal tile
// (j + 1, j) belongs to the owner of (j + 1, j + 1) instead, which keeps the
// chain panel -> update -> next diagonal factor inside one block), visiting
// them in column order at every step k:
//   diagonal (k, k): factor it (one wave), X = L_kk^{-1} (the block), write
//     L_kk, publish X as Dinv[k] and raise the step's diagonal flag;
//   panel (i, k), i > k: wait for the diagonal flag, L_ik = A_ik X^T on
//     MFMA, publish L_ik and raise the tile's panel flag;
//   update (i, j), k < j <= i: wait for the panel flags of (i, k) and (j, k),
//     A_ij -= L_ik L_jk^T on MFMA.
// Every tile of G is read and written only by its owner, so a tile's own
// updates are ordinary accesses; data one block hands to another (X and the
// panels) is written and read with device-scope accesses, coherent across the
// XCDs' L2s, and its flag is raised only after those stores have completed.
// The tasks of step k wait only on tasks of step k that come first in this
// order or on earlier steps, and the launch is cooperative (all blocks
// resident), so every wait ends; a wait that spins too long records an error
// and the block goes on, so the grid always drains.  Flags hold the call's
// epoch: a flag is raised when it equals the epoch, so no clearing is needed
// between calls with increasing epochs.
constexpr int CC_T = 256;
constexpr int CC_MAXOWN = 64;  // tiles per block at most
constexpr long CC_SPIN_LIMIT = 1L << 20;

__device__ __forceinline__ void cc_store(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double cc_load(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void cc_wait_stores()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ int cc_tile(int i, int j, int nb) { return j * nb - j * (j - 1) / 2 + (i - j); }

// Tile transfers: thread t moves elements (r, c) = (t / 64 + 4 s, t % 64) for
// s = 0..15 of a 64 x 64 tile.  Every load is issued unconditionally from a
// clamped address and zeroed by a select, so that all sixteen of a thread's
// loads are in flight at once (a masked load becomes a branch that waits for
// it).  Rows r >= nr read as zero.
constexpr int CC_E = NBMAX * NBMAX / CC_T;

__device__ __forceinline__ void cc_tile_to_lds(const double *src, int64_t ld, int nr, bool coherent, double *dst)
{
    const int c = threadIdx.x & 63, rb = threadIdx.x >> 6;
    double v[CC_E];
#pragma unroll
    for (int s = 0; s < CC_E; ++s) {
        const int r = rb + 4 * s;
        const double *q = src + (int64_t)min(r, nr - 1) * ld + c;
        v[s] = coherent ? cc_load(q) : *q;
    }
#pragma unroll
    for (int s = 0; s < CC_E; ++s) {
        const int r = rb + 4 * s;
        dst[r * LDP + c] = r < nr ? v[s] : 0.0;
    }
}

// Thread 0 waits until both flags hold the epoch (b may equal a).  A wait
// that spins too long sets *err = 3, and every wait gives up as soon as it
// sees that value, so after one timeout the grid drains quickly.  Then the
// block is released.
__device__ __forceinline__ void cc_wait(const unsigned *fa, const unsigned *fb, unsigned epoch, int *err)
{
    if (threadIdx.x == 0) {
        long spins = 0;
        while (__hip_atomic_load(const_cast<unsigned *>(fa), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch ||
               __hip_atomic_load(const_cast<unsigned *>(fb), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
            __builtin_amdgcn_s_sleep(1);
            ++spins;
            if (spins > CC_SPIN_LIMIT) {
                __hip_atomic_store(err, 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            if ((spins & 255) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 3) break;
        }
    }
    __syncthreads();
}

// All stores of the block have completed; then thread 0 raises the flag.
__device__ __forceinline__ void cc_raise(unsigned *f, unsigned epoch)
{
    cc_wait_stores();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(f, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// acc = P Q^T for 64 x 64 P, Q in LDS (row stride LDP); wave w holds the
// 32 x 32 quadrant (w / 2, w % 2) as 2 x 2 MFMA tiles.
__device__ __forceinline__ void cc_pqt(const double *P, const double *Q, double4v (&acc)[2][2])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wm = wave >> 1, wn = wave & 1;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = double4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int kk = 0; kk < NBMAX; kk += 4) {
        double av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = P[(wm * 32 + a * 16 + (lane & 15)) * LDP + kk + (lane >> 4)];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = Q[(wn * 32 + b * 16 + (lane & 15)) * LDP + kk + (lane >> 4)];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
}

// Row and column of element r of the accumulator (a, b) in this lane.
__device__ __forceinline__ int cc_row(int a, int r)
{
    return ((threadIdx.x >> 6) >> 1) * 32 + a * 16 + mfma16_row(threadIdx.x & 63, r);
}
__device__ __forceinline__ int cc_col(int b) { return ((threadIdx.x >> 6) & 1) * 32 + b * 16 + mfma16_col(threadIdx.x & 63); }

// Cholesky of the diagonal task's 64 x 64 tile (lower triangle of T, LDS) in
// place, blocked by 16 columns: wave w owns columns
// 16w .. 16w + 15 (lane = row).  Block column B is factored by wave B alone,
// column by column in registers (the pivot and the block's other entries of
// the new column come from the lanes that hold them, no block barrier), then
// published to LDS; after one block barrier the later waves subtract its
// rank-16 contribution from their columns.  Four barriers in all instead of
// one per column.  Wk: 2 x 64 x 17 doubles of LDS scratch.
__device__ __forceinline__ bool cc_chol64(double *T, double *Wk, int *s_bad)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double a[16];
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) a[cc] = T[lane * LDP + 16 * w + cc];
    if (threadIdx.x == 0) *s_bad = 0;
    bool bad = false;
#pragma unroll
    for (int B = 0; B < 4; ++B) {
        double *pb = Wk + (B & 1) * (NBMAX * 17);
        if (w == B) {
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                const int j = 16 * B + jj;
                const double d = lane_value(a[jj], j);
                bad |= !(d > 0.0 && d < INFINITY);
                // 1/sqrt(d): the hardware estimate and one Newton step
                // (e = 1 - d y^2, y += y e / 2), within an ulp or two;
                // l_jj = d / sqrt(d)
                const double y0 = __builtin_amdgcn_rsq(d);
                const double e0 = __builtin_fma(-d * y0, y0, 1.0);
                const double inv = __builtin_fma(0.5 * y0, e0, y0);
                const double ljj = d * inv;
                const double lij = (lane == j) ? ljj : (lane > j ? a[jj] * inv : 0.0);
                a[jj] = lij;
#pragma unroll
                for (int cc = jj + 1; cc < 16; ++cc) a[cc] = __builtin_fma(-lij, lane_value(lij, 16 * B + cc), a[cc]);
            }
#pragma unroll
            for (int cc = 0; cc < 16; ++cc) pb[lane * 17 + cc] = a[cc];
        }
        __syncthreads();
        if (w > B) {
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const double li = pb[lane * 17 + t];
#pragma unroll
                for (int cc = 0; cc < 16; ++cc) a[cc] = __builtin_fma(-li, pb[(16 * w + cc) * 17 + t], a[cc]);
            }
        }
    }
    if (bad) *s_bad = 1;
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
        const int c = 16 * w + cc;
        T[lane * LDP + c] = c <= lane ? a[cc] : 0.0;
    }
    __syncthreads();
    return *s_bad != 0;
}

// Blocked X = L^{-1} (64 x 64 lower, LDS stride LDP; X may not alias L):
// first wave w inverts the diagonal block L_ww (16 x 16) by forward
// substitution (a quad of lanes per column: lane q keeps rows 4 s + q) and
// zeroes its block row above the diagonal; then, for d = 1, 2, 3, wave j
// forms X_ij (i = j + d) = -X_ii sum_{k=j}^{i-1} L_ik X_kj from blocks of
// earlier levels, through a 16 x 16 scratch per wave (scr: 4 x 16 x 17).
__device__ __forceinline__ void cc_lower_inverse(const double *L, double *X, double *invd, double *scr)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x < NBMAX) invd[threadIdx.x] = 1.0 / L[threadIdx.x * LDP + threadIdx.x];
    __syncthreads();
    {
        const int jc = lane >> 2, q = lane & 3, o = 16 * w;
        double xr[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ii = 0; ii < 16; ++ii) {
            double sq = 0.0;
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) {
                if (4 * s2 >= ii) break;
                sq = __builtin_fma(L[(o + ii) * LDP + o + 4 * s2 + q], xr[s2], sq);
            }
            sq += __shfl_xor(sq, 1, 64);
            sq += __shfl_xor(sq, 2, 64);
            const double xi = ((ii == jc ? 1.0 : 0.0) - sq) * invd[o + ii];
            xr[ii >> 2] = (q == (ii & 3)) ? xi : xr[ii >> 2];
        }
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) X[(o + 4 * s2 + q) * LDP + o + jc] = xr[s2];
        for (int e = lane; e < 16 * (48 - o); e += 64) X[(o + e / (48 - o)) * LDP + o + 16 + e % (48 - o)] = 0.0;
    }
    __syncthreads();
    const int r = lane >> 2, c0 = 4 * (lane & 3);
    double *S = scr + w * (16 * 17);
#pragma unroll
    for (int d = 1; d < 4; ++d) {
        const int j = w, i = w + d;
        const bool act = i < 4;
        if (act) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int k = j; k < i; ++k) {
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const double lv = L[(16 * i + r) * LDP + 16 * k + t];
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc[u] = __builtin_fma(lv, X[(16 * k + t) * LDP + 16 * j + c0 + u], acc[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) S[r * 17 + c0 + u] = acc[u];
        }
        __syncthreads();
        if (act) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const double xv = X[(16 * i + r) * LDP + 16 * i + t];
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[u] = __builtin_fma(xv, S[t * 17 + c0 + u], acc[u]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) X[(16 * i + r) * LDP + 16 * j + c0 + u] = -acc[u];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(CC_T) void chol_coop_kernel(CholCoopArgs g)
{
    static_assert(CC_T == 4 * NBMAX, "four waves; a quad of lanes per column of the inverse");
    __shared__ double P[NBMAX * LDP];
    __shared__ double Q[NBMAX * LDP];
    __shared__ double invd[NBMAX];
    __shared__ double scr[4 * 16 * 17];
    __shared__ short own_i[CC_MAXOWN], own_j[CC_MAXOWN];
    __shared__ int s_nown, s_bad;
    const int m = g.m, nb = (m + NBMAX - 1) / NBMAX, ntiles = nb * (nb + 1) / 2;
    const int B = gridDim.x;
    unsigned *dflag = g.flags, *pflag = g.flags + nb;
    if (threadIdx.x == 0) {
        // the tiles t = b mod B except the sub-diagonal ones (j + 1, j), which
        // go to the owner of the diagonal tile (j + 1, j + 1) so that the
        // panel task on them, the update of that diagonal tile and its
        // factorization follow one another in one block; merged in column
        // order
        const int b = blockIdx.x;
        int n = 0, jr = 0, start = 0, t = b, js = 0;
        while (js < nb - 1 && cc_tile(js + 1, js + 1, nb) % B != b) ++js;
        for (;;) {
            int ir = -1;
            while (t < ntiles) {
                while (start + (nb - jr) <= t) { start += nb - jr; ++jr; }
                ir = jr + (t - start);
                if (ir != jr + 1) break;
                t += B;
            }
            const bool has_r = t < ntiles, has_s = js < nb - 1;
            if ((!has_r && !has_s) || n >= CC_MAXOWN) break;
            if (has_r && (!has_s || t < cc_tile(js + 1, js, nb))) {
                own_i[n] = (short)ir;
                own_j[n] = (short)jr;
                t += B;
            } else {
                own_i[n] = (short)(js + 1);
                own_j[n] = (short)js;
                ++js;
                while (js < nb - 1 && cc_tile(js + 1, js + 1, nb) % B != b) ++js;
            }
            ++n;
        }
        s_nown = n;
    }
    __syncthreads();
    const int nown = s_nown;
    const int tid = threadIdx.x;
    // factor the diagonal tile kk held in P (lower triangle, the identity
    // past m), invert the factor, store both and raise the tile's flag
    auto factor_publish = [&](int kk, int nr) {
        const int r0 = kk * NBMAX;
        __syncthreads();
        if (cc_chol64(P, Q, &s_bad) && tid == 0)
            __hip_atomic_store(g.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        cc_lower_inverse(P, Q, invd, scr);
        double *X = g.Dinv + (int64_t)kk * NBMAX * NBMAX;
        const int c = tid & 63, rb = tid >> 6;
#pragma unroll
        for (int s2 = 0; s2 < CC_E; ++s2) {
            const int r = rb + 4 * s2;
            cc_store(X + r * NBMAX + c, Q[r * LDP + c]);
            if (r < nr && c < nr && c <= r) g.L[(int64_t)(r0 + r) * g.ldl + r0 + c] = P[r * LDP + c];
        }
        cc_raise(dflag + kk, g.epoch);
    };
    // diagonal tile factored early (see the panel task below), -1: none
    int diag_done = -1;
    for (int k = 0; k < nb; ++k) {
        for (int q = 0; q < nown; ++q) {
            const int i = own_i[q], j = own_j[q];
            if (j < k) continue;
            if (i == j && diag_done == i) continue;  // its last update and factorization are done
            const int r0 = i * NBMAX, c0 = j * NBMAX;
            const int nr = min(NBMAX, m - r0), nc = min(NBMAX, m - c0);
            int fac = -1;  // diagonal tile to factor from P after this task
            __syncthreads();  // the previous task's LDS reads are done
            if (j == k && i == k) {
                // diagonal: factor, invert, publish
                {
                    const int c = tid & 63, rb = tid >> 6;
                    double v[CC_E];
#pragma unroll
                    for (int s2 = 0; s2 < CC_E; ++s2) {
                        const int r = rb + 4 * s2;
                        v[s2] = g.G[(int64_t)(r0 + min(r, nr - 1)) * g.ldg + r0 + min(c, nr - 1)];
                    }
#pragma unroll
                    for (int s2 = 0; s2 < CC_E; ++s2) {
                        const int r = rb + 4 * s2;
                        P[r * LDP + c] = (r < nr && c < nr) ? (c <= r ? v[s2] : 0.0) : (r == c ? 1.0 : 0.0);
                    }
                }
                fac = k;
            } else if (j == k) {
                // panel: L_ik = A_ik X^T
                cc_wait(dflag + k, dflag + k, g.epoch, g.err);
                cc_tile_to_lds(g.Dinv + (int64_t)k * NBMAX * NBMAX, NBMAX, NBMAX, true, Q);
                cc_tile_to_lds(g.G + (int64_t)r0 * g.ldg + c0, g.ldg, nr, false, P);  // nc = 64: k < nb - 1
                __syncthreads();
                double4v acc[2][2];
                cc_pqt(P, Q, acc);
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int rr = cc_row(a, r), cc = cc_col(b);
                            if (rr < nr && cc < nc) cc_store(g.L + (int64_t)(r0 + rr) * g.ldl + c0 + cc, acc[a][b][r]);
                        }
                if (i != k + 1) {
                    cc_raise(pflag + cc_tile(i, k, nb), g.epoch);
                    continue;
                }
                // (the diagonal tile has the panel's rows: nr)
                // This block also owns the diagonal tile (k + 1, k + 1), whose
                // last update is the one by this panel: apply it from LDS and
                // factor the tile at once, ahead of the step's other tasks
                // (it waits on nothing outside this block).
                __syncthreads();  // the panel product's LDS reads are done
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int rr = cc_row(a, r), cc = cc_col(b);
                            P[rr * LDP + cc] = rr < nr ? acc[a][b][r] : 0.0;
                        }
                cc_raise(pflag + cc_tile(i, k, nb), g.epoch);  // (its barrier also orders the LDS writes)
                // the diagonal tile's values load while the update product runs
                double gv[2][2][4];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            gv[a][b][r] = g.G[(int64_t)(r0 + min(cc_row(a, r), nr - 1)) * g.ldg + r0 +
                                              min(cc_col(b), nr - 1)];
                cc_pqt(P, P, acc);
                __syncthreads();  // the update product's LDS reads are done
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int rr = cc_row(a, r), cc = cc_col(b);
                            P[rr * LDP + cc] = (rr < nr && cc < nr) ? (cc <= rr ? gv[a][b][r] - acc[a][b][r] : 0.0)
                                                                    : (rr == cc ? 1.0 : 0.0);
                        }
                fac = k + 1;
                diag_done = k + 1;
            } else {
                // update: A_ij -= L_ik L_jk^T
                cc_wait(pflag + cc_tile(i, k, nb), pflag + cc_tile(j, k, nb), g.epoch, g.err);
                const int k0 = k * NBMAX;  // column block k is full: k < j <= nb - 1
                cc_tile_to_lds(g.L + (int64_t)r0 * g.ldl + k0, g.ldl, nr, true, P);
                cc_tile_to_lds(g.L + (int64_t)c0 * g.ldl + k0, g.ldl, nc, true, Q);
                __syncthreads();
                // this block's own tile of G: straight-line loads (clamped),
                // then the product, then the masked stores
                double gv[2][2][4];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            gv[a][b][r] = g.G[(int64_t)(r0 + min(cc_row(a, r), nr - 1)) * g.ldg + c0 +
                                              min(cc_col(b), nc - 1)];
                double4v acc[2][2];
                cc_pqt(P, Q, acc);
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int rr = cc_row(a, r), cc = cc_col(b);
                            if (rr < nr && cc < nc && (i > j || cc <= rr))
                                g.G[(int64_t)(r0 + rr) * g.ldg + c0 + cc] = gv[a][b][r] - acc[a][b][r];
                        }
            }
            if (fac >= 0) factor_publish(fac, nr);
        }
    }
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
    hipLaunchKernelGGL(tri_diag_inv_kernel, dim3(nblk), dim3(DT), 0, stream, T, t_i, t_j, m, nb, Dinv);
    return hipGetLastError();
}

hipError_t chol_diag_f64(const double *X, int64_t ldx, int m, int nb, int b, double *L, int64_t ldl, double *Dinv,
                         int *err, hipStream_t stream)
{
    if (nb != NBMAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(NBMAX), 0, stream, X, ldx, m, nb, b, L, ldl, Dinv, err);
    return hipGetLastError();
}

int chol_coop_blocks(int m, int device)
{
    const int nb = (m + NBMAX - 1) / NBMAX, ntiles = nb * (nb + 1) / 2;
    int cus = 0, per = 0, coop = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess || !coop) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, chol_coop_kernel, CC_T, 0) != hipSuccess || per < 1) return 0;
    const int blocks = std::min(ntiles, cus);  // one block per compute unit at most
    if ((ntiles + blocks - 1) / blocks + (nb + blocks - 1) / blocks > CC_MAXOWN) return 0;
    return blocks;
}

hipError_t chol_coop_f64(const CholCoopArgs &a, int blocks, hipStream_t stream)
{
    const int nb = (a.m + NBMAX - 1) / NBMAX, ntiles = nb * (nb + 1) / 2;
    if (a.m <= 0) return hipSuccess;
    if (blocks < 1 || (ntiles + blocks - 1) / blocks + (nb + blocks - 1) / blocks > CC_MAXOWN)
        return hipErrorInvalidValue;
    CholCoopArgs g = a;
    void *args[] = {(void *)&g};
    return hipLaunchCooperativeKernel((const void *)chol_coop_kernel, dim3(blocks), dim3(CC_T), args, 0, stream);
}

hipError_t shift_diag_f64(double *G, int64_t ld, int m, double c, hipStream_t stream)
{
    hipLaunchKernelGGL(shift_diag_kernel, dim3(1), dim3(256), 0, stream, G, ld, m, c);
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

hipError_t chol_diag_grouped_f64(const CholGroupArgs *d, int count, int nb, int b, hipStream_t stream)
{
    if (nb != NBMAX) return hipErrorInvalidValue;
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(chol_diag_grouped, dim3(count), dim3(NBMAX), 0, stream, d, nb, b);
    return hipGetLastError();
}

hipError_t tri_diag_inv_grouped_f64(const TriInvGroupArgs *d, int count, int max_m, int nb, hipStream_t stream)
{
    if (nb != NBMAX) return hipErrorInvalidValue;
    if (count <= 0 || max_m <= 0) return hipSuccess;
    hipLaunchKernelGGL(tri_diag_inv_grouped, dim3((max_m + nb - 1) / nb, count), dim3(DT), 0, stream, d, nb);
    return hipGetLastError();
}

hipError_t set_matrix_grouped_f64(const MatGroupArgs *d, int count, int64_t max_total, int ident, hipStream_t stream)
{
    if (count <= 0 || max_total <= 0) return hipSuccess;
    hipLaunchKernelGGL(set_matrix_grouped, dim3((unsigned)((max_total + 255) / 256), count), dim3(256), 0, stream, d,
                       ident);
    return hipGetLastError();
}

hipError_t iota_f64piv(int32_t *piv, int m, hipStream_t stream)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(iota_kernel, dim3((m + 255) / 256), dim3(256), 0, stream, piv, m);
    return hipGetLastError();
}

hipError_t iota_grouped_i32(const MatGroupArgs *d, int count, int max_m, hipStream_t stream)
{
    if (count <= 0 || max_m <= 0) return hipSuccess;
    hipLaunchKernelGGL(iota_grouped, dim3((max_m + 255) / 256, count), dim3(256), 0, stream, d);
    return hipGetLastError();
}

hipError_t shift_diag_grouped_f64(const MatGroupArgs *d, int count, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(shift_diag_grouped, dim3(count), dim3(256), 0, stream, d);
    return hipGetLastError();
}

hipError_t rdiag_grouped_f64(const MatGroupArgs *d, int count, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(rdiag_grouped, dim3(count), dim3(256), 0, stream, d);
    return hipGetLastError();
}

hipError_t form_tp_grouped_f64(const MatGroupArgs *d, int count, int64_t max_total, hipStream_t stream)
{
    if (count <= 0 || max_total <= 0) return hipSuccess;
    hipLaunchKernelGGL(form_tp_grouped, dim3((unsigned)((max_total + 255) / 256), count), dim3(256), 0, stream, d);
    return hipGetLastError();
}

hipError_t ns_norms_f64(const double *X, int m, unsigned long long *slots, hipStream_t stream)
{
    if (m <= 0) return hipSuccess;
    const int rows_per_block = 4 * NSN_ROWS_PER_WAVE;
    hipLaunchKernelGGL(ns_norms_kernel, dim3((unsigned)((m + rows_per_block - 1) / rows_per_block)), dim3(256), 0,
                       stream, X, m, slots);
    return hipGetLastError();
}

hipError_t ns_start_f64(const double *X, int m, const unsigned long long *slots, double *Y, hipStream_t stream)
{
    const int64_t total = (int64_t)m * m;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(ns_start_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, X, m, slots, Y);
    return hipGetLastError();
}

hipError_t reduce_affine_f64(const double *part, int64_t stride, int splits, int m, double *out, double scale,
                             double diag, double *bsum, hipStream_t stream)
{
    const int64_t total = (int64_t)m * m;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_affine_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, part,
                       stride, splits, m, out, scale, diag, bsum);
    return hipGetLastError();
}

hipError_t sum_blocks_sqrt_f64(const double *bsum, int nb, double *out, hipStream_t stream)
{
    hipLaunchKernelGGL(sum_blocks_sqrt_kernel, dim3(1), dim3(256), 0, stream, bsum, nb, out);
    return hipGetLastError();
}

hipError_t place_diag_blocks_f64(const double *Dinv, int m, int nb, double *X, int64_t ldx, hipStream_t stream)
{
    const int nblk = (m + nb - 1) / nb;
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(place_diag_blocks_kernel, dim3(4, nblk), dim3(256), 0, stream, Dinv, m, nb, X, ldx);
    return hipGetLastError();
}

}  // namespace rt
