// Randomized sketch S = A G (Sec. 4, eq. testing) with G a subsampled
// randomized Fourier transform: per row a of A, y = Pi D pad(a), Y = FFT(y),
// keep l entries of the orthonormal real packing of Y, scaled by sqrt(np/l).
//
// Two rows are transformed together as one complex signal (real part = row
// 2p, imaginary part = row 2p+1) and separated after the transform with the
// conjugate symmetry of real spectra.  The np-point transform is a four-step
// FFT over the n1 x n2 grid t = t1*n2 + t2, k = k1 + n1*k2:
//   pass 1: for each column t2: n1-point FFT over t1 (in LDS), times the
//           twiddle exp(-2 pi i t2 k1 / np);
//   pass 2: for each k1: n2-point FFT over t2 (in LDS), then unpack the two
//           real spectra and write only the l selected outputs.
// The permutation pi(t) = sigma[t1]*n2 + tau[t2] is folded into the loads:
// a pass-1 block takes the columns t2 = tau^{-1}(u) for a run of u, so each
// of its n1 gathers reads a contiguous run of A's row (coalesced); the
// intermediate stays in the tau-image order u and pass 2 places entry u at
// position tau^{-1}(u) in LDS.
#include <algorithm>

#include "rt_common.h"

namespace rt {

namespace {

template <typename R>
struct cpx { R re, im; };

template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b)
{
    return cpx<R>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

__device__ __forceinline__ unsigned bitrev(unsigned x, int bits)
{
    return bits == 0 ? 0u : (__builtin_bitreverse32(x) >> (32 - bits));
}

// In-place radix-2 decimation-in-time FFT of `cols` columns of length `len`
// stored column after column in LDS with column stride ld (input already in
// bit-reversed order).  tw: len/2 twiddles exp(-2 pi i j / len) in LDS.
//
// Up to MAXB consecutive radix-2 stages (half-sizes h, 2h, 4h, 8h) run in
// registers: a thread loads the 2^B elements base + j h (base = blk 2^B h +
// pos, pos < h) that those stages combine, applies the same butterflies the
// stage-by-stage form would, and writes them back; one block barrier per
// group of stages instead of one per stage.  Different groupings can still
// differ in the last bit, where the compiler fuses a product into a
// multiply-add in one shape of the code and not in another, so every kernel
// that must agree bitwise uses the same MAXB.
// Consecutive threads take consecutive columns, whose stride ld = len + 1
// puts their accesses on distinct banks.
template <typename R, int B>
__device__ __forceinline__ void fft_stage_group(cpx<R> *buf, int len, int ld, int cols, const cpx<R> *tw, int h)
{
    constexpr int G = 1 << B;
    const int tasks = (len / G) * cols;
    for (int t = threadIdx.x; t < tasks; t += blockDim.x) {
        const int c = t % cols, gi = t / cols;
        const int pos = gi % h, blk = gi / h;
        const int base = blk * G * h + pos;
        cpx<R> *col = buf + (int64_t)c * ld;
        cpx<R> x[G];
#pragma unroll
        for (int j = 0; j < G; ++j) x[j] = col[base + j * h];
#pragma unroll
        for (int st = 0; st < B; ++st) {
            const int hs = h << st;              // half-size of this stage
            const int tstep = len / (2 * hs);    // twiddle index step
#pragma unroll
            for (int j = 0; j < G; ++j) {
                if ((j >> st) & 1) continue;
                const int pj = pos + (j & ((1 << st) - 1)) * h;  // position inside the 2 hs block
                const cpx<R> w = tw[pj * tstep];
                const cpx<R> a = x[j];
                const cpx<R> b = cmul(x[j + (1 << st)], w);
                x[j] = cpx<R>{a.re + b.re, a.im + b.im};
                x[j + (1 << st)] = cpx<R>{a.re - b.re, a.im - b.im};
            }
        }
#pragma unroll
        for (int j = 0; j < G; ++j) col[base + j * h] = x[j];
    }
}

template <typename R, int MAXB = 4>
__device__ __forceinline__ void lds_fft_cols(cpx<R> *buf, int len, int ld, int cols, const cpx<R> *tw)
{
    for (int h = 1; h < len;) {
        int rem = 0;
        while ((h << rem) < len) ++rem;  // stages left
        switch (rem < MAXB ? rem : MAXB) {
        case 4: fft_stage_group<R, 4>(buf, len, ld, cols, tw, h); h <<= 4; break;
        case 3: fft_stage_group<R, 3>(buf, len, ld, cols, tw, h); h <<= 3; break;
        case 2: fft_stage_group<R, 2>(buf, len, ld, cols, tw, h); h <<= 2; break;
        default: fft_stage_group<R, 1>(buf, len, ld, cols, tw, h); h <<= 1; break;
        }
        __syncthreads();
    }
}

// Shared launch geometry of the two passes for one problem.
struct SketchGeom {
    int tw_cols, bits1, cp, bits2;
};

__host__ __device__ inline int ilog2(int64_t v)
{
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

template <typename R>
__host__ __device__ inline SketchGeom sketch_geom(const SketchTables &t)
{
    const int64_t csz = sizeof(cpx<R>);
    SketchGeom g;
    g.tw_cols = t.n2 < 16 ? (int)t.n2 : 16;
    while (g.tw_cols > 1 && (int64_t)g.tw_cols * t.n1 * csz > 64 * 1024) g.tw_cols >>= 1;
    g.cp = (int)((64 * 1024) / (2 * csz * t.n2));
    if (g.cp < 1) g.cp = 1;
    if (g.cp > 8) g.cp = 8;
    g.bits1 = ilog2(t.n1);
    g.bits2 = ilog2(t.n2);
    return g;
}

// Stages per register pass of the pass-1 column transforms: three in
// binary32, whose pipelined passes hold 32 gathered elements per thread in
// flight beside them, four in binary64; the plain, pipelined and grouped
// passes all use it, so a plan's sketch and a batch member's agree bitwise.
template <typename R>
struct Pass1Stages { static constexpr int value = sizeof(R) == 4 ? 3 : 4; };
// The same for the row transforms of pass 2.
template <typename R>
struct Pass2Stages { static constexpr int value = sizeof(R) == 4 ? 3 : 4; };

// Dynamic LDS of pass 1 (bytes), in this order: n1/2 twiddles of the
// n1-point FFT, the tw_cols x n1 columns, the two-level twiddle tables of
// the np-point product (np/tl and tl entries), sigma (n1) and the tw_cols
// in-block indices.  Pass 2: n2/2 twiddles, cp x 2 x n2 columns, tau^{-1} (n2).
template <typename R>
__host__ __device__ inline size_t pass1_smem(int64_t n1, int64_t n2, int tw_cols)
{
    const int64_t np = n1 * n2;
    const int tl_bits = (ilog2(np) + 1) / 2;
    const int64_t c = (n1 >> 1) + (int64_t)tw_cols * (n1 + 1) + (np >> tl_bits) + (int64_t(1) << tl_bits);
    return (size_t)(c * (int64_t)sizeof(cpx<R>) + (n1 + tw_cols) * 4);
}

template <typename R>
__host__ __device__ inline size_t pass2_smem(int64_t n2, int cp)
{
    return (size_t)(((n2 >> 1) + (int64_t)cp * 2 * (n2 + 1)) * (int64_t)sizeof(cpx<R>) + n2 * 4);
}

constexpr int SK_U = 8;  // gathers in flight per thread

template <typename R>
__device__ __forceinline__ void sketch_pass1_body(const SketchTables &t, const double *A, int64_t lda, int64_t m,
                                                  int64_t row0, cpx<R> *zbuf, int tw_cols, int bits1, int bx,
                                                  int64_t pair, const double *cs = nullptr)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    typedef cpx<R> cplx;
    cplx *smem = reinterpret_cast<cplx *>(smem_raw);
    const int n1 = (int)t.n1, n2 = (int)t.n2;
    const int nh = (int)(t.np >> t.tl_bits), nl = 1 << t.tl_bits;
    cplx *tw = smem;                           // n1/2
    const int ld1 = n1 + 1;                    // padded column stride (no bank conflicts across columns)
    cplx *buf = tw + (n1 >> 1);                // tw_cols x ld1
    cplx *th = buf + (int64_t)tw_cols * ld1;   // np / tl
    cplx *tlo = th + nh;                       // tl
    int *s_sigma = reinterpret_cast<int *>(tlo + nl);
    int *s_tinv = s_sigma + n1;
    const int64_t r0 = row0 + 2 * pair, r1 = r0 + 1;
    const int u0 = bx * tw_cols;
    if (u0 >= n2 || r0 >= m) return;  // whole block (grouped launches)
    const cplx *tw1 = reinterpret_cast<const cplx *>(sizeof(R) == 8 ? (const void *)t.tw1 : (const void *)t.tw1f);
    const cplx *twh = reinterpret_cast<const cplx *>(sizeof(R) == 8 ? (const void *)t.twh : (const void *)t.twhf);
    const cplx *twl = reinterpret_cast<const cplx *>(sizeof(R) == 8 ? (const void *)t.twl : (const void *)t.twlf);
    // stage the small tables once, so no gather below waits on a table load
    for (int e = threadIdx.x; e < (n1 >> 1); e += blockDim.x) tw[e] = tw1[e];
    for (int e = threadIdx.x; e < nh; e += blockDim.x) th[e] = twh[e];
    for (int e = threadIdx.x; e < nl; e += blockDim.x) tlo[e] = twl[e];
    for (int e = threadIdx.x; e < n1; e += blockDim.x) s_sigma[e] = t.sigma[e];
    for (int e = threadIdx.x; e < tw_cols; e += blockDim.x) s_tinv[e] = t.tau_inv[u0 + e];
    __syncthreads();
    const double *a0 = A + r0 * lda;
    const double *a1 = A + r1 * lda;
    const bool has1 = r1 < m;
    const int total = n1 * tw_cols;
    // gathers: SK_U independent loads per thread in flight at a time; each
    // run of tw_cols consecutive elements of a row is read contiguously
    for (int base = threadIdx.x; base < total; base += SK_U * blockDim.x) {
        double v0[SK_U], v1[SK_U], sg[SK_U];
        int dst[SK_U];
#pragma unroll
        for (int q = 0; q < SK_U; ++q) {
            const int e = base + q * blockDim.x;
            v0[q] = 0.0; v1[q] = 0.0; sg[q] = 0.0; dst[q] = -1;
            if (e < total) {
                const int t1 = e / tw_cols, j = e - t1 * tw_cols;
                const int64_t src = (int64_t)s_sigma[t1] * n2 + u0 + j;
                dst[q] = j * ld1 + (int)bitrev((unsigned)t1, bits1);
                if (src < t.n) {
                    // the sign of D, times the column scaling when A is scaled
                    // (sign * (a * c) rounds as a * (sign * c))
                    sg[q] = cs ? (double)t.sign[src] * cs[src] : (double)t.sign[src];
                    v0[q] = a0[src];
                    if (has1) v1[q] = a1[src];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < SK_U; ++q)
            if (dst[q] >= 0) buf[dst[q]] = cplx{(R)(sg[q] * v0[q]), (R)(sg[q] * v1[q])};
    }
    __syncthreads();
    lds_fft_cols<R, Pass1Stages<R>::value>(buf, n1, ld1, tw_cols, tw);
    const int tl_mask = nl - 1;
    cplx *zp = zbuf + pair * t.np;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int k1 = e / tw_cols, j = e - k1 * tw_cols;
        const int idx = s_tinv[j] * k1;  // < np, no reduction needed
        const cplx w = cmul(th[idx >> t.tl_bits], tlo[idx & tl_mask]);
        zp[(int64_t)k1 * n2 + u0 + j] = cmul(buf[(int64_t)j * ld1 + k1], w);
    }
}

template <typename R>
__global__ __launch_bounds__(256) void sketch_pass1(SketchTables t, const double *A, int64_t lda, int64_t m,
                                                    int64_t row0, cpx<R> *zbuf, int tw_cols, int bits1)
{
    sketch_pass1_body<R>(t, A, lda, m, row0, zbuf, tw_cols, bits1, blockIdx.x, blockIdx.y);
}

// Pass 1 for column group bx and a run of row pairs (pair = by, by + gy,
// ...), software-pipelined: the gathers of the next pair are
// issued right after the current pair is staged in LDS, so they stay in
// flight through its transform and its stores (block barriers wait for LDS
// only).  Q = n1 * tw_cols / 256 elements per thread, all of them loaded and
// stored unconditionally: rows past m and positions past n are read clamped
// and zeroed when staged, so the memory counters stay exact across the loop.
// A thread's elements share j = tid % tw_cols, so their signs and padding
// flags are two bit masks held for the whole run.  Same arithmetic per
// element and per column as sketch_pass1 (bitwise the same intermediate).
//
// With a column scaling cs (a batch member's A diag(cs)), each element is
// scaled when staged, cs re-read per row pair from the cache in groups of
// min(Q, 8) so that only that many scales are live beside the gathered data; the
// product rounds as the plain pass's sign * cs times the element does.
template <typename R, int Q>
__device__ __forceinline__ void pass1_pipe_body(const SketchTables &t, const double *A, int64_t lda, int64_t m,
                                                int64_t row0, int64_t npairs, cpx<R> *zbuf, int tw_cols, int bits1,
                                                int bx, int64_t by, int64_t gy, const double *cs)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    typedef cpx<R> cplx;
    cplx *smem = reinterpret_cast<cplx *>(smem_raw);
    const int n1 = (int)t.n1, n2 = (int)t.n2;
    const int nh = (int)(t.np >> t.tl_bits), nl = 1 << t.tl_bits;
    cplx *tw = smem;
    const int ld1 = n1 + 1;
    cplx *buf = tw + (n1 >> 1);
    cplx *th = buf + (int64_t)tw_cols * ld1;
    cplx *tlo = th + nh;
    int *s_sigma = reinterpret_cast<int *>(tlo + nl);
    int *s_tinv = s_sigma + n1;
    const int u0 = bx * tw_cols;
    if (u0 >= n2 || by >= npairs) return;
    const cplx *tw1 = reinterpret_cast<const cplx *>(sizeof(R) == 8 ? (const void *)t.tw1 : (const void *)t.tw1f);
    const cplx *twh = reinterpret_cast<const cplx *>(sizeof(R) == 8 ? (const void *)t.twh : (const void *)t.twhf);
    const cplx *twl = reinterpret_cast<const cplx *>(sizeof(R) == 8 ? (const void *)t.twl : (const void *)t.twlf);
    for (int e = threadIdx.x; e < (n1 >> 1); e += blockDim.x) tw[e] = tw1[e];
    for (int e = threadIdx.x; e < nh; e += blockDim.x) th[e] = twh[e];
    for (int e = threadIdx.x; e < nl; e += blockDim.x) tlo[e] = twl[e];
    for (int e = threadIdx.x; e < n1; e += blockDim.x) s_sigma[e] = t.sigma[e];
    for (int e = threadIdx.x; e < tw_cols; e += blockDim.x) s_tinv[e] = t.tau_inv[u0 + e];
    __syncthreads();
    // element q of this thread: e = tid + 256 q, t1 = e / tw_cols, j = tid % tw_cols
    const int j = threadIdx.x % tw_cols, t1_0 = threadIdx.x / tw_cols, t1_step = 256 / tw_cols;
    unsigned neg = 0, pad = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int64_t x = (int64_t)s_sigma[t1_0 + q * t1_step] * n2 + u0 + j;
        if (x >= t.n) pad |= 1u << q;
        else if (t.sign[x] < 0) neg |= 1u << q;
    }
    double v0[Q], v1[Q];
    // positions are re-read from the staged permutation at every gather
    // rather than held (registers go to the data in flight)
    // (32-bit byte offsets from the two row bases: the host takes this path
    // only when a row of A spans less than 4 GiB)
    auto gather = [&](int64_t pr) {
        const int64_t r0 = row0 + 2 * pr;
        const char *a0 = reinterpret_cast<const char *>(A + r0 * lda);
        const char *a1 = reinterpret_cast<const char *>(A + (r0 + 1 < m ? r0 + 1 : r0) * lda);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const unsigned x = (unsigned)s_sigma[t1_0 + q * t1_step] * (unsigned)n2 + (unsigned)(u0 + j);
            const unsigned off = (x < (unsigned)t.n ? x : (unsigned)t.n - 1u) * 8u;
            v0[q] = *reinterpret_cast<const double *>(a0 + off);
            v1[q] = *reinterpret_cast<const double *>(a1 + off);
        }
    };
    const int tl_mask = nl - 1;
    int64_t pair = by;
    gather(pair);
    for (; pair < npairs; pair += gy) {
        const bool has1 = row0 + 2 * pair + 1 < m;
        if (cs) {
            constexpr int CG = Q < 8 ? Q : 8;  // scales per group, never past the Q elements
            static_assert(Q % CG == 0, "whole groups of scales");
#pragma unroll
            for (int q0 = 0; q0 < Q; q0 += CG) {
                double c[CG];
#pragma unroll
                for (int i = 0; i < CG; ++i) {
                    const int64_t x = (int64_t)s_sigma[t1_0 + (q0 + i) * t1_step] * n2 + u0 + j;
                    c[i] = cs[x < t.n ? x : t.n - 1];
                }
#pragma unroll
                for (int i = 0; i < CG; ++i) {
                    const int q = q0 + i, t1 = t1_0 + q * t1_step;
                    const double s0 = c[i] * v0[q], s1 = c[i] * (has1 ? v1[q] : 0.0);
                    const double a = (pad >> q) & 1 ? 0.0 : ((neg >> q) & 1 ? -s0 : s0);
                    const double b = (pad >> q) & 1 ? 0.0 : ((neg >> q) & 1 ? -s1 : s1);
                    buf[j * ld1 + (int)bitrev((unsigned)t1, bits1)] = cplx{(R)a, (R)b};
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int t1 = t1_0 + q * t1_step;
                const double a = (pad >> q) & 1 ? 0.0 : ((neg >> q) & 1 ? -v0[q] : v0[q]);
                const double v = has1 ? v1[q] : 0.0;  // a missing odd row: a signed zero, as sign * 0
                const double b = (pad >> q) & 1 ? 0.0 : ((neg >> q) & 1 ? -v : v);
                buf[j * ld1 + (int)bitrev((unsigned)t1, bits1)] = cplx{(R)a, (R)b};
            }
        }
        __syncthreads();
        // the next pair of this block (the last one re-reads its own pair)
        const int64_t nxt = pair + gy;
        gather(nxt < npairs ? nxt : pair);
        lds_fft_cols<R, Pass1Stages<R>::value>(buf, n1, ld1, tw_cols, tw);
        cplx *zp = zbuf + pair * t.np;
#pragma unroll 2
        for (int q = 0; q < Q; ++q) {
            const int k1 = t1_0 + q * t1_step;
            const int idx = s_tinv[j] * k1;
            const cplx w = cmul(th[idx >> t.tl_bits], tlo[idx & tl_mask]);
            zp[(int64_t)k1 * n2 + u0 + j] = cmul(buf[(int64_t)j * ld1 + k1], w);
        }
        __syncthreads();
    }
}

template <typename R, int Q>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void sketch_pass1_pipe(
    SketchTables t, const double *A, int64_t lda, int64_t m, int64_t row0, int64_t npairs, cpx<R> *zbuf, int tw_cols,
    int bits1)
{
    pass1_pipe_body<R, Q>(t, A, lda, m, row0, npairs, zbuf, tw_cols, bits1, blockIdx.x, blockIdx.y, gridDim.y, nullptr);
}

template <typename R>
__device__ __forceinline__ void sketch_pass2_body(const SketchTables &t, int64_t m, int64_t row0, int64_t npairs,
                                                  const cpx<R> *zbuf, double *S, int64_t lds, int cp, int bits2,
                                                  int w, int64_t by)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    typedef cpx<R> cplx;
    cplx *smem = reinterpret_cast<cplx *>(smem_raw);
    const int n1 = (int)t.n1, n2 = (int)t.n2;
    cplx *tw = smem;               // n2/2
    const int ld2 = n2 + 1;        // padded column stride
    cplx *buf = smem + (n2 >> 1);  // cp x 2 x ld2
    // w: k1-pair index, ka = w, kb = (n1 - w) % n1
    const int ka = w, kb = (n1 - w) % n1;
    const int ncol = (ka == kb) ? 1 : 2;
    const int64_t p0 = by * cp;
    if (w > n1 / 2 || p0 >= npairs) return;  // whole block (grouped launches)
    const int pc = (int)min<int64_t>(cp, npairs - p0);
    int *s_tinv = reinterpret_cast<int *>(buf + (int64_t)cp * 2 * ld2);
    const cplx *tw2 = reinterpret_cast<const cplx *>(sizeof(R) == 8 ? (const void *)t.tw2 : (const void *)t.tw2f);
    for (int e = threadIdx.x; e < (n2 >> 1); e += blockDim.x) tw[e] = tw2[e];
    for (int e = threadIdx.x; e < n2; e += blockDim.x) s_tinv[e] = t.tau_inv[e];
    __syncthreads();
    const int total = pc * ncol * n2;
    for (int base = threadIdx.x; base < total; base += SK_U * blockDim.x) {
        cplx v[SK_U];
        int dst[SK_U];
#pragma unroll
        for (int q = 0; q < SK_U; ++q) {
            const int e = base + q * blockDim.x;
            dst[q] = -1;
            v[q] = cplx{0, 0};
            if (e < total) {
                const int c = e / n2, u = e - c * n2;
                const int p = c / ncol, col = c - p * ncol;
                const int k1 = col == 0 ? ka : kb;
                dst[q] = (p * 2 + col) * ld2 + (int)bitrev((unsigned)s_tinv[u], bits2);
                v[q] = zbuf[(p0 + p) * t.np + (int64_t)k1 * n2 + u];
            }
        }
#pragma unroll
        for (int q = 0; q < SK_U; ++q)
            if (dst[q] >= 0) buf[dst[q]] = v[q];
    }
    __syncthreads();
    // FFT every loaded column; columns are laid out p*2 + col, so transform
    // 2*pc columns (an unused second column is harmless zero work when ncol = 1).
    lds_fft_cols<R, Pass2Stages<R>::value>(buf, n2, ld2, pc * 2, tw);
    const int beg = t.sel_off[w], cnt = t.sel_off[w + 1] - beg;
    const double sc1 = 1.0 / __builtin_sqrt((double)t.l);
    const double sc2 = __builtin_sqrt(2.0) * sc1;
    const int64_t half = t.np >> 1;
    for (int e = threadIdx.x; e < cnt * pc; e += blockDim.x) {
        const int p = e / cnt, s = e - p * cnt;
        const int32_t *ent = t.sel + 3 * (beg + s);
        const int64_t k = ent[0];
        const int part = ent[1], q = ent[2];
        const int k1 = (int)(k % n1), k2 = (int)(k / n1);
        const int64_t kp = (t.np - k) % t.np;
        const int kp1 = (int)(kp % n1), kp2 = (int)(kp / n1);
        const cplx y = buf[(int64_t)(p * 2 + (k1 == ka ? 0 : 1)) * ld2 + k2];
        const cplx yp = buf[(int64_t)(p * 2 + (kp1 == ka ? 0 : 1)) * ld2 + kp2];
        // spectra of the two real rows: Ya = (Y_k + conj Y_{np-k})/2,
        // Yb = (Y_k - conj Y_{np-k})/(2i)
        const double ar = 0.5 * ((double)y.re + (double)yp.re), ai = 0.5 * ((double)y.im - (double)yp.im);
        const double br = 0.5 * ((double)y.im + (double)yp.im), bi = -0.5 * ((double)y.re - (double)yp.re);
        const double sc = (k == 0 || k == half) ? sc1 : sc2;
        const int64_t r0 = row0 + 2 * (p0 + p);
        S[r0 * lds + q] = sc * (part ? ai : ar);
        if (r0 + 1 < m) S[(r0 + 1) * lds + q] = sc * (part ? bi : br);
    }
}

template <typename R>
__global__ __launch_bounds__(256) void sketch_pass2(SketchTables t, int64_t m, int64_t row0, int64_t npairs,
                                                    const cpx<R> *zbuf, double *S, int64_t lds, int cp, int bits2)
{
    sketch_pass2_body<R>(t, m, row0, npairs, zbuf, S, lds, cp, bits2, blockIdx.x, blockIdx.y);
}

// Pass 2, software-pipelined like pass 1: the tasks (k1 pair w, group of cp
// row pairs), numbered w fastest, are dealt round-robin to nb blocks (block
// b0 takes tasks b0, b0 + nb, ...), and a
// block gathers its next task's columns while the current one is
// transformed and written out.  Q = 2 cp n2 / 256 elements per thread, all
// loaded unconditionally: a single-column pair (w = 0 or n1/2) loads its
// column twice and a short last group repeats its last row pair; neither
// copy is written out.  Same per-column arithmetic as sketch_pass2.
template <typename R, int Q>
__device__ __forceinline__ void pass2_pipe_body(const SketchTables &t, int64_t m, int64_t row0, int64_t npairs,
                                                const cpx<R> *zbuf, double *S, int64_t lds, int cp, int bits2,
                                                int64_t b0, int64_t nb)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    typedef cpx<R> cplx;
    cplx *smem = reinterpret_cast<cplx *>(smem_raw);
    const int n1 = (int)t.n1, n2 = (int)t.n2;
    cplx *tw = smem;
    const int ld2 = n2 + 1;
    cplx *buf = smem + (n2 >> 1);
    int *s_tinv = reinterpret_cast<int *>(buf + (int64_t)cp * 2 * ld2);
    const int gx = n1 / 2 + 1;
    const int64_t ngroups = (npairs + cp - 1) / cp, ntasks = ngroups * gx;
    if (b0 >= ntasks) return;
    const cplx *tw2 = reinterpret_cast<const cplx *>(sizeof(R) == 8 ? (const void *)t.tw2 : (const void *)t.tw2f);
    for (int e = threadIdx.x; e < (n2 >> 1); e += blockDim.x) tw[e] = tw2[e];
    for (int e = threadIdx.x; e < n2; e += blockDim.x) s_tinv[e] = t.tau_inv[e];
    __syncthreads();
    cplx v[Q];
    // (32-bit byte offsets from the group's base: the host takes this path
    // only when cp row pairs of the intermediate span less than 4 GiB)
    auto gather = [&](int64_t task) {
        const int w = (int)(task % gx);
        const int64_t p0 = task / gx * cp;
        const int ka = w, kb = (n1 - w) % n1;
        const int plast = (int)min<int64_t>(cp, npairs - p0) - 1;
        const char *zb = reinterpret_cast<const char *>(zbuf + p0 * t.np);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = threadIdx.x + 256 * q;
            const int c = e >> bits2, u = e & (n2 - 1);
            const int p = min(c >> 1, plast);
            const unsigned k1 = (unsigned)((c & 1) ? kb : ka);
            const unsigned off = ((unsigned)p * (unsigned)t.np + k1 * (unsigned)n2 + (unsigned)u) * (unsigned)sizeof(cplx);
            v[q] = *reinterpret_cast<const cplx *>(zb + off);
        }
    };
    const double sc1 = 1.0 / __builtin_sqrt((double)t.l);
    const double sc2 = __builtin_sqrt(2.0) * sc1;
    const int64_t half = t.np >> 1;
    int64_t task = b0;
    gather(task);
    for (; task < ntasks; task += nb) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = threadIdx.x + 256 * q;
            const int c = e >> bits2, u = e & (n2 - 1);
            buf[c * ld2 + (int)bitrev((unsigned)s_tinv[u], bits2)] = v[q];
        }
        __syncthreads();
        const int64_t nx = task + nb;
        gather(nx < ntasks ? nx : task);
        lds_fft_cols<R, Pass2Stages<R>::value>(buf, n2, ld2, cp * 2, tw);
        const int w = (int)(task % gx), ka = w;
        const int64_t p0 = task / gx * cp;
        const int pc = (int)min<int64_t>(cp, npairs - p0);
        const int beg = t.sel_off[w], cnt = t.sel_off[w + 1] - beg;
        for (int e = threadIdx.x; e < cnt * pc; e += blockDim.x) {
            const int p = e / cnt, s = e - p * cnt;
            const int32_t *ent = t.sel + 3 * (beg + s);
            const int64_t k = ent[0];
            const int part = ent[1], q = ent[2];
            const int k1 = (int)(k % n1), k2 = (int)(k / n1);
            const int64_t kp = (t.np - k) % t.np;
            const int kp1 = (int)(kp % n1), kp2 = (int)(kp / n1);
            const cplx y = buf[(int64_t)(p * 2 + (k1 == ka ? 0 : 1)) * ld2 + k2];
            const cplx yp = buf[(int64_t)(p * 2 + (kp1 == ka ? 0 : 1)) * ld2 + kp2];
            const double ar = 0.5 * ((double)y.re + (double)yp.re), ai = 0.5 * ((double)y.im - (double)yp.im);
            const double br = 0.5 * ((double)y.im + (double)yp.im), bi = -0.5 * ((double)y.re - (double)yp.re);
            const double sc = (k == 0 || k == half) ? sc1 : sc2;
            const int64_t r0 = row0 + 2 * (p0 + p);
            S[r0 * lds + q] = sc * (part ? ai : ar);
            if (r0 + 1 < m) S[(r0 + 1) * lds + q] = sc * (part ? bi : br);
        }
        __syncthreads();
    }
}

template <typename R, int Q>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void sketch_pass2_pipe(
    SketchTables t, int64_t m, int64_t row0, int64_t npairs, const cpx<R> *zbuf, double *S, int64_t lds, int cp,
    int bits2)
{
    pass2_pipe_body<R, Q>(t, m, row0, npairs, zbuf, S, lds, cp, bits2, blockIdx.x, gridDim.x);
}

// Grouped pipelined passes (members of one Fourier length, so one geometry):
// member blockIdx.z, chunk c of its rows; pass 1 walks the member's pairs in
// steps of gridDim.y, pass 2 its tasks in steps of gridDim.x.
template <typename R, int Q>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void sketch_pass1_pipe_grouped(
    const SketchGroupArgs *gs, int chunk, int tw_cols, int bits1)
{
    const SketchGroupArgs &g = gs[blockIdx.z];
    const int64_t row0 = (int64_t)chunk * g.rows_chunk;
    if (row0 >= g.m) return;
    const int64_t npairs = (min(g.rows_chunk, g.m - row0) + 1) / 2;
    pass1_pipe_body<R, Q>(g.t, g.A, g.lda, g.m, row0, npairs, reinterpret_cast<cpx<R> *>(g.zbuf), tw_cols, bits1,
                          blockIdx.x, blockIdx.y, gridDim.y, g.cs);
}

template <typename R, int Q>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void sketch_pass2_pipe_grouped(
    const SketchGroupArgs *gs, int chunk, int cp, int bits2)
{
    const SketchGroupArgs &g = gs[blockIdx.z];
    const int64_t row0 = (int64_t)chunk * g.rows_chunk;
    if (row0 >= g.m) return;
    const int64_t npairs = (min(g.rows_chunk, g.m - row0) + 1) / 2;
    pass2_pipe_body<R, Q>(g.t, g.m, row0, npairs, reinterpret_cast<const cpx<R> *>(g.zbuf), g.S, g.lds, cp, bits2,
                          blockIdx.x, gridDim.x);
}

// Grouped passes: member blockIdx.z; chunk c covers rows [c*rows_chunk, ...).
template <typename R>
__global__ __launch_bounds__(256) void sketch_pass1_grouped(const SketchGroupArgs *gs, int chunk)
{
    const SketchGroupArgs g = gs[blockIdx.z];
    const int64_t row0 = (int64_t)chunk * g.rows_chunk;
    if (row0 >= g.m) return;
    const int64_t rows = min(g.rows_chunk, g.m - row0);
    if ((int64_t)blockIdx.y >= (rows + 1) / 2) return;  // pairs of this member's chunk only
    const SketchGeom geo = sketch_geom<R>(g.t);
    sketch_pass1_body<R>(g.t, g.A, g.lda, g.m, row0, reinterpret_cast<cpx<R> *>(g.zbuf), geo.tw_cols, geo.bits1,
                         blockIdx.x, blockIdx.y, g.cs);
}

template <typename R>
__global__ __launch_bounds__(256) void sketch_pass2_grouped(const SketchGroupArgs *gs, int chunk)
{
    const SketchGroupArgs g = gs[blockIdx.z];
    const int64_t row0 = (int64_t)chunk * g.rows_chunk;
    if (row0 >= g.m) return;
    const int64_t rows = min(g.rows_chunk, g.m - row0);
    const SketchGeom geo = sketch_geom<R>(g.t);
    sketch_pass2_body<R>(g.t, g.m, row0, (rows + 1) / 2, reinterpret_cast<const cpx<R> *>(g.zbuf), g.S, g.lds, geo.cp,
                         geo.bits2, blockIdx.x, blockIdx.y);
}

// Blocks of kernel kf (256 threads, smem bytes of LDS) resident on the
// whole device at once.
hipError_t resident_blocks(const void *kf, size_t smem, int64_t *out)
{
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kf, 256, smem);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    *out = (int64_t)std::max(1, per_cu) * std::max(1, cus);
    return e;
}

// The pipelined kernels by elements per thread, 16 or 32 (32 in binary32
// only, where QB = 32), for launches through hipLaunchKernel.  Shorter rows
// (4 or 8 elements per thread, as in batches of short members) measured no
// gain over the plain passes and take those.
template <typename R, int QB>
const void *pass1_pipe_kernel(int q, bool grouped)
{
    if (q == 16) return grouped ? (const void *)sketch_pass1_pipe_grouped<R, 16> : (const void *)sketch_pass1_pipe<R, 16>;
    return grouped ? (const void *)sketch_pass1_pipe_grouped<R, QB> : (const void *)sketch_pass1_pipe<R, QB>;
}
template <typename R, int QB>
const void *pass2_pipe_kernel(int q, bool grouped)
{
    if (q == 16) return grouped ? (const void *)sketch_pass2_pipe_grouped<R, 16> : (const void *)sketch_pass2_pipe<R, 16>;
    return grouped ? (const void *)sketch_pass2_pipe_grouped<R, QB> : (const void *)sketch_pass2_pipe<R, QB>;
}
inline bool pipe_q(int q, int qb) { return q == 16 || q == qb; }

template <typename R>
hipError_t sketch_run(const SketchTables &t, const double *A, int64_t lda, int64_t m, double *S, int64_t lds,
                      void *zbuf, int64_t rows_chunk, hipStream_t stream)
{
    typedef cpx<R> cplx;
    const int n1 = (int)t.n1, n2 = (int)t.n2;
    const SketchGeom geo = sketch_geom<R>(t);
    const int bits1 = geo.bits1, bits2 = geo.bits2, tw_cols = geo.tw_cols, cp = geo.cp;
    const int64_t csz = sizeof(cplx);
    (void)csz;
    const size_t sm1 = pass1_smem<R>(n1, n2, tw_cols);
    const size_t sm2 = pass2_smem<R>(n2, cp);
    cplx *z = reinterpret_cast<cplx *>(zbuf);
    hipError_t ea = hipFuncSetAttribute((const void *)sketch_pass1<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm1);
    if (ea != hipSuccess) return ea;
    ea = hipFuncSetAttribute((const void *)sketch_pass2<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm2);
    if (ea != hipSuccess) return ea;
    // the pipelined pass 1 when each thread holds 16 or 32 elements of the
    // n1 x tw_cols column group, with as many blocks per pair range as fill
    // the device once (each then walks its share of the pairs)
    // (32 elements per thread occur in binary32 only: binary64 halves
    // tw_cols and cp for the same LDS, so its forms are not instantiated)
    constexpr int QB = sizeof(R) == 4 ? 32 : 16;
    const int q1 = (int)((int64_t)n1 * tw_cols / 256);
    const bool pipe = pipe_q(q1, QB) && (int64_t)q1 * 256 == (int64_t)n1 * tw_cols && t.np * 8 < (int64_t(1) << 32);
    const void *kp1 = pipe ? pass1_pipe_kernel<R, QB>(q1, false) : nullptr;
    int resident = 0;
    if (pipe) {
        const void *kf = kp1;
        if ((ea = hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm1)) != hipSuccess) return ea;
        int per_cu = 0, dev = 0, cus = 0;
        if ((ea = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kf, 256, sm1)) != hipSuccess) return ea;
        if ((ea = hipGetDevice(&dev)) != hipSuccess) return ea;
        if ((ea = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return ea;
        resident = std::max(1, per_cu) * std::max(1, cus);
    }
    // the pipelined pass 2 in binary32 when each thread holds 16 or 32
    // elements of the 2 cp columns, as many blocks as are resident at once
    // (in binary64 it measured slower than the plain pass 2: 6.5, or 6.4 with
    // three stages per register pass, against 5.7 ms for both passes at
    // 2048 x 262144)
    const int q2 = (int)((int64_t)2 * cp * n2 / 256);
    const bool pipe2 = sizeof(R) == 4 && pipe_q(q2, QB) && (int64_t)q2 * 256 == (int64_t)2 * cp * n2 &&
                       (int64_t)cp * t.np * csz < (int64_t(1) << 32);
    const void *kp2 = pipe2 ? pass2_pipe_kernel<R, QB>(q2, false) : nullptr;
    int64_t resident2 = 0;
    if (pipe2) {
        const void *kf = kp2;
        if ((ea = hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm2)) != hipSuccess) return ea;
        int per_cu = 0, dev = 0, cus = 0;
        if ((ea = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kf, 256, sm2)) != hipSuccess) return ea;
        if ((ea = hipGetDevice(&dev)) != hipSuccess) return ea;
        if ((ea = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return ea;
        resident2 = (int64_t)std::max(1, per_cu) * std::max(1, cus);
    }
    for (int64_t row0 = 0; row0 < m; row0 += rows_chunk) {
        const int64_t rows = std::min<int64_t>(rows_chunk, m - row0);
        const int64_t npairs = (rows + 1) / 2;
        if (pipe) {
            const int gx = n2 / tw_cols;
            const int64_t gy = std::min<int64_t>(npairs, std::max(1, resident / gx));
            SketchTables ta = t;
            const double *aa = A;
            int64_t la = lda, ma = m, ra = row0, pa = npairs;
            cplx *za = z;
            int twa = tw_cols, ba = bits1;
            void *args[] = {&ta, &aa, &la, &ma, &ra, &pa, &za, &twa, &ba};
            if ((ea = hipLaunchKernel(kp1, dim3(gx, (unsigned)gy), dim3(256), args, sm1, stream)) != hipSuccess) return ea;
        } else {
            hipLaunchKernelGGL(sketch_pass1<R>, dim3(n2 / tw_cols, (unsigned)npairs), dim3(256), sm1, stream, t, A, lda,
                               m, row0, z, tw_cols, bits1);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (pipe2) {
            const int64_t ntasks = (npairs + cp - 1) / cp * (n1 / 2 + 1);
            const unsigned gb = (unsigned)std::min<int64_t>(ntasks, resident2);
            SketchTables ta = t;
            int64_t ma = m, ra = row0, pa = npairs, la = lds;
            const cplx *za = z;
            double *sa = S;
            int cpa = cp, ba = bits2;
            void *args[] = {&ta, &ma, &ra, &pa, &za, &sa, &la, &cpa, &ba};
            if ((ea = hipLaunchKernel(kp2, dim3(gb), dim3(256), args, sm2, stream)) != hipSuccess) return ea;
        } else {
            hipLaunchKernelGGL(sketch_pass2<R>, dim3(n1 / 2 + 1, (unsigned)((npairs + cp - 1) / cp)), dim3(256), sm2,
                               stream, t, m, row0, npairs, (const cplx *)z, S, lds, cp, bits2);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename R>
hipError_t sketch_grouped_run(const SketchGroupArgs *d, int count, const SketchGroupShape &sh, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    typedef cpx<R> cplx;
    const int64_t csz = sizeof(cplx);
    // launch geometry covering every member: the largest n1, n2 and pairs
    SketchTables tmax{};
    tmax.n1 = sh.max_n1; tmax.n2 = sh.max_n2;
    size_t sm1 = 0, sm2 = 0;
    int gx1 = 0, gx2 = 0;
    for (int64_t n1 = 1; n1 <= sh.max_n1; n1 <<= 1)
        for (int64_t n2 = 1; n2 <= sh.max_n2; n2 <<= 1) {
            SketchTables tt{};
            tt.n1 = n1; tt.n2 = n2;
            const SketchGeom g = sketch_geom<R>(tt);
            sm1 = std::max(sm1, pass1_smem<R>(n1, n2, g.tw_cols));
            sm2 = std::max(sm2, pass2_smem<R>(n2, g.cp));
            gx1 = std::max(gx1, (int)(n2 / g.tw_cols));
            gx2 = std::max(gx2, (int)(n1 / 2 + 1));
        }
    hipError_t e = hipFuncSetAttribute((const void *)sketch_pass1_grouped<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)sm1);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)sketch_pass2_grouped<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm2);
    if (e != hipSuccess) return e;
    const int64_t max_pairs = (sh.max_rows_chunk + 1) / 2;
    // pipelined passes when every member has one geometry that qualifies (as
    // for a single plan), with the resident blocks shared among the members
    constexpr int QB = sizeof(R) == 4 ? 32 : 16;
    const SketchGeom geo = sketch_geom<R>(tmax);
    const int64_t n1 = sh.max_n1, n2 = sh.max_n2, np = n1 * n2;
    const int q1 = (int)(n1 * geo.tw_cols / 256), q2 = (int)(2 * geo.cp * n2 / 256);
    const bool pipe1 = sh.one_length && pipe_q(q1, QB) && (int64_t)q1 * 256 == n1 * geo.tw_cols &&
                       np * 8 < (int64_t(1) << 32);
    const bool pipe2 = sh.one_length && sizeof(R) == 4 && pipe_q(q2, QB) &&
                       (int64_t)q2 * 256 == 2 * geo.cp * n2 && geo.cp * np * csz < (int64_t(1) << 32);
    const size_t psm1 = pass1_smem<R>(n1, n2, geo.tw_cols), psm2 = pass2_smem<R>(n2, geo.cp);
    const void *k1 = pipe1 ? pass1_pipe_kernel<R, QB>(q1, true) : nullptr;
    const void *k2 = pipe2 ? pass2_pipe_kernel<R, QB>(q2, true) : nullptr;
    int64_t res1 = 0, res2 = 0;
    if (pipe1) {
        if ((e = hipFuncSetAttribute(k1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)psm1)) != hipSuccess) return e;
        if ((e = resident_blocks(k1, psm1, &res1)) != hipSuccess) return e;
    }
    if (pipe2) {
        if ((e = hipFuncSetAttribute(k2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)psm2)) != hipSuccess) return e;
        if ((e = resident_blocks(k2, psm2, &res2)) != hipSuccess) return e;
    }
    const int pgx = (int)(n2 / geo.tw_cols);
    const int64_t pgy = std::min<int64_t>(max_pairs, std::max<int64_t>(1, res1 / ((int64_t)pgx * count)));
    const int64_t ntasks = (max_pairs + geo.cp - 1) / geo.cp * (n1 / 2 + 1);
    const int64_t pnb = std::min<int64_t>(ntasks, std::max<int64_t>(1, res2 / count));
    for (int c = 0; c < sh.chunks; ++c) {
        if (pipe1) {
            const SketchGroupArgs *da = d;
            int ca = c, twa = geo.tw_cols, ba = geo.bits1;
            void *args[] = {&da, &ca, &twa, &ba};
            if ((e = hipLaunchKernel(k1, dim3(pgx, (unsigned)pgy, count), dim3(256), args, psm1, stream)) != hipSuccess)
                return e;
        } else {
            hipLaunchKernelGGL(sketch_pass1_grouped<R>, dim3(gx1, (unsigned)max_pairs, count), dim3(256), sm1, stream, d, c);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (pipe2) {
            const SketchGroupArgs *da = d;
            int ca = c, cpa = geo.cp, ba = geo.bits2;
            void *args[] = {&da, &ca, &cpa, &ba};
            if ((e = hipLaunchKernel(k2, dim3((unsigned)pnb, 1, count), dim3(256), args, psm2, stream)) != hipSuccess)
                return e;
        } else {
            hipLaunchKernelGGL(sketch_pass2_grouped<R>, dim3(gx2, (unsigned)max_pairs, count), dim3(256), sm2, stream, d, c);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t sketch_grouped_f64(const SketchGroupArgs *d, int count, const SketchGroupShape &sh, hipStream_t stream)
{
    return sketch_grouped_run<double>(d, count, sh, stream);
}

hipError_t sketch_grouped_f32(const SketchGroupArgs *d, int count, const SketchGroupShape &sh, hipStream_t stream)
{
    return sketch_grouped_run<float>(d, count, sh, stream);
}

hipError_t sketch_f64(const SketchTables &t, const double *A, int64_t lda, int64_t m, double *S, int64_t lds,
                      double *zbuf, int64_t rows_chunk, hipStream_t stream)
{
    return sketch_run<double>(t, A, lda, m, S, lds, zbuf, rows_chunk, stream);
}

hipError_t sketch_f32(const SketchTables &t, const double *A, int64_t lda, int64_t m, double *S, int64_t lds,
                      double *zbuf, int64_t rows_chunk, hipStream_t stream)
{
    return sketch_run<float>(t, A, lda, m, S, lds, zbuf, rows_chunk, stream);
}

}  // namespace rt
