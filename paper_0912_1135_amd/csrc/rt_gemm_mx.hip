// Reduced-precision GEMMs of the preconditioner on the gfx950 matrix cores,
// binary32 accumulation:
//   * MX_F32:  v_mfma_f32_16x16x4_f32   (binary32 operands)
//   * MX_BF16: v_mfma_f32_16x16x32_bf16 (bfloat16 operands)
//   * MX_BF16X3: three v_mfma_f32_16x16x32_bf16 per product, on binary32
//     operands split into bfloat16 halves (hi + lo)
// Operands are read from binary64 or binary32 storage and rounded on the way
// into LDS; an optional per-row (A) / per-column (B) power-of-two scale is
// applied before the rounding (exact).  Used for P^{-1}A in binary32 and for
// the Gram (P^{-1}A)(P^{-1}A)^T in binary32 or bfloat16.
#include "rt_common.h"

namespace rt {

namespace {

__device__ __forceinline__ double ld_any(const void *p, int is_dbl, int64_t idx)
{
    return is_dbl ? static_cast<const double *>(p)[idx] : (double)static_cast<const float *>(p)[idx];
}

// ---------------------------------------------------------------- binary32
constexpr int KC32 = 16;

template <int T, bool KCONTIG>
struct Lay32 {
    static constexpr int size = KCONTIG ? T * (KC32 + 1) : KC32 * (T + 32);
    __device__ static int at(int mn, int k) { return KCONTIG ? mn * (KC32 + 1) + k : k * (T + 32) + mn; }
};

// Element of binary64 (DBL) or binary32 storage, widened to binary64.
template <bool DBL>
__device__ __forceinline__ double ld_st(const void *p, int64_t idx)
{
    if constexpr (DBL) return static_cast<const double *>(p)[idx];
    else return (double)static_cast<const float *>(p)[idx];
}

// As the binary64 GEMM: every load is issued from a clamped address and
// zeroed by a select (straight-line loads, one chunk in flight behind the
// MFMAs), the loop-invariant address parts and scales are hoisted, and a
// gather of B's rows reads its indices one chunk ahead.  DBL: binary64
// storage of both operands (else binary32).
template <int BM, int BN, bool A_KC, bool B_KC, bool DBL, bool GB>
__device__ __forceinline__ void gemm_f32_tile(const GemmMxArgs &g, int bx, int by, int bz)
{
    using LA = Lay32<BM, A_KC>;
    using LB = Lay32<BN, B_KC>;
    __shared__ float As[2][LA::size];
    __shared__ float Bs[2][LB::size];
    constexpr int TM = BM / 32, TN = BN / 32;
    constexpr int NA = BM * KC32 / 256, NB = BN * KC32 / 256;
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    int ti, tj;
    if (g.c_lower) {
        const int t = bx;
        ti = (int)((__builtin_sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        while (ti * (ti + 1) / 2 > t) --ti;
        tj = t - ti * (ti + 1) / 2;
    } else {
        ti = by;
        tj = bx;
    }
    const int i0 = ti * BM, j0 = tj * BN;
    // tiles outside the problem (grouped launches cover the largest member)
    if (i0 >= g.M || j0 >= g.N || bz >= (g.ksplit > 1 ? g.ksplit : 1)) return;
    int kbeg = 0, kend = g.K;
    if (g.ksplit > 1) {
        int ks = (g.K + g.ksplit - 1) / g.ksplit;
        ks = (ks + KC32 - 1) / KC32 * KC32;
        kbeg = bz * ks;
        kend = min(g.K, kbeg + ks);
    }
    if (g.a_lower) kend = min(kend, i0 + BM);
    const int nch = kend > kbeg ? (kend - kbeg + KC32 - 1) / KC32 : 0;

    int a_ii[NA], a_kk[NA], b_jj[NB], b_kk[NB];
    int64_t a_row[NA], b_col[NB];
    bool a_in[NA], b_in[NB];
    double a_sc[NA], b_sc[NB];
#pragma unroll
    for (int e = 0; e < NA; ++e) {
        const int x = tid + 256 * e;
        a_ii[e] = A_KC ? x / KC32 : x % BM;
        a_kk[e] = A_KC ? x % KC32 : x / BM;
        const int i = i0 + a_ii[e];
        a_in[e] = i < g.M;
        const int ic = a_in[e] ? i : g.M - 1;
        a_row[e] = (g.a_gather ? (int64_t)g.a_gather[ic] : (int64_t)ic) * g.a_i;
        a_sc[e] = g.a_scale ? (double)g.a_scale[ic] : 1.0;
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
        const int x = tid + 256 * e;
        b_jj[e] = B_KC ? x / KC32 : x % BN;
        b_kk[e] = B_KC ? x % KC32 : x / BN;
        const int j = j0 + b_jj[e];
        b_in[e] = j < g.N;
        const int jc = b_in[e] ? j : g.N - 1;
        b_col[e] = (int64_t)jc * g.b_j;
        b_sc[e] = g.b_scale ? (double)g.b_scale[jc] : 1.0;
    }
    float ra[NA], rb[NB];
    int gi[NB];
    (void)gi;
    auto load_idx = [&](int c) {
        if constexpr (GB) {
#pragma unroll
            for (int e = 0; e < NB; ++e) {
                const int k = kbeg + c * KC32 + b_kk[e];
                gi[e] = g.b_gather[k < kend ? k : kend - 1];
            }
        }
    };
    auto load = [&](int c) {
        const int k0 = kbeg + c * KC32;
#pragma unroll
        for (int e = 0; e < NA; ++e) {
            const int k = k0 + a_kk[e];
            const bool ok = a_in[e] && k < kend && !(g.a_lower && k > i0 + a_ii[e]);
            const double v = ld_st<DBL>(g.A, a_row[e] + (int64_t)(k < kend ? k : kend - 1) * g.a_k) * a_sc[e];
            ra[e] = ok ? (float)v : 0.f;
        }
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            const int k = k0 + b_kk[e];
            const bool ok = b_in[e] && k < kend;
            int64_t kr;
            if constexpr (GB) kr = gi[e];
            else kr = k < kend ? k : kend - 1;
            const double v = ld_st<DBL>(g.B, kr * g.b_k + b_col[e]) * b_sc[e];
            rb[e] = ok ? (float)v : 0.f;
        }
    };
    f4 acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    if (nch > 0) {
        load_idx(0);
        load(0);
        load_idx(1);
    }
    for (int t = 0; t < nch; ++t) {
        const int buf = t & 1;
#pragma unroll
        for (int e = 0; e < NA; ++e) As[buf][LA::at(a_ii[e], a_kk[e])] = ra[e];
#pragma unroll
        for (int e = 0; e < NB; ++e) Bs[buf][LB::at(b_jj[e], b_kk[e])] = rb[e];
        __syncthreads();
        // next chunk's data (its indices were read a chunk ago), then the
        // indices of the chunk after it
        load(t + 1);
        load_idx(t + 2);
#pragma unroll
        for (int kk = 0; kk < KC32; kk += 4) {
            float av[TM], bv[TN];
#pragma unroll
            for (int a = 0; a < TM; ++a) av[a] = As[buf][LA::at(wm * (BM / 2) + a * 16 + (lane & 15), kk + (lane >> 4))];
#pragma unroll
            for (int b = 0; b < TN; ++b) bv[b] = Bs[buf][LB::at(wn * (BN / 2) + b * 16 + (lane & 15), kk + (lane >> 4))];
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
    }
    const int64_t coff = g.ksplit > 1 ? (int64_t)bz * g.c_split : 0;
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // binary32 MFMA tile: row = 4 * (lane / 16) + r, col = lane % 16
                const int i = i0 + wm * (BM / 2) + a * 16 + 4 * (lane >> 4) + r;
                const int j = j0 + wn * (BN / 2) + b * 16 + (lane & 15);
                if (i < g.M && j < g.N) {
                    const int64_t idx = coff + (int64_t)i * g.c_i + (int64_t)j * g.c_j;
                    const float v = g.alpha * acc[a][b][r];
                    if (g.c_dbl) static_cast<double *>(g.C)[idx] = (double)v;
                    else static_cast<float *>(g.C)[idx] = v;
                }
            }
}

template <int BM, int BN, bool A_KC, bool B_KC, bool DBL, bool GB>
__global__ __launch_bounds__(256) void gemm_f32_kernel(GemmMxArgs g)
{
    gemm_f32_tile<BM, BN, A_KC, B_KC, DBL, GB>(g, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Both operands K-contiguous binary32 (the Gram of a row-major matrix), no
// scales, no gather, K, the row strides and the base addresses multiples of
// 4 floats.  Each thread moves 16-byte pieces along k into LDS rows of KV + 4
// floats.  Inside every group of 16 k the contraction order is permuted the
// same way for both operands (lane group q takes k = 4 q + s at MFMA step s),
// so one 16-byte LDS read gives a lane its operands for four steps.  On a
// lower-triangle grid whose block count is a multiple of 8 the blocks are
// renumbered so that each XCD (blocks are dealt to the 8 XCDs in turn) runs a
// contiguous range of K splits: its L2 then serves every tile of a split from
// one read of the split's rows.
constexpr int KV = 32;

template <int BM, int BN>
__global__ __launch_bounds__(256) void gemm_f32_kc_kernel(GemmMxArgs g)
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    constexpr int LDK = KV + 4;
    __shared__ __attribute__((aligned(16))) float As[2][BM * LDK];
    __shared__ __attribute__((aligned(16))) float Bs[2][BN * LDK];
    constexpr int TM = BM / 32, TN = BN / 32;
    constexpr int Q = KV / 4;  // 16-byte pieces per row and chunk
    constexpr int NA = BM * Q / 256, NB = BN * Q / 256;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    int bx = blockIdx.x, bz = blockIdx.z;
    int ti, tj;
    if (g.c_lower) {
        const int64_t total = (int64_t)gridDim.x * gridDim.z;
        if ((total & 7) == 0) {
            const int64_t L = bx + (int64_t)gridDim.x * bz;
            const int64_t N = (L & 7) * (total >> 3) + (L >> 3);
            bx = (int)(N % gridDim.x);
            bz = (int)(N / gridDim.x);
        }
        const int t = bx;
        ti = (int)((__builtin_sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        while (ti * (ti + 1) / 2 > t) --ti;
        tj = t - ti * (ti + 1) / 2;
    } else {
        ti = blockIdx.y;
        tj = bx;
    }
    const int i0 = ti * BM, j0 = tj * BN;
    int kbeg = 0, kend = g.K;
    if (g.ksplit > 1) {
        int ks = (g.K + g.ksplit - 1) / g.ksplit;
        ks = (ks + KV - 1) / KV * KV;
        kbeg = bz * ks;
        kend = min(g.K, kbeg + ks);
    }
    const int nch = kend > kbeg ? (kend - kbeg + KV - 1) / KV : 0;
    const float *Ap = static_cast<const float *>(g.A);
    const float *Bp = static_cast<const float *>(g.B);
    // piece e of this thread: row x / Q, k offset 4 (x % Q), x = tid + 256 e
    int64_t a_off[NA], b_off[NB];
    bool a_in[NA], b_in[NB];
    const int kq = 4 * (tid % Q);
#pragma unroll
    for (int e = 0; e < NA; ++e) {
        const int i = i0 + (tid + 256 * e) / Q;
        a_in[e] = i < g.M;
        a_off[e] = (int64_t)(a_in[e] ? i : g.M - 1) * g.a_i;
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
        const int j = j0 + (tid + 256 * e) / Q;
        b_in[e] = j < g.N;
        b_off[e] = (int64_t)(b_in[e] ? j : g.N - 1) * g.b_j;
    }
    f4 ra[NA], rb[NB];
    // kend and every k below are multiples of 4: a piece is wholly in or out;
    // out-of-range pieces load from a clamped address and are zeroed
    auto load = [&](int c) {
        const int k = kbeg + c * KV + kq;
        const bool kin = k < kend;
        const int kc = kin ? k : kend - 4;
#pragma unroll
        for (int e = 0; e < NA; ++e) {
            const f4 v = *reinterpret_cast<const f4 *>(Ap + a_off[e] + kc);
            ra[e] = (kin && a_in[e]) ? v : f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            const f4 v = *reinterpret_cast<const f4 *>(Bp + b_off[e] + kc);
            rb[e] = (kin && b_in[e]) ? v : f4{0.f, 0.f, 0.f, 0.f};
        }
    };
    f4 acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    if (nch > 0) load(0);
    for (int t = 0; t < nch; ++t) {
        const int buf = t & 1;
#pragma unroll
        for (int e = 0; e < NA; ++e) *reinterpret_cast<f4 *>(&As[buf][((tid + 256 * e) / Q) * LDK + kq]) = ra[e];
#pragma unroll
        for (int e = 0; e < NB; ++e) *reinterpret_cast<f4 *>(&Bs[buf][((tid + 256 * e) / Q) * LDK + kq]) = rb[e];
        __syncthreads();
        if (t + 1 < nch) load(t + 1);
#pragma unroll
        for (int h = 0; h < KV / 16; ++h) {
            f4 av[TM], bv[TN];
#pragma unroll
            for (int a = 0; a < TM; ++a)
                av[a] = *reinterpret_cast<const f4 *>(
                    &As[buf][(wm * (BM / 2) + a * 16 + (lane & 15)) * LDK + 16 * h + 4 * (lane >> 4)]);
#pragma unroll
            for (int b = 0; b < TN; ++b)
                bv[b] = *reinterpret_cast<const f4 *>(
                    &Bs[buf][(wn * (BN / 2) + b * 16 + (lane & 15)) * LDK + 16 * h + 4 * (lane >> 4)]);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int a = 0; a < TM; ++a)
#pragma unroll
                    for (int b = 0; b < TN; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][s], bv[b][s], acc[a][b], 0, 0, 0);
        }
    }
    const int64_t coff = g.ksplit > 1 ? (int64_t)bz * g.c_split : 0;
    float *C = static_cast<float *>(g.C);
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wm * (BM / 2) + a * 16 + 4 * (lane >> 4) + r;
                const int j = j0 + wn * (BN / 2) + b * 16 + (lane & 15);
                if (i < g.M && j < g.N) C[coff + (int64_t)i * g.c_i + (int64_t)j * g.c_j] = g.alpha * acc[a][b][r];
            }
}

// Grouped launch (batches): member blockIdx.z / ksmax, split blockIdx.z % ksmax.
template <int BM, int BN, bool A_KC, bool B_KC, bool DBL>
__global__ __launch_bounds__(256) void gemm_f32_grouped_kernel(const GemmMxArgs *gs, int ksmax)
{
    const GemmMxArgs g = gs[blockIdx.z / ksmax];
    gemm_f32_tile<BM, BN, A_KC, B_KC, DBL, false>(g, blockIdx.x, blockIdx.y, blockIdx.z % ksmax);
}

// Split-bfloat16 product of binary32 operands (same operand conditions as
// gemm_f32_kc_kernel).  Each element w is written to LDS as two bfloat16
// halves, hi = bf16(w) and lo = bf16(w - hi) (w - hi is exact in binary32),
// and every 32 k of a 16 x 16 output tile take three bfloat16 MFMAs,
// lo hi^T + hi lo^T + hi hi^T, accumulated in binary32; the products of two
// bfloat16 values are exact in binary32, so the only error besides the
// accumulation is the dropped lo lo^T and the rounding of lo, together at
// most about 2^-16 |w| |v| per product.
//
// X3 = false is the plain bfloat16 product of the same operands, each scaled
// first by its optional power-of-two row (A) / column (B) scale: only hi,
// one MFMA per 32 k.
//
// LDS rows hold the KV = 32 bfloat16 of a row (64 bytes, no padding), their
// four 16-byte units XOR-swizzled by (row / 4) % 4: the 16 lanes of an MFMA
// operand read (16 rows, one unit) and the 32 lanes of an 8-byte store
// (4 rows, 8 slots) then hit distinct banks.  Global loads run two chunks
// ahead of the products (two register sets, the loop unrolled by two).
__device__ __forceinline__ int x3_off(int row, int unit)
{
    return row * KV + 8 * (unit ^ ((row >> 2) & 3));  // in bfloat16 elements
}

// Tiles of BM x BN with 64 x 64 per wave: 128 x 128 on four waves, or
// 256 x 128 on eight (a quarter less operand traffic per output); a lower-
// triangle grid of 256 x 128 tiles numbers tile (I, J), J <= 2I + 1, as
// I (I + 1) + J.
template <int BM, int BN, bool X3>
__device__ __forceinline__ void bf16_kc_tile(const GemmMxArgs &g, int bx, int by, int bz)
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
    typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
    constexpr int LO = X3 ? 1 : 0;  // the lo halves take no LDS in the plain form
    __shared__ __attribute__((aligned(16))) __bf16 Ah[2][BM * KV];
    __shared__ __attribute__((aligned(16))) __bf16 Al[2][LO ? BM * KV : 8];
    __shared__ __attribute__((aligned(16))) __bf16 Bh[2][BN * KV];
    __shared__ __attribute__((aligned(16))) __bf16 Bl[2][LO ? BN * KV : 8];
    static_assert(BN == 128 && (BM == 128 || BM == 256), "128 x 128 or 256 x 128 tiles");
    constexpr int NT = BM * BN / 64;  // threads: one wave per 64 x 64
    constexpr int WM = BM / 64;       // waves along M
    constexpr int TM = 4, TN = 4;
    constexpr int Q = KV / 4;
    constexpr int NA = BM * Q / NT, NB = BN * Q / NT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    int ti, tj;
    if (g.c_lower) {
        const int t = bx;
        if constexpr (BM == BN) {
            ti = (int)((__builtin_sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
            while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
            while (ti * (ti + 1) / 2 > t) --ti;
            tj = t - ti * (ti + 1) / 2;
        } else {
            ti = (int)((__builtin_sqrt(4.0 * t + 1.0) - 1.0) * 0.5);
            while ((ti + 1) * (ti + 2) <= t) ++ti;
            while (ti * (ti + 1) > t) --ti;
            tj = t - ti * (ti + 1);
        }
    } else {
        ti = by;
        tj = bx;
    }
    const int i0 = ti * BM, j0 = tj * BN;
    // (a 256 x 128 lower grid's last tiles can lie wholly right of column M,
    // and a grouped grid covers its largest member: the reduction never
    // reads such tiles)
    if (i0 >= g.M || j0 >= g.N) return;
    int kbeg = 0, kend = g.K;
    if (g.ksplit > 1) {
        int ks = (g.K + g.ksplit - 1) / g.ksplit;
        ks = (ks + KV - 1) / KV * KV;
        kbeg = bz * ks;
        kend = min(g.K, kbeg + ks);
    }
    const int nch = kend > kbeg ? (kend - kbeg + KV - 1) / KV : 0;
    const float *Ap = static_cast<const float *>(g.A);
    const float *Bp = static_cast<const float *>(g.B);
    // piece e of this thread: row (tid + NT e) / Q, 8-byte slot tid % Q
    int64_t a_off[NA], b_off[NB];
    bool a_in[NA], b_in[NB];
    float a_sc[NA], b_sc[NB];
    const int slot = tid % Q, kq = 4 * slot;
#pragma unroll
    for (int e = 0; e < NA; ++e) {
        const int i = i0 + (tid + NT * e) / Q;
        a_in[e] = i < g.M;
        const int ic = a_in[e] ? i : g.M - 1;
        a_off[e] = (int64_t)ic * g.a_i;
        a_sc[e] = (!X3 && g.a_scale) ? g.a_scale[ic] : 1.f;
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
        const int j = j0 + (tid + NT * e) / Q;
        b_in[e] = j < g.N;
        const int jc = b_in[e] ? j : g.N - 1;
        b_off[e] = (int64_t)jc * g.b_j;
        b_sc[e] = (!X3 && g.b_scale) ? g.b_scale[jc] : 1.f;
    }
    // raw loads (from clamped addresses); the range masks are applied when
    // the chunk is stored, so that no instruction waits on a load before the
    // products it runs behind
    f4 ra0[NA], rb0[NB], ra1[NA], rb1[NB];
    auto load = [&](int c, f4 (&ra)[NA], f4 (&rb)[NB]) {
        const int k = kbeg + c * KV + kq;
        const int kc = k < kend ? k : kend - 4;
#pragma unroll
        for (int e = 0; e < NA; ++e) ra[e] = *reinterpret_cast<const f4 *>(Ap + a_off[e] + kc);
#pragma unroll
        for (int e = 0; e < NB; ++e) rb[e] = *reinterpret_cast<const f4 *>(Bp + b_off[e] + kc);
    };
    auto store = [&](int buf, int c, const f4 (&ra)[NA], const f4 (&rb)[NB]) {
        const bool kin = kbeg + c * KV + kq < kend;
#pragma unroll
        for (int e = 0; e < NA + NB; ++e) {
            const bool ok = kin && (e < NA ? a_in[e] : b_in[e - NA]);
            const f4 v = ok ? (e < NA ? ra[e] : rb[e - NA]) : f4{0.f, 0.f, 0.f, 0.f};
            const float sc = X3 ? 1.f : (e < NA ? a_sc[e] : b_sc[e - NA]);
            bf4 hi, lo;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                hi[u] = (__bf16)(X3 ? v[u] : v[u] * sc);  // the scales are powers of two: exact
                if constexpr (X3) lo[u] = (__bf16)(v[u] - (float)hi[u]);
            }
            const int row = (tid + NT * (e < NA ? e : e - NA)) / Q;
            const int o = x3_off(row, slot >> 1) + 4 * (slot & 1);
            *reinterpret_cast<bf4 *>(e < NA ? &Ah[buf][o] : &Bh[buf][o]) = hi;
            if constexpr (X3) *reinterpret_cast<bf4 *>(e < NA ? &Al[buf][o] : &Bl[buf][o]) = lo;
        }
    };
    f4 acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    auto products = [&](int buf) {
        bf8 ah[TM], al[TM], bh[TN], bl[TN];
        (void)al;
        (void)bl;
#pragma unroll
        for (int a = 0; a < TM; ++a) {
            const int o = x3_off(wm * 64 + a * 16 + (lane & 15), lane >> 4);
            ah[a] = *reinterpret_cast<const bf8 *>(&Ah[buf][o]);
            if constexpr (X3) al[a] = *reinterpret_cast<const bf8 *>(&Al[buf][o]);
        }
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            const int o = x3_off(wn * 64 + b * 16 + (lane & 15), lane >> 4);
            bh[b] = *reinterpret_cast<const bf8 *>(&Bh[buf][o]);
            if constexpr (X3) bl[b] = *reinterpret_cast<const bf8 *>(&Bl[buf][o]);
        }
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
            for (int b = 0; b < TN; ++b) {
                if constexpr (X3) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
                }
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
            }
    };
    // chunk t comes from register set t % 2 and LDS buffer t % 2; the loads
    // of chunk t + 2 go into that set once it is in LDS
    if (nch > 0) {
        load(0, ra0, rb0);
        load(1, ra1, rb1);
    }
    // (loads past the last chunk read clamped, valid addresses and go
    // unused; issuing them unconditionally keeps the wait counts exact)
    int t = 0;
    for (; t + 1 < nch; t += 2) {
        store(0, t, ra0, rb0);
        __syncthreads();
        load(t + 2, ra0, rb0);
        __builtin_amdgcn_sched_barrier(0);
        products(0);
        store(1, t + 1, ra1, rb1);
        __syncthreads();
        load(t + 3, ra1, rb1);
        __builtin_amdgcn_sched_barrier(0);
        products(1);
    }
    if (t < nch) {
        store(0, t, ra0, rb0);
        __syncthreads();
        products(0);
    }
    const int64_t coff = g.ksplit > 1 ? (int64_t)bz * g.c_split : 0;
    float *C = static_cast<float *>(g.C);
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wm * 64 + a * 16 + 4 * (lane >> 4) + r;
                const int j = j0 + wn * 64 + b * 16 + (lane & 15);
                if (i < g.M && j < g.N) C[coff + (int64_t)i * g.c_i + (int64_t)j * g.c_j] = g.alpha * acc[a][b][r];
            }
}

template <int BM, int BN, bool X3>
__global__ __launch_bounds__(BM * BN / 64) __attribute__((amdgpu_waves_per_eu(2))) void gemm_bf16x3_kc_kernel(
    GemmMxArgs g)
{
    int bx = blockIdx.x, bz = blockIdx.z;
    if (g.c_lower) {
        const int64_t total = (int64_t)gridDim.x * gridDim.z;
        if ((total & 7) == 0) {
            const int64_t L = bx + (int64_t)gridDim.x * bz;
            const int64_t N = (L & 7) * (total >> 3) + (L >> 3);
            bx = (int)(N % gridDim.x);
            bz = (int)(N / gridDim.x);
        }
    }
    bf16_kc_tile<BM, BN, X3>(g, bx, blockIdx.y, bz);
}

// Grouped lower-triangle launch (batches): member blockIdx.z / ksmax, split
// blockIdx.z % ksmax; members with fewer splits or smaller m skip the rest.
template <int BM, int BN>
__global__ __launch_bounds__(BM * BN / 64) __attribute__((amdgpu_waves_per_eu(2))) void gemm_bf16x3_grouped_kernel(
    const GemmMxArgs *gs, int ksmax)
{
    const GemmMxArgs g = gs[blockIdx.z / ksmax];
    const int bz = blockIdx.z % ksmax;
    if (bz >= (g.ksplit > 1 ? g.ksplit : 1)) return;
    bf16_kc_tile<BM, BN, true>(g, blockIdx.x, 0, bz);
}

// ---------------------------------------------------------------- bfloat16
// Both operands K-contiguous (the Gram of a row-major matrix): LDS tiles are
// [mn][KB + 8] bfloat16, so each lane's 8 consecutive k are one 16-byte read
// and 16 lanes at 16 consecutive rows hit 64 distinct banks.
constexpr int KB = 32;

template <int BM, int BN, bool DBL>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmMxArgs g)
{
    typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
    typedef float f4 __attribute__((ext_vector_type(4)));
    constexpr int LDK = KB + 8;
    __shared__ __attribute__((aligned(16))) __bf16 As[2][BM * LDK];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][BN * LDK];
    constexpr int TM = BM / 32, TN = BN / 32;
    constexpr int NA = BM * KB / 8 / 256, NB = BN * KB / 8 / 256;  // 8-element groups per thread
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    int ti, tj;
    if (g.c_lower) {
        const int t = blockIdx.x;
        ti = (int)((__builtin_sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        while (ti * (ti + 1) / 2 > t) --ti;
        tj = t - ti * (ti + 1) / 2;
    } else {
        ti = blockIdx.y;
        tj = blockIdx.x;
    }
    const int i0 = ti * BM, j0 = tj * BN;
    int kbeg = 0, kend = g.K;
    if (g.ksplit > 1) {
        int ks = (g.K + g.ksplit - 1) / g.ksplit;
        ks = (ks + KB - 1) / KB * KB;
        kbeg = blockIdx.z * ks;
        kend = min(g.K, kbeg + ks);
    }
    // group e of this thread: row (x / 4), k-offset 8 * (x % 4), x = tid + 256 e;
    // row offsets and scales hoisted, loads from clamped addresses zeroed by
    // a select (straight-line, one chunk in flight)
    int64_t a_row[NA], b_row[NB];
    float a_sc[NA], b_sc[NB];
    bool a_in[NA], b_in[NB];
#pragma unroll
    for (int e = 0; e < NA; ++e) {
        const int x = tid + 256 * e, i = i0 + (x >> 2);
        a_in[e] = i < g.M;
        const int ic = a_in[e] ? i : g.M - 1;
        a_row[e] = (int64_t)ic * g.a_i;
        a_sc[e] = g.a_scale ? g.a_scale[ic] : 1.f;
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
        const int x = tid + 256 * e, j = j0 + (x >> 2);
        b_in[e] = j < g.N;
        const int jc = b_in[e] ? j : g.N - 1;
        b_row[e] = (int64_t)jc * g.b_j;
        b_sc[e] = g.b_scale ? g.b_scale[jc] : 1.f;
    }
    bf8 ra[NA], rb[NB];
    auto load = [&](int k0) {
#pragma unroll
        for (int e = 0; e < NA; ++e) {
            const int kk = 8 * ((tid + 256 * e) & 3);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = k0 + kk + u;
                const double v = ld_st<DBL>(g.A, a_row[e] + (int64_t)(k < kend ? k : kend - 1) * g.a_k) * a_sc[e];
                ra[e][u] = (a_in[e] && k < kend) ? (__bf16)(float)v : (__bf16)0.f;
            }
        }
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            const int kk = 8 * ((tid + 256 * e) & 3);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = k0 + kk + u;
                const double v = ld_st<DBL>(g.B, (int64_t)(k < kend ? k : kend - 1) * g.b_k + b_row[e]) * b_sc[e];
                rb[e][u] = (b_in[e] && k < kend) ? (__bf16)(float)v : (__bf16)0.f;
            }
        }
    };
    f4 acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    int buf = 0;
    if (kbeg < kend) load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += KB) {
#pragma unroll
        for (int e = 0; e < NA; ++e) {
            const int x = tid + 256 * e;
            *reinterpret_cast<bf8 *>(&As[buf][(x >> 2) * LDK + 8 * (x & 3)]) = ra[e];
        }
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            const int x = tid + 256 * e;
            *reinterpret_cast<bf8 *>(&Bs[buf][(x >> 2) * LDK + 8 * (x & 3)]) = rb[e];
        }
        __syncthreads();
        if (k0 + KB < kend) load(k0 + KB);
        bf8 av[TM], bv[TN];
#pragma unroll
        for (int a = 0; a < TM; ++a)
            av[a] = *reinterpret_cast<const bf8 *>(&As[buf][(wm * (BM / 2) + a * 16 + (lane & 15)) * LDK + 8 * (lane >> 4)]);
#pragma unroll
        for (int b = 0; b < TN; ++b)
            bv[b] = *reinterpret_cast<const bf8 *>(&Bs[buf][(wn * (BN / 2) + b * 16 + (lane & 15)) * LDK + 8 * (lane >> 4)]);
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
            for (int b = 0; b < TN; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
        buf ^= 1;
    }
    const int64_t coff = g.ksplit > 1 ? (int64_t)blockIdx.z * g.c_split : 0;
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wm * (BM / 2) + a * 16 + 4 * (lane >> 4) + r;
                const int j = j0 + wn * (BN / 2) + b * 16 + (lane & 15);
                if (i < g.M && j < g.N) {
                    const int64_t idx = coff + (int64_t)i * g.c_i + (int64_t)j * g.c_j;
                    const float v = g.alpha * acc[a][b][r];
                    if (g.c_dbl) static_cast<double *>(g.C)[idx] = (double)v;
                    else static_cast<float *>(g.C)[idx] = v;
                }
            }
}

template <int BM, int BN, bool DBL>
hipError_t launch32_st(const GemmMxArgs &g, dim3 grid, hipStream_t s)
{
    const bool akc = g.a_k == 1, bkc = g.b_k == 1;
    if (g.b_gather) {
        // the gathered product P^{-1}A: A K-contiguous, B's rows gathered
        if (!akc || bkc) return hipErrorInvalidValue;
        hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, true, false, DBL, true>), grid, dim3(256), 0, s, g);
    } else if (akc && bkc) {
        hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, true, true, DBL, false>), grid, dim3(256), 0, s, g);
    } else if (akc) {
        hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, true, false, DBL, false>), grid, dim3(256), 0, s, g);
    } else if (bkc) {
        hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, false, true, DBL, false>), grid, dim3(256), 0, s, g);
    } else {
        hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, false, false, DBL, false>), grid, dim3(256), 0, s, g);
    }
    return hipGetLastError();
}

// Operands that gemm_f32_kc_kernel and gemm_bf16x3_kc_kernel take: binary32,
// K-contiguous, unscaled (scaled allowed for the plain bfloat16 form),
// ungathered, full (not triangular), 16-byte aligned rows and K % 4 == 0.
bool kc_fast(const GemmMxArgs &g, bool scales_ok = false)
{
    return !g.a_dbl && !g.b_dbl && !g.c_dbl && g.a_k == 1 && g.b_k == 1 && !g.a_gather && !g.b_gather &&
           (scales_ok || (!g.a_scale && !g.b_scale)) && !g.a_lower && g.K % 4 == 0 && g.a_i % 4 == 0 &&
           g.b_j % 4 == 0 && (reinterpret_cast<uintptr_t>(g.A) & 15) == 0 &&
           (reinterpret_cast<uintptr_t>(g.B) & 15) == 0;
}

template <int BM, int BN>
hipError_t launch32(const GemmMxArgs &g, hipStream_t s)
{
    const int gm = (g.M + BM - 1) / BM, gn = (g.N + BN - 1) / BN;
    dim3 grid = g.c_lower ? dim3(gm * (gm + 1) / 2, 1, g.ksplit > 1 ? g.ksplit : 1)
                          : dim3(gn, gm, g.ksplit > 1 ? g.ksplit : 1);
    if (g.a_dbl != g.b_dbl) return hipErrorInvalidValue;  // operands share their storage type
    if (kc_fast(g)) {
        hipLaunchKernelGGL((gemm_f32_kc_kernel<BM, BN>), grid, dim3(256), 0, s, g);
        return hipGetLastError();
    }
    return g.a_dbl ? launch32_st<BM, BN, true>(g, grid, s) : launch32_st<BM, BN, false>(g, grid, s);
}

// out(i, j) = sum_s part[s][i][j] / (sa[i] sb[j]) in binary64 (fixed order);
// mirror: lower half summed, written to both halves.
__global__ void reduce_f32_kernel(const float *part, int64_t stride, int splits, int M, int N, int64_t ld,
                                  const float *sa, const float *sb, double *out, int64_t ldo, int mirror)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)M * N) return;
    const int i = (int)(e / N), j = (int)(e % N);
    if (mirror && j > i) return;
    double s = 0.0;
    for (int p = 0; p < splits; ++p) s += (double)part[p * stride + (int64_t)i * ld + j];
    if (sa) s /= (double)sa[i];
    if (sb) s /= (double)sb[j];
    out[(int64_t)i * ldo + j] = s;
    if (mirror) out[(int64_t)j * ldo + i] = s;
}

// scale[i] = 2^-e with e the smallest integer such that max_j |W_ij| <= 2^e
// (rows of a row-major m x n binary64/binary32 matrix; exact scaling).
__global__ __launch_bounds__(256) void row_scale_kernel(const void *W, int is_dbl, int64_t ldw, int n, float *scale)
{
    __shared__ double red[256];
    const int i = blockIdx.x;
    double mx = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) mx = fmax(mx, fabs(ld_any(W, is_dbl, (int64_t)i * ldw + j)));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int e = 0;
        if (red[0] > 0.0 && isfinite(red[0])) frexp(red[0], &e);  // red = f * 2^e, f in [0.5, 1)
        scale[i] = ldexpf(1.f, -e);
    }
}

// Round a binary64 row-major matrix to binary32.
__global__ void to_f32_kernel(const double *src, int64_t lds, float *dst, int64_t ldd, int m, int64_t n)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * n) return;
    const int i = (int)(e / n);
    const int64_t j = e % n;
    dst[(int64_t)i * ldd + j] = (float)src[(int64_t)i * lds + j];
}

// The split (X3) or plain bfloat16 product of binary32 operands: 256 x 128
// tiles for a lower-triangle grid unless tile == 128, else 128 x 128.
template <bool X3>
hipError_t launch_bf16_kc(const GemmMxArgs &g, hipStream_t stream)
{
    const unsigned ks = g.ksplit > 1 ? g.ksplit : 1;
    if (g.c_lower && g.tile != 128) {
        const int gi = (g.M + 255) / 256;
        hipLaunchKernelGGL((gemm_bf16x3_kc_kernel<256, 128, X3>), dim3(gi * (gi + 1), 1, ks), dim3(512), 0, stream,
                           g);
        return hipGetLastError();
    }
    const int gm = (g.M + 127) / 128, gn = (g.N + 127) / 128;
    const dim3 grid = g.c_lower ? dim3(gm * (gm + 1) / 2, 1, ks) : dim3(gn, gm, ks);
    hipLaunchKernelGGL((gemm_bf16x3_kc_kernel<128, 128, X3>), grid, dim3(256), 0, stream, g);
    return hipGetLastError();
}

}  // namespace

bool gemm_mx_bf16x3_ok(const GemmMxArgs &g) { return kc_fast(g); }

hipError_t gemm_bf16x3_grouped_lower(const GemmMxArgs *d_args, int count, int max_m, int ksmax, hipStream_t stream)
{
    if (count <= 0 || max_m <= 0) return hipSuccess;
    const int gi = (max_m + 255) / 256;
    hipLaunchKernelGGL((gemm_bf16x3_grouped_kernel<256, 128>), dim3(gi * (gi + 1), 1, count * ksmax), dim3(512), 0,
                       stream, d_args, ksmax);
    return hipGetLastError();
}

hipError_t gemm_mx(const GemmMxArgs &g, int mode, hipStream_t stream)
{
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (mode == MX_BF16X3) {
        if (!kc_fast(g)) return hipErrorInvalidValue;
        return launch_bf16_kc<true>(g, stream);
    }
    if (mode == MX_BF16) {
        if (g.a_k != 1 || g.b_k != 1 || g.a_gather || g.b_gather || g.a_lower) return hipErrorInvalidValue;
        const int gm = (g.M + 127) / 128, gn = (g.N + 127) / 128;
        dim3 grid = g.c_lower ? dim3(gm * (gm + 1) / 2, 1, g.ksplit > 1 ? g.ksplit : 1)
                              : dim3(gn, gm, g.ksplit > 1 ? g.ksplit : 1);
        if (g.a_dbl != g.b_dbl) return hipErrorInvalidValue;
        // binary32 operands with 16-byte rows: the LDS-swizzled kernel, one product
        if (kc_fast(g, true)) return launch_bf16_kc<false>(g, stream);
        if (g.a_dbl) hipLaunchKernelGGL((gemm_bf16_kernel<128, 128, true>), grid, dim3(256), 0, stream, g);
        else hipLaunchKernelGGL((gemm_bf16_kernel<128, 128, false>), grid, dim3(256), 0, stream, g);
        return hipGetLastError();
    }
    if (g.tile == 128) return launch32<128, 128>(g, stream);
    if (g.tile == 64) return launch32<64, 64>(g, stream);
    // triangular A (P^{-1}A): 64-row tiles measured faster than 128-row ones
    if (g.M >= 128 && g.N >= 128 && !g.a_lower) return launch32<128, 128>(g, stream);
    return launch32<64, 64>(g, stream);
}

hipError_t gemm_f32_grouped_lower(const GemmMxArgs *d_args, int count, int max_m, int ksmax, hipStream_t stream)
{
    if (count <= 0 || max_m <= 0) return hipSuccess;
    const int gm = (max_m + 63) / 64;
    const dim3 grid((unsigned)(gm * (gm + 1) / 2), 1, (unsigned)(count * ksmax));
    hipLaunchKernelGGL((gemm_f32_grouped_kernel<64, 64, true, true, true>), grid, dim3(256), 0, stream, d_args, ksmax);
    return hipGetLastError();
}

__global__ void reduce_f32_grouped_kernel(const ReduceF32GroupArgs *gs)
{
    const ReduceF32GroupArgs g = gs[blockIdx.y];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)g.m * g.m) return;
    const int i = (int)(e / g.m), j = (int)(e % g.m);
    if (j > i) return;
    double s = 0.0;
    for (int p = 0; p < g.splits; ++p) s += (double)g.part[p * g.stride + (int64_t)i * g.m + j];
    g.out[(int64_t)i * g.m + j] = s;
    g.out[(int64_t)j * g.m + i] = s;
}

hipError_t reduce_f32_grouped(const ReduceF32GroupArgs *d, int count, int max_m, hipStream_t stream)
{
    const int64_t total = (int64_t)max_m * max_m;
    if (count <= 0 || total == 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_f32_grouped_kernel, dim3((unsigned)((total + 255) / 256), count), dim3(256), 0, stream, d);
    return hipGetLastError();
}

hipError_t reduce_f32_splits(const float *part, int64_t stride, int splits, int M, int N, int64_t ld, const float *sa,
                             const float *sb, double *out, int64_t ldo, int mirror, hipStream_t stream)
{
    const int64_t total = (int64_t)M * N;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_f32_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, part, stride,
                       splits, M, N, ld, sa, sb, out, ldo, mirror);
    return hipGetLastError();
}

hipError_t row_pow2_scale(const void *W, int is_dbl, int64_t ldw, int m, int n, float *scale, hipStream_t stream)
{
    hipLaunchKernelGGL(row_scale_kernel, dim3(m), dim3(256), 0, stream, W, is_dbl, ldw, n, scale);
    return hipGetLastError();
}

hipError_t to_f32(const double *src, int64_t lds, float *dst, int64_t ldd, int m, int64_t n, hipStream_t stream)
{
    const int64_t total = (int64_t)m * n;
    hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, src, lds, dst, ldd,
                       m, n);
    return hipGetLastError();
}

}  // namespace rt
