// Reduced-precision GEMMs of the preconditioner on the gfx950 matrix cores,
// binary32 accumulation:
//   * MX_F32:  v_mfma_f32_16x16x4_f32   (binary32 operands)
//   * MX_BF16: v_mfma_f32_16x16x32_bf16 (bfloat16 operands)
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

template <int BM, int BN, bool A_KC, bool B_KC>
__global__ __launch_bounds__(256) void gemm_f32_kernel(GemmMxArgs g)
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
        ks = (ks + KC32 - 1) / KC32 * KC32;
        kbeg = blockIdx.z * ks;
        kend = min(g.K, kbeg + ks);
    }
    if (g.a_lower) kend = min(kend, i0 + BM);
    auto a_coord = [&](int e, int &ii, int &kk) {
        const int x = tid + 256 * e;
        if (A_KC) { ii = x / KC32; kk = x % KC32; } else { ii = x % BM; kk = x / BM; }
    };
    auto b_coord = [&](int e, int &jj, int &kk) {
        const int x = tid + 256 * e;
        if (B_KC) { jj = x / KC32; kk = x % KC32; } else { jj = x % BN; kk = x / BN; }
    };
    float ra[NA], rb[NB];
    auto load = [&](int k0) {
#pragma unroll
        for (int e = 0; e < NA; ++e) {
            int ii, kk;
            a_coord(e, ii, kk);
            const int i = i0 + ii, k = k0 + kk;
            double v = 0.0;
            if (i < g.M && k < kend && !(g.a_lower && k > i)) {
                const int64_t gi = g.a_gather ? (int64_t)g.a_gather[i] : (int64_t)i;
                v = ld_any(g.A, g.a_dbl, gi * g.a_i + (int64_t)k * g.a_k);
                if (g.a_scale) v *= (double)g.a_scale[i];
            }
            ra[e] = (float)v;
        }
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            int jj, kk;
            b_coord(e, jj, kk);
            const int j = j0 + jj, k = k0 + kk;
            double v = 0.0;
            if (j < g.N && k < kend) {
                const int64_t gk = g.b_gather ? (int64_t)g.b_gather[k] : (int64_t)k;
                v = ld_any(g.B, g.b_dbl, gk * g.b_k + (int64_t)j * g.b_j);
                if (g.b_scale) v *= (double)g.b_scale[j];
            }
            rb[e] = (float)v;
        }
    };
    f4 acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    int buf = 0;
    if (kbeg < kend) load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += KC32) {
#pragma unroll
        for (int e = 0; e < NA; ++e) {
            int ii, kk;
            a_coord(e, ii, kk);
            As[buf][LA::at(ii, kk)] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            int jj, kk;
            b_coord(e, jj, kk);
            Bs[buf][LB::at(jj, kk)] = rb[e];
        }
        __syncthreads();
        if (k0 + KC32 < kend) load(k0 + KC32);
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
        buf ^= 1;
    }
    const int64_t coff = g.ksplit > 1 ? (int64_t)blockIdx.z * g.c_split : 0;
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

// ---------------------------------------------------------------- bfloat16
// Both operands K-contiguous (the Gram of a row-major matrix): LDS tiles are
// [mn][KB + 8] bfloat16, so each lane's 8 consecutive k are one 16-byte read
// and 16 lanes at 16 consecutive rows hit 64 distinct banks.
constexpr int KB = 32;

template <int BM, int BN>
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
    // group e of this thread: row (x / 4), k-offset 8 * (x % 4), x = tid + 256 e
    bf8 ra[NA], rb[NB];
    auto load = [&](int k0) {
#pragma unroll
        for (int e = 0; e < NA; ++e) {
            const int x = tid + 256 * e, ii = x >> 2, kk = 8 * (x & 3);
            const int i = i0 + ii;
            const float sc = (i < g.M && g.a_scale) ? g.a_scale[i] : 1.f;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = k0 + kk + u;
                double v = 0.0;
                if (i < g.M && k < kend) v = ld_any(g.A, g.a_dbl, (int64_t)i * g.a_i + (int64_t)k * g.a_k) * sc;
                ra[e][u] = (__bf16)(float)v;
            }
        }
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            const int x = tid + 256 * e, jj = x >> 2, kk = 8 * (x & 3);
            const int j = j0 + jj;
            const float sc = (j < g.N && g.b_scale) ? g.b_scale[j] : 1.f;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = k0 + kk + u;
                double v = 0.0;
                if (j < g.N && k < kend) v = ld_any(g.B, g.b_dbl, (int64_t)k * g.b_k + (int64_t)j * g.b_j) * sc;
                rb[e][u] = (__bf16)(float)v;
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

template <int BM, int BN>
hipError_t launch32(const GemmMxArgs &g, hipStream_t s)
{
    const int gm = (g.M + BM - 1) / BM, gn = (g.N + BN - 1) / BN;
    dim3 grid = g.c_lower ? dim3(gm * (gm + 1) / 2, 1, g.ksplit > 1 ? g.ksplit : 1)
                          : dim3(gn, gm, g.ksplit > 1 ? g.ksplit : 1);
    const bool akc = g.a_k == 1, bkc = g.b_k == 1;
    if (akc && bkc) hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, true, true>), grid, dim3(256), 0, s, g);
    else if (akc) hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, true, false>), grid, dim3(256), 0, s, g);
    else if (bkc) hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, false, true>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, false, false>), grid, dim3(256), 0, s, g);
    return hipGetLastError();
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

}  // namespace

hipError_t gemm_mx(const GemmMxArgs &g, int mode, hipStream_t stream)
{
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (mode == MX_BF16) {
        if (g.a_k != 1 || g.b_k != 1 || g.a_gather || g.b_gather || g.a_lower) return hipErrorInvalidValue;
        const int gm = (g.M + 127) / 128, gn = (g.N + 127) / 128;
        dim3 grid = g.c_lower ? dim3(gm * (gm + 1) / 2, 1, g.ksplit > 1 ? g.ksplit : 1)
                              : dim3(gn, gm, g.ksplit > 1 ? g.ksplit : 1);
        hipLaunchKernelGGL((gemm_bf16_kernel<128, 128>), grid, dim3(256), 0, stream, g);
        return hipGetLastError();
    }
    if (g.M >= 128 && g.N >= 128 && !g.a_lower) return launch32<128, 128>(g, stream);
    return launch32<64, 64>(g, stream);
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
