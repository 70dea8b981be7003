// Compensated residual products of the refinement (Remark 4.3) on the int8
// matrix cores, exact in integer arithmetic (the splitting of Ozaki, Ogita,
// Oishi and Rump, 2012):
//
//   every dot product sum_k u_k v_k of a row of the A operand with a
//   right-hand side is taken on a common binary scale per row (2^e, all
//   |u_k| < 2^e) and per right-hand side (2^f); each value on the halved
//   scale, |u 2^-(e+1)| < 1/2, is written as a sum of OZ_S = 11 signed
//   base-128 digits, u 2^-(e+1) = sum_{s=0}^{10} alpha_s 128^-(s+1) + rho
//   with |alpha_s| <= 64 (65 for a double-binary64 right-hand side, whose
//   leading digit may carry) and |rho| <= 2^-78.  The digit products
//   P_st = sum_k alpha_s,k beta_t,k are exact in int32
//   (v_mfma_i32_16x16x64_i8 accumulates in int32; a diagonal holds at most
//   11 pairs, 11 * 65^2 * K < 2^31 for K <= OZ_KMAX = 32768), and
//   sum_k u_k v_k = 2^(e+f+2) sum_{s,t} 128^-(s+t+2) P_st
//   up to the digits and pairs left out.  The pairs on the OZ_NDIAG = 12
//   diagonals s + t <= 11 (76 of 121) are kept, summed per diagonal in
//   int32, and the diagonals combined in double-binary64 (TwoSum).  The
//   omitted pairs and the remainders rho add up to less than
//   2^(e+f) K 2^-75 in magnitude: about 2^-64 of the scale of the largest
//   term at K = 2048, 2^-57 at K = 262144.
//
// Two products use it: r = B - A^T x (x double-binary64; the A-operand rows
// are A's columns, K = m, the whole sum in one block) and s = A r (r binary64;
// the rows are A's rows, K = n split over blocks, double-binary64 partials
// summed by the compensated split reduction).  A's digits are formed on the
// fly from binary64 A for each 64 x 64 tile, three or four digits per
// binary64 rounding (oz_digit_group); the right-hand sides' digits come from
// a small digit kernel.
#include <algorithm>
#include <climits>

#include "rt_common.h"

namespace rt {

namespace {

constexpr int OZ_T = 512;
constexpr double OZ_ROUND = 6755399441055744.0;  // 1.5 * 2^52: x + OZ_ROUND rounds x to an integer for |x| < 2^51
constexpr int OZ_TILE = 64;        // A-operand rows and right-hand sides per block; K per chunk
constexpr int OZ_LD = OZ_TILE + 16;  // LDS row stride in bytes (16-byte reads of 8 lanes on distinct banks)
typedef int int4v __attribute__((ext_vector_type(4)));

// Exponent e with |v| < 2^e (frexp's), INT_MIN for zero.
__device__ __forceinline__ int oz_exp(double v)
{
    int e = 0;
    (void)frexp(v, &e);
    return v == 0.0 ? INT_MIN : e;
}

__global__ void oz_fill_kernel(int *p, int n, int v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Column and row exponents of the m x n row-major A, one 64 x 64 tile per
// block: thread t takes column j0 + t % 64 and rows i0 + 16 (t / 64) + u.
__global__ __launch_bounds__(256) void oz_aexp_kernel(const double *A, int64_t lda, int m, int n, int *colexp,
                                                      int *rowexp)
{
    __shared__ int cmax[64], rmax[64];
    const int t = threadIdx.x;
    if (t < 64) { cmax[t] = INT_MIN; rmax[t] = INT_MIN; }
    __syncthreads();
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int j = j0 + (t & 63), ib = 16 * (t >> 6);
    const bool jok = j < n;
    const int jc = jok ? j : n - 1;
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = A[(int64_t)min(i0 + ib + u, m - 1) * lda + jc];
    int cm = INT_MIN;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        // a wave holds one row's 64 columns: its maximum by shuffles, then
        // one LDS atomic per wave and row
        int e = (jok && i0 + ib + u < m) ? oz_exp(v[u]) : INT_MIN;
        cm = max(cm, e);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) e = max(e, __shfl_xor(e, o, 64));
        if ((t & 63) == 0 && e != INT_MIN) atomicMax(&rmax[ib + u], e);
    }
    if (jok && cm != INT_MIN) atomicMax(&cmax[t & 63], cm);
    __syncthreads();
    if (t < 64 && j0 + t < n && cmax[t] != INT_MIN) atomicMax(&colexp[j0 + t], cmax[t]);
    if (t >= 64 && t < 128 && i0 + t - 64 < m && rmax[t - 64] != INT_MIN) atomicMax(&rowexp[i0 + t - 64], rmax[t - 64]);
}

// Exponent of every column of the rows x k column-major V: blockIdx.x = column,
// blockIdx.y = a run of 8192 rows; max into exp[c] (cleared to INT_MIN).
__global__ __launch_bounds__(256) void oz_colexp_kernel(const double *V, int64_t ld, int rows, int *exp)
{
    __shared__ int red[256];
    const int c = blockIdx.x;
    const int r0 = blockIdx.y * 8192, r1 = min(rows, r0 + 8192);
    int e = INT_MIN;
    for (int i = r0 + threadIdx.x; i < r1; i += 256) e = max(e, oz_exp(V[(int64_t)c * ld + i]));
    red[threadIdx.x] = e;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] != INT_MIN) atomicMax(&exp[c], red[0]);
}

// Digits of the right-hand sides (vh + vl, or vh alone) on their halved
// column scales 2^(f+1): dig[(t kpad + c) rows_pad + row], t < OZ_S, zero
// past rows and k.  Each digit of a double-binary64 value is rounded from its
// high part and corrected by one when the low part carries the remainder
// past 1/2.
template <bool DD>
__global__ __launch_bounds__(256) void oz_digits_kernel(const double *vh, const double *vl, int64_t ld, int rows,
                                                        int k, int64_t rows_pad, int kpad, const int *exp,
                                                        int8_t *dig)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows_pad * kpad) return;
    const int c = (int)(e / rows_pad);
    const int64_t row = e % rows_pad;
    double h = 0.0, l = 0.0;
    const int ex = c < k ? exp[c] : INT_MIN;
    if (c < k && row < rows && ex != INT_MIN) {
        h = ldexp(vh[(int64_t)c * ld + row], -ex - 1);
        if (DD) l = ldexp(vl[(int64_t)c * ld + row], -ex - 1);
    }
#pragma unroll
    for (int t = 0; t < OZ_S; ++t) {
        h *= 128.0;
        l *= 128.0;
        double d = rint(h);
        if (DD) {
            double s, err;
            two_sum(h - d, l, s, err);  // h - d is exact
            if (s > 0.5) { d += 1.0; s -= 1.0; }
            else if (s < -0.5) { d -= 1.0; s += 1.0; }
            h = s;
            l = err;
        } else {
            h -= d;
        }
        dig[((int64_t)t * kpad + c) * rows_pad + row] = (int8_t)(int)d;
    }
}

// Digits s0 .. s0 + J - 1 of a value v with |v| <= 1/2 on the frame of digit
// s0: D = round(128^J v) in one binary64 rounding (adding 1.5 * 2^52, whose
// sum t keeps D, |D| <= 2^(7J-1) < 2^31, in two's complement in the low word
// of its bits), then D's balanced base-128 digits from the least
// significant: digit i is the signed 7-bit field at bit 7i of
// E_i = D + 64 (128^i - 1) / 127, the top digit all of E_{J-1} above bit
// 7(J-1) (so in [-64, 64]).  v becomes 128^J v - D, exact, |v| <= 1/2 on
// the next frame.  Digit s lands in byte u of wd[s].
static_assert(OZ_S == 11, "the digit groups below cover 4 + 4 + 3 digits");
template <int J, bool LAST>
__device__ __forceinline__ void oz_digit_group(double &v, int u, int (&wd)[OZ_S], int s0)
{
    constexpr double sc = (double)(1 << (7 * J));
    const double t = __builtin_fma(v, sc, OZ_ROUND);
    if (!LAST) v = __builtin_fma(v, sc, -(t - OZ_ROUND));
    int E = (int)(unsigned)__builtin_bit_cast(unsigned long long, t);
#pragma unroll
    for (int i = 0; i < J; ++i) {
        const int dg = i + 1 < J ? __builtin_amdgcn_sbfe(E, 7 * i, 7) : (E >> (7 * i));
        wd[s0 + J - 1 - i] |= (dg & 0xff) << (8 * u);
        E += 64 << (7 * i);
    }
}

// One 64 x 64 tile (A-operand rows r0.., right-hand sides c0..) over the K
// range of split blockIdx.z.  TRANS: the A-operand rows are A's columns (A^T x,
// K = m); otherwise A's rows (A r, K = n).  Eight waves: wave w takes the 16
// rows 16 (w % 4) .. and the 32 right-hand sides 32 (w / 4) .., so that its
// 12 x 2 accumulator tiles (96 registers) leave room for two waves per SIMD,
// which hide each other's issue and LDS stalls; each thread forms the digits
// of 8 of the tile's A values per chunk.
template <bool TRANS>
__global__ __launch_bounds__(OZ_T) void oz_mm_kernel(OzArgs g)
{
    __shared__ __attribute__((aligned(16))) int8_t As[OZ_S][OZ_TILE * OZ_LD];
    __shared__ __attribute__((aligned(16))) int8_t Bs[OZ_S][OZ_TILE * OZ_LD];
    typedef int int2v __attribute__((ext_vector_type(2)));
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int rw = w & 3, ch = w >> 2;
    const int r0 = blockIdx.x * OZ_TILE, c0 = blockIdx.y * OZ_TILE;
    const int64_t kbeg = (int64_t)blockIdx.z * g.kchunk;
    const int64_t kend = min((int64_t)g.K, kbeg + g.kchunk);
    // (an empty split of A r still writes its zero partials below)
    // this thread's part of the A tile: one A-operand row, 8 consecutive k
    const int lrow = TRANS ? (tid & 63) : (tid >> 3);
    const int lk = TRANS ? 8 * (tid >> 6) : 8 * (tid & 7);
    const int grow = r0 + lrow;
    const bool rok = grow < g.R;
    const int ex = rok ? g.rowexp[grow] : INT_MIN;
    const bool live = ex != INT_MIN;  // (an all-zero row has no scale)
    const int growc = rok ? grow : g.R - 1;
    // this thread's part of the B digits: right-hand side c0 + bc, 8 k from bk
    const int bc = tid >> 3, bk = 8 * (tid & 7);

    int4v acc[OZ_NDIAG][2];
#pragma unroll
    for (int d = 0; d < OZ_NDIAG; ++d)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) acc[d][ct] = int4v{0, 0, 0, 0};

    // chunk loads: raw A values (clamped addresses) and the B digits (padded:
    // always in range); issued one chunk ahead, before the current chunk's
    // products, and used only after them
    double av[8];
    int2v bl[OZ_S];
    auto load_chunk = [&](int64_t k0) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t kk = k0 + lk + u;
            const int64_t kc = kk < kend ? kk : kend - 1;
            av[u] = TRANS ? g.A[kc * g.lda + growc] : g.A[(int64_t)growc * g.lda + kc];
        }
#pragma unroll
        for (int t = 0; t < OZ_S; ++t)
            bl[t] = *reinterpret_cast<const int2v *>(g.dig + ((int64_t)t * g.kpad + c0 + bc) * g.Kpad + k0 + bk);
    };
    if (kbeg < kend) load_chunk(kbeg);
    for (int64_t k0 = kbeg; k0 < kend; k0 += OZ_TILE) {
        __syncthreads();  // the previous chunk's operand reads are done
#pragma unroll
        for (int t = 0; t < OZ_S; ++t) *reinterpret_cast<int2v *>(&Bs[t][bc * OZ_LD + bk]) = bl[t];
        // A digits of 8 elements: two 32-bit words per plane, one 8-byte store
        {
            int wd[2][OZ_S];
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int s2 = 0; s2 < OZ_S; ++s2) wd[q][s2] = 0;
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    // on the row's halved power-of-two scale (zero outside the
                    // range), |v| < 1/2; digits in groups of 4, 4 and 3
                    double v = (live && k0 + lk + 4 * q + u < kend) ? ldexp(av[4 * q + u], -ex - 1) : 0.0;
                    oz_digit_group<4, false>(v, u, wd[q], 0);
                    oz_digit_group<4, false>(v, u, wd[q], 4);
                    oz_digit_group<3, true>(v, u, wd[q], 8);
                }
#pragma unroll
            for (int s2 = 0; s2 < OZ_S; ++s2)
                *reinterpret_cast<int2v *>(&As[s2][lrow * OZ_LD + lk]) = int2v{wd[0][s2], wd[1][s2]};
        }
        __syncthreads();
        if (k0 + OZ_TILE < kend) load_chunk(k0 + OZ_TILE);  // in flight during the products
        int4v aop[OZ_S];
#pragma unroll
        for (int s = 0; s < OZ_S; ++s)
            aop[s] = *reinterpret_cast<const int4v *>(&As[s][(16 * rw + (lane & 15)) * OZ_LD + 16 * (lane >> 4)]);
        // digit plane t of the right-hand sides against every A plane s with
        // s + t on a kept diagonal; the next plane's operands are read while
        // these products run
        auto bop_at = [&](int t, int ct) {
            return *reinterpret_cast<const int4v *>(
                &Bs[t][(16 * (2 * ch + ct) + (lane & 15)) * OZ_LD + 16 * (lane >> 4)]);
        };
        int4v bcur[2], bnext[2];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) bcur[ct] = bop_at(0, ct);
#pragma unroll
        for (int t = 0; t < OZ_S; ++t) {
            if (t + 1 < OZ_S)
#pragma unroll
                for (int ct = 0; ct < 2; ++ct) bnext[ct] = bop_at(t + 1, ct);
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                for (int s = 0; s < OZ_S && s + t < OZ_NDIAG; ++s)
                    acc[s + t][ct] = __builtin_amdgcn_mfma_i32_16x16x64_i8(aop[s], bcur[ct], acc[s + t][ct], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) bcur[ct] = bnext[ct];
        }
    }

    // diagonals to double-binary64, smallest first: sum 128^-(d+2) Q_d, then
    // the scale 2^(e+f+2) (exact)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = r0 + 16 * rw + 4 * (lane >> 4) + r;
            const int c = c0 + 16 * (2 * ch + ct) + (lane & 15);
            if (row >= g.R || c >= g.k) continue;
            const int er = g.rowexp[row], ec = g.bexp[c];
            double hi = 0.0, lo = 0.0;
            if (er != INT_MIN && ec != INT_MIN) {
#pragma unroll
                for (int d = OZ_NDIAG - 1; d >= 0; --d) {
                    const double t = ldexp((double)acc[d][ct][r], -7 * (d + 2));
                    double s, err;
                    two_sum(hi, t, s, err);
                    hi = s;
                    lo += err;
                }
                double s, err;
                two_sum(hi, lo, s, err);
                hi = ldexp(s, er + ec + 2);
                lo = ldexp(err, er + ec + 2);
            }
            if (TRANS) {
                // r = B - (hi + lo), rounded once
                double d, e;
                two_sum(g.B[(int64_t)c * g.ldb + row], -hi, d, e);
                g.Rout[(int64_t)c * g.ldr + row] = d + (e - lo);
            } else {
                const int64_t idx = ((int64_t)blockIdx.z * g.k + c) * g.R + row;
                g.ph[idx] = hi;
                g.pl[idx] = lo;
            }
        }
}

}  // namespace

int oz_splits(int64_t K, int64_t tiles, int cu_count)
{
    // split K so that the grid holds about four blocks per compute unit, each
    // split at least 1024 long and at most OZ_KMAX (the int32 bound)
    int64_t s = std::max<int64_t>(1, (4 * (int64_t)cu_count + tiles - 1) / std::max<int64_t>(1, tiles));
    s = std::min<int64_t>(s, std::max<int64_t>(1, K / 1024));
    s = std::max<int64_t>(s, (K + OZ_KMAX - OZ_TILE - 1) / (OZ_KMAX - OZ_TILE));  // rounded chunks stay <= OZ_KMAX
    return (int)std::min<int64_t>(s, 64);
}

int64_t oz_kchunk(int64_t K, int splits)
{
    const int64_t c = (K + splits - 1) / splits;
    return (c + OZ_TILE - 1) / OZ_TILE * OZ_TILE;
}

hipError_t oz_exponents_f64(const double *A, int64_t lda, int m, int n, int *colexp, int *rowexp, hipStream_t s)
{
    hipLaunchKernelGGL(oz_fill_kernel, dim3((n + 255) / 256), dim3(256), 0, s, colexp, n, INT_MIN);
    hipLaunchKernelGGL(oz_fill_kernel, dim3((m + 255) / 256), dim3(256), 0, s, rowexp, m, INT_MIN);
    hipLaunchKernelGGL(oz_aexp_kernel, dim3((n + 63) / 64, (m + 63) / 64), dim3(256), 0, s, A, lda, m, n, colexp,
                       rowexp);
    return hipGetLastError();
}

hipError_t oz_digits_f64(const double *vh, const double *vl, int64_t ld, int rows, int k, int64_t rows_pad, int kpad,
                         int *exp, int8_t *dig, hipStream_t s)
{
    if (k <= 0 || rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(oz_fill_kernel, dim3((k + 255) / 256), dim3(256), 0, s, exp, k, INT_MIN);
    hipLaunchKernelGGL(oz_colexp_kernel, dim3(k, (rows + 8191) / 8192), dim3(256), 0, s, vh, ld, rows, exp);
    const int64_t total = rows_pad * kpad;
    if (vl)
        hipLaunchKernelGGL(oz_digits_kernel<true>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, vh, vl, ld,
                           rows, k, rows_pad, kpad, (const int *)exp, dig);
    else
        hipLaunchKernelGGL(oz_digits_kernel<false>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, vh, vl, ld,
                           rows, k, rows_pad, kpad, (const int *)exp, dig);
    return hipGetLastError();
}

hipError_t oz_mm(const OzArgs &g, int trans, int splits, hipStream_t s)
{
    if (g.R <= 0 || g.k <= 0) return hipSuccess;
    if (g.kchunk % OZ_TILE || g.Kpad % OZ_TILE || g.kpad % OZ_TILE || g.kchunk > OZ_KMAX) return hipErrorInvalidValue;
    if (trans && splits != 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((g.R + OZ_TILE - 1) / OZ_TILE), (unsigned)(g.kpad / OZ_TILE), (unsigned)splits);
    if (trans) hipLaunchKernelGGL(oz_mm_kernel<true>, grid, dim3(OZ_T), 0, s, g);
    else hipLaunchKernelGGL(oz_mm_kernel<false>, grid, dim3(OZ_T), 0, s, g);
    return hipGetLastError();
}

}  // namespace rt
