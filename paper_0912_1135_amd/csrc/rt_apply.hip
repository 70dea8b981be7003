// The passes over A of the projection (Sec. 4, steps 1 and 7) and of the
// refinement of the least-squares solution (Remark 4.3); the m x m products
// of steps 2-6 (x = M^{-1} c) are GEMMs issued by the plan.
//
//   c = A b                 ab_sx (plain, b in scalar registers) or
//                           ab_partial (LDS-staged; Dot2), then ab_reduce
//   b~ = A^T x, z = b - b~  atx_dd_sx (Dot2, x in scalar registers) or atx
//
// Refinement: r = b - A^T x and s = A r are accumulated with Dot2 (error-free
// products and sums, i.e. about twice binary64 precision) and x is kept as an
// unevaluated pair (x_hi, x_lo).  The contractions over the long dimension n
// are VALU kernels that stream A once per pass (or per block of right-hand
// sides) with coalesced loads kept in flight; the right-hand-side blocks are
// small and read from scalar registers or LDS.
#include "rt_common.h"

#include <algorithm>

namespace rt {

namespace {

constexpr int AB_RB = 32;   // rows of A per block
constexpr int AB_TC = 64;   // columns of A per LDS stage

// Zero read in place of an operand element outside the problem: the staging
// loads pick their address, not their value, so that every load is issued
// unconditionally (a load whose value is selected afterwards is compiled
// into a branch that waits for it).
__device__ double g_zero = 0.0;

// part[s][j][row] = sum_{t in split s} A[row][t] * B[t][j] (column-major m x k
// per split).  dd: Dot2 accumulation, hi in part_hi and error in part_lo.
// The next stage's A and B elements are loaded into registers while the
// current stage is multiplied out of LDS.
template <bool DD, int KJ>
__device__ __forceinline__ void ab_partial_body(const ApplyArgs &a, const double *B, int64_t ldb, int splits,
                                                double *part_hi, double *part_lo, int bx, int split, int bz)
{
    constexpr int NO = AB_RB * KJ / 256;      // outputs per thread
    constexpr int NA = AB_RB * AB_TC / 256;   // staged elements of A per thread
    constexpr int NB = AB_TC * KJ / 256;      // staged elements of B per thread
    static_assert(256 % KJ == 0 && 256 % AB_TC == 0, "thread coordinates assume these divide the block");
    __shared__ double As[AB_RB][AB_TC + 1];
    __shared__ double Bs[AB_TC][KJ];
    const int r0 = bx * AB_RB;
    const int j0 = bz * KJ;
    if (r0 >= a.m || split >= splits || j0 >= a.k) return;  // whole block (grouped launches)
    const int64_t len = ((int64_t)a.n + splits - 1) / splits;
    const int64_t t0 = (int64_t)split * len;
    const int64_t t1 = min<int64_t>(a.n, t0 + len);
    const int tid = threadIdx.x;
    // staged element e = tid + 256 q: A (rr, tt) = (e / AB_TC, e % AB_TC),
    // B (jj, tt) likewise; consecutive threads read consecutive t
    const int tt = tid % AB_TC;
    const double *arow[NA];
    const double *bcol[NB];
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        const int row = r0 + (tid + 256 * q) / AB_TC;
        arow[q] = row < a.m ? a.A + (int64_t)row * a.lda : nullptr;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int j = j0 + (tid + 256 * q) / AB_TC;
        bcol[q] = j < a.k ? B + (int64_t)j * ldb : nullptr;
    }
    double ra[NA], rb[NB];
    auto load = [&](int64_t tb) {
        const int64_t t = tb + tt;
        const bool tin = t < t1;
        // a column-scaled operand: each element rounded as A[i][t] * cs[t]
        const double ct = a.cs ? *(tin ? a.cs + t : &g_zero) : 1.0;
#pragma unroll
        for (int q = 0; q < NA; ++q) ra[q] = *((arow[q] && tin) ? arow[q] + t : &g_zero) * ct;
#pragma unroll
        for (int q = 0; q < NB; ++q) rb[q] = *((bcol[q] && tin) ? bcol[q] + t : &g_zero);
    };
    // NO outputs per thread: (row, j) = (o / KJ, o % KJ), o = tid + 256 q
    double s[NO], c[NO];
#pragma unroll
    for (int q = 0; q < NO; ++q) { s[q] = 0.0; c[q] = 0.0; }
    load(t0);
    for (int64_t tb = t0; tb < t1; tb += AB_TC) {
#pragma unroll
        for (int q = 0; q < NA; ++q) As[(tid + 256 * q) / AB_TC][tt] = ra[q];
#pragma unroll
        for (int q = 0; q < NB; ++q) Bs[tt][(tid + 256 * q) / AB_TC] = rb[q];
        __syncthreads();
        load(tb + AB_TC);  // past t1 every address is the zero
        // a thread's outputs share their column jj (256 is a multiple of
        // KJ): one LDS read of B per t serves all of them
        const int jj = tid % KJ;
#pragma unroll 8
        for (int t2 = 0; t2 < AB_TC; ++t2) {
            const double bv = Bs[t2][jj];
#pragma unroll
            for (int q = 0; q < NO; ++q) {
                const double av = As[(tid + 256 * q) / KJ][t2];
                if (DD) dot2_acc(av, bv, s[q], c[q]);
                else s[q] = __builtin_fma(av, bv, s[q]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NO; ++q) {
        const int o = tid + 256 * q;
        const int row = r0 + o / KJ, j = j0 + o % KJ;
        if (row < a.m && j < a.k) {
            const int64_t idx = (int64_t)split * a.m * a.k + (int64_t)j * a.m + row;
            part_hi[idx] = s[q];
            if (DD) part_lo[idx] = c[q];
        }
    }
}

template <bool DD, int KJ>
__global__ __launch_bounds__(256) void ab_partial_kernel(ApplyArgs a, const double *B, int64_t ldb, int splits,
                                                         double *part_hi, double *part_lo)
{
    ab_partial_body<DD, KJ>(a, B, ldb, splits, part_hi, part_lo, blockIdx.x, blockIdx.y, blockIdx.z);
}

// grouped: blockIdx.z = member * kbmax + right-hand-side block
template <bool DD, int KJ>
__global__ __launch_bounds__(256) void ab_partial_grouped(const AbGroupArgs *gs, int kbmax)
{
    const AbGroupArgs g = gs[blockIdx.z / kbmax];
    ab_partial_body<DD, KJ>(g.a, g.B, g.ldb, g.splits, g.ph, g.pl, blockIdx.x, blockIdx.y, blockIdx.z % kbmax);
}

// right-hand sides per block of the A B pass: every block reads its panel of
// A once for KJ columns of B (compensated accumulators need twice the registers)
inline int ab_kj(int k, int dd) { return k > 32 && !dd ? 64 : (k > 16 ? 32 : 16); }

// Sum of the split partials in split order; the loads of eight splits are
// issued before they are added (clamped indices, unconditional loads).
__device__ __forceinline__ void ab_reduce_body(const double *ph, const double *pl, int m, int k, int splits, int dd,
                                               double *out, int64_t ldo, int64_t e)
{
    const int64_t mk = (int64_t)m * k;
    if (e >= mk) return;
    const int j = (int)(e / m), row = (int)(e % m);
    constexpr int U = 8;
    double s = 0.0, c = 0.0;
    for (int p0 = 0; p0 < splits; p0 += U) {
        double vh[U], vl[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t idx = (int64_t)min(p0 + u, splits - 1) * mk + e;
            vh[u] = ph[idx];
            vl[u] = dd ? pl[idx] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (p0 + u >= splits) break;
            if (dd) {
                double t, err;
                two_sum(s, vh[u], t, err);
                s = t;
                c += err + vl[u];
            } else {
                s += vh[u];
            }
        }
    }
    out[(int64_t)j * ldo + row] = s + c;
}

__global__ void ab_reduce_kernel(const double *ph, const double *pl, int m, int k, int splits, int dd, double *out,
                                 int64_t ldo)
{
    ab_reduce_body(ph, pl, m, k, splits, dd, out, ldo, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void ab_reduce_grouped(const AbGroupArgs *gs, int dd)
{
    const AbGroupArgs g = gs[blockIdx.y];
    ab_reduce_body(g.ph, g.pl, g.a.m, g.a.k, g.splits, dd, g.out, g.ldo, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

constexpr int ATX_T = 128;  // columns t of A per block (one per thread)
constexpr int ATX_MC = 64;  // rows of x staged in LDS at a time

// y(t, j) = sum_i A[i][t] (xhi[i][j] + xlo[i][j]); then
//   mode 0: R = round(B - y)
//   mode 1: Y = round(y), Z = round(B - y)
template <bool DD, int KJ, bool SC = false>
__device__ __forceinline__ void atx_body(const ApplyArgs &a, const double *xhi, const double *xlo, int64_t ldx,
                                         const double *B, int64_t ldb, double *Rout, int64_t ldr, double *Y,
                                         int64_t ldy, double *Z, int64_t ldz, int bx, int by)
{
    __shared__ double xh[ATX_MC][KJ];
    __shared__ double xl[DD ? ATX_MC : 1][KJ];
    const int64_t t = (int64_t)bx * ATX_T + threadIdx.x;
    const int j0 = by * KJ;
    if ((int64_t)bx * ATX_T >= a.n || j0 >= a.k) return;  // whole block (grouped launches)
    const int kj = min(KJ, a.k - j0);
    double s[KJ], c[KJ];
#pragma unroll
    for (int j = 0; j < KJ; ++j) { s[j] = 0.0; c[j] = 0.0; }
    const bool active = t < a.n;
    // SC: a column-scaled operand, each element rounded as A[i][t] * cs[t]
    // (members without a scaling multiply by one)
    const double ct = (SC && a.cs && active) ? a.cs[t] : 1.0;
    for (int i0 = 0; i0 < a.m; i0 += ATX_MC) {
        const int mc = min(ATX_MC, a.m - i0);
        for (int e = threadIdx.x; e < ATX_MC * KJ; e += ATX_T) {
            const int ii = e / KJ, jj = e % KJ;
            const bool ok = ii < mc && jj < kj;
            xh[ii][jj] = ok ? xhi[(int64_t)(j0 + jj) * ldx + i0 + ii] : 0.0;
            if (DD) xl[ii][jj] = (ok && xlo) ? xlo[(int64_t)(j0 + jj) * ldx + i0 + ii] : 0.0;
        }
        __syncthreads();
        if (active) {
            const double *ap = a.A + (int64_t)i0 * a.lda + t;
            for (int ii = 0; ii < mc; ii += 8) {
                // eight loads in flight before the 8 x 16 compensated updates
                double av[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    av[u] = (ii + u < mc) ? ap[(int64_t)(ii + u) * a.lda] : 0.0;
                    if (SC) av[u] *= ct;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
#pragma unroll
                    for (int j = 0; j < KJ; ++j) {
                        if (DD) {
                            dot2_acc(av[u], xh[ii + u][j], s[j], c[j]);
                            c[j] = __builtin_fma(av[u], xl[ii + u][j], c[j]);
                        } else {
                            s[j] = __builtin_fma(av[u], xh[ii + u][j], s[j]);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (!active) return;
    for (int j = 0; j < kj; ++j) {
        const int col = j0 + j;
        double zr = 0.0;
        if (B) {
            double d, e;
            two_sum(B[(int64_t)col * ldb + t], -s[j], d, e);
            zr = d + (e - c[j]);
        }
        if (Rout) Rout[(int64_t)col * ldr + t] = zr;
        if (Y) Y[(int64_t)col * ldy + t] = s[j] + c[j];
        if (Z) Z[(int64_t)col * ldz + t] = zr;
    }
}

template <bool DD, int KJ>
__global__ __launch_bounds__(ATX_T) void atx_kernel(ApplyArgs a, const double *xhi, const double *xlo, int64_t ldx,
                                                    const double *B, int64_t ldb, double *Rout, int64_t ldr,
                                                    double *Y, int64_t ldy, double *Z, int64_t ldz)
{
    atx_body<DD, KJ>(a, xhi, xlo, ldx, B, ldb, Rout, ldr, Y, ldy, Z, ldz, blockIdx.x, blockIdx.y);
}

template <bool DD, int KJ, bool SC>
__global__ __launch_bounds__(ATX_T) void atx_grouped(const AtxGroupArgs *gs)
{
    const AtxGroupArgs g = gs[blockIdx.z];
    atx_body<DD, KJ, SC>(g.a, g.xhi, g.xlo, g.ldx, g.B, g.ldb, g.Rout, g.ldr, g.Y, g.ldy, g.Z, g.ldz, blockIdx.x,
                     blockIdx.y);
}

// Compensated A^T x with x in scalar registers.  x (hi and lo) is packed per
// block of 8 right-hand sides as xpk[jb][i][0..8) = hi and [8..16) = lo, rows
// padded with zeros to a multiple of 8 (m8).  The packed addresses are
// uniform across the wave, so they are read with scalar loads and the Dot2
// updates take x as scalar operands: the pass reads no LDS, and its rate is
// set by the vector FP64 instructions.  One thread per column t of A; A is
// read once per block of 8 right-hand sides.
constexpr int ATS_T = 256;
constexpr int ATS_KJ = 8;

__global__ void pack_x_kernel(const double *xhi, const double *xlo, int64_t ldx, int m, int m8, int k, double *xpk)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int kb = (k + ATS_KJ - 1) / ATS_KJ;
    if (e >= (int64_t)kb * m8 * 2 * ATS_KJ) return;
    const int w = (int)(e % (2 * ATS_KJ));
    const int64_t r = e / (2 * ATS_KJ);
    const int i = (int)(r % m8), jb = (int)(r / m8);
    const int j = jb * ATS_KJ + (w % ATS_KJ);
    double v = 0.0;
    if (i < m && j < k) {
        if (w < ATS_KJ) v = xhi[(int64_t)j * ldx + i];
        else if (xlo) v = xlo[(int64_t)j * ldx + i];
    }
    xpk[e] = v;
}

__global__ __launch_bounds__(ATS_T) void atx_dd_sx_kernel(int m, int m8, int n, int k, const double *__restrict__ A,
                                                          int64_t lda, const double *__restrict__ xpk,
                                                          const double *__restrict__ B, int64_t ldb,
                                                          double *__restrict__ Rout, int64_t ldr,
                                                          double *__restrict__ Y, int64_t ldy,
                                                          double *__restrict__ Z, int64_t ldz)
{
    const int64_t t = (int64_t)blockIdx.x * ATS_T + threadIdx.x;
    const int jb = blockIdx.y, j0 = jb * ATS_KJ;
    const int kj = min(ATS_KJ, k - j0);
    const double *xp = xpk + (int64_t)jb * m8 * 2 * ATS_KJ;
    const bool active = t < n;
    const double *ap = A + (active ? t : 0);
    double s[ATS_KJ], c[ATS_KJ];
#pragma unroll
    for (int j = 0; j < ATS_KJ; ++j) { s[j] = 0.0; c[j] = 0.0; }
    auto update = [&](const double (&av)[8], int i0) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double *xr = xp + (int64_t)(i0 + u) * 2 * ATS_KJ;
#pragma unroll
            for (int j = 0; j < ATS_KJ; ++j) {
                dot2_acc(av[u], xr[j], s[j], c[j]);
                c[j] = __builtin_fma(av[u], xr[ATS_KJ + j], c[j]);
            }
        }
    };
    // Groups of 8 rows inside m: straight-line, two register slots taken in
    // turn, the next group's loads in flight during this group's updates (the
    // last pair reloads its final group rather than branch: a conditional or
    // masked load is compiled into a branch that waits for it, and a copy
    // between slots waits at the loop's back edge).  Then the ragged group,
    // masked.
    const int full = m / 8;
    auto load8 = [&](double (&av)[8], int g) {
#pragma unroll
        for (int u = 0; u < 8; ++u) av[u] = ap[(int64_t)(8 * g + u) * lda];
    };
    int g = 0;
    if (full > 0) {
        double a0[8], a1[8];
        load8(a0, 0);
        for (; g + 2 <= full; g += 2) {
            load8(a1, g + 1);
            update(a0, 8 * g);
            load8(a0, min(g + 2, full - 1));
            update(a1, 8 * g + 8);
        }
        if (g < full) {  // odd count: slot 0 holds the last full group
            update(a0, 8 * g);
            ++g;
        }
    }
    const int i0 = 8 * g;
    if (i0 < m8) {
        double av[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u;
            const double v = ap[(int64_t)(i < m ? i : m - 1) * lda];
            av[u] = i < m ? v : 0.0;
        }
        update(av, i0);
    }
    if (!active) return;
    for (int j = 0; j < kj; ++j) {
        const int col = j0 + j;
        double zr = 0.0;
        if (B) {
            double d, e;
            two_sum(B[(int64_t)col * ldb + t], -s[j], d, e);
            zr = d + (e - c[j]);
        }
        if (Rout) Rout[(int64_t)col * ldr + t] = zr;
        if (Y) Y[(int64_t)col * ldy + t] = s[j] + c[j];
        if (Z) Z[(int64_t)col * ldz + t] = zr;
    }
}

// Plain binary64 A B with B in scalar registers.  B is packed as
// bpk[jb][t][16] (16 right-hand sides per block jb, zero past n and k), so
// the 16 values of one t are uniform across the wave and are read with scalar
// loads.  A block is
// four waves on one 64-row strip of A and one split of the columns t; the
// split is cut into chunks of 16 columns dealt to the waves in turn.  A wave
// loads its chunk (64 rows x 16 doubles) with coalesced pair loads, one
// chunk ahead, into a tile of its own in LDS, and each lane reads back its
// row: one LDS read per 16 FMAs, so the pass is bound by reading A.  The
// four waves' sums are combined in LDS in wave order and written as
// part[split][j][row].  (A compensated form of this kernel, 8 right-hand
// sides per block to fit the accumulator pairs, measured slower than the
// LDS-staged Dot2 pass above, which the refinement keeps.)
constexpr int ABS_RH = 16;           // right-hand sides per block (packed width)
constexpr int ABS_TC = 16;           // columns of A per chunk
constexpr int ABS_LD = ABS_TC + 1;   // LDS row stride in doubles: row reads free of bank conflicts
constexpr int ABS_WAVES = 4;

__global__ void pack_rhs_kernel(const double *B, int64_t ldb, int n, int k, int64_t tpad, double *bpk)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int kb = (k + ABS_RH - 1) / ABS_RH;
    if (e >= (int64_t)kb * tpad * ABS_RH) return;
    const int jj = (int)(e % ABS_RH);
    const int64_t r = e / ABS_RH;
    const int64_t t = r % tpad;
    const int j = (int)(r / tpad) * ABS_RH + jj;
    bpk[e] = (t < n && j < k) ? B[(int64_t)j * ldb + t] : 0.0;
}

// V2: A 16-byte aligned with even lda, so full chunks load as double pairs
template <bool V2>
__global__ __launch_bounds__(256) void ab_sx_kernel(int m, int n, int k, const double *__restrict__ A, int64_t lda,
                                                    const double *__restrict__ bpk, int64_t tpad, int splits,
                                                    double *__restrict__ part)
{
    constexpr int RH = ABS_RH;
    constexpr int TILE = 64 * ABS_LD;
    constexpr int RED = (ABS_WAVES - 1) * RH * 64;
    __shared__ double lds[ABS_WAVES * TILE > RED ? ABS_WAVES * TILE : RED];
    // the wave index through readfirstlane, so that chunk and B addresses are
    // known to be uniform and B is read with scalar loads
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r0 = blockIdx.x * 64, split = blockIdx.y, jb = blockIdx.z;
    const int64_t nch = (n + ABS_TC - 1) / ABS_TC;
    const int64_t per = (nch + splits - 1) / splits;
    const int64_t c0 = (int64_t)split * per, c1 = min(nch, c0 + per);
    double *tile = lds + w * TILE;
    const double *bp = bpk + (int64_t)jb * tpad * RH;

    // loader: lane (rsub, seg) takes columns 2 seg, 2 seg + 1 of rows
    // rsub + 8 q, q = 0..7 (rows past m are clamped and read as zero)
    const int seg = lane & 7, rsub = lane >> 3;
    int64_t roff[8];
    bool rok[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int row = r0 + rsub + 8 * q;
        rok[q] = row < m;
        roff[q] = (int64_t)(rok[q] ? row : m - 1) * lda;
    }
    double2 nx[8];
    auto load = [&](int64_t ch) {
        const int64_t t = ch * ABS_TC + 2 * seg;
        if (V2 && (ch + 1) * ABS_TC <= n) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double2 v = *reinterpret_cast<const double2 *>(A + roff[q] + t);
                nx[q].x = rok[q] ? v.x : 0.0;
                nx[q].y = rok[q] ? v.y : 0.0;
            }
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double v0 = A[roff[q] + (t < n ? t : n - 1)];
                const double v1 = A[roff[q] + (t + 1 < n ? t + 1 : n - 1)];
                nx[q].x = (rok[q] && t < n) ? v0 : 0.0;
                nx[q].y = (rok[q] && t + 1 < n) ? v1 : 0.0;
            }
        }
    };

    double s[RH];
#pragma unroll
    for (int j = 0; j < RH; ++j) s[j] = 0.0;
    int64_t ch = c0 + w;
    if (ch < c1) load(ch);
    for (; ch < c1; ch += ABS_WAVES) {
        // one wave writes and reads its own tile, in program order: no barrier
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            tile[(rsub + 8 * q) * ABS_LD + 2 * seg] = nx[q].x;
            tile[(rsub + 8 * q) * ABS_LD + 2 * seg + 1] = nx[q].y;
        }
        if (ch + ABS_WAVES < c1) load(ch + ABS_WAVES);
        double a[ABS_TC];
#pragma unroll
        for (int tt = 0; tt < ABS_TC; ++tt) a[tt] = tile[lane * ABS_LD + tt];
        const double *bt = bp + ch * ABS_TC * RH;
#pragma unroll
        for (int tt = 0; tt < ABS_TC; ++tt) {
#pragma unroll
            for (int j = 0; j < RH; ++j) s[j] = __builtin_fma(a[tt], bt[tt * RH + j], s[j]);
        }
    }
    // combine the four waves in order 0, 1, 2, 3
    __syncthreads();
    if (w > 0) {
        double *rp = lds + (w - 1) * RH * 64;
#pragma unroll
        for (int j = 0; j < RH; ++j) rp[j * 64 + lane] = s[j];
    }
    __syncthreads();
    if (w != 0) return;
    for (int v = 0; v < ABS_WAVES - 1; ++v) {
        const double *rp = lds + v * RH * 64;
#pragma unroll
        for (int j = 0; j < RH; ++j) s[j] += rp[j * 64 + lane];
    }
    const int row = r0 + lane;
    if (row >= m) return;
    const int64_t base = (int64_t)split * m * k;
#pragma unroll
    for (int j = 0; j < RH; ++j) {
        const int col = jb * RH + j;
        if (col < k) part[base + (int64_t)col * m + row] = s[j];
    }
}

// right-hand sides per block of the A^T x pass (accumulators per thread)
// (the compensated form keeps 16: twice the accumulators cost more in
// occupancy than the extra pass over A)
inline int atx_kj(int k, int dd) { return dd ? 16 : (k > 32 ? 64 : (k > 16 ? 32 : 16)); }

// x = (xhi, xlo) + d in double-double, and norms = (|d|^2, |x_hi|^2), by one
// block (any multiple of 64 threads, at most 1024).  Each thread loads U
// elements' operands before any arithmetic; indices past total are clamped
// for the loads and masked out of the stores and the norms.
__device__ __forceinline__ void dd_update_body(double *__restrict__ xhi, double *__restrict__ xlo,
                                               const double *__restrict__ D, int total, double *norms)
{
#pragma clang fp contract(off)
    constexpr int U = 4;
    __shared__ double red[2][16];
    const int nt = blockDim.x;
    double nd = 0.0, nx = 0.0;
    for (int e0 = threadIdx.x; e0 < total; e0 += U * nt) {
        double d[U], h[U], l[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = min(e0 + u * nt, total - 1);
            d[u] = D[e];
            h[u] = xhi[e];
            l[u] = xlo[e];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * nt;
            double sm, err;
            two_sum(h[u], d[u], sm, err);
            const double lo = l[u] + err;
            const double hi = sm + lo;
            const double in = e < total ? 1.0 : 0.0;
            nd += in * (d[u] * d[u]);
            nx += in * (hi * hi);
            if (e < total) {
                xlo[e] = lo - (hi - sm);
                xhi[e] = hi;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        nd += __shfl_xor(nd, o, 64);
        nx += __shfl_xor(nx, o, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = nd;
        red[1][w] = nx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int v = 0; v < nt / 64; ++v) {
            a += red[0][v];
            b += red[1][v];
        }
        norms[0] = a;
        norms[1] = b;
    }
}

__global__ __launch_bounds__(1024) void dd_update_kernel(double *xhi, double *xlo, const double *D, int total,
                                                        double *norms)
{
    dd_update_body(xhi, xlo, D, total, norms);
}

__global__ __launch_bounds__(256) void dd_update_grouped(const DdGroupArgs *gs)
{
    const DdGroupArgs g = gs[blockIdx.x];
    dd_update_body(g.xhi, g.xlo, g.D, g.total, g.norms);
}

__device__ __forceinline__ void copy_cols_body(const double *src, int64_t lds, double *dst, int64_t ldd, int rows,
                                               int cols, double *zero_out, int64_t ldz, int64_t e,
                                               const double *rs = nullptr)
{
    if (e >= (int64_t)rows * cols) return;
    const int j = (int)(e / rows), i = (int)(e % rows);
    const double v = src[(int64_t)j * lds + i];
    dst[(int64_t)j * ldd + i] = rs ? v * rs[i] : v;
    if (zero_out) zero_out[(int64_t)j * ldz + i] = 0.0;
}

__global__ void copy_cols_kernel(const double *src, int64_t lds, double *dst, int64_t ldd, int rows, int cols,
                                 double *zero_out, int64_t ldz)
{
    copy_cols_body(src, lds, dst, ldd, rows, cols, zero_out, ldz, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void sub_cols_kernel(const double *B, int64_t ldb, const double *C, int64_t ldc, double *out, int64_t ldo,
                                int rows, int cols)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cols) return;
    const int j = (int)(e / rows), i = (int)(e % rows);
    const double v = B[(int64_t)j * ldb + i] - C[(int64_t)j * ldc + i];
    out[(int64_t)j * ldo + i] = v;
}

// Outputs from a final null projection r: Y = B - r and Z = r, each
// optional.  One thread reads B and r at an index before it writes there, so
// Y or Z may be B itself.
__device__ __forceinline__ void finish_cols_body(const FinishGroupArgs &g, int64_t e)
{
    if (e >= (int64_t)g.rows * g.cols) return;
    const int j = (int)(e / g.rows), i = (int)(e % g.rows);
    const double r = g.r[(int64_t)j * g.ldr + i];
    const double y = g.Y ? g.B[(int64_t)j * g.ldb + i] - r : 0.0;
    if (g.Y) g.Y[(int64_t)j * g.ldy + i] = y;
    if (g.Z) g.Z[(int64_t)j * g.ldz + i] = r;
}

__global__ void finish_cols_kernel(FinishGroupArgs g)
{
    finish_cols_body(g, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void finish_cols_grouped(const FinishGroupArgs *gs)
{
    finish_cols_body(gs[blockIdx.y], (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void copy_cols_grouped(const CopyGroupArgs *gs)
{
    const CopyGroupArgs g = gs[blockIdx.y];
    copy_cols_body(g.src, g.lds, g.dst, g.ldd, g.rows, g.cols, g.zero_out, g.ldz,
                   (int64_t)blockIdx.x * blockDim.x + threadIdx.x, g.rs);
}

}  // namespace

hipError_t ab_partial_f64(const ApplyArgs &a, const double *B, int64_t ldb, int splits, double *part_hi,
                          double *part_lo, int dd, hipStream_t stream)
{
    const int kj = ab_kj(a.k, dd);
    dim3 grid((a.m + AB_RB - 1) / AB_RB, splits, (a.k + kj - 1) / kj);
#define AB_CASE(DD_, KJ_)                                                                                            \
    if (!!dd == DD_ && kj == KJ_)                                                                                    \
        hipLaunchKernelGGL((ab_partial_kernel<DD_, KJ_>), grid, dim3(256), 0, stream, a, B, ldb, splits, part_hi, \
                           part_lo);
    AB_CASE(true, 16) AB_CASE(true, 32) AB_CASE(false, 16) AB_CASE(false, 32) AB_CASE(false, 64)
#undef AB_CASE
    return hipGetLastError();
}

int ab_sx_splits(int64_t m, int64_t n, int64_t k, int cu_count)
{
    // about two blocks per compute unit, at least four chunks per wave
    const int64_t tiles = ((m + 63) / 64) * ((k + ABS_RH - 1) / ABS_RH);
    const int64_t nch = (n + ABS_TC - 1) / ABS_TC;
    const int64_t want = (2 * (int64_t)cu_count + tiles - 1) / tiles;
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, nch / (4 * ABS_WAVES)));
}

hipError_t ab_sx_f64(const ApplyArgs &a, const double *B, int64_t ldb, double *bpk, int splits, double *part,
                     hipStream_t stream)
{
    if (a.m <= 0 || a.n <= 0 || a.k <= 0) return hipSuccess;
    if (splits < 1) return hipErrorInvalidValue;
    const int64_t tpad = (a.n + ABS_TC - 1) / ABS_TC * ABS_TC;
    const int kb = (a.k + ABS_RH - 1) / ABS_RH;
    const int64_t total = (int64_t)kb * tpad * ABS_RH;
    hipLaunchKernelGGL(pack_rhs_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, B, ldb, a.n, a.k,
                       tpad, bpk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const bool v2 = (a.lda % 2 == 0) && (reinterpret_cast<uintptr_t>(a.A) % 16 == 0);
    const dim3 grid((unsigned)((a.m + 63) / 64), (unsigned)splits, (unsigned)kb);
    if (v2)
        hipLaunchKernelGGL((ab_sx_kernel<true>), grid, dim3(64 * ABS_WAVES), 0, stream, a.m, a.n, a.k, a.A, a.lda,
                           bpk, tpad, splits, part);
    else
        hipLaunchKernelGGL((ab_sx_kernel<false>), grid, dim3(64 * ABS_WAVES), 0, stream, a.m, a.n, a.k, a.A, a.lda,
                           bpk, tpad, splits, part);
    return hipGetLastError();
}

hipError_t ab_reduce_f64(const double *part_hi, const double *part_lo, int m, int k, int splits, int dd, double *out,
                         int64_t ldo, hipStream_t stream)
{
    const int64_t total = (int64_t)m * k;
    // 64-thread blocks: m k is small (thousands), so spread it over more CUs
    hipLaunchKernelGGL(ab_reduce_kernel, dim3((unsigned)((total + 63) / 64)), dim3(64), 0, stream, part_hi, part_lo, m,
                       k, splits, dd, out, ldo);
    return hipGetLastError();
}

hipError_t atx_f64(const ApplyArgs &a, const double *Xhi, const double *Xlo, int64_t ldx, const double *B,
                   int64_t ldb, double *Rout, int64_t ldr, double *Y, int64_t ldy, double *Z, int64_t ldz, int dd,
                   hipStream_t stream, double *xpk)
{
    if (dd && xpk) {
        const int m8 = (a.m + 7) / 8 * 8, kb = (a.k + ATS_KJ - 1) / ATS_KJ;
        const int64_t total = (int64_t)kb * m8 * 2 * ATS_KJ;
        hipLaunchKernelGGL(pack_x_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, Xhi, Xlo, ldx,
                           a.m, m8, a.k, xpk);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        dim3 grid((unsigned)((a.n + ATS_T - 1) / ATS_T), kb);
        hipLaunchKernelGGL(atx_dd_sx_kernel, grid, dim3(ATS_T), 0, stream, a.m, m8, a.n, a.k, a.A, a.lda, xpk, B,
                           ldb, Rout, ldr, Y, ldy, Z, ldz);
        return hipGetLastError();
    }
    const int kj = atx_kj(a.k, dd);
    dim3 grid((unsigned)((a.n + ATX_T - 1) / ATX_T), (a.k + kj - 1) / kj);
#define ATX_CASE(DD_, KJ_)                                                                                          \
    if (!!dd == DD_ && kj == KJ_)                                                                                   \
        hipLaunchKernelGGL((atx_kernel<DD_, KJ_>), grid, dim3(ATX_T), 0, stream, a, Xhi, Xlo, ldx, B, ldb, Rout, ldr, \
                           Y, ldy, Z, ldz);
    ATX_CASE(true, 16) ATX_CASE(false, 16) ATX_CASE(false, 32) ATX_CASE(false, 64)
#undef ATX_CASE
    return hipGetLastError();
}

hipError_t dd_update_f64(double *Xhi, double *Xlo, const double *D, int m, int k, double *norms, hipStream_t stream)
{
    hipLaunchKernelGGL(dd_update_kernel, dim3(1), dim3(1024), 0, stream, Xhi, Xlo, D, m * k, norms);
    return hipGetLastError();
}

hipError_t sub_cols_f64(const double *B, int64_t ldb, const double *C, int64_t ldc, double *out, int64_t ldo, int rows,
                        int cols, hipStream_t stream)
{
    const int64_t total = (int64_t)rows * cols;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(sub_cols_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, B, ldb, C, ldc,
                       out, ldo, rows, cols);
    return hipGetLastError();
}

hipError_t copy_cols_f64(const double *src, int64_t lds, double *dst, int64_t ldd, int rows, int cols,
                         double *zero_out, int64_t ldz, hipStream_t stream)
{
    const int64_t total = (int64_t)rows * cols;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(copy_cols_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, src, lds, dst,
                       ldd, rows, cols, zero_out, ldz);
    return hipGetLastError();
}

hipError_t ab_partial_grouped_f64(const AbGroupArgs *d, int count, int max_m, int max_k, int max_splits, int dd,
                                  hipStream_t stream)
{
    if (count <= 0 || max_m <= 0 || max_k <= 0) return hipSuccess;
    const int kj = ab_kj(max_k, dd);
    const int kb = (max_k + kj - 1) / kj;
    dim3 grid((max_m + AB_RB - 1) / AB_RB, max_splits, count * kb);
#define AB_CASE(DD_, KJ_) \
    if (!!dd == DD_ && kj == KJ_) hipLaunchKernelGGL((ab_partial_grouped<DD_, KJ_>), grid, dim3(256), 0, stream, d, kb);
    AB_CASE(true, 16) AB_CASE(true, 32) AB_CASE(false, 16) AB_CASE(false, 32) AB_CASE(false, 64)
#undef AB_CASE
    return hipGetLastError();
}

hipError_t ab_reduce_grouped_f64(const AbGroupArgs *d, int count, int64_t max_mk, int dd, hipStream_t stream)
{
    if (count <= 0 || max_mk <= 0) return hipSuccess;
    hipLaunchKernelGGL(ab_reduce_grouped, dim3((unsigned)((max_mk + 255) / 256), count), dim3(256), 0, stream, d, dd);
    return hipGetLastError();
}

hipError_t atx_grouped_f64(const AtxGroupArgs *d, int count, int64_t max_n, int max_k, int dd, int scaled,
                           hipStream_t stream)
{
    if (count <= 0 || max_n <= 0 || max_k <= 0) return hipSuccess;
    const int kj = atx_kj(max_k, dd);
    dim3 grid((unsigned)((max_n + ATX_T - 1) / ATX_T), (max_k + kj - 1) / kj, count);
#define ATX_CASE(DD_, KJ_) \
    if (!!dd == DD_ && kj == KJ_)                                                                                    \
        hipLaunchKernelGGL(scaled ? (atx_grouped<DD_, KJ_, true>) : (atx_grouped<DD_, KJ_, false>), grid, dim3(ATX_T), \
                           0, stream, d);
    ATX_CASE(true, 16) ATX_CASE(false, 16) ATX_CASE(false, 32) ATX_CASE(false, 64)
#undef ATX_CASE
    return hipGetLastError();
}

hipError_t dd_update_grouped_f64(const DdGroupArgs *d, int count, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(dd_update_grouped, dim3(count), dim3(256), 0, stream, d);
    return hipGetLastError();
}

hipError_t finish_cols_f64(const FinishGroupArgs &g, hipStream_t stream)
{
    const int64_t total = (int64_t)g.rows * g.cols;
    if (total == 0 || (!g.Y && !g.Z)) return hipSuccess;
    hipLaunchKernelGGL(finish_cols_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, g);
    return hipGetLastError();
}

hipError_t finish_cols_grouped_f64(const FinishGroupArgs *d, int count, int64_t max_total, hipStream_t stream)
{
    if (count <= 0 || max_total <= 0) return hipSuccess;
    hipLaunchKernelGGL(finish_cols_grouped, dim3((unsigned)((max_total + 255) / 256), count), dim3(256), 0, stream, d);
    return hipGetLastError();
}

hipError_t copy_cols_grouped_f64(const CopyGroupArgs *d, int count, int64_t max_total, hipStream_t stream)
{
    if (count <= 0 || max_total <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_cols_grouped, dim3((unsigned)((max_total + 255) / 256), count), dim3(256), 0, stream, d);
    return hipGetLastError();
}

}  // namespace rt
