// Binary64 GEMM on the gfx950 matrix cores (v_mfma_f64_16x16x4_f64), LDS-tiled.
//
// One kernel serves every dense contraction of the preconditioner: the
// triangular products with the explicitly inverted factor (P^- of eq. scary),
// the Gram (P^{-1}A)(P^{-1}A)^T (steps a-e of Sec. 4), the blocked Cholesky
// updates and the right-looking triangular solves.  256 threads = 4 waves in
// a 2 x 2 arrangement; each wave owns (BM/2) x (BN/2) of the output as
// 16 x 16 MFMA tiles; K advances in chunks of 16 staged through LDS.
#include "rt_common.h"

namespace rt {

namespace {

// K per chunk: 16 for 64 x 64 tiles, 32 for 128 x 128 tiles (each measured
// faster for its tile: the larger tile has the MFMA work to cover the deeper
// loads, the smaller one keeps two blocks per compute unit).
template <int BM>
struct Chunk { static constexpr int value = BM >= 128 ? 32 : 16; };

// LDS layout of an operand tile with MN extent T: a K-contiguous operand is
// kept MN-major ([T][KC+1], k fastest, as loaded), an MN-contiguous one
// K-major ([KC][T+16]); both paddings make the coalesced stores and the MFMA
// operand reads (16 consecutive MN indices x 4 consecutive k per wave)
// bank-conflict free.
template <int T, bool KCONTIG, int KC>
struct TileLayout {
    static constexpr int size = KCONTIG ? T * (KC + 1) : KC * (T + 16);
    __device__ static int at(int mn, int k) { return KCONTIG ? mn * (KC + 1) + k : k * (T + 16) + mn; }
};

// Chunks of K in flight: the loads of chunk t + RING - 1 are issued before
// chunk t is multiplied, so RING - 1 chunk products hide a load's latency.
// Two slots (one chunk ahead, LDS double buffered): deeper rings defeat the
// compiler's memory counters at the loop back edge (it then waits for every
// load before issuing the next), so small products get their latency hiding
// from more resident blocks instead (more K splits).
template <int BM>
struct Ring { static constexpr int value = 2; };

// One BM x BN output tile (bx, by) of split bz.  Tiles outside the problem
// (possible in grouped launches, whose grid covers the largest member)
// return at once; the whole block takes the same branch.
//
// Operand chunks travel global -> registers (a ring of RING slots) -> LDS
// (double buffered).  Every load is issued unconditionally from a clamped
// address and zeroed by a select when out of range, so the loads stay
// straight-line and the compiler's counters let RING - 1 chunks remain in
// flight.  A row gather of B (along K) reads its indices one chunk ahead of
// the data they address, in a ring of their own; a row gather of A (along M)
// is resolved once.
template <int BM, int BN, bool A_KC, bool B_KC, bool GB>
__device__ __forceinline__ void gemm_f64_tile(const GemmArgs &g, int bx, int by, int bz)
{
    constexpr int KC = Chunk<BM>::value;
    using LA = TileLayout<BM, A_KC, KC>;
    using LB = TileLayout<BN, B_KC, KC>;
    __shared__ double As[2][LA::size];
    __shared__ double Bs[2][LB::size];
    constexpr int TM = BM / 32, TN = BN / 32;
    constexpr int NA = BM * KC / 256, NB = BN * KC / 256;  // elements per thread and chunk
    constexpr int R = Ring<BM>::value;
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
    if (i0 >= g.M || j0 >= g.N || bz >= (g.ksplit > 1 ? g.ksplit : 1)) return;
    int kbeg = 0, kend = g.K;
    if (g.ksplit > 1) {
        int ks = (g.K + g.ksplit - 1) / g.ksplit;
        ks = (ks + KC - 1) / KC * KC;
        kbeg = bz * ks;
        kend = min(g.K, kbeg + ks);
    }
    if (g.a_lower) kend = min(kend, i0 + BM);
    const int nch = kend > kbeg ? (kend - kbeg + KC - 1) / KC : 0;

    // per-element coordinates (consecutive threads along the operand's
    // contiguous dimension) and the loop-invariant parts of the addresses
    int a_ii[NA], a_kk[NA], b_jj[NB], b_kk[NB];
    int64_t a_row[NA], b_col[NB];
    bool a_in[NA], b_in[NB];
#pragma unroll
    for (int e = 0; e < NA; ++e) {
        const int x = tid + 256 * e;
        a_ii[e] = A_KC ? x / KC : x % BM;
        a_kk[e] = A_KC ? x % KC : x / BM;
        const int i = i0 + a_ii[e];
        a_in[e] = i < g.M;
        const int ic = a_in[e] ? i : g.M - 1;
        a_row[e] = (g.a_gather ? (int64_t)g.a_gather[ic] : (int64_t)ic) * g.a_i;
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
        const int x = tid + 256 * e;
        b_jj[e] = B_KC ? x / KC : x % BN;
        b_kk[e] = B_KC ? x % KC : x / BN;
        const int j = j0 + b_jj[e];
        b_in[e] = j < g.N;
        b_col[e] = (int64_t)(b_in[e] ? j : g.N - 1) * g.b_j;
    }

    double ra[R][NA], rb[R][NB];
    int gi[R][NB];
    (void)gi;
    auto load_idx = [&](int s, int c) {
        if constexpr (GB) {
#pragma unroll
            for (int e = 0; e < NB; ++e) {
                const int k = kbeg + c * KC + b_kk[e];
                gi[s][e] = g.b_gather[k < kend ? k : kend - 1];
            }
        }
    };
    auto load = [&](int s, int c) {
        const int k0 = kbeg + c * KC;
#pragma unroll
        for (int e = 0; e < NA; ++e) {
            const int k = k0 + a_kk[e];
            const bool ok = a_in[e] && k < kend && !(g.a_lower && k > i0 + a_ii[e]);
            const double v = g.A[a_row[e] + (int64_t)(k < kend ? k : kend - 1) * g.a_k];
            ra[s][e] = ok ? v : 0.0;
        }
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            const int k = k0 + b_kk[e];
            const bool ok = b_in[e] && k < kend;
            int64_t kr;
            if constexpr (GB) kr = gi[s][e];
            else kr = k < kend ? k : kend - 1;
            const double v = g.B[kr * g.b_k + b_col[e]];
            rb[s][e] = ok ? v : 0.0;
        }
    };
    auto stage = [&](int s, int buf) {
#pragma unroll
        for (int e = 0; e < NA; ++e) As[buf][LA::at(a_ii[e], a_kk[e])] = ra[s][e];
#pragma unroll
        for (int e = 0; e < NB; ++e) Bs[buf][LB::at(b_jj[e], b_kk[e])] = rb[s][e];
    };

    double4v acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = double4v{0.0, 0.0, 0.0, 0.0};

    if (nch > 0) {
        // prologue: indices of chunks 0..R-1, data of chunks 0..R-2, chunk 0 staged
#pragma unroll
        for (int s = 0; s < R; ++s) load_idx(s, s);
#pragma unroll
        for (int s = 0; s < R - 1; ++s) load(s, s);
        stage(0, 0);
        __syncthreads();
    }
    for (int t0 = 0; t0 < nch; t0 += R) {
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int t = t0 + u;
            if (t >= nch) break;
            // indices of chunk t + R (slot u held chunk t's), data of chunk t + R - 1
            load_idx(u, t + R);
            load((u + R - 1) % R, t + R - 1);
            const int buf = t & 1;
#pragma unroll
            for (int kk = 0; kk < KC; kk += 4) {
                double av[TM], bv[TN];
#pragma unroll
                for (int a = 0; a < TM; ++a)
                    av[a] = As[buf][LA::at(wm * (BM / 2) + a * 16 + (lane & 15), kk + (lane >> 4))];
#pragma unroll
                for (int b = 0; b < TN; ++b)
                    bv[b] = Bs[buf][LB::at(wn * (BN / 2) + b * 16 + (lane & 15), kk + (lane >> 4))];
#pragma unroll
                for (int a = 0; a < TM; ++a)
#pragma unroll
                    for (int b = 0; b < TN; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
            }
            if (t + 1 < nch) stage((u + 1) % R, buf ^ 1);
            __syncthreads();
        }
    }

    double *C = g.C + (g.ksplit > 1 ? (int64_t)bz * g.c_split : 0);
    const bool use_beta = (g.ksplit <= 1) && (g.beta != 0.0);
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wm * (BM / 2) + a * 16 + mfma16_row(lane, r);
                const int j = j0 + wn * (BN / 2) + b * 16 + mfma16_col(lane);
                if (i < g.M && j < g.N) {
                    const int64_t off = (int64_t)i * g.c_i + (int64_t)j * g.c_j;
                    double v = g.alpha * acc[a][b][r];
                    if (g.c_rs) v *= g.c_rs[i];
                    if (g.c_cs) v *= g.c_cs[j];
                    if (g.c_f32) {
                        reinterpret_cast<float *>(g.C)[off] = (float)v;
                    } else {
                        double *p = C + off;
                        if (use_beta) v += g.beta * *p;
                        *p = v;
                    }
                }
            }
}

// One-dimensional grid.  Tiles that read the same operand panel form a
// group (the M tiles of one N tile and K split, which share B; or all lower
// tiles of one K split, which share the panels of W).  In the plain order
// block b runs tile b: N tile fastest, then M tile, then split (lower tiles,
// then split, for a triangular C).  In the XCD order the tiles, numbered
// t = group * members + member, are cut into runs of `chunk` consecutive
// numbers and block b runs position (b / 8) % chunk of run
// ((b / 8) / chunk) * 8 + b % 8: the device deals consecutive workgroups
// round-robin to its 8 XCDs, each with its own L2, so each run executes on
// one XCD and reuses its panels from that XCD's L2.  chunk is the group size,
// or smaller when there are too few groups to occupy every XCD.
constexpr int XCDS = 8;

struct TileMap {
    int members, total, chunk, gn, gm, xcd;
};

template <int BM, int BN, bool A_KC, bool B_KC, bool GB>
__global__ __launch_bounds__(256) void gemm_f64_kernel(GemmArgs g, TileMap tm)
{
    const int b = blockIdx.x, q = b / XCDS;
    const int t = tm.xcd ? ((q / tm.chunk) * XCDS + b % XCDS) * tm.chunk + q % tm.chunk : b;
    if (t >= tm.total) return;
    if (g.c_lower) {
        gemm_f64_tile<BM, BN, A_KC, B_KC, GB>(g, t % tm.members, 0, t / tm.members);
    } else if (tm.xcd) {
        const int group = t / tm.members;
        gemm_f64_tile<BM, BN, A_KC, B_KC, GB>(g, group % tm.gn, t % tm.members, group / tm.gn);
    } else {
        const int r = t / tm.gn;
        gemm_f64_tile<BM, BN, A_KC, B_KC, GB>(g, t % tm.gn, r % tm.gm, r / tm.gm);
    }
}

// Grouped launch: member blockIdx.z / ksmax, split blockIdx.z % ksmax.
template <int BM, int BN, bool A_KC, bool B_KC, bool GB>
__global__ __launch_bounds__(256) void gemm_f64_grouped_kernel(const GemmArgs *gs, int ksmax)
{
    const GemmArgs g = gs[blockIdx.z / ksmax];
    gemm_f64_tile<BM, BN, A_KC, B_KC, GB>(g, blockIdx.x, blockIdx.y, blockIdx.z % ksmax);
}

template <int BM, int BN, bool GB>
hipError_t launch_tile_g(const GemmArgs &g, const TileMap &tm, hipStream_t s)
{
    const int64_t runs = (tm.total + tm.chunk - 1) / tm.chunk;
    const int64_t nb = tm.xcd ? (int64_t)tm.chunk * ((runs + XCDS - 1) / XCDS) * XCDS : tm.total;
    if (nb > INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nb);
    const bool akc = (g.a_k == 1), bkc = (g.b_k == 1);
    if (akc && bkc) hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, true, true, GB>), grid, dim3(256), 0, s, g, tm);
    else if (akc) hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, true, false, GB>), grid, dim3(256), 0, s, g, tm);
    else if (bkc) hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, false, true, GB>), grid, dim3(256), 0, s, g, tm);
    else hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, false, false, GB>), grid, dim3(256), 0, s, g, tm);
    return hipGetLastError();
}

template <int BM, int BN>
hipError_t launch_tile(const GemmArgs &g, hipStream_t s)
{
    const int gm = (g.M + BM - 1) / BM, gn = (g.N + BN - 1) / BN;
    const int ks = g.ksplit > 1 ? g.ksplit : 1;
    // groups sharing a panel: lower tiles of one split, or the M tiles of one
    // (N tile, split)
    TileMap tm;
    tm.members = g.c_lower ? gm * (gm + 1) / 2 : gm;
    const int ngroups = g.c_lower ? ks : gn * ks;
    tm.total = tm.members * ngroups;
    tm.gn = gn;
    tm.gm = gm;
    tm.chunk = ngroups >= XCDS ? tm.members : (tm.total + XCDS - 1) / XCDS;
    // measured: the XCD order pays for a triangular C and for 16 or more M
    // tiles per panel; with 8 M tiles (a 512-row product) the plain order
    // runs the same product about 20% faster
    tm.xcd = (g.c_lower || gm >= 16) ? 1 : 0;
    if (g.order == 1 && !g.c_lower) tm.xcd = 0;
    if (g.order == 2) tm.xcd = 1;
    return g.b_gather ? launch_tile_g<BM, BN, true>(g, tm, s) : launch_tile_g<BM, BN, false>(g, tm, s);
}

__device__ __forceinline__ void reduce_splits_body(const double *part, int64_t stride, int splits, int M, int N,
                                                   int64_t ld, double *out, int64_t ldo, int mirror, int64_t e)
{
    if (e >= (int64_t)M * N) return;
    const int i = (int)(e / N), j = (int)(e % N);
    if (mirror && j > i) return;
    double s = 0.0;
    for (int p = 0; p < splits; ++p) s += part[p * stride + (int64_t)i * ld + j];
    out[(int64_t)i * ldo + j] = s;
    if (mirror) out[(int64_t)j * ldo + i] = s;
}

__global__ void reduce_splits_kernel(const double *part, int64_t stride, int splits, int M, int N,
                                     int64_t ld, double *out, int64_t ldo, int mirror)
{
    reduce_splits_body(part, stride, splits, M, N, ld, out, ldo, mirror, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void reduce_splits_grouped(const ReduceGroupArgs *gs)
{
    const ReduceGroupArgs g = gs[blockIdx.y];
    reduce_splits_body(g.part, g.stride, g.splits, g.M, g.N, g.ld, g.out, g.ldo, g.mirror,
                       (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Square products of the Newton-Schulz iteration: out = scale (A B) +
// diag I for row-major m x m A, B and out.  One wave per 16 x 16 output tile
// over the whole of K: no split, hence no partials to write and reduce.  The
// operands (a few MB) are read straight from L2, k = k0 + 4 u + (lane / 16)
// for k-step u, so an A load covers 16 rows x 4 consecutive k and a B load
// 4 rows x 16 consecutive columns; the loads of the next 64 k are in flight
// while the 16 MFMAs of the current 64 run, alternating two accumulators.
// Groups inside the matrix run in a straight-line two-slot pipeline of
// unmasked loads (masked loads get turned into branches that wait for each
// load, and a conditional prefetch makes the compiler wait for it before
// the other slot's products); ragged groups follow one at a time, masked.
// With bsum the wave also writes the sum over its tile of (out - I)^2 to
// bsum[tile], tile = ti * ceil(m / 16) + tj.
constexpr int SQ_U = 16;  // k-steps of 4 per group

__device__ __forceinline__ void sq_load_full(double (&av)[SQ_U], double (&bv)[SQ_U], const double *ap,
                                             const double *bp, int m, int k0, int q)
{
#pragma unroll
    for (int u = 0; u < SQ_U; ++u) {
        const int k = k0 + 4 * u + q;
        av[u] = ap[k];
        bv[u] = bp[(int64_t)k * m];
    }
}

__device__ __forceinline__ void sq_load(double (&av)[SQ_U], double (&bv)[SQ_U], const double *ap, const double *bp,
                                        bool aok, bool bok, int m, int k0, int q)
{
#pragma unroll
    for (int u = 0; u < SQ_U; ++u) {
        const int k = k0 + 4 * u + q;
        const int kc = k < m ? k : m - 1;
        const double x = ap[kc];
        const double y = bp[(int64_t)kc * m];
        av[u] = (aok && k < m) ? x : 0.0;
        bv[u] = (bok && k < m) ? y : 0.0;
    }
}

__device__ __forceinline__ void sq_mma(const double (&av)[SQ_U], const double (&bv)[SQ_U], double4v &acc0,
                                       double4v &acc1)
{
#pragma unroll
    for (int u = 0; u < SQ_U; u += 2) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u + 1], bv[u + 1], acc1, 0, 0, 0);
    }
}

__global__ __launch_bounds__(64) void sq_mm_kernel(int m, const double *__restrict__ A, const double *__restrict__ B,
                                                   double *__restrict__ out, double scale, double diag,
                                                   double *__restrict__ bsum)
{
    const int tiles = (m + 15) / 16;
    const int ti = blockIdx.x / tiles, tj = blockIdx.x % tiles;
    const int lane = threadIdx.x, r = lane & 15, q = lane >> 4;
    const int ia = ti * 16 + r, jb = tj * 16 + r;
    const bool aok = ia < m, bok = jb < m;
    const double *ap = A + (int64_t)(aok ? ia : m - 1) * m;
    const double *bp = B + (bok ? jb : m - 1);
    double4v acc0 = double4v{0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
    double a0[SQ_U], b0[SQ_U], a1[SQ_U], b1[SQ_U];
    constexpr int KG = 4 * SQ_U;
    const int groups = (m + KG - 1) / KG;
    // groups with every k inside m, for a tile with every row and column inside
    const int full_groups = (ti * 16 + 16 <= m && tj * 16 + 16 <= m) ? m / KG : 0;
    int gi = 0;
    if (full_groups > 0) {
        sq_load_full(a0, b0, ap, bp, m, 0, q);
        for (; gi + 2 <= full_groups; gi += 2) {
            sq_load_full(a1, b1, ap, bp, m, (gi + 1) * KG, q);
            sq_mma(a0, b0, acc0, acc1);
            // the last pair reloads its final group instead of branching
            sq_load_full(a0, b0, ap, bp, m, min(gi + 2, full_groups - 1) * KG, q);
            sq_mma(a1, b1, acc0, acc1);
        }
        if (gi < full_groups) {  // odd count: slot 0 holds the last full group
            sq_mma(a0, b0, acc0, acc1);
            ++gi;
        }
    }
    for (; gi < groups; ++gi) {
        sq_load(a0, b0, ap, bp, aok, bok, m, gi * KG, q);
        sq_mma(a0, b0, acc0, acc1);
    }
    double qs = 0.0;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int i = ti * 16 + mfma16_row(lane, rr), j = tj * 16 + mfma16_col(lane);
        if (i < m && j < m) {
            const double id = (i == j) ? 1.0 : 0.0;
            const double v = scale * (acc0[rr] + acc1[rr]) + diag * id;
            out[(int64_t)i * m + j] = v;
            qs += (v - id) * (v - id);
        }
    }
    if (!bsum) return;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) qs += __shfl_xor(qs, o, 64);
    if (lane == 0) bsum[blockIdx.x] = qs;
}

// Skinny products of the M^{-1} application: out(i, j) = sum_r A[i lda + r]
// B[j ldb + r] for i < M, j < N (A row-major, B and out column-major, out[j
// ldo + i]), N a block of right-hand sides.  One block of 4 waves per 16 x 16
// tile of out; the waves take quarters of K and add their tiles through LDS
// in wave order, so one launch does the whole product.  Elements outside the
// problem are read from a shared zero (the address is selected, not the
// value), so every load is unconditional and the two register slots of 64 k
// stay in flight in turn.
__device__ double g_zero_mm = 0.0;

constexpr int SK_U = 16;  // k-steps of 4 per slot

__device__ __forceinline__ void skinny_load(double (&av)[SK_U], double (&bv)[SK_U], const double *ap,
                                            const double *bp, bool iok, bool jok, int k0, int ke, int q)
{
#pragma unroll
    for (int u = 0; u < SK_U; ++u) {
        const int k = k0 + 4 * u + q;
        const bool kin = k < ke;
        av[u] = *((iok && kin) ? ap + k : &g_zero_mm);
        bv[u] = *((jok && kin) ? bp + k : &g_zero_mm);
    }
}

__global__ __launch_bounds__(256) void skinny_mm_kernel(int M, int N, int K, const double *__restrict__ A,
                                                        int64_t lda, const double *__restrict__ B, int64_t ldb,
                                                        double *__restrict__ out, int64_t ldo)
{
    __shared__ double red[3][4][64];
    const int tm = (M + 15) / 16;
    const int ti = blockIdx.x % tm, tj = blockIdx.x / tm;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int i = ti * 16 + r, j = tj * 16 + r;
    const bool iok = i < M, jok = j < N;
    const double *ap = A + (int64_t)(iok ? i : 0) * lda;
    const double *bp = B + (int64_t)(jok ? j : 0) * ldb;
    constexpr int KG = 4 * SK_U;
    const int kq = ((K + 3) / 4 + KG - 1) / KG * KG;  // this wave's quarter, whole slots
    const int kb = w * kq, ke = min(K, kb + kq);
    double4v acc0 = double4v{0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
    double a0[SK_U], b0[SK_U], a1[SK_U], b1[SK_U];
    skinny_load(a0, b0, ap, bp, iok, jok, kb, ke, q);
    for (int k0 = kb; k0 < ke; k0 += 2 * KG) {
        skinny_load(a1, b1, ap, bp, iok, jok, k0 + KG, ke, q);
#pragma unroll
        for (int u = 0; u < SK_U; u += 2) {
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], b0[u], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u + 1], b0[u + 1], acc1, 0, 0, 0);
        }
        skinny_load(a0, b0, ap, bp, iok, jok, k0 + 2 * KG, ke, q);
#pragma unroll
        for (int u = 0; u < SK_U; u += 2) {
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], b1[u], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u + 1], b1[u + 1], acc1, 0, 0, 0);
        }
    }
    double v[4];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) v[rr] = acc0[rr] + acc1[rr];
    if (w > 0) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) red[w - 1][rr][lane] = v[rr];
    }
    __syncthreads();
    if (w != 0) return;
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) v[rr] += red[x][rr][lane];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int oi = ti * 16 + mfma16_row(lane, rr), oj = tj * 16 + mfma16_col(lane);
        if (oi < M && oj < N) out[(int64_t)oj * ldo + oi] = v[rr];
    }
}

}  // namespace

hipError_t skinny_mm_f64(int M, int N, int K, const double *A, int64_t lda, const double *B, int64_t ldb, double *out,
                         int64_t ldo, hipStream_t stream)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    if (K <= 0) return hipErrorInvalidValue;
    const int64_t nb = (int64_t)((M + 15) / 16) * ((N + 15) / 16);
    if (nb > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(skinny_mm_kernel, dim3((unsigned)nb), dim3(256), 0, stream, M, N, K, A, lda, B, ldb, out, ldo);
    return hipGetLastError();
}

hipError_t sq_mm_f64(int m, const double *A, const double *B, double *out, double scale, double diag, double *bsum,
                     hipStream_t stream)
{
    if (m <= 0) return hipSuccess;
    const int64_t nb = sq_mm_blocks(m);
    if (nb > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sq_mm_kernel, dim3((unsigned)nb), dim3(64), 0, stream, m, A, B, out, scale, diag, bsum);
    return hipGetLastError();
}

hipError_t gemm_f64(const GemmArgs &g, hipStream_t stream)
{
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (g.c_f32 && (g.beta != 0.0 || g.ksplit > 1)) return hipErrorInvalidValue;
    if (g.tile == 64 && g.tile_n == 128) return launch_tile<64, 128>(g, stream);
    if (g.tile == 128 && g.tile_n == 64) return launch_tile<128, 64>(g, stream);
    if (g.tile == 128) return launch_tile<128, 128>(g, stream);
    if (g.tile == 64) return launch_tile<64, 64>(g, stream);
    // triangular A (P^{-1}A): 64-row tiles measured faster than 128-row ones
    if (g.M >= 128 && g.N >= 128 && !g.a_lower && !g.small_tiles) return launch_tile<128, 128>(g, stream);
    return launch_tile<64, 64>(g, stream);
}

template <bool GB>
void launch_grouped(const GemmArgs *d_args, const GemmShape &shape, dim3 grid, int ks, hipStream_t stream)
{
    constexpr int BM = 64, BN = 64;
    if (shape.a_kc && shape.b_kc)
        hipLaunchKernelGGL((gemm_f64_grouped_kernel<BM, BN, true, true, GB>), grid, dim3(256), 0, stream, d_args, ks);
    else if (shape.a_kc)
        hipLaunchKernelGGL((gemm_f64_grouped_kernel<BM, BN, true, false, GB>), grid, dim3(256), 0, stream, d_args, ks);
    else if (shape.b_kc)
        hipLaunchKernelGGL((gemm_f64_grouped_kernel<BM, BN, false, true, GB>), grid, dim3(256), 0, stream, d_args, ks);
    else
        hipLaunchKernelGGL((gemm_f64_grouped_kernel<BM, BN, false, false, GB>), grid, dim3(256), 0, stream, d_args,
                           ks);
}

hipError_t gemm_f64_grouped(const GemmArgs *d_args, int count, const GemmShape &shape, hipStream_t stream)
{
    if (count <= 0 || shape.M <= 0 || shape.N <= 0) return hipSuccess;
    constexpr int BM = 64, BN = 64;
    const int gm = (shape.M + BM - 1) / BM, gn = (shape.N + BN - 1) / BN;
    const int ks = shape.ksplit > 1 ? shape.ksplit : 1;
    dim3 grid = shape.c_lower ? dim3(gm * (gm + 1) / 2, 1, count * ks) : dim3(gn, gm, count * ks);
    if (shape.b_gather) launch_grouped<true>(d_args, shape, grid, ks, stream);
    else launch_grouped<false>(d_args, shape, grid, ks, stream);
    return hipGetLastError();
}

hipError_t reduce_splits_f64(const double *part, int64_t stride, int splits, int M, int N, int64_t ld,
                             double *out, int64_t ldo, int mirror, hipStream_t stream)
{
    const int64_t total = (int64_t)M * N;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_splits_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream,
                       part, stride, splits, M, N, ld, out, ldo, mirror);
    return hipGetLastError();
}

hipError_t reduce_splits_grouped_f64(const ReduceGroupArgs *d, int count, int64_t max_total, hipStream_t stream)
{
    if (count <= 0 || max_total <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_splits_grouped, dim3((unsigned)((max_total + 255) / 256), count), dim3(256), 0, stream, d);
    return hipGetLastError();
}

}  // namespace rt
