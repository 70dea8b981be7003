// Internal declarations shared by the gfx950 kernels and the host runtime of
// the randomized orthogonal projection library.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace rt {

// ---------------------------------------------------------------- device
// Four binary64 accumulators of one lane of a 16x16x4 f64 MFMA.
typedef double double4v __attribute__((ext_vector_type(4)));

// Output element (row, col) held by lane `lane`, register r of a 16x16x4 f64
// MFMA tile: col = lane % 16, row = lane / 16 + 4 * r (measured on gfx950).
__device__ __forceinline__ int mfma16_row(int lane, int r) { return (lane >> 4) + 4 * r; }
__device__ __forceinline__ int mfma16_col(int lane) { return lane & 15; }

// Error-free transformations (Knuth's TwoSum, FMA-based TwoProd).  FMA
// contraction is switched off inside them: fusing the rounded product into a
// following sum would break the error-free property.
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
#pragma clang fp contract(off)
    s = a + b;
    double z = s - a;
    e = (a - (s - z)) + (b - z);
}
__device__ __forceinline__ void two_prod(double a, double b, double &p, double &e)
{
#pragma clang fp contract(off)
    p = a * b;
    e = __builtin_fma(a, b, -p);
}
// (s, c) += a*b, with s the running sum and c the accumulated error
// (Ogita-Rump-Oishi Dot2).
__device__ __forceinline__ void dot2_acc(double a, double b, double &s, double &c)
{
#pragma clang fp contract(off)
    double p, ep, t, es;
    two_prod(a, b, p, ep);
    two_sum(s, p, t, es);
    s = t;
    c += ep + es;
}

// ---------------------------------------------------------------- GEMM
// C(i,j) = alpha * sum_k A(i,k) B(k,j) + beta * C(i,j), binary64 on MFMA.
//   A(i,k) = A[ga(i)*a_i + k*a_k], ga(i) = a_gather ? a_gather[i] : i
//   B(k,j) = B[gb(k)*b_k + j*b_j], gb(k) = b_gather ? b_gather[k] : k
//   C(i,j) = C[i*c_i + j*c_j] (+ split * c_split for split-K partials)
// a_lower: A is lower triangular (A(i,k) = 0 for k > i, never read).
// c_lower: only output tiles on or below the diagonal are computed.
// ksplit > 1: grid.z = ksplit; each split writes alpha*partial (beta ignored)
// to C + split*c_split.
struct GemmArgs {
    int M, N, K;
    const double *A; int64_t a_i, a_k; const int32_t *a_gather;
    const double *B; int64_t b_k, b_j; const int32_t *b_gather;
    double *C; int64_t c_i, c_j; int64_t c_split;
    double alpha, beta;
    int a_lower, c_lower, ksplit;
    int small_tiles;  // 1: 64 x 64 tiles whatever M, N (more blocks for small products)
    int tile;         // 0: chosen from the shape; 64 or 128 forces the square tile size
    int tile_n;       // with tile: 0 square; 128 (tile 64) or 64 (tile 128) for a 64 x 128 or 128 x 64 tile
    int order;        // 0: tile order chosen from the shape; 1 plain; 2 XCD-grouped
    int c_f32;        // 1: C is binary32 (each result rounded once; beta must be 0, no K split)
    // optional output scalings: C[i][j] = alpha (A B)[i][j] c_rs[i] c_cs[j] (+ beta C)
    const double *c_rs = nullptr, *c_cs = nullptr;
};

// Launches GEMM with 64x64 or 128x128 tiles (chosen from M, N unless
// small_tiles is set).
hipError_t gemm_f64(const GemmArgs &g, hipStream_t stream);

// out = scale (A B) + diag I for row-major m x m A, B, out (leading dimension
// m; out must not alias A or B), one wave per 16 x 16 tile over the whole K.
// With bsum (sq_mm_blocks(m) doubles), bsum[tile] = sum over the tile of
// (out - I)^2.
hipError_t sq_mm_f64(int m, const double *A, const double *B, double *out, double scale, double diag, double *bsum,
                     hipStream_t stream);
inline int64_t sq_mm_blocks(int64_t m) { return ((m + 15) / 16) * ((m + 15) / 16); }

// out(i, j) = sum_r A[i lda + r] B[j ldb + r], i < M, j < N, r < K: A
// row-major, B and out column-major (out[j ldo + i]; out must not alias A or
// B).  One launch, one block per 16 x 16 tile of out, K split over its waves.
hipError_t skinny_mm_f64(int M, int N, int K, const double *A, int64_t lda, const double *B, int64_t ldb, double *out,
                         int64_t ldo, hipStream_t stream);

// Grouped GEMM: one launch over `count` problems whose GemmArgs live in
// device memory.  Every member must share the operand layouts (a_k == 1,
// b_k == 1) and c_lower given here; M, N and ksplit here are the maxima
// over the members (the grid covers them; smaller members skip the tiles
// they do not have).  64 x 64 tiles.
struct GemmShape {
    int M, N, ksplit;
    int a_kc, b_kc, c_lower;
    int b_gather;  // 1 when the members gather B's rows (all or none do)
};
hipError_t gemm_f64_grouped(const GemmArgs *d_args, int count, const GemmShape &shape, hipStream_t stream);
struct ReduceGroupArgs {
    const double *part; int64_t stride; int splits, M, N; int64_t ld; double *out; int64_t ldo; int mirror;
};
hipError_t reduce_splits_grouped_f64(const ReduceGroupArgs *d, int count, int64_t max_total, hipStream_t stream);

// out(i,j) = sum_{s<splits} part[s*stride + i*ld + j] for i,j < M x N
// (row-major, fixed summation order); if mirror, out(j,i) = out(i,j) too and
// only i >= j is summed.
hipError_t reduce_splits_f64(const double *part, int64_t stride, int splits, int M, int N,
                             int64_t ld, double *out, int64_t ldo, int mirror, hipStream_t stream);

// ---------------------------------------------------------------- reduced precision
// C(i,j) = alpha * sum_k A(i,k) B(k,j) on binary32 or bfloat16 MFMA with
// binary32 accumulation.  A/B are read from binary64 (x_dbl = 1) or binary32
// storage, multiplied by the optional power-of-two scales a_scale[i] /
// b_scale[j] and rounded; C is written as binary64 (c_dbl = 1) or binary32.
enum { MX_F32 = 0, MX_BF16 = 1, MX_BF16X3 = 2 };
struct GemmMxArgs {
    int M, N, K;
    const void *A; int a_dbl; int64_t a_i, a_k; const int32_t *a_gather; const float *a_scale;
    const void *B; int b_dbl; int64_t b_k, b_j; const int32_t *b_gather; const float *b_scale;
    void *C; int c_dbl; int64_t c_i, c_j, c_split;
    float alpha;
    int a_lower, c_lower, ksplit;
    int tile;         // binary32: 0 chosen from the shape; 64 or 128 forces it
};
hipError_t gemm_mx(const GemmMxArgs &g, int mode, hipStream_t stream);
// MX_BF16X3 takes binary32, K-contiguous, unscaled, ungathered, full operands
// with 16-byte aligned rows and K % 4 == 0 (the Gram of a row-major binary32
// matrix whose row length is a multiple of 4).
bool gemm_mx_bf16x3_ok(const GemmMxArgs &g);
// Grouped split-bfloat16 Gram (batches): the lower 256 x 128 tiles of each
// member's binary32 partials C = A B (binary32 A, B as MX_BF16X3 takes them),
// K split ksmax ways (members with fewer splits skip the extra ones).
hipError_t gemm_bf16x3_grouped_lower(const GemmMxArgs *d_args, int count, int max_m, int ksmax, hipStream_t stream);
// Grouped binary32 Gram of binary64 operands (batches): the lower 64 x 64
// tiles of each member's C = A B (A, B K-contiguous), K split ksmax ways
// (members with fewer splits skip the extra ones); then the binary64
// reduction of each member's binary32 partials into both triangles of its
// m x m output.
hipError_t gemm_f32_grouped_lower(const GemmMxArgs *d_args, int count, int max_m, int ksmax, hipStream_t stream);
struct ReduceF32GroupArgs { const float *part; int64_t stride; int splits; int m; double *out; };
hipError_t reduce_f32_grouped(const ReduceF32GroupArgs *d, int count, int max_m, hipStream_t stream);
// out(i,j) = sum_s part[s*stride + i*ld + j] / (sa[i] sb[j]) in binary64.
hipError_t reduce_f32_splits(const float *part, int64_t stride, int splits, int M, int N, int64_t ld,
                             const float *sa, const float *sb, double *out, int64_t ldo, int mirror,
                             hipStream_t stream);
// scale[i] = 2^-e, e = exponent of max_j |W_ij| (row-major m x n).
hipError_t row_pow2_scale(const void *W, int is_dbl, int64_t ldw, int m, int n, float *scale, hipStream_t stream);
hipError_t to_f32(const double *src, int64_t lds, float *dst, int64_t ldd, int m, int64_t n, hipStream_t stream);

// ---------------------------------------------------------------- exact int8 products
// Compensated residual products on the int8 matrix cores (digit splitting, see
// rt_ozaki.hip).  OZ_S signed base-128 digits per operand, digit pairs on the
// OZ_NDIAG diagonals s + t < OZ_NDIAG (digits counted from 0) kept, at most
// OZ_KMAX terms per int32 partial sum.
constexpr int OZ_S = 11;
constexpr int OZ_NDIAG = 12;
constexpr int64_t OZ_KMAX = 32768;
struct OzArgs {
    int R, K, k;               // A-operand rows, reduction length, right-hand sides
    const double *A; int64_t lda;
    const int *rowexp;         // exponent per A-operand row (columns of A for A^T x, rows for A r)
    const int8_t *dig;         // right-hand-side digits dig[(t kpad + c) Kpad + kk]
    int kpad; int64_t Kpad;    // right-hand sides and K padded to multiples of 64
    const int *bexp;           // exponent per right-hand side
    int64_t kchunk;            // K per split (multiple of 64, at most OZ_KMAX)
    const double *B; int64_t ldb; double *Rout; int64_t ldr;  // A^T x: Rout = B - A^T x
    double *ph, *pl;           // A r: double-binary64 partials [split][c][row]
};
// Splits of K for the A r product and the K per split.
int oz_splits(int64_t K, int64_t tiles, int cu_count);
int64_t oz_kchunk(int64_t K, int splits);
// colexp[j] (n) and rowexp[i] (m): exponents e with |A_ij| < 2^e over A's
// columns and rows (INT_MIN for an all-zero one).
hipError_t oz_exponents_f64(const double *A, int64_t lda, int m, int n, int *colexp, int *rowexp, hipStream_t s);
// Digits of the columns of the rows x k column-major vh (+ vl when not null)
// on per-column scales exp[c] (computed here): dig[(t kpad + c) rows_pad + row].
hipError_t oz_digits_f64(const double *vh, const double *vl, int64_t ld, int rows, int k, int64_t rows_pad, int kpad,
                         int *exp, int8_t *dig, hipStream_t s);
// trans = 1: Rout = B - A^T x (K = m, one split); trans = 0: split partials of A r.
hipError_t oz_mm(const OzArgs &g, int trans, int splits, hipStream_t s);

// ---------------------------------------------------------------- sketch
struct SketchTables {
    int64_t n, np, n1, n2, l;
    const int8_t *sign;      // np
    const int32_t *sigma;    // n1
    const int32_t *tau_inv;  // n2: tau_inv[u] = t2 with tau[t2] = u
    const double *tw1;       // n1/2 complex (re,im): exp(-2 pi i j / n1)
    const double *tw2;       // n2/2 complex: exp(-2 pi i j / n2)
    const double *twh;       // (np / tl) complex: exp(-2 pi i (j*tl) / np)
    const double *twl;       // tl complex: exp(-2 pi i j / np)
    const float *tw1f, *tw2f, *twhf, *twlf;  // binary32 copies of the four tables
    int tl_bits;             // log2(tl)
    const int32_t *sel_off;  // n1/2 + 2 offsets (CSR by k1-pair)
    const int32_t *sel;      // l entries of (k, part, q) triples
};
// S (m x l row-major, lds) = A G for the SRFT; Zbuf holds one row chunk of
// the intermediate (rows_chunk/2 x np complex binary64).
hipError_t sketch_f64(const SketchTables &t, const double *A, int64_t lda, int64_t m,
                      double *S, int64_t lds, double *zbuf, int64_t rows_chunk, hipStream_t stream);
// Grouped sketch over many problems (one launch pair per row chunk).
struct SketchGroupArgs {
    SketchTables t; const double *A; int64_t lda, m; double *S; int64_t lds;
    double *zbuf; int64_t rows_chunk;
    const double *cs = nullptr;  // optional: sketch of A diag(cs), each element scaled on load
};
// one_length: every member has the same padded Fourier length, hence one
// transform geometry (the pipelined passes need it).
struct SketchGroupShape { int64_t max_n1, max_n2, max_rows_chunk; int chunks; bool one_length = false; };
hipError_t sketch_grouped_f64(const SketchGroupArgs *d, int count, const SketchGroupShape &sh, hipStream_t stream);
// The same in binary32 arithmetic (binary32 tables and intermediate; S
// written in binary64 as the binary32 plan sketch does).
hipError_t sketch_grouped_f32(const SketchGroupArgs *d, int count, const SketchGroupShape &sh, hipStream_t stream);
// Same sketch with the transform in binary32 (A rounded on load; S written in
// binary64).
hipError_t sketch_f32(const SketchTables &t, const double *A, int64_t lda, int64_t m,
                      double *S, int64_t lds, double *zbuf, int64_t rows_chunk, hipStream_t stream);

// ---------------------------------------------------------------- pivoted QR
struct QrcpWork {
    unsigned *counter = nullptr;  // grid-barrier arrival counter (zeroed by the launcher)
    unsigned *flag = nullptr;     // spare
    int *err = nullptr;           // 1: wait timeout, 2: no finite pivot
    double *slots = nullptr;      // 2 * blocks * 2 doubles: candidate (norm^2, column)
    double *vbuf = nullptr;       // 2 * blocks * rows doubles: candidate columns
    double *cols = nullptr;       // null: columns kept in LDS; else blocks * 16 * rows doubles
    // optional Householder reflectors: step k writes v (v[k] = 1) to
    // V[k * rows + i] for rows i >= k, and its scalar to tau[k], so that
    // M Pi = H_0 ... H_{cols-1} R with H_k = I - tau_k v v^T (null: not kept)
    double *V = nullptr;
    double *tau = nullptr;
};
// Column-pivoted Householder QR of M = S^T (rows = l, cols = m; column j of M
// is row j of S, S row-major with ld lds).  R: m x m row-major, upper part
// written (the caller clears the strictly lower part).  piv: m int32.
hipError_t qrcp_f64(const double *S, int64_t lds, int rows, int cols, double *R, int32_t *piv,
                    const QrcpWork &w, int blocks, size_t lds_bytes_max, hipStream_t stream);
// Number of cooperative blocks for an l x m factorization (-1: unsupported);
// *global_cols = 1 when the columns must live in global memory (w.cols).
int qrcp_max_blocks(int rows, int cols, int cu_count, size_t lds_max, int *global_cols);
hipError_t zero_u32(unsigned *p, int n, hipStream_t stream);
// Register-resident cooperative form (256 or 512 threads per block; rows <= 8192).
// Block count from qrcp_reg_shape; the workspace is that of qrcp_f64 with
// G blocks (slots 4 G doubles, vbuf 2 G rows doubles).
bool qrcp_reg_shape(int rows, int cols, int cu_count, int *nc, int *rpt, int *blocks, int *threads);
hipError_t qrcp_reg_f64(const double *S, int64_t lds, int rows, int cols, double *R, int32_t *piv,
                        const QrcpWork &w, int cu_count, hipStream_t stream);

// Grouped register-resident form for a batch: member i is factored by its own
// group of G_i = ceil(cols_i / nc) blocks (the shape chosen for the largest
// member), synchronized only among themselves through the member's own
// workspace w (counter zeroed beforehand; slots 4 G_i and vbuf 2 G_i rows_i
// doubles).  A launch holds at most per_launch members, so that every group
// is resident at once; the same outputs and error codes as qrcp_reg_f64.
struct QrcpGrpArgs {
    const double *S; int64_t lds; int rows, cols;
    double *R; int32_t *piv;
    QrcpWork w;
    int G;
};
struct QrcpGrpShape {
    int nc = 0, rpt = 0, threads = 0, gmax = 0, per_launch = 0;
};
bool qrcp_grp_shape(int max_rows, int max_cols, int cu_count, QrcpGrpShape *sh);
hipError_t qrcp_grp_f64(const QrcpGrpArgs *d_args, int count, const QrcpGrpShape &sh, hipStream_t stream);

// Column-pivoted QR of one matrix per workgroup (no grid synchronization):
// M is column-major rows x cols (ld ldm) and is overwritten; R (cols x cols
// row-major, upper part written) and piv (cols) as for qrcp_f64; *err = 2
// when only NaN norms remain.  rows <= qrcp_wg_max_rows(), cols <=
// qrcp_wg_max_cols().
struct QrcpWgArgs {
    double *M; int64_t ldm; int rows, cols;
    double *R; int32_t *piv; int *err;
};
hipError_t qrcp_wg_f64(const QrcpWgArgs *d_args, int count, hipStream_t stream);
int qrcp_wg_max_rows();
int qrcp_wg_max_cols();

// ---------------------------------------------------------------- factor
// Inverse of each nb x nb diagonal block of the lower-triangular matrix
// L(i,j) = T[i*t_i + j*t_j] (j <= i), m x m; Dinv: nblk blocks of nb*nb
// row-major; the tail block is padded with the identity.
hipError_t tri_diag_inv_f64(const double *T, int64_t t_i, int64_t t_j, int m, int nb,
                            double *Dinv, hipStream_t stream);
// Cholesky of the nb x nb (or smaller tail) diagonal block at (b*nb, b*nb) of
// X (row-major, ldx): writes L's diagonal block into L (row-major, ldl, zeros
// above) and its inverse into Dinv + b*nb*nb; sets *err = 1 on breakdown.
hipError_t chol_diag_f64(const double *X, int64_t ldx, int m, int nb, int b, double *L, int64_t ldl,
                         double *Dinv, int *err, hipStream_t stream);
// Set a row-major m x n matrix to the identity (or zero if ident = 0).
// grouped forms of the factor kernels (one problem per blockIdx.y or .x)
struct CholGroupArgs { const double *X; int64_t ldx; int m; double *L; int64_t ldl; double *Dinv; int *err; };
// Cholesky G = L L^T of a row-major m x m SPD matrix in one cooperative
// launch (64 x 64 tiles owned by blocks, flags between tasks).  G's lower
// triangle is read and overwritten by the trailing updates; L's lower
// triangle is written (the caller clears the rest); Dinv gets the inverses of
// L's 64 x 64 diagonal blocks (identity-padded past m).  flags: nb + nb (nb +
// 1) / 2 words (nb = ceil(m / 64)) that hold no value equal to epoch before
// the call.  *err: 1 a pivot not positive and finite, 3 a wait timed out.
struct CholCoopArgs { double *G; int64_t ldg; int m; double *L; int64_t ldl; double *Dinv; int *err; unsigned *flags; unsigned epoch; };
// Blocks for the cooperative Cholesky on this device (0: not available).
int chol_coop_blocks(int m, int device);
hipError_t chol_coop_f64(const CholCoopArgs &a, int blocks, hipStream_t stream);
hipError_t chol_diag_grouped_f64(const CholGroupArgs *d, int count, int nb, int b, hipStream_t stream);
struct TriInvGroupArgs { const double *T; int64_t t_i, t_j; int m; double *Dinv; };
hipError_t tri_diag_inv_grouped_f64(const TriInvGroupArgs *d, int count, int max_m, int nb, hipStream_t stream);
struct MatGroupArgs { double *X; int64_t ld; int m, n; double c; const int32_t *piv; double *out; };
// X = 0 (ident = 0) or I (ident = 1), m x n
hipError_t set_matrix_grouped_f64(const MatGroupArgs *d, int count, int64_t max_total, int ident, hipStream_t stream);
// piv[i] = i, i < m (the pivot vector given as MatGroupArgs::piv)
hipError_t iota_grouped_i32(const MatGroupArgs *d, int count, int max_m, hipStream_t stream);
hipError_t iota_f64piv(int32_t *piv, int m, hipStream_t stream);
// X[i][i] += c * trace(X), m x m
hipError_t shift_diag_grouped_f64(const MatGroupArgs *d, int count, hipStream_t stream);
// out[0..3] as rdiag_ends_f64 for the m x m X
hipError_t rdiag_grouped_f64(const MatGroupArgs *d, int count, hipStream_t stream);
// out = [T'^T; T'] for T = X (m x m), T' = T Pi with piv
hipError_t form_tp_grouped_f64(const MatGroupArgs *d, int count, int64_t max_total, hipStream_t stream);

// G[i][i] += c * trace(G) for the m x m matrix G (one block).
hipError_t shift_diag_f64(double *G, int64_t ld, int m, double c, hipStream_t stream);
hipError_t set_matrix_f64(double *X, int64_t ld, int m, int n, int ident, hipStream_t stream);
// Zero the strictly upper (upper = 1) or strictly lower part of a row-major m x m matrix.
hipError_t zero_triangle_f64(double *X, int64_t ld, int m, int upper, hipStream_t stream);
// X's diagonal nb-blocks (row-major, ld ldx) from the inverted blocks Dinv of
// tri_diag_inv_f64; the rest of X is untouched.
hipError_t place_diag_blocks_f64(const double *Dinv, int m, int nb, double *X, int64_t ldx, hipStream_t stream);
// out = [T'^T ; T'] (two row-major m x m blocks) with T' = T Pi.
hipError_t form_tp_f64(const double *T, const int32_t *piv, int m, double *out, hipStream_t stream);
// |R_11| and |R_mm| of the row-major R (for the rank test), written to out[0..1].
hipError_t rdiag_ends_f64(const double *R, int64_t ldr, int m, double *out, hipStream_t stream);

// Newton-Schulz inverse of the SPD Gram (row-major m x m, both triangles).
// slots[0] = |X|_inf and slots[1] = max_i X_ii as bit patterns of
// non-negative doubles (atomic maxima; the caller clears the two slots).
hipError_t ns_norms_f64(const double *X, int m, unsigned long long *slots, hipStream_t stream);
// Y = 2 a I - a^2 X with a = 1 / slots[0]: the first iterate from Y_0 = a I.
hipError_t ns_start_f64(const double *X, int m, const unsigned long long *slots, double *Y, hipStream_t stream);
// out = scale * sum_s part[s] + diag * I for splits partials of an m x m
// matrix (stride apart); with bsum, block b also writes the sum of squares of
// (out - I) over its 256 entries to bsum[b] (ceil(m^2 / 256) blocks).
hipError_t reduce_affine_f64(const double *part, int64_t stride, int splits, int m, double *out, double scale,
                             double diag, double *bsum, hipStream_t stream);
// out[0] = sqrt(sum of bsum[0..nb)), summed in a fixed order (one block).
hipError_t sum_blocks_sqrt_f64(const double *bsum, int nb, double *out, hipStream_t stream);

// ---------------------------------------------------------------- apply
// C (m x k, column-major, ldc) partials: P[s] = A(:, split s) * B(split s, :)
// in binary64 (ddot = 0) or Dot2 (ddot = 1: hi in P, lo in P2).
struct ApplyArgs {
    int m, n, k;
    const double *A; int64_t lda;
    // optional column scaling: element (i, t) of the operand is the binary64
    // product A[i][t] * cs[t] (a column-scaled A without a scaled copy)
    const double *cs = nullptr;
};
hipError_t ab_partial_f64(const ApplyArgs &a, const double *B, int64_t ldb, int splits,
                          double *part_hi, double *part_lo, int dd, hipStream_t stream);
// The same partials in plain binary64 with B in scalar registers: B is first
// packed into bpk (ab_pack_size(n, k) doubles) as [block of 16 right-hand
// sides][t][16], zero past n and k; each wave streams a 64-row strip of A
// through its own LDS tile.  splits comes from ab_sx_splits.
hipError_t ab_sx_f64(const ApplyArgs &a, const double *B, int64_t ldb, double *bpk, int splits,
                     double *part, hipStream_t stream);
inline int64_t ab_pack_size(int64_t n, int64_t k) { return (k + 15) / 16 * ((n + 15) / 16 * 16) * 16; }
int ab_sx_splits(int64_t m, int64_t n, int64_t k, int cu_count);
// out (m x k, col-major ldo) = sum of partials (dd: compensated, rounded once).
hipError_t ab_reduce_f64(const double *part_hi, const double *part_lo, int m, int k, int splits,
                         int dd, double *out, int64_t ldo, hipStream_t stream);
// R = B - A^T (Xhi + Xlo) (n x k, col-major), Dot2 over m; mode 0: write
// r = round(B - A^T x) to Rout; mode 1: write Y = round(A^T x) and
// Z = round(B - A^T x) (either may be NULL); dd = 0 uses plain binary64 and
// ignores Xlo.  With dd and a workspace xpk of atx_pack_size(m, k) doubles,
// x is packed for scalar loads and the pass reads no LDS.
hipError_t atx_f64(const ApplyArgs &a, const double *Xhi, const double *Xlo, int64_t ldx,
                   const double *B, int64_t ldb, double *Rout, int64_t ldr,
                   double *Y, int64_t ldy, double *Z, int64_t ldz, int dd, hipStream_t stream,
                   double *xpk = nullptr);
inline int64_t atx_pack_size(int64_t m, int64_t k) { return (k + 7) / 8 * ((m + 7) / 8 * 8) * 16; }
// ---- grouped (batched) forms: one launch over many problems whose
// arguments live in device memory; the grid covers the largest member and
// smaller members skip the blocks they do not have.
struct AbGroupArgs {       // c = A B (partials + reduction)
    ApplyArgs a; const double *B; int64_t ldb; int splits;
    double *ph, *pl;       // splits * m * k partials
    double *out; int64_t ldo;
};
hipError_t ab_partial_grouped_f64(const AbGroupArgs *d, int count, int max_m, int max_k, int max_splits, int dd,
                                  hipStream_t stream);
hipError_t ab_reduce_grouped_f64(const AbGroupArgs *d, int count, int64_t max_mk, int dd, hipStream_t stream);
struct AtxGroupArgs {      // as atx_f64
    ApplyArgs a; const double *xhi, *xlo; int64_t ldx; const double *B; int64_t ldb;
    double *Rout; int64_t ldr; double *Y; int64_t ldy; double *Z; int64_t ldz;
};
// scaled: some member has a column scaling (a.cs)
hipError_t atx_grouped_f64(const AtxGroupArgs *d, int count, int64_t max_n, int max_k, int dd, int scaled,
                           hipStream_t stream);
struct DdGroupArgs { double *xhi, *xlo; const double *D; int total; double *norms; };
hipError_t dd_update_grouped_f64(const DdGroupArgs *d, int count, hipStream_t stream);
// dst = src (column-major rows x cols; rs: optional row scaling, dst[i][j] =
// src[i][j] * rs[i], src may be dst); zero_out: optional, set to zero alike
struct CopyGroupArgs {
    const double *src; int64_t lds; double *dst; int64_t ldd; int rows, cols; double *zero_out; int64_t ldz;
    const double *rs = nullptr;
};
// Y = B - r and Z = r (column-major rows x cols; Y or Z null to skip; either may be B)
struct FinishGroupArgs { const double *r; int64_t ldr; const double *B; int64_t ldb; double *Y; int64_t ldy; double *Z; int64_t ldz; int rows, cols; };
hipError_t finish_cols_f64(const FinishGroupArgs &g, hipStream_t stream);
hipError_t finish_cols_grouped_f64(const FinishGroupArgs *d, int count, int64_t max_total, hipStream_t stream);
hipError_t copy_cols_grouped_f64(const CopyGroupArgs *d, int count, int64_t max_total, hipStream_t stream);

// (Xhi, Xlo) += D (double-binary64 update); norms[0] = |D|_F^2, norms[1] = |Xhi|_F^2.
hipError_t dd_update_f64(double *Xhi, double *Xlo, const double *D, int m, int k, double *norms,
                         hipStream_t stream);
// Copy an m x k column-major block (ld -> ld2), optionally zeroing `zero_out`.
// Classical scheme: X (m x k, column-major) = Pi R^{-1} Q^T C for the
// Householder pivoted QR M Pi = Q R of an m x m matrix with reflectors V
// (QrcpWork::V layout), scalars tau, row-major upper-triangular R and piv.
// m <= 8192 (the vector is kept in LDS).
hipError_t qr_solve_f64(int m, const double *V, const double *tau, const double *R, const int32_t *piv,
                        const double *C, int64_t ldc, double *X, int64_t ldx, int k, hipStream_t stream);
// Conjugate gradients on k columns (m x k column-major blocks, ld m): init
// r = t, pp = t, u = 0, gamma = r.r; step with q = (operator) pp.
hipError_t cg_init_f64(int m, int k, const double *t, double *u, double *r, double *pp, double *gamma,
                       hipStream_t stream);
hipError_t cg_step_f64(int m, int k, double *u, double *r, double *pp, const double *q, double *gamma,
                       hipStream_t stream);
// out = B - C for column-major rows x cols blocks (out may be B or C).
hipError_t sub_cols_f64(const double *B, int64_t ldb, const double *C, int64_t ldc, double *out, int64_t ldo, int rows,
                        int cols, hipStream_t stream);
hipError_t copy_cols_f64(const double *src, int64_t lds, double *dst, int64_t ldd, int rows, int cols,
                         double *zero_out, int64_t ldz, hipStream_t stream);

}  // namespace rt
