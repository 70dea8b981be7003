/*
 * oracle.c -- CPU reference for the randomized orthogonal projection of
 * Rokhlin & Tygert, "A fast randomized algorithm for orthogonal projection".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call this
 * file; only the test-suite, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code, header or table with the GPU library: every
 * routine here is written from the paper's definitions, plainly and slowly,
 * in IEEE double precision, with an extended-precision (binary128) residual
 * where the definition must be evaluated beyond double rounding.
 *
 * Contents
 *   orc_splitmix64_*     SplitMix64 (Steele, Lea, Flood 2014) and the draw
 *                        order of the sketch's random tables.
 *   orc_srft_tables      signs, block/in-block permutations, sorted subset J
 *                        of the subsampled randomized Fourier sketch.
 *   orc_qrcp             Businger-Golub column-pivoted Householder QR
 *                        (Sec. 4, eq. QR_decomp; Householder reflections as
 *                        stated at the end of Sec. 5).
 *   orc_project          The three outputs of the problem statement (Sec. 1,
 *                        items 1-3; Sec. 4, first paragraph): x = argmin
 *                        |A^T x - b| (Remark 4.1), row projection A^T x and
 *                        null projection b - A^T x (eq. basic_identity).
 *                        Evaluated by Householder QR of A^T plus iterative
 *                        refinement (the refinement of Remark 4.3) with the
 *                        residuals in binary128.
 *   orc_project_r        The same outputs from a triangular factor of A^T
 *                        supplied by the caller (LAPACK's Householder QR
 *                        as a library step), refined the same way.
 *   orc_project_complex_r  The same for complex A (conjugate transpose A^*),
 *                        with binary128 complex residuals.
 *
 * Conventions
 *   A is row-major m x n with leading dimension lda (element (i,j) at
 *   A[i*lda + j]).  Right-hand sides are column-major n x k (column c at
 *   B + c*ldb).  X is column-major m x k.
 */
#include <complex.h>
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __float128 quad;

/* ------------------------------------------------------------------------ */
/* SplitMix64: state advances by the golden-ratio increment; each output is  */
/* the published 64-bit finalizer of the new state.                          */
/* ------------------------------------------------------------------------ */
static uint64_t sm64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Uniform integer in [0, range): high word of the 128-bit product. */
static uint64_t sm64_below(uint64_t *state, uint64_t range)
{
    unsigned __int128 p = (unsigned __int128)sm64_next(state) * range;
    return (uint64_t)(p >> 64);
}

void orc_splitmix64_stream(uint64_t seed, int64_t count, uint64_t *out)
{
    uint64_t s = seed;
    for (int64_t i = 0; i < count; ++i) out[i] = sm64_next(&s);
}

/* Seed of batch instance i: first output of a generator started at seed^i. */
uint64_t orc_instance_seed(uint64_t seed, int64_t i)
{
    uint64_t s = seed ^ (uint64_t)i;
    return sm64_next(&s);
}

/* Padded length and grid split of the sketch's Fourier transform:
 * np = max(4, 2^ceil(log2 n)), n2 = 2^floor(e/2), n1 = np/n2. */
void orc_srft_dims(int64_t n, int64_t *np, int64_t *n1, int64_t *n2)
{
    int64_t p = 4;
    int e = 2;
    while (p < n) { p <<= 1; ++e; }
    *np = p;
    *n2 = (int64_t)1 << (e / 2);
    *n1 = p / *n2;
}

/*
 * Random tables of the sketch, drawn from one SplitMix64 stream started at
 * `seed`, in this order:
 *   1. np signs: draw t gives sign[t] = -1 if its top bit is set, else +1;
 *   2. sigma, a permutation of [0,n1): Fisher-Yates from the top
 *      (for j = n1-1..1: r = below(j+1); swap sigma[j], sigma[r]);
 *   3. tau, a permutation of [0,n2), drawn the same way;
 *   4. J, an l-subset of [0,np) in increasing order by selection sampling
 *      (for t = 0,1,..: keep t iff below(np - t) < l - kept).
 * The permutation of the padded row is pi(t) = sigma[t / n2]*n2 + tau[t % n2].
 */
int orc_srft_tables(uint64_t seed, int64_t n, int64_t l, int8_t *sign,
                    int32_t *sigma, int32_t *tau, int32_t *J)
{
    int64_t np, n1, n2;
    orc_srft_dims(n, &np, &n1, &n2);
    if (l < 1 || l > np) return 1;
    uint64_t s = seed;
    for (int64_t t = 0; t < np; ++t)
        sign[t] = (sm64_next(&s) >> 63) ? (int8_t)-1 : (int8_t)1;
    for (int64_t j = 0; j < n1; ++j) sigma[j] = (int32_t)j;
    for (int64_t j = n1 - 1; j >= 1; --j) {
        int64_t r = (int64_t)sm64_below(&s, (uint64_t)(j + 1));
        int32_t tmp = sigma[j]; sigma[j] = sigma[r]; sigma[r] = tmp;
    }
    for (int64_t j = 0; j < n2; ++j) tau[j] = (int32_t)j;
    for (int64_t j = n2 - 1; j >= 1; --j) {
        int64_t r = (int64_t)sm64_below(&s, (uint64_t)(j + 1));
        int32_t tmp = tau[j]; tau[j] = tau[r]; tau[r] = tmp;
    }
    int64_t kept = 0;
    for (int64_t t = 0; t < np && kept < l; ++t) {
        if ((int64_t)sm64_below(&s, (uint64_t)(np - t)) < l - kept) J[kept++] = (int32_t)t;
    }
    return kept == l ? 0 : 2;
}

/* ------------------------------------------------------------------------ */
/* Column-pivoted Householder QR (Businger-Golub), eq. QR_decomp:            */
/*   M Pi^T = Q R, M is rows x cols column-major (ld = ldm), rows >= cols.   */
/* At step k the pivot is the not-yet-chosen column whose trailing part      */
/* M[k:, j] has the largest 2-norm (recomputed from scratch every step; ties */
/* go to the lowest original column index).  The reflector is               */
/* H = I - tau v v^T with v[0] = 1, beta = -sign(alpha)*|x| (sign(0) = +1).  */
/* Outputs: R (cols x cols, row-major, upper triangle; zeros below) and piv, */
/* with column k of M Pi^T equal to column piv[k] of M.  M is overwritten.   */
/* ------------------------------------------------------------------------ */
int orc_qrcp(int64_t rows, int64_t cols, double *M, int64_t ldm, double *R, int32_t *piv)
{
    if (rows < cols || cols < 1) return 1;
    char *done = (char *)calloc((size_t)cols, 1);
    double *nrm = (double *)malloc(sizeof(double) * (size_t)cols);
    double *v = (double *)malloc(sizeof(double) * (size_t)rows);
    if (!done || !nrm || !v) { free(done); free(nrm); free(v); return 3; }
    memset(R, 0, sizeof(double) * (size_t)(cols * cols));
    for (int64_t k = 0; k < cols; ++k) {
        /* norms of the trailing parts of the remaining columns */
        #pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < cols; ++j) {
            if (done[j]) continue;
            const double *c = M + j * ldm;
            double s = 0.0;
            for (int64_t i = k; i < rows; ++i) s += c[i] * c[i];
            nrm[j] = s;
        }
        int64_t p = -1;
        for (int64_t j = 0; j < cols; ++j) {
            if (done[j]) continue;
            if (p < 0 || nrm[j] > nrm[p]) p = j;
        }
        done[p] = 1;
        piv[k] = (int32_t)p;
        double *x = M + p * ldm;
        /* R entries above the diagonal were produced by earlier reflectors */
        for (int64_t i = 0; i < k; ++i) R[i * cols + k] = x[i];
        double alpha = x[k];
        double xnorm = sqrt(nrm[p]);
        double beta, tau;
        if (xnorm == 0.0) {
            beta = 0.0; tau = 0.0;
            for (int64_t i = k; i < rows; ++i) v[i] = 0.0;
            v[k] = 1.0;
        } else {
            beta = (alpha >= 0.0) ? -xnorm : xnorm;
            tau = (beta - alpha) / beta;
            double inv = 1.0 / (alpha - beta);
            v[k] = 1.0;
            for (int64_t i = k + 1; i < rows; ++i) v[i] = x[i] * inv;
        }
        R[k * cols + k] = beta;
        x[k] = beta;
        for (int64_t i = k + 1; i < rows; ++i) x[i] = 0.0;
        /* apply H_k to every other remaining column */
        #pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < cols; ++j) {
            if (done[j]) continue;
            double *c = M + j * ldm;
            double w = 0.0;
            for (int64_t i = k; i < rows; ++i) w += v[i] * c[i];
            w *= tau;
            for (int64_t i = k; i < rows; ++i) c[i] -= w * v[i];
        }
    }
    free(done); free(nrm); free(v);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Projection, row projection and least squares (Sec. 1; Sec. 4; Rem. 4.1).  */
/* ------------------------------------------------------------------------ */

/* Householder QR of A^T (n x m): the columns of A^T are the rows of A.     */
/* H holds them as m vectors of length n; on return H[j][j+1:] holds the     */
/* reflector tails (v[0] = 1 implied), tau[j] the scalar, Rd the diagonal.   */
static void householder_at(int64_t m, int64_t n, double *H, double *tau, double *Rd)
{
    for (int64_t j = 0; j < m; ++j) {
        double *x = H + j * n;
        double s = 0.0;
        for (int64_t i = j; i < n; ++i) s += x[i] * x[i];
        double xnorm = sqrt(s), alpha = x[j];
        double beta, t;
        if (xnorm == 0.0) { beta = 0.0; t = 0.0; }
        else {
            beta = (alpha >= 0.0) ? -xnorm : xnorm;
            t = (beta - alpha) / beta;
            double inv = 1.0 / (alpha - beta);
            for (int64_t i = j + 1; i < n; ++i) x[i] *= inv;
        }
        tau[j] = t;
        Rd[j] = beta;
        x[j] = 1.0; /* temporarily v[0] */
        #pragma omp parallel for schedule(static)
        for (int64_t c = j + 1; c < m; ++c) {
            double *y = H + c * n;
            double w = 0.0;
            for (int64_t i = j; i < n; ++i) w += x[i] * y[i];
            w *= t;
            for (int64_t i = j; i < n; ++i) y[i] -= w * x[i];
        }
        x[j] = beta;
    }
}

/* Triangular solves with an upper-triangular m x m R addressed through
 * strides: R[i][j] = Rp[i*ri + j*rj] for i <= j (the diagonal included).   */

/* Solve R y = c (back substitution), y overwritten. */
static void solve_r(int64_t m, const double *Rp, int64_t ri, int64_t rj, double *y)
{
    for (int64_t i = m - 1; i >= 0; --i) {
        double s = y[i];
        for (int64_t j = i + 1; j < m; ++j) s -= Rp[i * ri + j * rj] * y[j];
        y[i] = s / Rp[i * ri + i * rj];
    }
}

/* Solve R^T y = c (forward substitution), y overwritten. */
static void solve_rt(int64_t m, const double *Rp, int64_t ri, int64_t rj, double *y)
{
    for (int64_t i = 0; i < m; ++i) {
        double s = y[i];
        for (int64_t j = 0; j < i; ++j) s -= Rp[j * ri + i * rj] * y[j];
        y[i] = s / Rp[i * ri + i * rj];
    }
}

/*
 * Refinement (Remark 4.3) of the k least-squares solutions x (binary128,
 * m x k column-major, in: the starting point) and the outputs formed from
 * them.  For each column b:
 *   r = b - A^T x and s = A r in binary128 (s rounded once to double),
 *   d = R^{-1} R^{-T} s in double (R from a Householder QR of A^T, so that
 *   R^T R = A A^T up to rounding), x += d kept in binary128;
 *   stop when |d| <= 1e-22 |x|, when |d| stops decreasing, or after maxit
 *   steps.  Then p = A^T x and z = b - A^T x in binary128, rounded once.
 * The columns are taken one after another; inside a column the loops over
 * independent entries (t for r, i for s) run in parallel, and every entry is
 * accumulated in the same order as a sequential loop would.
 */
static int refine_and_form(int64_t m, int64_t n, const double *A, int64_t lda,
                           const double *Rp, int64_t ri, int64_t rj, int64_t k,
                           const double *B, int64_t ldb, quad *xq, double *Z, int64_t ldz,
                           double *P, int64_t ldp, double *X, int64_t ldx, int maxit, double *info)
{
    quad *r = (quad *)malloc(sizeof(quad) * (size_t)n);
    double *d = (double *)malloc(sizeof(double) * (size_t)m);
    if (!r || !d) { free(r); free(d); return 3; }
    int steps_max = 0;
    double last_ratio = 0.0;
    for (int64_t c = 0; c < k; ++c) {
        const double *b = B + c * ldb;
        quad *x = xq + c * m;
        double prev = INFINITY, ratio = 0.0;
        int steps = 0;
        for (int it = 0; it < maxit; ++it) {
            /* r = b - A^T x in binary128: entry t subtracts a_it x_i for i = 0..m-1 */
            #pragma omp parallel for schedule(static)
            for (int64_t t = 0; t < n; ++t) {
                quad acc = (quad)b[t];
                for (int64_t i = 0; i < m; ++i) acc -= (quad)A[i * lda + t] * x[i];
                r[t] = acc;
            }
            /* s = A r in binary128, rounded once to double */
            #pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < m; ++i) {
                const double *a = A + i * lda;
                quad s = 0;
                for (int64_t t = 0; t < n; ++t) s += (quad)a[t] * r[t];
                d[i] = (double)s;
            }
            solve_rt(m, Rp, ri, rj, d);
            solve_r(m, Rp, ri, rj, d);
            double dn = 0.0, xn = 0.0;
            for (int64_t i = 0; i < m; ++i) {
                x[i] += (quad)d[i];
                dn += d[i] * d[i];
                double xd = (double)x[i];
                xn += xd * xd;
            }
            dn = sqrt(dn); xn = sqrt(xn);
            ++steps;
            ratio = xn > 0.0 ? dn / xn : 0.0;
            if (dn <= 1e-22 * xn || dn >= prev) break;
            prev = dn;
        }
        /* p = A^T x and z = b - A^T x in binary128 */
        #pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < n; ++t) {
            quad acc = 0;
            for (int64_t i = 0; i < m; ++i) acc += (quad)A[i * lda + t] * x[i];
            if (P) P[c * ldp + t] = (double)acc;
            if (Z) Z[c * ldz + t] = (double)((quad)b[t] - acc);
        }
        if (X) for (int64_t i = 0; i < m; ++i) X[c * ldx + i] = (double)x[i];
        if (steps > steps_max) steps_max = steps;
        if (ratio > last_ratio) last_ratio = ratio;
    }
    if (info) { info[0] = steps_max; info[1] = last_ratio; }
    free(r); free(d);
    return 0;
}

/*
 * For each of the k columns b of B:
 *   x = argmin_h |A^T h - b|        (written to X if X != NULL)
 *   p = A^T x                       (row-space projection, to P if != NULL)
 *   z = b - A^T x                   (null-space projection, to Z if != NULL)
 * Start: x0 from the Householder QR of A^T (x0 = R^{-1} [Q^T b]_{0:m}),
 * then the binary128 refinement of refine_and_form.
 * info (length >= 2, may be NULL): info[0] = refinement steps taken,
 * info[1] = |d|/|x| of the last step (maximum over columns).
 */
int orc_project(int64_t m, int64_t n, const double *A, int64_t lda, int64_t k,
                const double *B, int64_t ldb, double *Z, int64_t ldz,
                double *P, int64_t ldp, double *X, int64_t ldx, int maxit, double *info)
{
    if (m < 1 || n < m || lda < n || k < 0 || (k > 0 && ldb < n)) return 1;
    double *H = (double *)malloc(sizeof(double) * (size_t)(m * n));
    double *tau = (double *)malloc(sizeof(double) * (size_t)m);
    double *Rd = (double *)malloc(sizeof(double) * (size_t)m);
    quad *xq = (quad *)malloc(sizeof(quad) * (size_t)(m * (k > 0 ? k : 1)));
    if (!H || !tau || !Rd || !xq) { free(H); free(tau); free(Rd); free(xq); return 3; }
    for (int64_t i = 0; i < m; ++i) memcpy(H + i * n, A + i * lda, sizeof(double) * (size_t)n);
    householder_at(m, n, H, tau, Rd);

    /* x0 per column: apply H_0 .. H_{m-1} to b, then back-substitute with R,
     * whose entries are R[i][j] = H[j*n + i] (i <= j; the diagonal is beta) */
    int bad = 0;
    #pragma omp parallel for schedule(dynamic, 1) reduction(|:bad)
    for (int64_t c = 0; c < k; ++c) {
        const double *b = B + c * ldb;
        double *w = (double *)malloc(sizeof(double) * (size_t)n);
        if (!w) { bad = 1; continue; }
        memcpy(w, b, sizeof(double) * (size_t)n);
        for (int64_t j = 0; j < m; ++j) {
            const double *v = H + j * n;
            double s = w[j];
            for (int64_t i = j + 1; i < n; ++i) s += v[i] * w[i];
            s *= tau[j];
            w[j] -= s;
            for (int64_t i = j + 1; i < n; ++i) w[i] -= s * v[i];
        }
        solve_r(m, H, 1, n, w);
        for (int64_t i = 0; i < m; ++i) xq[c * m + i] = (quad)w[i];
        free(w);
    }
    int rc = bad ? 3 : refine_and_form(m, n, A, lda, H, 1, n, k, B, ldb, xq, Z, ldz, P, ldp, X, ldx, maxit, info);
    free(H); free(tau); free(Rd); free(xq);
    return rc;
}

/*
 * As orc_project, with the triangular factor of the Householder QR of A^T
 * supplied by the caller (R, m x m upper triangular, row-major, ld ldr;
 * e.g. LAPACK's): x starts at 0, so the first refinement step is the
 * semi-normal solve x1 = R^{-1} R^{-T} A b, and the binary128 refinement of
 * refine_and_form continues from there (it contracts by about u cond(A)
 * per step for any backward-stable R).
 */
int orc_project_r(int64_t m, int64_t n, const double *A, int64_t lda, const double *R, int64_t ldr,
                  int64_t k, const double *B, int64_t ldb, double *Z, int64_t ldz,
                  double *P, int64_t ldp, double *X, int64_t ldx, int maxit, double *info)
{
    if (m < 1 || n < m || lda < n || ldr < m || k < 0 || (k > 0 && ldb < n)) return 1;
    quad *xq = (quad *)calloc((size_t)(m * (k > 0 ? k : 1)), sizeof(quad));
    if (!xq) return 3;
    int rc = refine_and_form(m, n, A, lda, R, ldr, 1, k, B, ldb, xq, Z, ldz, P, ldp, X, ldx, maxit, info);
    free(xq);
    return rc;
}

/*
 * Complex-valued A (Sec. 1: the method extends to complex entries), with
 * A^* the conjugate transpose.  Data are interleaved (re, im) binary64
 * pairs: A row-major m x n (element (i,j) at 2*(i*lda + j)), B/Z/P column-
 * major n x k, X column-major m x k, R upper triangular m x m row-major (a
 * Householder factor of A^*, so that R^* R = A A^*, from the caller).
 * x starts at 0; per step r = b - A^* x and s = A r in binary128 complex,
 * d = R^{-1} R^{-*} s in binary64 complex, x += d kept in binary128; stop
 * as refine_and_form does.  Then p = A^* x, z = b - p, rounded once.
 */
typedef __complex128 cquad;

static void csolve_rh(int64_t m, const double *R, int64_t ldr, double _Complex *y)
{   /* R^* y = c: forward substitution with the conjugate transpose */
    for (int64_t i = 0; i < m; ++i) {
        double _Complex s = y[i];
        for (int64_t j = 0; j < i; ++j) {
            const double _Complex rji = R[2 * (j * ldr + i)] + R[2 * (j * ldr + i) + 1] * 1.0i;
            s -= conj(rji) * y[j];
        }
        const double _Complex rii = R[2 * (i * ldr + i)] + R[2 * (i * ldr + i) + 1] * 1.0i;
        y[i] = s / conj(rii);
    }
}

static void csolve_r(int64_t m, const double *R, int64_t ldr, double _Complex *y)
{   /* R y = c: back substitution */
    for (int64_t i = m - 1; i >= 0; --i) {
        double _Complex s = y[i];
        for (int64_t j = i + 1; j < m; ++j) s -= (R[2 * (i * ldr + j)] + R[2 * (i * ldr + j) + 1] * 1.0i) * y[j];
        y[i] = s / (R[2 * (i * ldr + i)] + R[2 * (i * ldr + i) + 1] * 1.0i);
    }
}

static cquad cq(const double *v) { cquad z; __real__ z = v[0]; __imag__ z = v[1]; return z; }

int orc_project_complex_r(int64_t m, int64_t n, const double *A, int64_t lda, const double *R, int64_t ldr,
                          int64_t k, const double *B, int64_t ldb, double *Z, int64_t ldz, double *P, int64_t ldp,
                          double *X, int64_t ldx, int maxit, double *info)
{
    if (m < 1 || n < m || lda < n || ldr < m || k < 0 || (k > 0 && ldb < n)) return 1;
    cquad *r = (cquad *)malloc(sizeof(cquad) * (size_t)n);
    cquad *x = (cquad *)malloc(sizeof(cquad) * (size_t)m);
    double _Complex *d = (double _Complex *)malloc(sizeof(double _Complex) * (size_t)m);
    if (!r || !x || !d) { free(r); free(x); free(d); return 3; }
    int steps_max = 0;
    double last_ratio = 0.0;
    for (int64_t c = 0; c < k; ++c) {
        const double *b = B + 2 * c * ldb;
        for (int64_t i = 0; i < m; ++i) x[i] = 0;
        double prev = INFINITY, ratio = 0.0;
        int steps = 0;
        for (int it = 0; it < maxit; ++it) {
            /* r = b - A^* x: entry t subtracts conj(a_it) x_i for i = 0..m-1 */
            #pragma omp parallel for schedule(static)
            for (int64_t t = 0; t < n; ++t) {
                cquad acc = cq(b + 2 * t);
                for (int64_t i = 0; i < m; ++i) acc -= conjq(cq(A + 2 * (i * lda + t))) * x[i];
                r[t] = acc;
            }
            /* s = A r, rounded once to binary64 */
            #pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < m; ++i) {
                cquad s = 0;
                for (int64_t t = 0; t < n; ++t) s += cq(A + 2 * (i * lda + t)) * r[t];
                d[i] = (double)crealq(s) + (double)cimagq(s) * 1.0i;
            }
            csolve_rh(m, R, ldr, d);
            csolve_r(m, R, ldr, d);
            double dn = 0.0, xn = 0.0;
            for (int64_t i = 0; i < m; ++i) {
                cquad di;
                __real__ di = creal(d[i]);
                __imag__ di = cimag(d[i]);
                x[i] += di;
                dn += creal(d[i]) * creal(d[i]) + cimag(d[i]) * cimag(d[i]);
                const double xr = (double)crealq(x[i]), xim = (double)cimagq(x[i]);
                xn += xr * xr + xim * xim;
            }
            dn = sqrt(dn); xn = sqrt(xn);
            ++steps;
            ratio = xn > 0.0 ? dn / xn : 0.0;
            if (dn <= 1e-22 * xn || dn >= prev) break;
            prev = dn;
        }
        /* p = A^* x and z = b - A^* x in binary128 complex */
        #pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < n; ++t) {
            cquad acc = 0;
            for (int64_t i = 0; i < m; ++i) acc += conjq(cq(A + 2 * (i * lda + t))) * x[i];
            if (P) { P[2 * (c * ldp + t)] = (double)crealq(acc); P[2 * (c * ldp + t) + 1] = (double)cimagq(acc); }
            if (Z) {
                const cquad zt = cq(b + 2 * t) - acc;
                Z[2 * (c * ldz + t)] = (double)crealq(zt);
                Z[2 * (c * ldz + t) + 1] = (double)cimagq(zt);
            }
        }
        if (X)
            for (int64_t i = 0; i < m; ++i) {
                X[2 * (c * ldx + i)] = (double)crealq(x[i]);
                X[2 * (c * ldx + i) + 1] = (double)cimagq(x[i]);
            }
        if (steps > steps_max) steps_max = steps;
        if (ratio > last_ratio) last_ratio = ratio;
    }
    if (info) { info[0] = steps_max; info[1] = last_ratio; }
    free(r); free(x); free(d);
    return 0;
}

/* Number of OpenMP threads the oracle runs with. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
