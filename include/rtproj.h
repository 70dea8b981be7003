/*
 * rtproj.h -- randomized, preconditioned orthogonal projection on AMD gfx950.
 *
 * Implements the method of Rokhlin & Tygert, "A fast randomized algorithm for
 * orthogonal projection": for a full-rank m x n matrix A with m <= n and right-
 * hand sides b (length n) it returns
 *   - the least-squares solution x = argmin |A^T x - b|        (Remark 4.1),
 *   - the projection onto the row space of A,  A^T x           (Sec. 4),
 *   - the projection onto the null space of A, b - A^T x       (eq. basic_identity),
 * through the preconditioned identity (eq. basic_precond) with P = Pi^T R^T
 * taken from a column-pivoted QR (eq. QR_decomp) of a randomized sketch
 * S = A G (eq. testing).
 *
 * Layouts (all matrices live in device memory unless stated otherwise):
 *   A   row-major m x n, element (i, j) at A[i*lda + j], lda >= n.
 *   B   column-major n x k: right-hand side c starts at B + c*ldb, ldb >= n.
 *       (A C-contiguous torch tensor of shape (k, n).)  Same for Z and Y.
 *   X   column-major m x k, ldx >= m.
 * All floating-point data at the interface is IEEE binary64.
 *
 * Ownership and lifetime: a plan owns its device workspaces (allocated with
 * hipMalloc at creation and grown on demand).  A is BORROWED by
 * rtproj_precondition: every projection applies A and A^T again (the costs
 * C_A and C_{A^*} of Sec. 4.1), so A must stay valid and unchanged until the
 * next rtproj_precondition or rtproj_plan_destroy.  Outputs are owned by the
 * caller.  Z (or Y) may alias B only with identical pointer and leading
 * dimension.
 *
 * Streams and synchronisation: every call enqueues its work on the plan's
 * stream (rtproj_plan_set_stream; default: the null stream).
 * rtproj_precondition blocks until the sketch's pivoted QR has finished, to
 * read the rank test (a few bytes), and until the Gram's inverse is done.
 * The project calls are asynchronous unless refinement runs with a
 * convergence test (set_refinement with rtol > 0), which reads one flag per
 * refinement step; otherwise whether the refinement converged is read at the
 * next rtproj_plan_status or rtproj_plan_info.  A plan is not thread-safe;
 * distinct plans are independent.
 *
 * Errors: every entry point returns an rtproj_status; nothing is thrown and
 * nothing aborts.  Argument errors are detected on the host before any device
 * work and leave the plan unchanged.  rtproj_last_error() returns a
 * thread-local message for the last failure.
 */
#ifndef RTPROJ_H
#define RTPROJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rtproj_plan_s *rtproj_plan;

typedef enum {
    RTPROJ_OK = 0,
    RTPROJ_ERR_INVALID_ARG = 1, /* bad size, leading dimension or null pointer */
    RTPROJ_ERR_ALLOC = 2,       /* device allocation failed                      */
    RTPROJ_ERR_DEVICE = 3,      /* HIP runtime or kernel failure                 */
    RTPROJ_ERR_STATE = 4,       /* projection requested before preconditioning   */
    RTPROJ_ERR_RANK = 5,        /* A (numerically) rank deficient: the pivoted QR
                                   of the sketch failed, or the Gram's inverse
                                   (Cholesky breakdown, or no Newton-Schulz
                                   convergence)                                  */
    RTPROJ_ERR_NOCONV = 6,      /* refinement did not contract                   */
    RTPROJ_ERR_UNSUPPORTED = 7  /* size or mode the library does not handle      */
} rtproj_status;

/* Arithmetic used by the preconditioner (the projection's residuals, the
 * solves with R and Pi, and the Gram's inverse are always binary64). */
typedef enum {
    RTPROJ_PREC_FP64 = 0,       /* sketch, P^{-1}A and its Gram in binary64           */
    RTPROJ_PREC_MIXED_FP32 = 1, /* binary32 sketch and Gram (binary32 MFMA); P^{-1}A
                                   in binary32 when kappa_est <= 1e5, else binary64;
                                   the sketch is redone in binary64 when its rank
                                   estimate shows it too coarse (2^-24 kappa_est >
                                   1) or the Gram shows cond(P^{-1}A) > 10          */
    RTPROJ_PREC_MIXED_BF16 = 2, /* binary32 sketch; Gram from row-scaled (powers of
                                   two) bfloat16 P^{-1}A on MFMA with binary32
                                   accumulation; P^{-1}A as in MIXED_FP32             */
    RTPROJ_PREC_MIXED_BF16X3 = 3 /* as MIXED_FP32, the Gram from binary32 P^{-1}A split
                                   into bfloat16 halves w = hi + lo (+ about 2^-16 w):
                                   hi lo^T + lo hi^T + hi hi^T on bfloat16 MFMA with
                                   binary32 accumulation (about 2^-16 relative per
                                   product).  Needs n % 4 == 0; otherwise the Gram
                                   is binary32 as in MIXED_FP32 (gram_bits 32)       */
} rtproj_precision;

/* How the pivoted QR of the sketch (eq. QR_decomp) is computed.  All modes
 * give the same R and pivots in exact arithmetic; the two-stage modes are
 * backward stable in the normwise sense (the QR of the small factor R0 of
 * S^T = Q0 R0 has the same column norms as S^T at every step). */
typedef enum {
    RTPROJ_QR_AUTO = 0,         /* chosen by the plan from the sizes              */
    RTPROJ_QR_DIRECT = 1,       /* Householder QRCP of S^T (l x m), one
                                   cooperative launch                            */
    RTPROJ_QR_TWO_STAGE = 2,    /* the factor R0 of S^T = Q0 R0 by shifted
                                   Cholesky QR and one unshifted pass (two
                                   Gram/Cholesky passes on MFMA, binary64;
                                   Q0 is not formed; a third pass when the
                                   second factor's diagonal spans more than
                                   1e5, a nearly rank-deficient sketch), then
                                   the cooperative QRCP of R0 (m x m)            */
    RTPROJ_QR_TWO_STAGE_WG = 3  /* as 2, the QRCP of R0 in one workgroup         */
} rtproj_qr_mode;

/* How Y = X^{-1} of the Gram X = (P^{-1}A)(P^{-1}A)^* (eq. inversion) enters
 * the projections.  Both give (A A^*)^{-1} up to rounding; the refinement
 * removes what is left. */
typedef enum {
    RTPROJ_INV_AUTO = 0,           /* Newton-Schulz for m <= 1024, else Cholesky   */
    RTPROJ_INV_NEWTON_SCHULZ = 1,  /* Y_{k+1} = Y_k (2I - X Y_k), Y_0 = I/|X|_inf,
                                      iterated until |I - X Y_k|_F <= 1e-6 (then
                                      one more step); applications use
                                      T'^T (Y (T' c)) with T' = R^{-T} Pi         */
    RTPROJ_INV_CHOLESKY = 2        /* X = L L^T (blocked, binary64); applications
                                      use T' = L^{-1} R^{-T} Pi, T'^T (T' c)      */
} rtproj_inverse;

/* Arithmetic of the refinement residuals (Remark 4.3).  r = b - A^T x is the
 * residual, s = A r the contraction the correction is solved from, and the
 * final A^T x gives the row and null projections.  A residual evaluated in
 * plain binary64 stalls at a relative error of x of about u cond(A);
 * compensated (double-binary64, Dot2) evaluation removes that floor at
 * about ten times the instruction count. */
typedef enum {
    RTPROJ_RESID_AUTO = 0,     /* chosen from the rank estimate (see
                                  rtproj_plan_set_refinement)                   */
    RTPROJ_RESID_PLAIN = 1,    /* every residual in plain binary64              */
    RTPROJ_RESID_S_ONLY = 2,   /* r and the final A^T x plain, s = A r
                                  compensated in the compensated steps          */
    RTPROJ_RESID_FULL = 3      /* r and s compensated in the compensated steps
                                  (x kept double-binary64); the final
                                  z = b - A^T x is the last compensated r minus
                                  A^T d for that step's correction d, a plain
                                  product (|d| is the error left in x before
                                  it); the iterative variant recomputes
                                  A^T x compensated                            */
} rtproj_residual;

/* Arithmetic of the compensated products r = b - A^T x and s = A r inside
 * the compensated refinement steps (Remark 4.3).  Both evaluate the same
 * quantities to well beyond binary64; the integer form is exact on the digit
 * grid it keeps: every dot product is taken on one power-of-two scale per
 * row of the operand and per right-hand side, its operands are split into
 * 13 signed 6-bit digits, the digit products are summed exactly in int32 on
 * the int8 matrix cores, and the pairs of digit positions s + t <= 14 are
 * combined in double-binary64 (omitted terms below about 2^-62 of the
 * largest term's scale at 2048 terms). */
typedef enum {
    RTPROJ_COMP_AUTO = 0,      /* the integer form from 16 right-hand sides on
                                  (and m <= 32768), Dot2 below                 */
    RTPROJ_COMP_DOT2 = 1,      /* Dot2 (TwoProd and TwoSum) on the vector units */
    RTPROJ_COMP_INT8 = 2       /* exact digit products on the int8 matrix cores
                                  (m <= 32768; else Dot2)                       */
} rtproj_compensation;

/* Method of a plan.  Both return the same x, A^* x and b - A^* x in exact
 * arithmetic; they differ in rounding (Sec. 1) and cost (Sec. 5). */
typedef enum {
    RTPROJ_METHOD_RANDOMIZED = 0, /* the preconditioned identity (eq. basic_precond)
                                     with P from the randomized sketch, and the
                                     refinement of Remark 4.3 (the default)          */
    RTPROJ_METHOD_CLASSICAL = 1,  /* eq. basic_identity evaluated directly: A A^*
                                     (binary64 MFMA), its Householder pivoted QR,
                                     x = Pi R^{-1} Q^T (A b), no refinement; the
                                     comparison scheme of Sec. 5 (s_pre, s_pro,
                                     delta_norm, epsilon_norm); m <= 4096          */
    RTPROJ_METHOD_KRYLOV = 2      /* the iterative variant (Sec. 1: a
                                     preconditioned iterative approach is also
                                     feasible): the sketch, its pivoted QR and
                                     R^{-T} only (no P^{-1}A, Gram or inverse);
                                     every solve with A A^* = P (W W^*) P^* runs
                                     conjugate gradients on the well-conditioned
                                     W W^*, W = P^{-1}A, applying W and W^* as
                                     R^{-T} Pi A and A^* Pi^T R^{-1} (two passes
                                     over A per iteration; the iteration count is
                                     set by rtproj_plan_set_krylov), inside the
                                     refinement of Remark 4.3                      */
} rtproj_method;

typedef struct {
    int64_t m, n, l;           /* sizes of the plan                                  */
    int64_t np;                /* padded Fourier length of the sketch               */
    double kappa_est;          /* |R_11 / R_mm| of the pivoted QR of the sketch      */
    double rdiag_min;          /* |R_mm|                                             */
    int precision;             /* rtproj_precision of the last precondition          */
    int refine_steps;          /* refinement steps taken by the last projection     */
    double refine_last_ratio;  /* |dx| / |x| of the last refinement step             */
    int qrcp_blocks;           /* workgroups of the cooperative pivoted QR           */
    int sketch_bits, w_bits, gram_bits; /* precisions used by the last precondition:
                                   64 binary64, 32 binary32, 16 bfloat16, 17 split
                                   bfloat16 (hi + lo halves)                         */
    int sketch_escalated;      /* a binary32 sketch was redone in binary64: 1 right
                                  after the pivoted QR (2^-24 kappa_est > 1, or a
                                  failed rank test), 2 after the Gram (gram_cond_est
                                  > 10); 0 otherwise                                */
    double gram_cond_est;      /* a lower bound on cond(P^{-1}A): Newton-Schulz
                                   sqrt(max_i X_ii max_i Y_ii); Cholesky max/min
                                   of diag(L)                                        */
    /* Per-stage device time, accumulated since rtproj_plan_set_timing(plan, 1),
     * measured with HIP events on the plan's stream (zero while timing is off).
     * Stages: 0 sketch, 1 pivoted QR, 2 R^{-T} solve, 3 P^{-1}A product, 4 Gram,
     * 5 inverse of the Gram (Newton-Schulz iterations, or the Cholesky),
     * 6 the factor T' of M^{-1} (Newton-Schulz: R^{-T} Pi; Cholesky: the
     * solve L^{-1}R^{-T}), 7 A b, 8 applications of (AA^T)^{-1},
     * 9 refinement residual b - A^T x, 10 refinement product A r,
     * 11 final A^T x and b - A^T x, 12 the small factor R0 of the two-stage
     * pivoted QR; 9, 10 and 11 count the compensated passes, and the plain
     * binary64 ones are 13 (residual), 14 (product A r) and 15 (final,
     * including the final pass formed from the last compensated residual). */
    double t_stage_ms[16];
    int64_t stage_calls[16];
    int qr_mode;               /* rtproj_qr_mode used by the last precondition       */
    int inverse;               /* rtproj_inverse used by the last precondition
                                  (1 or 2)                                          */
    int inverse_iters;         /* Newton-Schulz iterations (0 for Cholesky)          */
    double inverse_resid;      /* Newton-Schulz: |I - X Y_k|_F of the last iterate
                                  before the final step (the final residual is
                                  about its square, down to rounding); 0 for
                                  Cholesky                                          */
    int refine_plain;          /* steps of the last projection with plain residuals */
    int refine_comp;           /* steps with compensated residuals after them        */
    int resid_mode;            /* rtproj_residual used by the last projection
                                  (1, 2 or 3; 0 before any)                         */
    int refine_status;         /* RTPROJ_OK or RTPROJ_ERR_NOCONV for the last
                                  projection (evaluated by rtproj_plan_status or
                                  rtproj_plan_info)                                 */
    double refine_rho_est;     /* contraction per step estimated from the steps'
                                  corrections (|d_1|/|x_1| and ratios of
                                  successive same-kind corrections)                 */
    double refine_err_est;     /* relative error of x estimated after the last step:
                                  refine_rho_est times the last |d| / |x|            */
    double refine_rho_model;   /* contraction per step the schedule was planned with
                                  (see rtproj_plan_set_refinement)                  */
    int method;                /* rtproj_method of the last precondition             */
    int comp_method;           /* rtproj_compensation of the last projection's
                                  compensated steps (0 when none ran)            */
} rtproj_info;

/*
 * Create a plan for m x n matrices (1 <= m <= l <= n, Sec. 4: "m <= l <= n")
 * sketched to l columns; `seed` fixes the random sketch (signs, permutations,
 * subsample; see rtproj_sketch_tables).  Allocates device memory on the
 * current HIP device.  On error *out is NULL.
 */
rtproj_status rtproj_plan_create(int64_t m, int64_t n, int64_t l, uint64_t seed, rtproj_plan *out);

/* Release every resource of the plan (NULL is accepted). */
rtproj_status rtproj_plan_destroy(rtproj_plan plan);

/* Stream (a hipStream_t) on which the plan enqueues its work. */
rtproj_status rtproj_plan_set_stream(rtproj_plan plan, void *hip_stream);

/* Precision of the preconditioner (rtproj_precision).  Takes effect at the
 * next rtproj_precondition; projections plan their refinement for the
 * precision the preconditioner in use was built with. */
rtproj_status rtproj_plan_set_precision(rtproj_plan plan, int precision);

/* Precision of P^{-1}A in the reduced-precision modes: 0 (default) binary32
 * while the rank estimate allows it (kappa_est <= 1e5), else binary64; 32 or
 * 64 forces it.  Forcing binary32 on an ill-conditioned A makes the
 * preconditioner too poor for the refinement to contract (Remarks 4.2 and
 * 4.3), which rtproj_plan_status then reports as RTPROJ_ERR_NOCONV.  Takes
 * effect at the next rtproj_precondition; RTPROJ_ERR_INVALID_ARG for other
 * values. */
rtproj_status rtproj_plan_set_w_bits(rtproj_plan plan, int bits);

/* Method (rtproj_method); default RTPROJ_METHOD_RANDOMIZED.  Takes effect
 * at the next rtproj_precondition.  RTPROJ_ERR_INVALID_ARG for an unknown
 * value; RTPROJ_ERR_UNSUPPORTED for the classical scheme with m > 4096.
 * With RTPROJ_METHOD_CLASSICAL, rtproj_precondition forms A A^* and its
 * pivoted QR (kappa_est then reports |R_11 / R_mm| of that QR, about
 * cond(A)^2, and fails only on a zero or non-finite pivot), the projections
 * compute x = Pi R^{-1} Q^T A b and A^* x, b - A^* x in plain binary64, and
 * the refinement and residual settings do not apply. */
rtproj_status rtproj_plan_set_method(rtproj_plan plan, int method);

/* Sketch with the caller's dense n x l matrix G (device, row-major, element
 * (t, j) at G[t*ldg + j], ldg >= l) in place of the subsampled randomized
 * Fourier transform: S = A G (eq. testing) in binary64 on MFMA, as the
 * paper's experiments draw G (i.i.d. Gaussian, or lagged Fibonacci uniform
 * on [-1, 1]; Sec. 5).  G is borrowed from the next rtproj_precondition
 * until G is replaced or cleared (G = NULL restores the SRFT).  The
 * projections do not depend on G (eq. basic_precond is an identity); only
 * the conditioning of P^{-1}A does (Lemma 2.4).  Costs 2 m n l flops per
 * precondition. */
rtproj_status rtproj_plan_set_sketch_matrix(rtproj_plan plan, const double *G, int64_t ldg);

/* Conjugate-gradient iterations per solve of the iterative method
 * (RTPROJ_METHOD_KRYLOV); default 30, which takes the error of a solve to
 * about 2 (0.6)^30 = 4e-7 when cond(P^{-1}A) <= 4 (Observation 3.2 with
 * l = 4m); 1 to 500, else RTPROJ_ERR_INVALID_ARG.  Takes effect at the next
 * projection. */
rtproj_status rtproj_plan_set_krylov(rtproj_plan plan, int iters);

/* Autotuning of the preconditioner's large contractions (1 on, 0 off, the
 * default).  When on, the first rtproj_precondition of a shape times every
 * candidate configuration of the product P^{-1}A (64 or 128 square tiles,
 * plain or XCD-grouped tile order) and of its Gram (split-K counts, tile
 * size) on the plan's stream with the real operands, keeps the fastest in a
 * process-wide table keyed by operation, number type and sizes, and uses it
 * for every later preconditioning of that shape (on any plan with autotuning
 * on).  The tuning precondition takes the candidates' extra time and waits
 * on the stream once per candidate. */
rtproj_status rtproj_plan_set_autotune(rtproj_plan plan, int enable);
/* Save or load the autotuner's table (text, one entry per line: key and
 * integers).  Loading adds to (and overrides entries of) the table in
 * memory; RTPROJ_ERR_INVALID_ARG for an unreadable file or a malformed line. */
rtproj_status rtproj_autotune_save(const char *path);
rtproj_status rtproj_autotune_load(const char *path);
/* Entries in the autotuner's table. */
int rtproj_autotune_entries(void);

/* Arithmetic of the refinement residuals (rtproj_residual); default
 * RTPROJ_RESID_AUTO.  Takes effect at the next projection. */
rtproj_status rtproj_plan_set_residual(rtproj_plan plan, int mode);

/* Form of the compensated products (rtproj_compensation); default
 * RTPROJ_COMP_AUTO.  Takes effect at the next projection (the integer form
 * allocates its digit buffers then). */
rtproj_status rtproj_plan_set_compensation(rtproj_plan plan, int method);

/* Method of the pivoted QR of the sketch (rtproj_qr_mode).  Takes effect at
 * the next rtproj_precondition; RTPROJ_ERR_UNSUPPORTED if the mode cannot
 * handle the plan's sizes. */
rtproj_status rtproj_plan_set_qr(rtproj_plan plan, int mode);

/* Method of the Gram's inverse (rtproj_inverse).  Takes effect at the next
 * rtproj_precondition; RTPROJ_ERR_INVALID_ARG for an unknown value. */
rtproj_status rtproj_plan_set_inverse(rtproj_plan plan, int method);

/*
 * Iterative refinement of the least-squares solution (Remark 4.3): up to
 * `max_steps` steps x <- x + M^{-1} A (b - A^T x) with M = P X P^T the
 * preconditioned normal matrix.  rtol > 0 stops early once |dx| <= rtol |x|
 * (one device-to-host read per step) and returns RTPROJ_ERR_NOCONV from the
 * projection itself when the steps stopped contracting; rtol = 0 runs
 * exactly the scheduled steps without any host synchronisation.
 * max_steps = 0 returns the unrefined projection (the seven steps of Sec. 4
 * in binary64); max_steps = -1 (the default) chooses the schedule from the
 * rank estimate kappa_est of the pivoted QR, with the contraction per step
 * modelled as rho = 16 u kappa_est (binary64 P^{-1}A) or 2 u_32 kappa_est
 * (binary32 P^{-1}A), plus the Gram's rounding (u_32 K / 32 for a Gram
 * accumulated in binary32 over K terms per split, plus 4e-3 for bfloat16
 * inputs), and the floor of a plain binary64 residual as 16 u kappa_est
 * (relative error of x; rtproj_info.refine_rho_model reports rho): plain
 * steps while the
 * error is above that floor, then, unless the floor itself is below the goal
 * 1e-11, compensated steps until rho^s times the error is <= 1e-11.  In
 * RTPROJ_RESID_AUTO the compensated steps compensate r and s, and after
 * them the final projections come from the last compensated residual as in
 * RTPROJ_RESID_FULL.  An explicit
 * max_steps runs that many compensated steps (plain ones in
 * RTPROJ_RESID_PLAIN).
 */
rtproj_status rtproj_plan_set_refinement(rtproj_plan plan, int max_steps, double rtol);

/*
 * Build the preconditioner for A (row-major m x n, lda >= n, device):
 * sketch S = A G (eq. testing), pivoted QR S^T = Q R Pi (eq. QR_decomp),
 * P^- = Pi^T R^{-1} (eq. scary) in its transposed form R^{-T}, the
 * preconditioned matrix P^{-1}A = R^{-T} Pi A, its Gram X (the matrix X of
 * Sec. 4, steps a-e) and Y = X^{-1} (eq. inversion): by default Newton-
 * Schulz iterations for m <= 1024 and a Cholesky factor of X above that
 * (rtproj_plan_set_inverse).  Blocks the host until the pivoted QR is done
 * (rank test) and until the inverse is formed (its residual or breakdown).
 * In the reduced-precision modes a binary32 sketch is redone in binary64
 * when the rank estimate shows it too coarse (2^-24 kappa_est > 1), or when
 * the Gram shows a poorly conditioned P^{-1}A.  Returns RTPROJ_ERR_RANK if
 * |R_mm| <= m * 2^-52 * |R_11|, the Cholesky breaks down or Newton-Schulz
 * does not converge.  A is borrowed (see above).
 */
rtproj_status rtproj_precondition(rtproj_plan plan, const double *A, int64_t lda);

/*
 * Apply the projector to k right-hand sides (B column-major n x k, ldb >= n):
 *   rtproj_project_null: Z = B - A^T X   (ldz >= n)
 *   rtproj_project_row:  Y = A^T X       (ldy >= n)
 *   rtproj_lstsq:        X               (ldx >= m)
 *   rtproj_project_all:  any of Z, Y, X (NULL to skip)
 * following the seven steps of Sec. 4 (c = A b, d = Pi c, R^T e = d,
 * f = Y e, R g = f, h = Pi^T g, b~ = A^T h) plus the refinement configured by
 * rtproj_plan_set_refinement.  k = 0 is a no-op.  RTPROJ_ERR_STATE before
 * the first successful rtproj_precondition.
 */
rtproj_status rtproj_project_null(rtproj_plan plan, const double *B, int64_t ldb, int64_t k,
                                  double *Z, int64_t ldz);
rtproj_status rtproj_project_row(rtproj_plan plan, const double *B, int64_t ldb, int64_t k,
                                 double *Y, int64_t ldy);
rtproj_status rtproj_lstsq(rtproj_plan plan, const double *B, int64_t ldb, int64_t k,
                           double *X, int64_t ldx);
rtproj_status rtproj_project_all(rtproj_plan plan, const double *B, int64_t ldb, int64_t k,
                                 double *Z, int64_t ldz, double *Y, int64_t ldy,
                                 double *X, int64_t ldx);

/*
 * As rtproj_project_all, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the projection's workspace (for k right-hand sides) is taken
 * from a static 64 MiB device array that the library holds on every GPU it
 * runs on until the process ends, not from buffers the plan grows.  The
 * call allocates nothing; the plan itself (created and preconditioned
 * beforehand) and the caller's B and outputs are used as by
 * rtproj_project_all.  RTPROJ_ERR_UNSUPPORTED for a plan preconditioned
 * with RTPROJ_METHOD_KRYLOV, and when the workspace for (m, n, k) exceeds
 * 64 MiB (about m k (5 + 2 splits) + 2 n k doubles; split
 * the right-hand sides over several calls).  All calls on one GPU share the
 * array and every call overwrites it: calls that overlap in time on one GPU
 * (different streams, threads) race; order them on one stream.
 */
rtproj_status rtproj_project_all_noalloc(rtproj_plan plan, const double *B, int64_t ldb, int64_t k,
                                         double *Z, int64_t ldz, double *Y, int64_t ldy, double *X, int64_t ldx);

/* Enable (1, also resets the accumulated stage times) or disable (0) the
 * per-stage event timing reported in rtproj_info.t_stage_ms. */
rtproj_status rtproj_plan_set_timing(rtproj_plan plan, int enable);

/* Sizes, rank estimate, refinement and stage-timing statistics (synchronises
 * the stream and evaluates the last projection's convergence check). */
rtproj_status rtproj_plan_info(rtproj_plan plan, rtproj_info *out);

/* Waits for the plan's stream and returns the outcome of the last
 * projection's refinement (Remarks 4.2 and 4.3): RTPROJ_ERR_NOCONV when a
 * step's correction did not shrink to at most half the previous one while
 * corrections were still above 1e-11 |x|, or when the error estimated after
 * the last step (the estimated contraction times the last |dx| / |x|) is
 * above 1e-10; the outputs then hold the last iterate.  RTPROJ_OK otherwise,
 * and when nothing was refined. */
rtproj_status rtproj_plan_status(rtproj_plan plan);

/*
 * Copy plan state to device buffers supplied by the caller (synchronous):
 *   S    m x l row-major sketch (lds >= l; NULL to skip)
 *   R    m x m row-major upper-triangular factor of the pivoted QR (NULL to skip)
 *   piv  m int32: column k of S^T Pi^T is column piv[k] of S^T (NULL to skip)
 *   Minv m x m row-major M^{-1} = (P^*)^{-1} Y P^{-1}, the approximation of
 *        (A A^*)^{-1} the projections apply (NULL to skip)
 * RTPROJ_ERR_STATE before preconditioning.
 */
rtproj_status rtproj_plan_export(rtproj_plan plan, double *S, int64_t lds, double *R,
                                 int32_t *piv, double *Minv);

/*
 * Host copies of the plan's random sketch tables (for inspection):
 * sign[np] (+1/-1), sigma[n1], tau[n2] (permutations), J[l] (sorted subset of
 * [0, np)), with np = max(4, 2^ceil(log2 n)), n2 = 2^floor(log2(np)/2),
 * n1 = np / n2.  Any pointer may be NULL; dims may be NULL.
 */
rtproj_status rtproj_sketch_tables(rtproj_plan plan, int64_t *dims3, int8_t *sign,
                                   int32_t *sigma, int32_t *tau, int32_t *J);

/*
 * Batches: `count` independent problems of uneven sizes (member i is an
 * m[i] x n[i] matrix sketched to l[i] columns, 1 <= m[i] <= l[i] <= n[i],
 * m[i] <= 2048), preconditioned and projected together with ONE grouped
 * launch per stage of the path for all members.  The pivoted QR of member i
 * is the two-stage form (R0 of S^T = Q0 R0 by shifted Cholesky QR, then the QRCP of
 * R0, in one workgroup per member or, for few large members, in a group of
 * blocks per member that synchronize only among themselves; the batch picks
 * the faster from the sizes and rtproj_batch_info reports it as qr_mode
 * RTPROJ_QR_TWO_STAGE_WG or RTPROJ_QR_TWO_STAGE), so no step waits on the host: rank tests
 * and factorization breakdowns are reported afterwards by
 * rtproj_batch_status.  Member i's sketch seed is the first output of
 * SplitMix64 seeded with seed XOR i.  Arithmetic is binary64 with
 * compensated refinement residuals, as for a plan, except for a binary32
 * Gram with rtproj_batch_set_precision.
 *
 * Array arguments (A, lda, B, ldb, k, Z, ...) are HOST arrays of `count`
 * entries; the pointers in them are device pointers with the layouts of
 * the single-problem calls.  A[i] is borrowed as for rtproj_precondition.
 * With rtproj_batch_set_graph(batch, 1) each entry point records its grouped
 * launches into a HIP graph on first use and replays it while the arguments
 * (pointers, sizes, k) stay the same.  Calls are asynchronous on the batch's
 * stream except when new arguments must be uploaded (a short host wait).
 */
typedef struct rtproj_batch_s *rtproj_batch;

rtproj_status rtproj_batch_create(int64_t count, const int64_t *m, const int64_t *n, const int64_t *l, uint64_t seed,
                                  rtproj_batch *out);
rtproj_status rtproj_batch_destroy(rtproj_batch batch);
rtproj_status rtproj_batch_set_stream(rtproj_batch batch, void *hip_stream);
/* Refinement of every member (Remark 4.3): steps >= 0 compensated steps
 * x <- x + M^{-1} A (b - A^T x); -1 (the default) the schedule of
 * rtproj_plan_set_refinement for the least favourable member's rank
 * estimate (plain binary64 residuals above their floor, compensated after),
 * which reads the estimates once per projection call (a short host wait). */
rtproj_status rtproj_batch_set_refinement(rtproj_batch batch, int steps);
/* Precision of every member's preconditioner: RTPROJ_PREC_FP64 (default);
 * RTPROJ_PREC_MIXED_FP32, whose Gram of P^{-1}A runs on binary32 MFMA
 * (grouped over the members) with binary64 operands and reduction; or
 * RTPROJ_PREC_MIXED_BF16X3, whose P^{-1}A is stored in binary32 and whose
 * Gram is the split-bfloat16 one (hi + lo halves, three bfloat16 products,
 * grouped over the members) when every member has n % 4 == 0, else the
 * binary32 one (member info reports gram_bits 17 or 32).  Both reduced
 * precisions sketch in binary32 arithmetic and then read every member's rank
 * estimate once (a short host wait in rtproj_batch_precondition): when a
 * member's sketch proves too coarse (2^-24 kappa_est > 1, a failed rank test,
 * or a Gram condition estimate above 10) all members are sketched again in
 * binary64 (member info: sketch_bits, sketch_escalated).  The products
 * themselves, the factorizations and the refinement residuals stay binary64,
 * and the refinement schedule accounts for the Gram's rounding (Remark 4.3).
 * RTPROJ_ERR_UNSUPPORTED for RTPROJ_PREC_MIXED_BF16.  Takes effect at the
 * next rtproj_batch_precondition. */
rtproj_status rtproj_batch_set_precision(rtproj_batch batch, int precision);
/* 1: capture each entry point's launches into a HIP graph and replay it. */
rtproj_status rtproj_batch_set_graph(rtproj_batch batch, int enable);
rtproj_status rtproj_batch_precondition(rtproj_batch batch, const double *const *A, const int64_t *lda);
/* As rtproj_batch_precondition for the column-scaled matrices A[i] diag(d[i])
 * (an interior-point step rescales a fixed A by a positive diagonal):
 * col_scale[i] points to n[i] doubles on the device, or is NULL for an
 * unscaled member.  No scaled copy is made: every pass that reads a scaled
 * member's A forms its elements A[i][r][t] * d[t] as it loads them (the
 * products with A rounded element by element as a scaled copy would be), so
 * col_scale[i] is borrowed like A[i] and must stay valid and unchanged until
 * the last projection that uses this preconditioning. */
rtproj_status rtproj_batch_precondition_scaled(rtproj_batch batch, const double *const *A, const int64_t *lda,
                                              const double *const *col_scale);
/* As rtproj_project_all per member; Z, Y, X (or their entries) may be NULL;
 * k[i] = 0 skips member i. */
rtproj_status rtproj_batch_project_all(rtproj_batch batch, const double *const *B, const int64_t *ldb,
                                       const int64_t *k, double *const *Z, const int64_t *ldz, double *const *Y,
                                       const int64_t *ldy, double *const *X, const int64_t *ldx);
/* Waits for the batch's stream and reports, per member (per_member may be
 * NULL), RTPROJ_OK, RTPROJ_ERR_RANK (|R_mm| <= m 2^-52 |R_11|, a NaN in A,
 * or a Cholesky breakdown), RTPROJ_ERR_DEVICE (a block barrier of the grouped
 * pivoted QR timed out) or RTPROJ_ERR_NOCONV (the member's refinement in
 * the last rtproj_batch_project_all did not converge, judged as in
 * rtproj_plan_status); returns RTPROJ_ERR_RANK if any member has it, else
 * RTPROJ_ERR_DEVICE if any member has it, else RTPROJ_ERR_NOCONV if any
 * member has it, else RTPROJ_OK. */
rtproj_status rtproj_batch_status(rtproj_batch batch, int *per_member);
/* Per-stage device time of the batch (stage indices as in rtproj_info),
 * accumulated while enabled; only eager (non-graph) calls are timed, and a
 * timed call waits for its stream. */
rtproj_status rtproj_batch_set_timing(rtproj_batch batch, int enable);
/* Batch totals: largest m, n, l; refinement steps; stage times. */
rtproj_status rtproj_batch_info(rtproj_batch batch, rtproj_info *out);
/* Host copies of member i's sketch tables, as rtproj_sketch_tables for a
 * plan (member i draws them from instance seed i, see above). */
rtproj_status rtproj_batch_member_tables(rtproj_batch batch, int64_t i, int64_t *dims3, int8_t *sign, int32_t *sigma,
                                         int32_t *tau, int32_t *J);
/* Sizes and the rank estimates of member i (valid after rtproj_batch_status). */
rtproj_status rtproj_batch_member_info(rtproj_batch batch, int64_t i, rtproj_info *out);

/*
 * Complex-valued A (Sec. 1: the method and its analysis extend to complex
 * entries).  x = argmin |A^* x - b| with A^* the conjugate transpose, the
 * row projection A^* x and the null projection b - A^* x, for a complex
 * m x n A of rank m.  Complex arrays are interleaved (re, im) binary64
 * pairs in device memory, 16-byte aligned (std::complex<double>,
 * torch.complex128), with leading dimensions in complex elements and the
 * layouts of the real calls: A row-major m x n (lda >= n), B, Z, Y
 * column-major n x k, X column-major m x k.
 *
 * A complex plan runs a real plan of sizes (2m, 2n, 2l) on the real 2m x 2n
 * matrix [Re A, -Im A; Im A, Re A], which maps [Re b; Im b] to [Re Ab; Im Ab]
 * and whose transpose acts as A^*; the embedding is an isometry, so its
 * projections and least-squares solution are those of A, and its condition
 * number is cond(A).  The plan owns the embedded copy (4 m n doubles, formed
 * at each rtproj_cprecondition, so A is not borrowed) and embedded
 * right-hand sides and outputs (grown with k).  rtproj_cplan_real returns
 * the real plan for the setters, rtproj_plan_info and rtproj_plan_status
 * (its sizes are 2m, 2n, 2l).  Errors as for the real calls.
 */
typedef struct rtproj_cplan_s *rtproj_cplan;
rtproj_status rtproj_cplan_create(int64_t m, int64_t n, int64_t l, uint64_t seed, rtproj_cplan *out);
rtproj_status rtproj_cplan_destroy(rtproj_cplan plan);
rtproj_plan rtproj_cplan_real(rtproj_cplan plan);
rtproj_status rtproj_cprecondition(rtproj_cplan plan, const double *A, int64_t lda);
rtproj_status rtproj_cproject_all(rtproj_cplan plan, const double *B, int64_t ldb, int64_t k, double *Z, int64_t ldz,
                                  double *Y, int64_t ldy, double *X, int64_t ldx);

const char *rtproj_status_string(rtproj_status status);
const char *rtproj_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RTPROJ_H */
