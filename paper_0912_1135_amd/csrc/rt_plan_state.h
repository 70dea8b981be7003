// Internal state of a plan, shared by the single-problem runtime (rt_plan.hip)
// and the batched runtime (rt_batch.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "../../include/rtproj.h"
#include "rt_common.h"

namespace rtp {


// Records the message returned by rtproj_last_error() and returns s.
rtproj_status fail(rtproj_status s, const std::string &msg);
extern thread_local std::string g_last_error;

#define RT_HIP(expr)                                                                                  \
    do {                                                                                              \
        hipError_t _e = (expr);                                                                       \
        if (_e != hipSuccess)                                                                         \
            return fail(RTPROJ_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));        \
    } while (0)

constexpr int NB = 64;  // block size of the triangular solves and the Cholesky
// right-hand sides from which the plain binary64 A-passes run as MFMA GEMMs
constexpr int64_t RT_MFMA_KMIN = 32;
// right-hand sides from which the compensated products take the int8-MFMA form
constexpr int64_t RT_OZ_KMIN = 16;
// P^{-1}A is formed in binary32 only while the rank estimate of the pivoted QR
// is at most this: its rounding error grows like 2^-24 kappa and must leave
// the refinement a contraction well below 1.
constexpr double RT_W32_KAPPA_MAX = 1e5;
// Reduced-precision modes redo the sketch in binary64 when max/min diag of
// the Gram's Cholesky factor exceeds this (a healthy preconditioner gives ~3).
constexpr double RT_COND_ESCALATE = 10.0;
// Two-stage QR: a third Cholesky QR pass runs when the second factor's
// diagonal spans more than 1 / RT_CQR_THIRD (its iterate nearly rank
// deficient, so the two-pass R0 would resolve the smallest singular values
// of the sketch only to about sqrt(u) |S|).
constexpr double RT_CQR_THIRD = 1e-5;
// Automatic choice of the Gram inverse: Newton-Schulz (about a dozen pairs of
// m^3 products, latency-light) up to this m, the blocked Cholesky (m^3 / 3,
// but a chain of small diagonal steps) above it.
constexpr int64_t RT_NS_MAX_M = 1024;
// Newton-Schulz: iterations of the first round, after the first step from
// a I (a = 1 / |X|_inf) that the start kernel forms elementwise (a Gram
// sketched at l = 4m has |X|_inf about 5 lambda_max and condition about 8.5;
// its residual is below 1e-10 after these; harder Grams take further rounds
// sized from the measured residual), the residual
// |I - X Y_k|_F below which Y_{k+1} is final, the largest residual accepted
// as a rounding floor once it stops squaring, and the iteration cap.  The
// iterates are used as computed, never symmetrised: I - X Y_{k+1} =
// (I - X Y_k)^2 holds for any Y_k, while a symmetrised product drifts when the
// computed Y_k does not commute with X.
constexpr int RT_NS_FIRST = 10;
constexpr double RT_NS_DONE = 1e-6;
constexpr double RT_NS_FLOOR = 1e-4;
constexpr int RT_NS_MAX_IT = 64;
// Largest m whose Newton-Schulz products run as one fused launch per product
// (one wave per 16 x 16 tile, whole K; its L2 reads grow as m^3).
constexpr int64_t RT_NS_FUSED_MAX_M = 256;
// Largest block of right-hand sides whose M^{-1} products run as one launch
// each (skinny product kernel) instead of a split GEMM and its reduction.
constexpr int64_t RT_SKINNY_KMAX = 64;
// Refinement planner.  Accuracy goal of the automatic schedule: a tenth of
// the 1e-10 relative error the projections are specified to (room for the
// model's constants).  The rank estimate |R_11 / R_mm| of the pivoted QR
// understates cond(A) (by 18 to 40 times in the measured workloads); the
// planner's constants below absorb that factor.
constexpr double RT_REFINE_GOAL = 1e-11;
// Relative error of x at which a refinement with a plain binary64 residual
// stalls: about RT_FLOOR_C u kappa_est (measured 7e-9 at cond(A) = 1e8,
// kappa_est = 4.7e6: RT_FLOOR_C u kappa_est = 8.3e-9).
constexpr double RT_FLOOR_C = 16.0;
// A binary32 sketch is redone in binary64 before anything else is built on
// it when 2^-24 kappa_est exceeds this (the sketch's rounding then reaches
// the small singular directions: healthy at 0.15, degraded at 6, measured).
constexpr double RT_SKETCH32_MAX = 1.0;
// Refinement steps recorded per projection for the convergence check.
constexpr int RT_MAX_STEPS = 80;
// Convergence check of a projection's refinement (Remarks 4.2 and 4.3): the
// iteration did not converge when a step's correction did not shrink to at
// most this fraction of the previous one while corrections are still above
// RT_NC_ACTIVE |x|, or when the error estimated after the last step
// (contraction estimate times the last relative correction) is above
// RT_NC_TOL.
constexpr double RT_NC_RATIO = 0.5;
constexpr double RT_NC_ACTIVE = 1e-11;
constexpr double RT_NC_TOL = 1e-10;

// ------------------------------------------------------------ random tables
// SplitMix64 (Steele, Lea and Flood, 2014): the state advances by the golden
// ratio increment and each output is the finalizer of the new state.
struct SplitMix64 {
    uint64_t s;
    uint64_t next()
    {
        s += 0x9e3779b97f4a7c15ULL;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        return z ^ (z >> 31);
    }
    // uniform in [0, range): high half of next() * range
    uint64_t below(uint64_t range) { return (uint64_t)(((unsigned __int128)next() * range) >> 64); }
};

struct HostTables {
    int64_t np = 0, n1 = 0, n2 = 0;
    std::vector<int8_t> sign;
    std::vector<int32_t> sigma, tau, J;
};

// Draw order: np signs (top bit set -> -1), Fisher-Yates of sigma over
// [0, n1) from the top, the same for tau over [0, n2), then the sorted
// l-subset J of [0, np) by selection sampling.
inline void draw_tables(uint64_t seed, int64_t n, int64_t l, HostTables &t)
{
    int64_t np = 4;
    int e = 2;
    while (np < n) { np <<= 1; ++e; }
    t.np = np;
    t.n2 = int64_t(1) << (e / 2);
    t.n1 = np / t.n2;
    SplitMix64 g{seed};
    t.sign.resize(np);
    for (int64_t i = 0; i < np; ++i) t.sign[i] = (g.next() >> 63) ? int8_t(-1) : int8_t(1);
    t.sigma.resize(t.n1);
    for (int64_t i = 0; i < t.n1; ++i) t.sigma[i] = (int32_t)i;
    for (int64_t j = t.n1 - 1; j >= 1; --j) std::swap(t.sigma[j], t.sigma[g.below((uint64_t)j + 1)]);
    t.tau.resize(t.n2);
    for (int64_t i = 0; i < t.n2; ++i) t.tau[i] = (int32_t)i;
    for (int64_t j = t.n2 - 1; j >= 1; --j) std::swap(t.tau[j], t.tau[g.below((uint64_t)j + 1)]);
    t.J.clear();
    t.J.reserve(l);
    for (int64_t i = 0; i < np && (int64_t)t.J.size() < l; ++i)
        if ((int64_t)g.below((uint64_t)(np - i)) < l - (int64_t)t.J.size()) t.J.push_back((int32_t)i);
}

inline void twiddles(int64_t len, int64_t count, int64_t step, std::vector<double> &out)
{
    // out[j] = exp(-2 pi i j*step / len), j < count, from long-double cos/sin
    out.resize(2 * count);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int64_t j = 0; j < count; ++j) {
        const long double ang = -2.0L * pi * (long double)((j * step) % len) / (long double)len;
        out[2 * j] = (double)cosl(ang);
        out[2 * j + 1] = (double)sinl(ang);
    }
}

template <class T>
hipError_t dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void **)p, count * sizeof(T));
}


}  // namespace rtp

// Grouped products of the recursive-doubling inverse X = L^{-1} of an m x m
// lower-triangular L (see build_tri_inverse): per level, the pairs joined and
// the launch shapes of its two grouped products; d_args holds every level's
// argument blocks (first products, then second products, level by level).
struct TriInverse {
    rt::GemmArgs *d_args = nullptr;
    std::vector<int> count;
    std::vector<rt::GemmShape> shape1, shape2;
};

struct rtproj_plan_s {
    int64_t m = 0, n = 0, l = 0;
    uint64_t seed = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    int cu_count = 0;
    size_t lds_max = 0;
    int precision = RTPROJ_PREC_FP64;
    int refine_steps = -1;  // -1: chosen from the rank estimate of the pivoted QR
    double refine_rtol = 0.0;
    int resid_mode = RTPROJ_RESID_AUTO;  // rtproj_residual requested
    int w_bits_req = 0;        // 0: P^{-1}A precision from the rank estimate; 32 or 64 forced
    int prec_used = RTPROJ_PREC_FP64;    // precision of the last precondition
    // convergence check of the last projection: per-step |d|^2, |x|^2 copied
    // to pinned memory; evaluated at the next call that waits on the stream
    double *h_norms = nullptr;  // pinned, 2 RT_MAX_STEPS
    int nc_steps = 0;           // steps recorded (0: nothing pending)
    int nc_plain = 0;           // of which plain (the first ones)
    bool nc_pending = false;
    bool resketch = false;      // the binary32 sketch must be redone in binary64
    int method = RTPROJ_METHOD_RANDOMIZED;  // requested (rtproj_method)
    int method_used = RTPROJ_METHOD_RANDOMIZED;  // of the last precondition
    double *d_V = nullptr, *d_tau = nullptr;  // classical scheme: reflectors of the QR of A A^T
    bool autotune = false;         // time candidate configurations of new shapes (rt_tune.hip)
    int part_cap = 0;              // split partials d_part holds (m x m doubles each)
    int krylov_iters = 30;         // CG iterations per solve of the iterative method
    double *d_kry = nullptr;       // its vectors: u, r, pp, q, w (m x kcap each) and kcap gammas
    int64_t kry_cap = 0;
    const double *Gmat = nullptr;  // caller's dense sketch matrix (n x l row-major), borrowed; null: SRFT
    int64_t ldg = 0;
    double *d_gpart = nullptr;     // split partials of S = A G
    int64_t gpart_cap = 0;
    rtp::HostTables tab;
    // device tables
    int8_t *d_sign = nullptr;
    int32_t *d_sigma = nullptr, *d_tauinv = nullptr, *d_sel_off = nullptr, *d_sel = nullptr;
    double *d_tw1 = nullptr, *d_tw2 = nullptr, *d_twh = nullptr, *d_twl = nullptr;
    float *d_tw1f = nullptr, *d_tw2f = nullptr, *d_twhf = nullptr, *d_twlf = nullptr;
    int tl_bits = 0;
    // preconditioner state
    double *d_zbuf = nullptr;
    int64_t rows_chunk = 0;
    double *d_S = nullptr, *d_R = nullptr, *d_Y = nullptr, *d_W = nullptr, *d_part = nullptr;
    int64_t ldw = 0;           // row stride of d_W (elements of its storage type)
    double *d_G = nullptr, *d_L = nullptr, *d_Tp = nullptr, *d_DinvR = nullptr, *d_DinvL = nullptr;
    int32_t *d_piv = nullptr;
    unsigned *d_sync = nullptr;
    double *d_slots = nullptr, *d_vbuf = nullptr, *d_qrcols = nullptr, *d_scal = nullptr, *d_diag = nullptr;
    int *d_err = nullptr;
    float *d_rowscale = nullptr;
    // the cooperative Cholesky: blocks on this device (0: the blocked
    // multi-launch form), its task flags and the epoch of the last call
    int chol_blocks = 0;
    unsigned *d_cflags = nullptr;
    unsigned chol_epoch = 0;
    int qr_blocks = 0;         // cooperative blocks for the l x m QRCP (direct mode)
    int qr_blocks0 = 0;        // cooperative blocks for the m x m QRCP of R0
    int qr_reg_l = 0, qr_reg_m = 0;  // blocks of the register-resident form (0: not applicable)
    int qr_mode = RTPROJ_QR_AUTO;
    int inv_method = RTPROJ_INV_AUTO;  // inverse of the Gram requested
    int inv_used = 0;          // RTPROJ_INV_NEWTON_SCHULZ or RTPROJ_INV_CHOLESKY, last precondition
    double *d_bsum = nullptr;  // block sums of squares of the Newton-Schulz residual (ns_bsum_count(m))
    double *d_Yq = nullptr;    // two-stage: the m x l iterate of the Cholesky QR
    double *d_Yq2 = nullptr;   // two-stage: the third pass's m x l iterate
    int r0_passes = 0;         // two-stage: Cholesky QR passes of the last R0 (2 or 3)
    double *d_R0 = nullptr;    // two-stage: R0^T (lower, row-major m x m)
    rt::QrcpWgArgs *d_wgargs = nullptr;
    // R^{-T} by recursive doubling: per level, the grouped products
    // T = L21 X11 and X21 = -X22 T over all block pairs (device argument
    // arrays built at plan creation)
    TriInverse rinv;           // R^{-T} into d_Y (scratch d_L)
    TriInverse linv[2];        // L^{-1} of the Cholesky factors in d_L and d_Y into d_Linv (scratch d_G)
    double *d_Linv = nullptr;  // two-stage: inverse of the current Cholesky factor
    bool w32 = false;          // P^{-1}A held in binary32 by the last precondition
    int syrk_splits = 1;
    int wgram_splits = 1;  // K splits of the Gram of P^-1 A (balanced over the compute units)
    int gram_splits_used = 1;  // those of the last precondition (the refinement schedule's Gram term)
    // projection workspace
    int64_t kcap = 0;
    int ab_splits = 1;
    int ab_mma_splits = 1;     // K splits of the MFMA form of A B (many right-hand sides)
    int oz_splits = 1;         // K splits of the int8-MFMA compensated A r
    bool oz_ready = false;     // the int8-MFMA buffers are sized for kcap
    double *d_oz_xdig = nullptr, *d_oz_rdig = nullptr, *d_oz_bexp = nullptr;  // (byte and int storage)
    int comp_method = RTPROJ_COMP_AUTO;
    int comp_used = 0;         // compensation form of the last projection's compensated steps
    int *d_colexp = nullptr, *d_rowexp = nullptr;  // exponents of A's columns and rows (int8-MFMA form)
    bool oz_exp_valid = false; // they describe the current A
    double *d_c = nullptr, *d_tmp = nullptr, *d_xhi = nullptr, *d_xlo = nullptr, *d_d = nullptr, *d_r = nullptr;
    double *d_ph = nullptr, *d_pl = nullptr, *d_norms = nullptr;
    double *d_bpk = nullptr;   // right-hand sides packed for the scalar-load A B pass (ab_pack_size(n, k))
    int ab_sx_splits = 1;      // column splits of that pass
    double *d_xpk = nullptr;   // x packed for the scalar-load A^T x pass (atx_pack_size(m, k))
    // borrowed operand
    const double *A = nullptr;
    int64_t lda = 0;
    bool ready = false;
    rtproj_info info{};
    // binary64 preconditions copy the Newton-Schulz norm slots here without
    // waiting (the refinement planner does not use the conditioning estimate
    // at binary64); rtproj_plan_info waits on the stream and derives it
    unsigned long long *h_scal = nullptr;  // pinned, 4 slots
    bool cond_pending = false;
    // stage timing (HIP events on the plan's stream)
    bool timing = false;
    struct StageEvents { int stage; hipEvent_t start, stop; };
    std::vector<StageEvents> pending;

    rt::SketchTables sketch_tables() const
    {
        rt::SketchTables t;
        t.n = n; t.np = tab.np; t.n1 = tab.n1; t.n2 = tab.n2; t.l = l;
        t.sign = d_sign; t.sigma = d_sigma; t.tau_inv = d_tauinv;
        t.tw1 = d_tw1; t.tw2 = d_tw2; t.twh = d_twh; t.twl = d_twl; t.tl_bits = tl_bits;
        t.tw1f = d_tw1f; t.tw2f = d_tw2f; t.twhf = d_twhf; t.twlf = d_twlf;
        t.sel_off = d_sel_off; t.sel = d_sel;
        return t;
    }
};

namespace rtp {

// Projection workspace for k right-hand sides: the split counts of the A B
// passes and the element count (doubles) of each buffer, in the order c,
// tmp, xhi, xlo, d, r, ph, pl, bpk, norms, xpk, and for the int8-MFMA
// compensated products (oz) the digits of x, the digits of r and the
// right-hand-side exponents.
struct ProjLayout {
    static constexpr int NBUF = 14;
    int ab_splits = 1, ab_sx_splits = 1, ab_mma_splits = 1;
    int oz_splits = 1;         // K splits of the int8-MFMA A r (when oz)
    bool oz = false;           // the int8-MFMA buffers are sized (else one element each)
    int64_t count[NBUF] = {};
    size_t bytes() const;  // every buffer rounded up to 256 bytes
};
ProjLayout proj_layout(int64_t m, int64_t n, int64_t k, int cu_count, bool oz);
// Whether the compensated products of a projection with k right-hand sides
// take the int8-MFMA form (the plan's setting; automatic: from 16 right-hand
// sides on, when m fits one int32 partial sum).
bool use_oz(rtproj_plan p, int64_t k);
// The plan's pointer to projection buffer i (order of ProjLayout::count).
double **proj_buffers(rtproj_plan p, int i);
// Grows the projection workspace of p to k right-hand sides.
rtproj_status ensure_k(rtproj_plan p, int64_t k);
// Projection of k right-hand sides through the plan's current workspace
// pointers (the body of rtproj_project_all).
rtproj_status project(rtproj_plan p, const double *B, int64_t ldb, int64_t k, double *Z, int64_t ldz, double *Y,
                      int64_t ldy, double *X, int64_t ldx);
// Device address of the library's static projection workspace on the
// current device, resolved once per device (at plan creation).
rtproj_status resolve_static_workspace(int device);
// A refinement schedule (see rtproj_plan_set_refinement): `plain` steps with
// binary64 residuals, then `comp` steps whose contraction s = A r (and, with
// comp_r, the residual r = b - A^T x) is compensated; the final A^T x is
// compensated when comp_final.  rho is the modelled contraction per step.
struct RefinePlan {
    int plain = 0, comp = 0;
    bool comp_r = true, comp_final = true;
    double rho = 0.5;
};
// Modelled contraction per refinement step (gram_k: terms per split-K
// partial sum of a reduced-precision Gram), and the schedule built on it.
double refine_rho_model(double kappa_est, int precision, bool w32, double cond_w, double gram_k);
RefinePlan refine_schedule(double kappa_est, int precision, bool w32, double cond_w, double gram_k, int mode,
                           int max_steps);
// Autotuner: key of an operation and its sizes; the process-wide table of
// chosen configurations; timing of `count` candidates on the plan's stream
// (run(c) enqueues candidate c), index of the fastest in *best.
std::string tune_key(const char *op, int64_t m, int64_t n, int64_t k);
bool tune_lookup(const std::string &key, std::vector<int> &choice);
void tune_store(const std::string &key, const std::vector<int> &choice);
rtproj_status tune_pick(rtproj_plan p, int count, const std::function<hipError_t(int)> &run, int *best,
                        std::vector<float> *times);
// The schedule for a given contraction rho.
RefinePlan refine_schedule_rho(double rho, double kappa_est, int mode, int max_steps);
// Status of a finished refinement from its per-step norms (|d_j|^2, |x_j|^2
// pairs, `steps` of them, the first `plain` from plain steps): RTPROJ_OK or
// RTPROJ_ERR_NOCONV, with the contraction and error estimates.
rtproj_status refine_verdict(const double *norms, int steps, int plain, double *rho_est, double *err_est);
// First output of SplitMix64 seeded with seed XOR i: the sketch seed of
// member i of a batch.
uint64_t instance_seed(uint64_t seed, int64_t i);

}  // namespace rtp
