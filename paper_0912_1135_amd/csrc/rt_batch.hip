// Batched runtime: many independent problems of uneven sizes (m_i, n_i, l_i,
// k_i) run through the same path as a single plan, stage by stage, with ONE
// grouped launch per stage for all members (the launch grid covers the
// largest member; smaller members skip the blocks they do not have).
//
// A call is recorded as a program: a list of grouped launches whose
// per-member arguments live in one device arena.  The program is rebuilt on
// the host for every call (cheap), uploaded only when its bytes changed, and
// either launched op by op or captured once into a HIP graph and replayed
// while neither the program nor the buffers change.  Nothing in a program
// waits on the host: rank tests and breakdowns are evaluated afterwards by
// rtproj_batch_status.
//
// Per member the path is the one of rt_plan.hip with the two-stage pivoted
// QR (S^T = Q0 R0 by shifted Cholesky QR, then the pivoted QR of R0).  That
// QR runs either one workgroup per member (no grid-wide barrier; best for
// many small members) or as the register-resident form with a group of
// blocks per member, each group synchronized on its own (best for few large
// members), whichever a cost estimate finds faster for the batch.
#include "rt_plan_state.h"

#include <map>

using namespace rtp;

namespace {

enum OpKind {
    OP_GEMM, OP_REDUCE, OP_SKETCH, OP_COPY, OP_SET0, OP_SET1, OP_SHIFT, OP_CHOL, OP_TRIINV, OP_QRCPWG, OP_RDIAG,
    OP_FORMTP, OP_ZERO, OP_AB, OP_ABRED, OP_ATX, OP_DDUPD, OP_IOTA, OP_GEMM32, OP_RED32, OP_FINISH,
    OP_QRCPGRP, OP_GEMMX3
};

struct Op {
    OpKind kind;
    size_t off;         // descriptor array offset in the arena (bytes)
    int count;
    rt::GemmShape gs{};
    rt::SketchGroupShape ss{};
    int64_t total = 0;  // element counts for the elementwise ops
    int i0 = 0, i1 = 0, i2 = 0, dd = 0;
    int stage = -1;     // rtproj_info stage index the op is accounted to
};

struct Program {
    std::vector<unsigned char> bytes;
    std::vector<Op> ops;
    int stage = -1;  // stage of the ops recorded next
    void push(Op o)
    {
        o.stage = stage;
        ops.push_back(o);
    }
    template <class T>
    size_t add(const std::vector<T> &v)
    {
        size_t off = (bytes.size() + 255) & ~size_t(255);
        bytes.resize(off + v.size() * sizeof(T));
        if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
        return off;
    }
};

struct DevBuf {
    unsigned char *d = nullptr;
    size_t cap = 0;
    std::vector<unsigned char> shadow;  // bytes currently on the device
    ~DevBuf() { if (d) (void)hipFree(d); }
};

}  // namespace

struct rtproj_batch_s {
    int64_t count = 0;
    std::vector<rtproj_plan> sub;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // graph capture (the null stream cannot be captured)
    int refine_steps = -1;  // -1: schedule from the members' rank estimates
    int precision = RTPROJ_PREC_FP64;  // the preconditioner's Gram: binary64 or binary32 (MIXED_FP32)
    int prec_used = RTPROJ_PREC_FP64;  // of the last precondition
    bool x3 = false;                   // the last precondition's Grams were split bfloat16
    bool sketch64 = true;              // the last precondition sketched in binary64
    bool escalated = false;            // ... after a binary32 sketch proved too coarse
    int plain_steps = 0, comp_steps = 2;  // schedule of the last projection
    bool comp_final = true;               // its final pass after compensated steps
    int last_steps = 0, last_plain = 0;   // steps of the last projection (norms recorded)
    std::vector<int64_t> last_k;          // right-hand sides per member in it
    int use_graph = 0;
    int timing = 0;                 // per-stage HIP events (eager mode only)
    double t_stage_ms[16] = {};
    int64_t stage_calls[16] = {};
    int64_t max_m = 0, max_n = 0, max_l = 0;
    double *d_diag_all = nullptr;  // count x 8: |R| ends of R (4), of the Gram factor (4)
    std::vector<const double *> cscale;  // per member: d of A diag(d) (borrowed), or null
    rt::QrcpGrpShape qr_grp;        // grouped pivoted QR of R0 (per_launch 0: one workgroup per member)
    double *d_qrw = nullptr;        // its candidate slots and columns, per member from qrw_off[i]
    std::vector<int64_t> qrw_off;
    bool ready = false;
    // one program and arena per entry point, plus its captured graph
    struct Slot {
        DevBuf arena;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        std::vector<unsigned char> graph_key;
        ~Slot()
        {
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
        }
    } pre, pro;
};

namespace {

constexpr int NBB = 64;  // block size of the grouped triangular solves and Cholesky

// ------------------------------------------------------------- recording
rt::GemmShape shape_of(const std::vector<rt::GemmArgs> &v)
{
    rt::GemmShape s{};
    s.a_kc = v.empty() ? 1 : (v[0].a_k == 1);
    s.b_kc = v.empty() ? 1 : (v[0].b_k == 1);
    s.c_lower = v.empty() ? 0 : v[0].c_lower;
    // the members of one recorded product all gather B's rows or none do
    s.b_gather = v.empty() ? 0 : (v[0].b_gather != nullptr);
    for (const auto &g : v) {
        s.M = std::max(s.M, g.M);
        s.N = std::max(s.N, g.N);
        s.ksplit = std::max(s.ksplit, std::max(1, g.ksplit));
    }
    return s;
}

void rec_gemm(Program &P, const std::vector<rt::GemmArgs> &v)
{
    Op o{OP_GEMM, P.add(v), (int)v.size()};
    o.gs = shape_of(v);
    P.push(o);
}

void rec_reduce(Program &P, const std::vector<rt::ReduceGroupArgs> &v)
{
    Op o{OP_REDUCE, P.add(v), (int)v.size()};
    for (const auto &r : v) o.total = std::max<int64_t>(o.total, (int64_t)r.M * r.N);
    P.push(o);
}

void rec_mat(Program &P, OpKind kind, const std::vector<rt::MatGroupArgs> &v)
{
    Op o{kind, P.add(v), (int)v.size()};
    for (const auto &r : v) o.total = std::max<int64_t>(o.total, (int64_t)r.m * std::max(r.n, r.m));
    P.push(o);
}

// C (m x m, both triangles) = X X^T for each member's row-major m x K X.
// Binary32 Gram on MFMA of the binary64 X (lower 64 x 64 tiles, split over
// K), reduced in binary64 into both triangles of C.
void rec_gram32(Program &P, rtproj_batch b, const std::vector<const double *> &X, const std::vector<int64_t> &ldx,
                const std::vector<int64_t> &K, const std::vector<double *> &C)
{
    std::vector<rt::GemmMxArgs> g(b->count);
    std::vector<rt::ReduceF32GroupArgs> r(b->count);
    int ksmax = 1, mmax = 0;
    for (int64_t i = 0; i < b->count; ++i) {
        rtproj_plan p = b->sub[i];
        const int64_t m = p->m;
        rt::GemmMxArgs &a = g[i];
        a.M = (int)m; a.N = (int)m; a.K = (int)K[i];
        a.A = X[i]; a.a_dbl = 1; a.a_i = ldx[i]; a.a_k = 1;
        a.B = X[i]; a.b_dbl = 1; a.b_k = 1; a.b_j = ldx[i];
        a.C = p->d_part; a.c_dbl = 0; a.c_i = m; a.c_j = 1; a.c_split = m * m;
        a.alpha = 1.f; a.c_lower = 1;
        a.ksplit = (int)std::max<int64_t>(1, std::min<int64_t>(p->syrk_splits, K[i] / 256));
        r[i] = rt::ReduceF32GroupArgs{reinterpret_cast<const float *>(p->d_part), m * m, a.ksplit, (int)m, C[i]};
        ksmax = std::max(ksmax, a.ksplit);
        mmax = std::max<int>(mmax, (int)m);
    }
    Op o{OP_GEMM32, P.add(g), (int)b->count};
    o.i0 = mmax;
    o.i1 = ksmax;
    P.push(o);
    Op q{OP_RED32, P.add(r), (int)b->count};
    q.i0 = mmax;
    P.push(q);
}

// C as rec_gram32, from binary32 X (row stride ldx floats, 16-byte rows):
// the split-bfloat16 Gram on MFMA (hi + lo halves, three products), lower
// 256 x 128 tiles split over K, reduced in binary64 into both triangles.
void rec_gram_x3(Program &P, rtproj_batch b, const std::vector<const float *> &X, const std::vector<int64_t> &ldx,
                 const std::vector<int64_t> &K, const std::vector<double *> &C)
{
    std::vector<rt::GemmMxArgs> g(b->count);
    std::vector<rt::ReduceF32GroupArgs> r(b->count);
    int ksmax = 1, mmax = 0;
    for (int64_t i = 0; i < b->count; ++i) {
        rtproj_plan p = b->sub[i];
        const int64_t m = p->m;
        rt::GemmMxArgs &a = g[i];
        a.M = (int)m; a.N = (int)m; a.K = (int)K[i];
        a.A = X[i]; a.a_dbl = 0; a.a_i = ldx[i]; a.a_k = 1;
        a.B = X[i]; a.b_dbl = 0; a.b_k = 1; a.b_j = ldx[i];
        a.C = p->d_part; a.c_dbl = 0; a.c_i = m; a.c_j = 1; a.c_split = m * m;
        a.alpha = 1.f; a.c_lower = 1;
        a.ksplit = (int)std::max<int64_t>(1, std::min<int64_t>(p->syrk_splits, K[i] / 256));
        r[i] = rt::ReduceF32GroupArgs{reinterpret_cast<const float *>(p->d_part), m * m, a.ksplit, (int)m, C[i]};
        ksmax = std::max(ksmax, a.ksplit);
        mmax = std::max<int>(mmax, (int)m);
    }
    Op o{OP_GEMMX3, P.add(g), (int)b->count};
    o.i0 = mmax;
    o.i1 = ksmax;
    P.push(o);
    Op q{OP_RED32, P.add(r), (int)b->count};
    q.i0 = mmax;
    P.push(q);
}

void rec_gram(Program &P, rtproj_batch b, const std::vector<const double *> &X, const std::vector<int64_t> &ldx,
              const std::vector<int64_t> &K, const std::vector<double *> &C)
{
    std::vector<rt::GemmArgs> g(b->count);
    std::vector<rt::ReduceGroupArgs> r(b->count);
    for (int64_t i = 0; i < b->count; ++i) {
        rtproj_plan p = b->sub[i];
        const int64_t m = p->m;
        rt::GemmArgs &a = g[i];
        a.M = (int)m; a.N = (int)m; a.K = (int)K[i];
        a.A = X[i]; a.a_i = ldx[i]; a.a_k = 1;
        a.B = X[i]; a.b_k = 1; a.b_j = ldx[i];
        a.C = p->d_part; a.c_i = m; a.c_j = 1; a.c_split = m * m;
        a.alpha = 1.0; a.c_lower = 1;
        a.ksplit = (int)std::max<int64_t>(1, std::min<int64_t>(p->syrk_splits, K[i] / 256));
        r[i] = rt::ReduceGroupArgs{p->d_part, m * m, a.ksplit, (int)m, (int)m, m, C[i], m, 1};
    }
    rec_gemm(P, g);
    rec_reduce(P, r);
}

// Blocked right-looking Cholesky C = L L^T per member (C overwritten below
// its diagonal blocks by the trailing updates); Dinv gets L's diagonal-block
// inverses; a failed pivot sets the member's error flag.
void rec_cholesky(Program &P, rtproj_batch b, const std::vector<double *> &C, const std::vector<double *> &L)
{
    const int64_t cnt = b->count;
    std::vector<rt::MatGroupArgs> z(cnt);
    std::vector<rt::CholGroupArgs> ch(cnt);
    for (int64_t i = 0; i < cnt; ++i) {
        rtproj_plan p = b->sub[i];
        z[i] = rt::MatGroupArgs{L[i], p->m, (int)p->m, (int)p->m, 0.0, nullptr, nullptr};
        ch[i] = rt::CholGroupArgs{C[i], p->m, (int)p->m, L[i], p->m, p->d_DinvL, p->d_err};
    }
    rec_mat(P, OP_SET0, z);
    const size_t choff = P.add(ch);
    const int64_t nblk = (b->max_m + NBB - 1) / NBB;
    for (int64_t bk = 0; bk < nblk; ++bk) {
        Op o{OP_CHOL, choff, (int)cnt};
        o.i0 = (int)bk;
        P.push(o);
        std::vector<rt::GemmArgs> pan(cnt), upd(cnt);
        for (int64_t i = 0; i < cnt; ++i) {
            rtproj_plan p = b->sub[i];
            const int64_t m = p->m, r0 = bk * NBB, nbb = std::max<int64_t>(0, std::min<int64_t>(NBB, m - r0));
            const int64_t rest = std::max<int64_t>(0, m - r0 - nbb);
            rt::GemmArgs &g = pan[i];
            g.M = (int)rest; g.N = (int)nbb; g.K = (int)nbb;
            g.A = C[i] + (r0 + nbb) * m + r0; g.a_i = m; g.a_k = 1;
            g.B = p->d_DinvL + bk * NBB * NBB; g.b_k = 1; g.b_j = NBB;
            g.C = L[i] + (r0 + nbb) * m + r0; g.c_i = m; g.c_j = 1;
            g.alpha = 1.0; g.ksplit = 1;
            rt::GemmArgs &u = upd[i];
            u.M = (int)rest; u.N = (int)rest; u.K = (int)nbb;
            u.A = L[i] + (r0 + nbb) * m + r0; u.a_i = m; u.a_k = 1;
            u.B = L[i] + (r0 + nbb) * m + r0; u.b_k = 1; u.b_j = m;
            u.C = C[i] + (r0 + nbb) * m + (r0 + nbb); u.c_i = m; u.c_j = 1;
            u.alpha = -1.0; u.beta = 1.0; u.c_lower = 1; u.ksplit = 1;
            if (rest == 0) { g.M = 0; u.M = 0; }
        }
        rec_gemm(P, pan);
        rec_gemm(P, upd);
    }
}

// In place B <- L^{-1} B (row-major m x ncols) per member, with L read as
// L[i*l_i + j*l_j] and Dinv its diagonal-block inverses; rhs_lower: B lower
// triangular (columns past the block's last row are zero and skipped).
void rec_trsm(Program &P, rtproj_batch b, const std::vector<const double *> &Lp, int64_t l_i_mul, int64_t l_j_mul,
              const std::vector<const double *> &Dinv, const std::vector<double *> &B, const std::vector<int64_t> &ldb,
              const std::vector<int64_t> &ncols, bool rhs_lower)
{
    const int64_t cnt = b->count;
    const int64_t nblk = (b->max_m + NBB - 1) / NBB;
    for (int64_t bk = 0; bk < nblk; ++bk) {
        std::vector<rt::GemmArgs> dg(cnt), up(cnt);
        for (int64_t i = 0; i < cnt; ++i) {
            rtproj_plan p = b->sub[i];
            const int64_t m = p->m;
            // l_i / l_j are given as multiples of m (0, 1) plus a unit stride
            const int64_t l_i = l_i_mul ? m : 1, l_j = l_j_mul ? m : 1;
            const int64_t r0 = bk * NBB, nbb = std::max<int64_t>(0, std::min<int64_t>(NBB, m - r0));
            const int64_t cols = rhs_lower ? std::min<int64_t>(ncols[i], r0 + nbb) : ncols[i];
            rt::GemmArgs &g = dg[i];
            g.M = (int)nbb; g.N = (int)cols; g.K = (int)nbb;
            g.A = Dinv[i] + bk * NBB * NBB; g.a_i = NBB; g.a_k = 1;
            g.B = B[i] + r0 * ldb[i]; g.b_k = ldb[i]; g.b_j = 1;
            g.C = B[i] + r0 * ldb[i]; g.c_i = ldb[i]; g.c_j = 1;
            g.alpha = 1.0; g.ksplit = 1;
            const int64_t rest = std::max<int64_t>(0, m - r0 - nbb);
            rt::GemmArgs &u = up[i];
            u.M = (int)rest; u.N = (int)cols; u.K = (int)nbb;
            u.A = Lp[i] + (r0 + nbb) * l_i + r0 * l_j; u.a_i = l_i; u.a_k = l_j;
            u.B = B[i] + r0 * ldb[i]; u.b_k = ldb[i]; u.b_j = 1;
            u.C = B[i] + (r0 + nbb) * ldb[i]; u.c_i = ldb[i]; u.c_j = 1;
            u.alpha = -1.0; u.beta = 1.0; u.ksplit = 1;
            if (nbb == 0) { g.M = 0; u.M = 0; }
        }
        rec_gemm(P, dg);
        rec_gemm(P, up);
    }
}

void build_precondition(Program &P, rtproj_batch b, const double *const *A, const int64_t *lda,
                        const double *const *cs)
{
    const int64_t cnt = b->count;
    // 1. sketches: one grouped launch pair per padded Fourier length and band
    // of 128 rows, so that each grid (sized for the largest member it covers)
    // wastes few blocks on smaller transforms or fewer row pairs
    P.stage = 0;
    {
        std::map<std::pair<int64_t, int64_t>, std::vector<int64_t>> by_np;
        for (int64_t i = 0; i < cnt; ++i) by_np[{b->sub[i]->tab.np, (b->sub[i]->m + 127) / 128}].push_back(i);
        for (const auto &cls : by_np) {
            std::vector<rt::SketchGroupArgs> v;
            Op o{OP_SKETCH, 0, (int)cls.second.size()};
            o.i0 = b->sketch64 ? 0 : 1;  // 1: binary32 arithmetic
            o.ss.one_length = true;      // the class shares its padded length
            for (int64_t i : cls.second) {
                rtproj_plan p = b->sub[i];
                v.push_back(rt::SketchGroupArgs{p->sketch_tables(), A[i], lda[i], p->m, p->d_S, p->l, p->d_zbuf,
                                                p->rows_chunk, cs[i]});
                o.ss.max_n1 = std::max(o.ss.max_n1, p->tab.n1);
                o.ss.max_n2 = std::max(o.ss.max_n2, p->tab.n2);
                o.ss.max_rows_chunk = std::max(o.ss.max_rows_chunk, p->rows_chunk);
                o.ss.chunks = std::max<int>(o.ss.chunks, (int)((p->m + p->rows_chunk - 1) / p->rows_chunk));
            }
            o.off = P.add(v);
            P.push(o);
        }
    }
    std::vector<double *> G(cnt), Yq(cnt), L1(cnt), L2(cnt), L3(cnt), R0(cnt), S(cnt), Rm(cnt), Ym(cnt), Lm(cnt);
    std::vector<const double *> cYq(cnt);
    std::vector<int64_t> ll(cnt), mm(cnt);
    for (int64_t i = 0; i < cnt; ++i) {
        rtproj_plan p = b->sub[i];
        G[i] = p->d_G; Yq[i] = p->d_Yq; cYq[i] = p->d_Yq; L1[i] = p->d_L; L2[i] = p->d_Y; L3[i] = p->d_Tp;
        R0[i] = p->d_R0; S[i] = p->d_S; Rm[i] = p->d_R; Ym[i] = p->d_Y; Lm[i] = p->d_L;
        ll[i] = p->l; mm[i] = p->m;
    }
    // flags
    {
        Op o{OP_ZERO, 0, (int)cnt};
        std::vector<unsigned *> flags;
        for (int64_t i = 0; i < cnt; ++i) {
            flags.push_back(reinterpret_cast<unsigned *>(b->sub[i]->d_err));
            flags.push_back(b->sub[i]->d_sync);      // the grouped QR's arrival counter
            flags.push_back(b->sub[i]->d_sync + 2);
        }
        o.off = P.add(flags);
        o.count = (int)flags.size();
        P.push(o);
    }
    // 2a. R0 by shifted Cholesky QR with all three passes: a graph cannot
    // skip the third on a device-side test, and it is what resolves a
    // member's numerical rank deficiency to about u |S|
    P.stage = 12;
    {
        std::vector<rt::CopyGroupArgs> c(cnt);
        int64_t tot = 0;
        for (int64_t i = 0; i < cnt; ++i) {
            rtproj_plan p = b->sub[i];
            c[i] = rt::CopyGroupArgs{p->d_S, p->l, p->d_Yq, p->l, (int)p->l, (int)p->m, nullptr, 0};
            tot = std::max(tot, p->l * p->m);
        }
        Op o{OP_COPY, P.add(c), (int)cnt};
        o.total = tot;
        P.push(o);
    }
    std::vector<double *> Ls[3] = {L1, L2, L3};
    std::vector<const double *> Dl(cnt);
    for (int64_t i = 0; i < cnt; ++i) Dl[i] = b->sub[i]->d_DinvL;
    for (int it = 0; it < 3; ++it) {
        rec_gram(P, b, cYq, ll, ll, G);
        if (it == 0) {
            std::vector<rt::MatGroupArgs> sh(cnt);
            for (int64_t i = 0; i < cnt; ++i) {
                rtproj_plan p = b->sub[i];
                const double c = 11.0 * ((double)p->l * p->m + (double)p->m * (p->m + 1)) * std::ldexp(1.0, -53);
                sh[i] = rt::MatGroupArgs{p->d_G, p->m, (int)p->m, (int)p->m, c, nullptr, nullptr};
            }
            rec_mat(P, OP_SHIFT, sh);
        }
        rec_cholesky(P, b, G, Ls[it]);
        if (it < 2) {
            std::vector<const double *> Lc(Ls[it].begin(), Ls[it].end());
            rec_trsm(P, b, Lc, 1, 0, Dl, Yq, ll, ll, false);
        }
    }
    for (int pass = 0; pass < 2; ++pass) {
        std::vector<rt::GemmArgs> g(cnt);
        for (int64_t i = 0; i < cnt; ++i) {
            const int64_t m = mm[i];
            rt::GemmArgs &a = g[i];
            a.M = (int)m; a.N = (int)m; a.K = (int)m;
            a.A = pass == 0 ? L1[i] : G[i]; a.a_i = m; a.a_k = 1; a.a_lower = 1;
            a.B = pass == 0 ? L2[i] : L3[i]; a.b_k = m; a.b_j = 1;
            a.C = pass == 0 ? G[i] : R0[i]; a.c_i = m; a.c_j = 1;
            a.alpha = 1.0; a.ksplit = 1;
        }
        rec_gemm(P, g);
    }
    // 2b. pivoted QR of R0, one workgroup per member
    P.stage = 1;
    {
        std::vector<rt::MatGroupArgs> z(cnt), pv(cnt);
        for (int64_t i = 0; i < cnt; ++i) {
            z[i] = rt::MatGroupArgs{Rm[i], mm[i], (int)mm[i], (int)mm[i], 0.0, nullptr, nullptr};
            pv[i] = rt::MatGroupArgs{nullptr, 0, (int)mm[i], 0, 0.0, b->sub[i]->d_piv, nullptr};
        }
        rec_mat(P, OP_SET0, z);
        // valid pivots even if a member's QR stops early on non-finite data
        Op io{OP_IOTA, P.add(pv), (int)cnt};
        io.i0 = (int)b->max_m;
        P.push(io);
        if (b->qr_grp.per_launch > 0) {
            // groups of blocks per member, as many members per launch as stay resident
            const rt::QrcpGrpShape &sh = b->qr_grp;
            for (int64_t c0 = 0; c0 < cnt; c0 += sh.per_launch) {
                std::vector<rt::QrcpGrpArgs> q;
                for (int64_t i = c0; i < std::min<int64_t>(cnt, c0 + sh.per_launch); ++i) {
                    rtproj_plan p = b->sub[i];
                    const int G = (int)((p->m + sh.nc - 1) / sh.nc);
                    rt::QrcpWork w;
                    w.counter = p->d_sync;
                    w.flag = p->d_sync + 1;
                    w.err = reinterpret_cast<int *>(p->d_sync + 2);
                    w.slots = b->d_qrw + b->qrw_off[i];
                    w.vbuf = w.slots + 4 * G;
                    q.push_back(rt::QrcpGrpArgs{p->d_R0, p->m, (int)p->m, (int)p->m, p->d_R, p->d_piv, w, G});
                }
                Op o{OP_QRCPGRP, P.add(q), (int)q.size()};
                o.i0 = sh.nc;
                o.i1 = sh.rpt;
                o.i2 = sh.threads;
                o.dd = sh.gmax;
                o.total = sh.per_launch;
                P.push(o);
            }
        } else {
            std::vector<rt::QrcpWgArgs> q(cnt);
            for (int64_t i = 0; i < cnt; ++i) {
                rtproj_plan p = b->sub[i];
                q[i] = rt::QrcpWgArgs{p->d_R0, p->m, (int)p->m, (int)p->m, p->d_R, p->d_piv,
                                      reinterpret_cast<int *>(p->d_sync + 2)};
            }
            P.push(Op{OP_QRCPWG, P.add(q), (int)cnt});
        }
        std::vector<rt::MatGroupArgs> rd(cnt);
        for (int64_t i = 0; i < cnt; ++i)
            rd[i] = rt::MatGroupArgs{Rm[i], mm[i], (int)mm[i], (int)mm[i], 0.0, nullptr, b->d_diag_all + 8 * i};
        rec_mat(P, OP_RDIAG, rd);
    }
    // 3. R^{-T} in d_Y: diagonal-block inverses, identity, blocked solve
    P.stage = 2;
    {
        std::vector<rt::TriInvGroupArgs> t(cnt);
        for (int64_t i = 0; i < cnt; ++i) t[i] = rt::TriInvGroupArgs{Rm[i], 1, mm[i], (int)mm[i], b->sub[i]->d_DinvR};
        Op o{OP_TRIINV, P.add(t), (int)cnt};
        o.i0 = (int)b->max_m;
        P.push(o);
        std::vector<rt::MatGroupArgs> id(cnt);
        for (int64_t i = 0; i < cnt; ++i) id[i] = rt::MatGroupArgs{Ym[i], mm[i], (int)mm[i], (int)mm[i], 0.0, nullptr, nullptr};
        rec_mat(P, OP_SET1, id);
        std::vector<const double *> Rc(cnt), Dr(cnt);
        for (int64_t i = 0; i < cnt; ++i) { Rc[i] = Rm[i]; Dr[i] = b->sub[i]->d_DinvR; }
        rec_trsm(P, b, Rc, 0, 1, Dr, Ym, mm, mm, true);
    }
    // 4. W = R^{-T} (Pi A)
    P.stage = 3;
    {
        std::vector<rt::GemmArgs> g(cnt);
        for (int64_t i = 0; i < cnt; ++i) {
            rtproj_plan p = b->sub[i];
            rt::GemmArgs &a = g[i];
            a.M = (int)p->m; a.N = (int)p->n; a.K = (int)p->m;
            a.A = p->d_Y; a.a_i = p->m; a.a_k = 1; a.a_lower = 1;
            a.B = A[i]; a.b_k = lda[i]; a.b_j = 1; a.b_gather = p->d_piv;
            a.C = p->d_W; a.c_i = b->x3 ? p->ldw : p->n; a.c_j = 1;
            a.c_f32 = b->x3 ? 1 : 0;  // binary32 W (padded rows) for the split-bfloat16 Gram
            a.c_cs = cs[i];  // R^{-T} Pi (A D) = (R^{-T} Pi A) D
            a.alpha = 1.0; a.ksplit = 1;
        }
        rec_gemm(P, g);
    }
    // 5. Gram of W, 6. its Cholesky
    {
        std::vector<const double *> W(cnt);
        std::vector<int64_t> nn(cnt);
        for (int64_t i = 0; i < cnt; ++i) { W[i] = b->sub[i]->d_W; nn[i] = b->sub[i]->n; }
        P.stage = 4;
        if (b->x3) {
            std::vector<const float *> Wf(cnt);
            std::vector<int64_t> lw(cnt);
            for (int64_t i = 0; i < cnt; ++i) {
                Wf[i] = reinterpret_cast<const float *>(b->sub[i]->d_W);
                lw[i] = b->sub[i]->ldw;
            }
            rec_gram_x3(P, b, Wf, lw, nn, G);
        } else if (b->prec_used != RTPROJ_PREC_FP64) {
            rec_gram32(P, b, W, nn, nn, G);
        } else {
            rec_gram(P, b, W, nn, nn, G);
        }
        P.stage = 5;
        rec_cholesky(P, b, G, Lm);
    }
    // 7. T = L^{-1} R^{-T} (in d_Y), T' = T Pi
    P.stage = 6;
    {
        std::vector<const double *> Lc(cnt);
        for (int64_t i = 0; i < cnt; ++i) Lc[i] = Lm[i];
        rec_trsm(P, b, Lc, 1, 0, Dl, Ym, mm, mm, true);
        std::vector<rt::MatGroupArgs> f(cnt), rd(cnt);
        for (int64_t i = 0; i < cnt; ++i) {
            rtproj_plan p = b->sub[i];
            f[i] = rt::MatGroupArgs{p->d_Y, p->m, (int)p->m, (int)p->m, 0.0, p->d_piv, p->d_Tp};
            rd[i] = rt::MatGroupArgs{p->d_L, p->m, (int)p->m, (int)p->m, 0.0, nullptr, b->d_diag_all + 8 * i + 4};
        }
        rec_mat(P, OP_FORMTP, f);
        rec_mat(P, OP_RDIAG, rd);
    }
}

// x (m x k per member) = T'^T (T' c) into H, via split-K GEMMs and reductions.
void rec_minv(Program &P, rtproj_batch b, const std::vector<int64_t> &k, const std::vector<const double *> &C,
              const std::vector<double *> &H)
{
    const int64_t cnt = b->count;
    for (int pass = 0; pass < 2; ++pass) {
        std::vector<rt::GemmArgs> g(cnt);
        std::vector<rt::ReduceGroupArgs> r(cnt);
        for (int64_t i = 0; i < cnt; ++i) {
            rtproj_plan p = b->sub[i];
            const int64_t m = p->m;
            const int splits = (int)std::max<int64_t>(1, std::min<int64_t>(p->ab_splits, (m + 63) / 64));
            rt::GemmArgs &a = g[i];
            a.M = (int)m; a.N = (int)k[i]; a.K = (int)m;
            a.A = p->d_Tp + (pass == 0 ? m * m : 0); a.a_i = m; a.a_k = 1;
            a.B = pass == 0 ? C[i] : p->d_tmp; a.b_k = 1; a.b_j = m;
            a.C = p->d_ph; a.c_i = 1; a.c_j = m; a.c_split = m * k[i];
            a.alpha = 1.0; a.ksplit = splits;
            r[i] = rt::ReduceGroupArgs{p->d_ph, m * k[i], splits, (int)k[i], (int)m, m, pass == 0 ? p->d_tmp : H[i], m, 0};
            if (k[i] == 0) { a.M = 0; r[i].M = 0; }
        }
        rec_gemm(P, g);
        rec_reduce(P, r);
    }
}

// c = A B per member (A column-scaled by cs[i] when given).  The MFMA form
// takes a scaled member as A (D B), with D B written to d_r first (B may be
// d_r itself: scaled in place).
void rec_ab(Program &P, rtproj_batch b, const std::vector<int64_t> &k, const double *const *A, const int64_t *lda,
            const double *const *cs, std::vector<const double *> B, std::vector<int64_t> ldb, int dd)
{
    const int64_t cnt = b->count;
    const int64_t kmax = *std::max_element(k.begin(), k.end());
    if (!dd && kmax >= RT_MFMA_KMIN) {
        // plain product with many right-hand sides: MFMA GEMM split over n
        std::vector<rt::CopyGroupArgs> sc;
        int64_t tot = 0;
        for (int64_t i = 0; i < cnt; ++i) {
            rtproj_plan p = b->sub[i];
            if (!cs[i] || k[i] == 0) continue;
            sc.push_back(rt::CopyGroupArgs{B[i], ldb[i], p->d_r, p->n, (int)p->n, (int)k[i], nullptr, 0, cs[i]});
            tot = std::max(tot, p->n * k[i]);
            B[i] = p->d_r;
            ldb[i] = p->n;
        }
        if (!sc.empty()) {
            Op o{OP_COPY, P.add(sc), (int)sc.size()};
            o.total = tot;
            P.push(o);
        }
        std::vector<rt::GemmArgs> g(cnt);
        std::vector<rt::ReduceGroupArgs> r(cnt);
        for (int64_t i = 0; i < cnt; ++i) {
            rtproj_plan p = b->sub[i];
            const int64_t m = p->m;
            rt::GemmArgs &a = g[i];
            a.M = (int)m; a.N = (int)k[i]; a.K = (int)p->n;
            a.A = A[i]; a.a_i = lda[i]; a.a_k = 1;
            a.B = B[i]; a.b_k = 1; a.b_j = ldb[i];
            a.C = p->d_ph; a.c_i = 1; a.c_j = m; a.c_split = m * k[i];
            a.alpha = 1.0; a.ksplit = p->ab_splits;
            r[i] = rt::ReduceGroupArgs{p->d_ph, m * k[i], p->ab_splits, (int)k[i], (int)m, m, p->d_c, m, 0};
            if (k[i] == 0) { a.M = 0; r[i].M = 0; }
        }
        rec_gemm(P, g);
        rec_reduce(P, r);
        return;
    }
    std::vector<rt::AbGroupArgs> v(cnt);
    Op o{OP_AB, 0, (int)cnt};
    o.dd = dd;
    for (int64_t i = 0; i < cnt; ++i) {
        rtproj_plan p = b->sub[i];
        v[i] = rt::AbGroupArgs{rt::ApplyArgs{(int)p->m, (int)p->n, (int)k[i], A[i], lda[i], cs[i]}, B[i], ldb[i],
                               p->ab_splits, p->d_ph, p->d_pl, p->d_c, p->m};
        o.i0 = std::max<int>(o.i0, (int)p->m);
        o.i1 = std::max<int>(o.i1, (int)k[i]);
        o.i2 = std::max<int>(o.i2, p->ab_splits);
        o.total = std::max<int64_t>(o.total, p->m * k[i]);
    }
    o.off = P.add(v);
    P.push(o);
    Op r = o;
    r.kind = OP_ABRED;
    P.push(r);
}

void rec_atx(Program &P, rtproj_batch b, const std::vector<rt::AtxGroupArgs> &v, int dd)
{
    Op o{OP_ATX, P.add(v), (int)v.size()};
    o.dd = dd;
    for (const auto &a : v) {
        o.total = std::max<int64_t>(o.total, a.a.n);
        o.i1 = std::max(o.i1, a.a.k);
        if (a.a.cs) o.i0 = 1;  // some member is column-scaled
    }
    (void)b;
    P.push(o);
}

void build_project(Program &P, rtproj_batch b, const double *const *A, const int64_t *lda, const double *const *cs,
                   const double *const *B,
                   const int64_t *ldb, const int64_t *k, double *const *Z, const int64_t *ldz, double *const *Y,
                   const int64_t *ldy, double *const *X, const int64_t *ldx)
{
    const int64_t cnt = b->count;
    std::vector<int64_t> kk(k, k + cnt), lb(ldb, ldb + cnt), nn(cnt), mm(cnt);
    std::vector<const double *> Bv(B, B + cnt), c(cnt), r(cnt);
    std::vector<double *> xhi(cnt), dd(cnt);
    for (int64_t i = 0; i < cnt; ++i) {
        rtproj_plan p = b->sub[i];
        c[i] = p->d_c; r[i] = p->d_r; xhi[i] = p->d_xhi; dd[i] = p->d_d; nn[i] = p->n; mm[i] = p->m;
    }
    // c = A b; x = M^{-1} c; xlo = 0
    P.stage = 7;
    rec_ab(P, b, kk, A, lda, cs, Bv, lb, 0);
    P.stage = 8;
    rec_minv(P, b, kk, c, xhi);
    {
        std::vector<rt::MatGroupArgs> z(cnt);
        for (int64_t i = 0; i < cnt; ++i) z[i] = rt::MatGroupArgs{b->sub[i]->d_xlo, mm[i], (int)kk[i], (int)mm[i], 0.0, nullptr, nullptr};
        rec_mat(P, OP_SET0, z);
    }
    const int nsteps = std::min(b->plain_steps + b->comp_steps, RT_MAX_STEPS);
    for (int it = 0; it < nsteps; ++it) {
        const int comp = it >= b->plain_steps ? 1 : 0;  // plain residuals first, compensated last
        std::vector<rt::AtxGroupArgs> a(cnt);
        for (int64_t i = 0; i < cnt; ++i) {
            rtproj_plan p = b->sub[i];
            a[i] = rt::AtxGroupArgs{rt::ApplyArgs{(int)p->m, (int)p->n, (int)kk[i], A[i], lda[i], cs[i]}, p->d_xhi, p->d_xlo,
                                    p->m, B[i], ldb[i], p->d_r, p->n, nullptr, 0, nullptr, 0};
        }
        P.stage = comp ? 9 : 13;  // compensated or plain residual
        if (comp || *std::max_element(kk.begin(), kk.end()) < RT_MFMA_KMIN) {
            rec_atx(P, b, a, comp);
        } else {
            // plain residual r = b - A^T x_hi with many right-hand sides:
            // copy b, then the MFMA GEMM with alpha = -1, beta = 1
            std::vector<rt::CopyGroupArgs> cp(cnt);
            std::vector<rt::GemmArgs> g(cnt);
            int64_t tot = 0;
            for (int64_t i = 0; i < cnt; ++i) {
                rtproj_plan p = b->sub[i];
                cp[i] = rt::CopyGroupArgs{B[i], ldb[i], p->d_r, p->n, (int)p->n, (int)kk[i], nullptr, 0};
                tot = std::max(tot, p->n * kk[i]);
                rt::GemmArgs &q = g[i];
                q.M = (int)p->n; q.N = (int)kk[i]; q.K = (int)p->m;
                q.A = A[i]; q.a_i = 1; q.a_k = lda[i]; q.c_rs = cs[i];  // (A D)^T x = D (A^T x)
                q.B = p->d_xhi; q.b_k = 1; q.b_j = p->m;
                q.C = p->d_r; q.c_i = 1; q.c_j = p->n;
                q.alpha = -1.0; q.beta = 1.0; q.ksplit = 1;
                if (kk[i] == 0) q.M = 0;
            }
            Op o{OP_COPY, P.add(cp), (int)cnt};
            o.total = tot;
            P.push(o);
            rec_gemm(P, g);
        }
        P.stage = comp ? 10 : 14;
        rec_ab(P, b, kk, A, lda, cs, r, nn, comp);
        P.stage = 8;
        rec_minv(P, b, kk, c, dd);
        std::vector<rt::DdGroupArgs> u(cnt);
        for (int64_t i = 0; i < cnt; ++i) {
            rtproj_plan p = b->sub[i];
            u[i] = rt::DdGroupArgs{p->d_xhi, p->d_xlo, p->d_d, (int)(p->m * kk[i]), p->d_norms + 2 * it};
        }
        P.push(Op{OP_DDUPD, P.add(u), (int)cnt});
    }
    const bool from_r = nsteps > 0 && b->comp_final && nsteps - 1 >= b->plain_steps;
    if (from_r) {
        // the last step was compensated: its residual r = b - A^T x_prev is in
        // d_r and its correction d in d_d, so z = r - A^T d with a plain
        // product (|d| is the error of x_prev), Y = B - z, Z = z
        P.stage = 15;
        if (*std::max_element(kk.begin(), kk.end()) < RT_MFMA_KMIN) {
            std::vector<rt::AtxGroupArgs> a(cnt);
            for (int64_t i = 0; i < cnt; ++i) {
                rtproj_plan p = b->sub[i];
                a[i] = rt::AtxGroupArgs{rt::ApplyArgs{(int)p->m, (int)p->n, (int)kk[i], A[i], lda[i], cs[i]}, p->d_d, nullptr,
                                        p->m, p->d_r, p->n, p->d_r, p->n, nullptr, 0, nullptr, 0};
            }
            rec_atx(P, b, a, 0);
        } else {
            std::vector<rt::GemmArgs> g(cnt);
            for (int64_t i = 0; i < cnt; ++i) {
                rtproj_plan p = b->sub[i];
                rt::GemmArgs &q = g[i];
                q.M = (int)p->n; q.N = (int)kk[i]; q.K = (int)p->m;
                q.A = A[i]; q.a_i = 1; q.a_k = lda[i]; q.c_rs = cs[i];  // (A D)^T x = D (A^T x)
                q.B = p->d_d; q.b_k = 1; q.b_j = p->m;
                q.C = p->d_r; q.c_i = 1; q.c_j = p->n;
                q.alpha = -1.0; q.beta = 1.0; q.ksplit = 1;
                if (kk[i] == 0) q.M = 0;
            }
            rec_gemm(P, g);
        }
        std::vector<rt::FinishGroupArgs> f(cnt);
        int64_t tot = 0;
        for (int64_t i = 0; i < cnt; ++i) {
            rtproj_plan p = b->sub[i];
            double *yi = Y ? Y[i] : nullptr, *zi = Z ? Z[i] : nullptr;
            f[i] = rt::FinishGroupArgs{p->d_r, p->n, B[i], ldb[i], yi, yi ? ldy[i] : 0, zi, zi ? ldz[i] : 0,
                                       (int)p->n, (int)kk[i]};
            if (!yi && !zi) f[i].cols = 0;
            tot = std::max(tot, (int64_t)f[i].rows * f[i].cols);
        }
        Op o{OP_FINISH, P.add(f), (int)cnt};
        o.total = tot;
        P.push(o);
    }
    const bool final_comp = nsteps > 0 && b->comp_final;
    if (!from_r && !final_comp && *std::max_element(kk.begin(), kk.end()) >= RT_MFMA_KMIN) {
        // plain final pass with many right-hand sides on MFMA: d_r = B, then
        // d_r -= A^T x_hi (grouped GEMM), then Y = B - d_r and Z = d_r
        P.stage = 15;
        std::vector<rt::CopyGroupArgs> cp(cnt);
        std::vector<rt::GemmArgs> g(cnt);
        std::vector<rt::FinishGroupArgs> f(cnt);
        int64_t tot = 0;
        for (int64_t i = 0; i < cnt; ++i) {
            rtproj_plan p = b->sub[i];
            cp[i] = rt::CopyGroupArgs{B[i], ldb[i], p->d_r, p->n, (int)p->n, (int)kk[i], nullptr, 0};
            rt::GemmArgs &q = g[i];
            q.M = (int)p->n; q.N = (int)kk[i]; q.K = (int)p->m;
            q.A = A[i]; q.a_i = 1; q.a_k = lda[i]; q.c_rs = cs[i];  // (A D)^T x = D (A^T x)
            q.B = p->d_xhi; q.b_k = 1; q.b_j = p->m;
            q.C = p->d_r; q.c_i = 1; q.c_j = p->n;
            q.alpha = -1.0; q.beta = 1.0; q.ksplit = 1;
            if (kk[i] == 0) q.M = 0;
            double *yi = Y ? Y[i] : nullptr, *zi = Z ? Z[i] : nullptr;
            f[i] = rt::FinishGroupArgs{p->d_r, p->n, B[i], ldb[i], yi, yi ? ldy[i] : 0, zi, zi ? ldz[i] : 0,
                                       (int)p->n, (int)kk[i]};
            if (!yi && !zi) { f[i].cols = 0; cp[i].cols = 0; q.M = 0; }
            tot = std::max(tot, p->n * kk[i]);
        }
        Op oc{OP_COPY, P.add(cp), (int)cnt};
        oc.total = tot;
        P.push(oc);
        rec_gemm(P, g);
        Op of{OP_FINISH, P.add(f), (int)cnt};
        of.total = tot;
        P.push(of);
    } else if (!from_r) {
        P.stage = final_comp ? 11 : 15;
        std::vector<rt::AtxGroupArgs> a(cnt);
        for (int64_t i = 0; i < cnt; ++i) {
            rtproj_plan p = b->sub[i];
            a[i] = rt::AtxGroupArgs{rt::ApplyArgs{(int)p->m, (int)p->n, (int)kk[i], A[i], lda[i], cs[i]}, p->d_xhi, p->d_xlo,
                                    p->m, B[i], ldb[i], nullptr, 0, Y ? Y[i] : nullptr, Y ? ldy[i] : 0,
                                    Z ? Z[i] : nullptr, Z ? ldz[i] : 0};
            if (!(Y && Y[i]) && !(Z && Z[i])) a[i].a.k = 0;
        }
        rec_atx(P, b, a, final_comp ? 1 : 0);
    }
    // x to the outputs, accounted to the final pass that ran
    P.stage = (!from_r && final_comp) ? 11 : 15;
    if (X) {
        std::vector<rt::CopyGroupArgs> cp(cnt);
        int64_t tot = 0;
        for (int64_t i = 0; i < cnt; ++i) {
            rtproj_plan p = b->sub[i];
            const int rows = X[i] ? (int)p->m : 0;
            cp[i] = rt::CopyGroupArgs{p->d_xhi, p->m, X[i], X[i] ? ldx[i] : 0, rows, (int)kk[i], nullptr, 0};
            tot = std::max(tot, (int64_t)rows * kk[i]);
        }
        Op o{OP_COPY, P.add(cp), (int)cnt};
        o.total = tot;
        P.push(o);
    }
}

// ------------------------------------------------------------- execution
__global__ void zero_flags_kernel(unsigned *const *flags, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) *flags[i] = 0u;
}

hipError_t run_op(const Op &o, const unsigned char *arena, hipStream_t s)
{
    const void *d = arena + o.off;
    switch (o.kind) {
    case OP_GEMM: return rt::gemm_f64_grouped((const rt::GemmArgs *)d, o.count, o.gs, s);
    case OP_REDUCE: return rt::reduce_splits_grouped_f64((const rt::ReduceGroupArgs *)d, o.count, o.total, s);
    case OP_SKETCH:
        return o.i0 ? rt::sketch_grouped_f32((const rt::SketchGroupArgs *)d, o.count, o.ss, s)
                    : rt::sketch_grouped_f64((const rt::SketchGroupArgs *)d, o.count, o.ss, s);
    case OP_COPY: return rt::copy_cols_grouped_f64((const rt::CopyGroupArgs *)d, o.count, o.total, s);
    case OP_SET0: return rt::set_matrix_grouped_f64((const rt::MatGroupArgs *)d, o.count, o.total, 0, s);
    case OP_SET1: return rt::set_matrix_grouped_f64((const rt::MatGroupArgs *)d, o.count, o.total, 1, s);
    case OP_SHIFT: return rt::shift_diag_grouped_f64((const rt::MatGroupArgs *)d, o.count, s);
    case OP_CHOL: return rt::chol_diag_grouped_f64((const rt::CholGroupArgs *)d, o.count, NBB, o.i0, s);
    case OP_TRIINV: return rt::tri_diag_inv_grouped_f64((const rt::TriInvGroupArgs *)d, o.count, o.i0, NBB, s);
    case OP_QRCPWG: return rt::qrcp_wg_f64((const rt::QrcpWgArgs *)d, o.count, s);
    case OP_QRCPGRP: {
        rt::QrcpGrpShape sh;
        sh.nc = o.i0; sh.rpt = o.i1; sh.threads = o.i2; sh.gmax = o.dd; sh.per_launch = (int)o.total;
        return rt::qrcp_grp_f64((const rt::QrcpGrpArgs *)d, o.count, sh, s);
    }
    case OP_RDIAG: return rt::rdiag_grouped_f64((const rt::MatGroupArgs *)d, o.count, s);
    case OP_FORMTP: return rt::form_tp_grouped_f64((const rt::MatGroupArgs *)d, o.count, o.total, s);
    case OP_ZERO:
        hipLaunchKernelGGL(zero_flags_kernel, dim3((o.count + 255) / 256), dim3(256), 0, s, (unsigned *const *)d, o.count);
        return hipGetLastError();
    case OP_AB: return rt::ab_partial_grouped_f64((const rt::AbGroupArgs *)d, o.count, o.i0, o.i1, o.i2, o.dd, s);
    case OP_ABRED: return rt::ab_reduce_grouped_f64((const rt::AbGroupArgs *)d, o.count, o.total, o.dd, s);
    case OP_ATX: return rt::atx_grouped_f64((const rt::AtxGroupArgs *)d, o.count, o.total, o.i1, o.dd, o.i0, s);
    case OP_DDUPD: return rt::dd_update_grouped_f64((const rt::DdGroupArgs *)d, o.count, s);
    case OP_IOTA: return rt::iota_grouped_i32((const rt::MatGroupArgs *)d, o.count, o.i0, s);
    case OP_GEMM32: return rt::gemm_f32_grouped_lower((const rt::GemmMxArgs *)d, o.count, o.i0, o.i1, s);
    case OP_GEMMX3: return rt::gemm_bf16x3_grouped_lower((const rt::GemmMxArgs *)d, o.count, o.i0, o.i1, s);
    case OP_RED32: return rt::reduce_f32_grouped((const rt::ReduceF32GroupArgs *)d, o.count, o.i0, s);
    case OP_FINISH: return rt::finish_cols_grouped_f64((const rt::FinishGroupArgs *)d, o.count, o.total, s);
    }
    return hipErrorInvalidValue;
}

// Everything a launch sequence depends on: the descriptor bytes and every
// op's own launch parameters (kind, offset, counts, shapes, flags), so that
// two programs with equal descriptors but different flags (a compensated
// against a plain pass) never share a captured graph.
std::vector<unsigned char> program_key(const Program &P)
{
    std::vector<unsigned char> key(P.bytes);
    auto put = [&key](const void *v, size_t n) {
        const unsigned char *c = static_cast<const unsigned char *>(v);
        key.insert(key.end(), c, c + n);
    };
    for (const Op &o : P.ops) {
        const int ints[] = {(int)o.kind, o.count, o.i0, o.i1, o.i2, o.dd, o.gs.M, o.gs.N, o.gs.ksplit, o.gs.a_kc,
                            o.gs.b_kc, o.gs.c_lower, o.gs.b_gather, o.ss.chunks};
        const int64_t longs[] = {(int64_t)o.off, o.total, o.ss.max_n1, o.ss.max_n2, o.ss.max_rows_chunk};
        put(ints, sizeof(ints));
        put(longs, sizeof(longs));
    }
    return key;
}

// Upload the program's descriptors (only if they changed) and run it, from
// the captured graph when enabled and still valid.
rtproj_status run_program(rtproj_batch b, rtproj_batch_s::Slot &slot, const Program &P)
{
    hipStream_t s = b->stream;
    DevBuf &a = slot.arena;
    const bool same = a.shadow == P.bytes;
    if (!same) {
        if (P.bytes.size() > a.cap) {
            if (a.d) RT_HIP(hipFree(a.d));
            a.d = nullptr;
            a.cap = 0;
            RT_HIP(hipMalloc((void **)&a.d, P.bytes.size()));
            a.cap = P.bytes.size();
        }
        RT_HIP(hipMemcpyAsync(a.d, P.bytes.data(), P.bytes.size(), hipMemcpyHostToDevice, s));
        RT_HIP(hipStreamSynchronize(s));  // the host copy is released after this call
        a.shadow = P.bytes;
    }
    if (!b->use_graph) {
        if (!b->timing) {
            for (const Op &o : P.ops) RT_HIP(run_op(o, a.d, s));
            return RTPROJ_OK;
        }
        // per-stage events around each run of ops of one stage
        struct Ev { int stage; hipEvent_t e0, e1; };
        std::vector<Ev> evs;
        size_t i = 0;
        hipError_t err = hipSuccess;
        while (i < P.ops.size() && err == hipSuccess) {
            const int st = P.ops[i].stage;
            Ev ev{st, nullptr, nullptr};
            (void)hipEventCreate(&ev.e0);
            (void)hipEventCreate(&ev.e1);
            (void)hipEventRecord(ev.e0, s);
            for (; i < P.ops.size() && P.ops[i].stage == st; ++i)
                if ((err = run_op(P.ops[i], a.d, s)) != hipSuccess) break;
            (void)hipEventRecord(ev.e1, s);
            evs.push_back(ev);
        }
        (void)hipStreamSynchronize(s);
        for (Ev &ev : evs) {
            float ms = 0.f;
            if (ev.stage >= 0 && ev.stage < 16 && hipEventElapsedTime(&ms, ev.e0, ev.e1) == hipSuccess) {
                b->t_stage_ms[ev.stage] += ms;
                b->stage_calls[ev.stage] += 1;
            }
            (void)hipEventDestroy(ev.e0);
            (void)hipEventDestroy(ev.e1);
        }
        RT_HIP(err);
        return RTPROJ_OK;
    }
    std::vector<unsigned char> key = program_key(P);
    if (!slot.exec || slot.graph_key != key) {
        if (slot.exec) { (void)hipGraphExecDestroy(slot.exec); slot.exec = nullptr; }
        if (slot.graph) { (void)hipGraphDestroy(slot.graph); slot.graph = nullptr; }
        if (!b->cap_stream) RT_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
        hipStream_t cs = b->cap_stream;
        RT_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (const Op &o : P.ops)
            if ((e = run_op(o, a.d, cs)) != hipSuccess) break;
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (e != hipSuccess) { if (g) (void)hipGraphDestroy(g); RT_HIP(e); }
        RT_HIP(e2);
        slot.graph = g;
        RT_HIP(hipGraphInstantiate(&slot.exec, slot.graph, nullptr, nullptr, 0));
        slot.graph_key = std::move(key);
    }
    RT_HIP(hipGraphLaunch(slot.exec, s));
    return RTPROJ_OK;
}

// Whether the grouped pivoted QR of the R0 factors beats one workgroup per
// member, from per-step costs measured on this part: a workgroup streams its
// trailing matrix through L2 at every step (read and write at about 27 GB/s
// per workgroup, plus about 1.5 us of block barriers), while a group of
// blocks is bound by its exchange between blocks (about 8 us per step at
// m = 1024) and runs as many members at once as stay resident.
bool grouped_qr_faster(const int64_t *m, int64_t count, int cu, const rt::QrcpGrpShape &sh)
{
    double wg = 0.0, grp = 0.0;
    for (int64_t i = 0; i < count; ++i) {
        const double mi = (double)m[i];
        wg = std::max(wg, mi * mi * mi * 16.0 / (3.0 * 27e9) + 1.5e-6 * mi);
        grp = std::max(grp, 8e-6 * mi);
    }
    wg *= (double)((count + cu - 1) / cu);
    grp *= (double)((count + sh.per_launch - 1) / sh.per_launch);
    return grp < wg;
}

}  // namespace

extern "C" {

rtproj_status rtproj_batch_create(int64_t count, const int64_t *m, const int64_t *n, const int64_t *l, uint64_t seed,
                                  rtproj_batch *out)
{
    if (!out) return fail(RTPROJ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (count < 1) return fail(RTPROJ_ERR_INVALID_ARG, "count < 1");
    if (!m || !n || !l) return fail(RTPROJ_ERR_INVALID_ARG, "size arrays are NULL");
    for (int64_t i = 0; i < count; ++i) {
        if (m[i] < 1 || n[i] < m[i] || l[i] < m[i] || l[i] > n[i])
            return fail(RTPROJ_ERR_INVALID_ARG, "member " + std::to_string(i) + ": need 1 <= m <= l <= n");
        // (the grouped form of the QR of R0 reaches no further on 256 compute units)
        if (m[i] > rt::qrcp_wg_max_cols() || m[i] > rt::qrcp_wg_max_rows())
            return fail(RTPROJ_ERR_UNSUPPORTED, "member " + std::to_string(i) + ": m above the batched QR limit");
    }
    rtproj_batch b = new (std::nothrow) rtproj_batch_s;
    if (!b) return fail(RTPROJ_ERR_ALLOC, "host allocation failed");
    b->count = count;
    b->sub.assign(count, nullptr);
    for (int64_t i = 0; i < count; ++i) {
        rtproj_status st = rtproj_plan_create(m[i], n[i], l[i], instance_seed(seed, i), &b->sub[i]);
        if (st != RTPROJ_OK) {
            const std::string msg = g_last_error;
            rtproj_batch_destroy(b);
            return fail(st, "member " + std::to_string(i) + ": " + msg);
        }
        b->max_m = std::max(b->max_m, m[i]);
        b->max_n = std::max(b->max_n, n[i]);
        b->max_l = std::max(b->max_l, l[i]);
    }
    if (hipMalloc((void **)&b->d_diag_all, (size_t)count * 8 * sizeof(double)) != hipSuccess) {
        b->d_diag_all = nullptr;
        rtproj_batch_destroy(b);
        return fail(RTPROJ_ERR_ALLOC, "device allocation failed");
    }
    // the pivoted QR of R0: one workgroup per member or a group of blocks per member
    {
        const int cu = b->sub[0]->cu_count;
        const bool wg_ok = b->max_m <= rt::qrcp_wg_max_cols() && b->max_m <= rt::qrcp_wg_max_rows();
        rt::QrcpGrpShape sh;
        const bool grp_ok = rt::qrcp_grp_shape((int)b->max_m, (int)b->max_m, cu, &sh);
        if (!wg_ok && !grp_ok) {
            rtproj_batch_destroy(b);
            return fail(RTPROJ_ERR_UNSUPPORTED, "a member's m is above the batched QR limits");
        }
        if (grp_ok && (!wg_ok || grouped_qr_faster(m, count, cu, sh))) {
            b->qr_grp = sh;
            b->qrw_off.resize(count);
            int64_t tot = 0;
            for (int64_t i = 0; i < count; ++i) {
                const int64_t G = (m[i] + sh.nc - 1) / sh.nc;
                b->qrw_off[i] = tot;
                tot += 4 * G + 2 * G * m[i];
            }
            if (hipMalloc((void **)&b->d_qrw, (size_t)tot * sizeof(double)) != hipSuccess) {
                b->d_qrw = nullptr;
                rtproj_batch_destroy(b);
                return fail(RTPROJ_ERR_ALLOC, "device allocation failed");
            }
        }
    }
    *out = b;
    return RTPROJ_OK;
}

rtproj_status rtproj_batch_destroy(rtproj_batch b)
{
    if (!b) return RTPROJ_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    else (void)hipDeviceSynchronize();
    for (rtproj_plan p : b->sub)
        if (p) rtproj_plan_destroy(p);
    if (b->d_diag_all) (void)hipFree(b->d_diag_all);
    if (b->d_qrw) (void)hipFree(b->d_qrw);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return RTPROJ_OK;
}

rtproj_status rtproj_batch_set_stream(rtproj_batch b, void *stream)
{
    if (!b) return fail(RTPROJ_ERR_INVALID_ARG, "null batch");
    b->stream = (hipStream_t)stream;
    for (rtproj_plan p : b->sub) rtproj_plan_set_stream(p, stream);
    return RTPROJ_OK;
}

rtproj_status rtproj_batch_set_refinement(rtproj_batch b, int steps)
{
    if (!b) return fail(RTPROJ_ERR_INVALID_ARG, "null batch");
    if (steps < -1 || steps > 64) return fail(RTPROJ_ERR_INVALID_ARG, "steps outside [-1, 64]");
    b->refine_steps = steps;
    return RTPROJ_OK;
}

rtproj_status rtproj_batch_set_precision(rtproj_batch b, int precision)
{
    if (!b) return fail(RTPROJ_ERR_INVALID_ARG, "null batch");
    if (precision != RTPROJ_PREC_FP64 && precision != RTPROJ_PREC_MIXED_FP32 && precision != RTPROJ_PREC_MIXED_BF16X3)
        return fail(precision == RTPROJ_PREC_MIXED_BF16 ? RTPROJ_ERR_UNSUPPORTED : RTPROJ_ERR_INVALID_ARG,
                    "batches take RTPROJ_PREC_FP64, RTPROJ_PREC_MIXED_FP32 or RTPROJ_PREC_MIXED_BF16X3");
    b->precision = precision;
    return RTPROJ_OK;
}

rtproj_status rtproj_batch_set_graph(rtproj_batch b, int enable)
{
    if (!b) return fail(RTPROJ_ERR_INVALID_ARG, "null batch");
    b->use_graph = enable ? 1 : 0;
    return RTPROJ_OK;
}

rtproj_status rtproj_batch_set_timing(rtproj_batch b, int enable)
{
    if (!b) return fail(RTPROJ_ERR_INVALID_ARG, "null batch");
    b->timing = enable ? 1 : 0;
    for (int s = 0; s < 16; ++s) { b->t_stage_ms[s] = 0.0; b->stage_calls[s] = 0; }
    return RTPROJ_OK;
}

rtproj_status rtproj_batch_info(rtproj_batch b, rtproj_info *out)
{
    if (!b || !out) return fail(RTPROJ_ERR_INVALID_ARG, "null batch or output");
    std::memset(out, 0, sizeof(*out));
    out->m = b->max_m; out->n = b->max_n; out->l = b->max_l;
    out->refine_steps = b->plain_steps + b->comp_steps;
    out->qr_mode = b->qr_grp.per_launch > 0 ? RTPROJ_QR_TWO_STAGE : RTPROJ_QR_TWO_STAGE_WG;
    for (int s = 0; s < 16; ++s) { out->t_stage_ms[s] = b->t_stage_ms[s]; out->stage_calls[s] = b->stage_calls[s]; }
    return RTPROJ_OK;
}

rtproj_status rtproj_batch_precondition_scaled(rtproj_batch b, const double *const *A, const int64_t *lda,
                                              const double *const *col_scale)
{
    if (!b) return fail(RTPROJ_ERR_INVALID_ARG, "null batch");
    if (!A || !lda) return fail(RTPROJ_ERR_INVALID_ARG, "A or lda is NULL");
    for (int64_t i = 0; i < b->count; ++i) {
        if (!A[i]) return fail(RTPROJ_ERR_INVALID_ARG, "member " + std::to_string(i) + ": A is NULL");
        if (lda[i] < b->sub[i]->n) return fail(RTPROJ_ERR_INVALID_ARG, "member " + std::to_string(i) + ": lda < n");
    }
    b->ready = false;
    // a column-scaled member borrows d as it borrows A: every pass that reads
    // A applies the scaling itself, and no scaled copy is made
    b->cscale.assign(b->count, nullptr);
    if (col_scale)
        for (int64_t i = 0; i < b->count; ++i) b->cscale[i] = col_scale[i];
    b->prec_used = b->precision;
    // the split-bfloat16 Gram reads 16-byte rows of binary32 W: every member
    // needs n % 4 == 0, else the batch takes the binary32 Gram
    b->x3 = b->prec_used == RTPROJ_PREC_MIXED_BF16X3;
    for (int64_t i = 0; i < b->count && b->x3; ++i) b->x3 = b->sub[i]->n % 4 == 0;
    // the reduced precisions sketch in binary32; when that proves too coarse
    // for any member (as for plans: 2^-24 kappa_est above RT_SKETCH32_MAX, a
    // failed rank test, or a Gram condition estimate above RT_COND_ESCALATE),
    // every member is sketched again in binary64
    b->sketch64 = b->prec_used == RTPROJ_PREC_FP64;
    b->escalated = false;
    for (;;) {
        Program P;
        build_precondition(P, b, A, lda, b->cscale.data());
        rtproj_status st = run_program(b, b->pre, P);
        if (st != RTPROJ_OK) return st;
        if (b->sketch64) break;
        std::vector<double> diag((size_t)b->count * 8);
        RT_HIP(hipMemcpyAsync(diag.data(), b->d_diag_all, diag.size() * sizeof(double), hipMemcpyDeviceToHost,
                              b->stream));
        RT_HIP(hipStreamSynchronize(b->stream));
        bool coarse = false;
        for (int64_t i = 0; i < b->count && !coarse; ++i) {
            const double *d = diag.data() + 8 * i;
            const double kap = d[2] > 0 ? d[3] / d[2] : INFINITY;
            const double cw = d[6] > 0 ? d[7] / d[6] : INFINITY;
            coarse = !(std::ldexp(kap, -24) <= RT_SKETCH32_MAX) ||
                     !(d[2] > (double)b->sub[i]->m * std::ldexp(1.0, -52) * d[3]) || !(cw <= RT_COND_ESCALATE);
        }
        if (!coarse) break;
        b->sketch64 = true;
        b->escalated = true;
    }
    for (int64_t i = 0; i < b->count; ++i) {
        b->sub[i]->A = A[i];
        b->sub[i]->lda = lda[i];
    }
    b->ready = true;
    return RTPROJ_OK;
}

rtproj_status rtproj_batch_precondition(rtproj_batch b, const double *const *A, const int64_t *lda)
{
    return rtproj_batch_precondition_scaled(b, A, lda, nullptr);
}

rtproj_status rtproj_batch_project_all(rtproj_batch b, const double *const *B, const int64_t *ldb, const int64_t *k,
                                       double *const *Z, const int64_t *ldz, double *const *Y, const int64_t *ldy,
                                       double *const *X, const int64_t *ldx)
{
    if (!b) return fail(RTPROJ_ERR_INVALID_ARG, "null batch");
    if (!b->ready) return fail(RTPROJ_ERR_STATE, "batch projection before a successful rtproj_batch_precondition");
    if (!B || !ldb || !k) return fail(RTPROJ_ERR_INVALID_ARG, "B, ldb or k is NULL");
    for (int64_t i = 0; i < b->count; ++i) {
        rtproj_plan p = b->sub[i];
        const std::string who = "member " + std::to_string(i) + ": ";
        if (k[i] < 0) return fail(RTPROJ_ERR_INVALID_ARG, who + "k < 0");
        if (k[i] == 0) continue;
        if (!B[i] || ldb[i] < p->n) return fail(RTPROJ_ERR_INVALID_ARG, who + "B is NULL or ldb < n");
        if (Z && Z[i] && (!ldz || ldz[i] < p->n)) return fail(RTPROJ_ERR_INVALID_ARG, who + "ldz < n");
        if (Y && Y[i] && (!ldy || ldy[i] < p->n)) return fail(RTPROJ_ERR_INVALID_ARG, who + "ldy < n");
        if (X && X[i] && (!ldx || ldx[i] < p->m)) return fail(RTPROJ_ERR_INVALID_ARG, who + "ldx < m");
        if ((Z && Z[i] == B[i] && ldz[i] != ldb[i]) || (Y && Y[i] == B[i] && ldy[i] != ldb[i]))
            return fail(RTPROJ_ERR_INVALID_ARG, who + "an output aliases B with a different leading dimension");
    }
    for (int64_t i = 0; i < b->count; ++i) {
        rtproj_status st = ensure_k(b->sub[i], std::max<int64_t>(1, k[i]));
        if (st != RTPROJ_OK) return st;
    }
    if (b->refine_steps >= 0) {
        b->plain_steps = 0;
        b->comp_steps = b->refine_steps;
        b->comp_final = b->refine_steps > 0;
    } else {
        // one schedule for all members (one program): the most demanding one,
        // from the rank estimates the preconditioner left on the device
        std::vector<double> diag((size_t)b->count * 8);
        RT_HIP(hipMemcpyAsync(diag.data(), b->d_diag_all, diag.size() * sizeof(double), hipMemcpyDeviceToHost,
                              b->stream));
        RT_HIP(hipStreamSynchronize(b->stream));
        int pl = 0, cp = 0;
        bool cf = false;
        for (int64_t i = 0; i < b->count; ++i) {
            const double *d = diag.data() + 8 * i;
            const double kap = d[2] > 0 ? d[3] / d[2] : 1e16;
            const double cw = d[6] > 0 ? d[7] / d[6] : 1e3;
            rtproj_plan p = b->sub[i];
            const double gram_k = (double)p->n / std::max<int64_t>(1, std::min<int64_t>(p->syrk_splits, p->n / 256));
            const RefinePlan rp = refine_schedule(std::isfinite(kap) ? kap : 1e16, b->prec_used, false,
                                                  std::isfinite(cw) ? cw : 1e3, gram_k, RTPROJ_RESID_FULL, -1);
            pl = std::max(pl, rp.plain);
            cp = std::max(cp, rp.comp);
            cf = cf || rp.comp_final;
        }
        b->plain_steps = pl;
        b->comp_steps = cp;
        b->comp_final = cf;
    }
    std::vector<const double *> A(b->count);
    std::vector<int64_t> lda(b->count);
    for (int64_t i = 0; i < b->count; ++i) { A[i] = b->sub[i]->A; lda[i] = b->sub[i]->lda; }
    Program P;
    build_project(P, b, A.data(), lda.data(), b->cscale.data(), B, ldb, k, Z, ldz, Y, ldy, X, ldx);
    b->last_steps = std::min(b->plain_steps + b->comp_steps, RT_MAX_STEPS);
    b->last_plain = std::min(b->plain_steps, b->last_steps);
    b->last_k.assign(k, k + b->count);
    return run_program(b, b->pro, P);
}

rtproj_status rtproj_batch_status(rtproj_batch b, int *per_member)
{
    if (!b) return fail(RTPROJ_ERR_INVALID_ARG, "null batch");
    std::vector<double> diag((size_t)b->count * 8);
    std::vector<int> cerr(b->count), qerr(b->count);
    hipStream_t s = b->stream;
    RT_HIP(hipMemcpyAsync(diag.data(), b->d_diag_all, diag.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    for (int64_t i = 0; i < b->count; ++i) {
        RT_HIP(hipMemcpyAsync(&cerr[i], b->sub[i]->d_err, sizeof(int), hipMemcpyDeviceToHost, s));
        RT_HIP(hipMemcpyAsync(&qerr[i], b->sub[i]->d_sync + 2, sizeof(int), hipMemcpyDeviceToHost, s));
    }
    // per-step refinement norms of the last projection (members with k > 0)
    const int ns = b->last_k.size() == (size_t)b->count ? b->last_steps : 0;
    std::vector<double> norms((size_t)b->count * 2 * std::max(ns, 1), 0.0);
    for (int64_t i = 0; i < b->count && ns > 0; ++i)
        if (b->last_k[i] > 0)
            RT_HIP(hipMemcpyAsync(norms.data() + (size_t)i * 2 * ns, b->sub[i]->d_norms, (size_t)ns * 2 * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
    RT_HIP(hipStreamSynchronize(s));
    rtproj_status worst = RTPROJ_OK;
    for (int64_t i = 0; i < b->count; ++i) {
        rtproj_plan p = b->sub[i];
        const double *d = diag.data() + 8 * i;
        rtproj_status st = RTPROJ_OK;
        if (ns > 0 && b->last_k[i] > 0) {
            double rho, err;
            st = refine_verdict(norms.data() + (size_t)i * 2 * ns, ns, b->last_plain, &rho, &err);
            p->info.refine_rho_est = rho;
            p->info.refine_err_est = err;
            p->info.refine_status = st;
        }
        if (qerr[i] || cerr[i] || !(d[2] > (double)p->m * std::ldexp(1.0, -52) * d[3])) st = RTPROJ_ERR_RANK;
        if (qerr[i] == 1) st = RTPROJ_ERR_DEVICE;  // the grouped QR's barrier timed out
        p->info.kappa_est = d[2] > 0 ? d[3] / d[2] : INFINITY;
        p->info.rdiag_min = d[2];
        p->info.gram_cond_est = d[6] > 0 ? d[7] / d[6] : INFINITY;
        p->info.inverse = RTPROJ_INV_CHOLESKY;
        p->inv_used = RTPROJ_INV_CHOLESKY;
        p->info.precision = b->prec_used;
        p->info.gram_bits = b->x3 ? 17 : (b->prec_used != RTPROJ_PREC_FP64 ? 32 : 64);
        p->info.w_bits = 64;
        p->info.sketch_bits = b->sketch64 ? 64 : 32;
        p->info.sketch_escalated = b->escalated ? 1 : 0;
        if (per_member) per_member[i] = st;
        // precedence: rank deficiency, then a device error, then non-convergence
        if (st == RTPROJ_ERR_RANK || (st == RTPROJ_ERR_DEVICE && worst != RTPROJ_ERR_RANK) ||
            (st != RTPROJ_OK && worst == RTPROJ_OK))
            worst = st;
    }
    if (worst == RTPROJ_ERR_RANK)
        return fail(worst, "at least one member is rank deficient or its factorization broke down");
    if (worst == RTPROJ_ERR_DEVICE) return fail(worst, "pivoted QR: a member's block barrier timed out");
    if (worst != RTPROJ_OK) return fail(worst, "the refinement of at least one member did not converge");
    return RTPROJ_OK;
}

rtproj_status rtproj_batch_member_tables(rtproj_batch b, int64_t i, int64_t *dims3, int8_t *sign, int32_t *sigma,
                                         int32_t *tau, int32_t *J)
{
    if (!b || i < 0 || i >= b->count) return fail(RTPROJ_ERR_INVALID_ARG, "bad batch or member");
    return rtproj_sketch_tables(b->sub[i], dims3, sign, sigma, tau, J);
}

rtproj_status rtproj_batch_member_info(rtproj_batch b, int64_t i, rtproj_info *out)
{
    if (!b || !out || i < 0 || i >= b->count) return fail(RTPROJ_ERR_INVALID_ARG, "bad batch, member or output");
    *out = b->sub[i]->info;
    out->m = b->sub[i]->m; out->n = b->sub[i]->n; out->l = b->sub[i]->l; out->np = b->sub[i]->tab.np;
    out->refine_steps = b->plain_steps + b->comp_steps;
    out->refine_plain = b->plain_steps;
    out->refine_comp = b->comp_steps;
    out->qr_mode = b->qr_grp.per_launch > 0 ? RTPROJ_QR_TWO_STAGE : RTPROJ_QR_TWO_STAGE_WG;
    return RTPROJ_OK;
}

}  // extern "C"
