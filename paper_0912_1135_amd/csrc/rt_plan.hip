// Host runtime and C ABI of the randomized orthogonal projection library
// (see include/rtproj.h for the contract).
//
// Preconditioning (Sec. 4, first two step lists):
//   1. S = A G, the SRFT sketch of eq. testing              sketch_f64
//   2. S^T = Q R Pi, eq. QR_decomp                           qrcp_f64 (cooperative)
//   3. R^{-T}, the transposed P^- of eq. scary               blocked TRSM on MFMA
//   4. W = P^{-1} A = R^{-T} (Pi A)                          triangular GEMM on MFMA
//   5. X = W W^T (steps a-e)                                 SYRK on MFMA, split-K
//   6. X = L L^T (replaces the inverse of eq. inversion)     blocked Cholesky
//   7. T = L^{-1} R^{-T}, T' = T Pi, so that
//      (A A^T)^{-1} = Pi^T R^{-1} X^{-1} R^{-T} Pi = T'^T T'
// Projection (the seven steps of Sec. 4; Remark 4.1; Remark 4.3):
//   c = A b, x = T'^T (T' c), then refinement steps
//   x += T'^T T' A (b - A^T x) with Dot2 residuals, then
//   A^T x (row projection) and b - A^T x (null projection).
#include "rt_plan_state.h"
namespace rtp {

thread_local std::string g_last_error;

rtproj_status fail(rtproj_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

uint64_t instance_seed(uint64_t seed, int64_t i)
{
    SplitMix64 g{seed ^ (uint64_t)i};
    return g.next();
}

}  // namespace rtp

using namespace rtp;

namespace rtp {

// Records a start event on construction and a stop event on destruction
// when the plan's stage timing is enabled.
struct StageScope {
    rtproj_plan p;
    int stage;
    hipEvent_t start = nullptr, stop = nullptr;
    StageScope(rtproj_plan plan, int st) : p(plan), stage(st)
    {
        if (p->timing && hipEventCreate(&start) == hipSuccess && hipEventCreate(&stop) == hipSuccess)
            (void)hipEventRecord(start, p->stream);
    }
    ~StageScope()
    {
        if (start && stop) {
            (void)hipEventRecord(stop, p->stream);
            p->pending.push_back({stage, start, stop});
        }
    }
};

void collect_timing(rtproj_plan p)
{
    for (auto &e : p->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e.start, e.stop) == hipSuccess) {
            p->info.t_stage_ms[e.stage] += ms;
            p->info.stage_calls[e.stage] += 1;
        }
        (void)hipEventDestroy(e.start);
        (void)hipEventDestroy(e.stop);
    }
    p->pending.clear();
}

// Argument blocks of the recursive-doubling inverse X = L^{-1} of the m x m
// lower-triangular L read as L(i, j) = Lp[i l_i + j l_j], X and the scratch T
// row-major m x m: level s joins pairs of inverted diagonal blocks of size
// S = NB 2^s; for the pair at rows/cols c0 .. c0 + S (X11) and r0 = c0 + S ..
// r0 + s2 (X22), T = L21 X11 goes to T's block (r0, c0), then X21 = -X22 T
// to the same block of X (the inverse of [L11 0; L21 L22] is
// [X11 0; -X22 L21 X11 X22]).
hipError_t build_tri_inverse(int64_t m, const double *Lp, int64_t l_i, int64_t l_j, double *X, double *T,
                             TriInverse &out)
{
    std::vector<rt::GemmArgs> all;
    out.count.clear();
    out.shape1.clear();
    out.shape2.clear();
    for (int64_t S = NB; S < m; S *= 2) {
        std::vector<rt::GemmArgs> g1, g2;
        for (int64_t c0 = 0; c0 + S < m; c0 += 2 * S) {
            const int64_t r0 = c0 + S, s1 = S, s2 = std::min<int64_t>(S, m - r0);
            rt::GemmArgs a{};
            a.M = (int)s2; a.N = (int)s1; a.K = (int)s1;
            a.A = Lp + r0 * l_i + c0 * l_j; a.a_i = l_i; a.a_k = l_j;
            a.B = X + c0 * m + c0; a.b_k = m; a.b_j = 1;
            a.C = T + r0 * m + c0; a.c_i = m; a.c_j = 1;
            a.alpha = 1.0; a.ksplit = 1;
            g1.push_back(a);
            rt::GemmArgs b{};
            b.M = (int)s2; b.N = (int)s1; b.K = (int)s2;
            b.A = X + r0 * m + r0; b.a_i = m; b.a_k = 1;
            b.B = T + r0 * m + c0; b.b_k = m; b.b_j = 1;
            b.C = X + r0 * m + c0; b.c_i = m; b.c_j = 1;
            b.alpha = -1.0; b.ksplit = 1;
            g2.push_back(b);
        }
        rt::GemmShape h1{}, h2{};
        h1.M = h2.M = (int)S; h1.N = h2.N = (int)S; h1.ksplit = h2.ksplit = 1;
        h1.a_kc = l_j == 1 ? 1 : 0; h1.b_kc = 0; h2.a_kc = 1; h2.b_kc = 0;
        out.count.push_back((int)g1.size());
        out.shape1.push_back(h1);
        out.shape2.push_back(h2);
        all.insert(all.end(), g1.begin(), g1.end());
        all.insert(all.end(), g2.begin(), g2.end());
    }
    if (all.empty()) return hipSuccess;
    hipError_t e = hipMalloc(&out.d_args, all.size() * sizeof(rt::GemmArgs));
    if (e != hipSuccess) return e;
    return hipMemcpy(out.d_args, all.data(), all.size() * sizeof(rt::GemmArgs), hipMemcpyHostToDevice);
}

// X = L^{-1} from the inverted diagonal blocks Dinv (placed into a cleared X)
// and the levels of t, on the plan's stream.
hipError_t run_tri_inverse(rtproj_plan p, const TriInverse &t, const double *Dinv, double *X)
{
    const int64_t m = p->m;
    hipStream_t s = p->stream;
    hipError_t e = rt::set_matrix_f64(X, m, (int)m, (int)m, 0, s);
    if (e == hipSuccess) e = rt::place_diag_blocks_f64(Dinv, (int)m, NB, X, m, s);
    size_t off = 0;
    for (size_t lv = 0; lv < t.count.size() && e == hipSuccess; ++lv) {
        const int cnt = t.count[lv];
        e = rt::gemm_f64_grouped(t.d_args + off, cnt, t.shape1[lv], s);
        if (e == hipSuccess) e = rt::gemm_f64_grouped(t.d_args + off + cnt, cnt, t.shape2[lv], s);
        off += 2 * (size_t)cnt;
    }
    return e;
}

void release(rtproj_plan p)
{
    for (auto &e : p->pending) {
        (void)hipEventDestroy(e.start);
        (void)hipEventDestroy(e.stop);
    }
    p->pending.clear();
    void *bufs[] = {p->d_sign, p->d_sigma, p->d_tauinv, p->d_sel_off, p->d_sel, p->d_tw1, p->d_tw2, p->d_twh,
                    p->d_twl, p->d_tw1f, p->d_tw2f, p->d_twhf, p->d_twlf, p->d_rowscale, p->d_zbuf, p->d_S, p->d_R, p->d_Y, p->d_W, p->d_part, p->d_G, p->d_L, p->d_Tp,
                    p->d_DinvR, p->d_DinvL, p->d_piv, p->d_sync, p->d_slots, p->d_vbuf, p->d_qrcols, p->d_Yq, p->d_R0, p->d_wgargs, p->rinv.d_args, p->linv[0].d_args, p->linv[1].d_args, p->d_Linv, p->d_Yq2, p->d_scal, p->d_diag,
                    p->d_bsum, p->d_c, p->d_tmp, p->d_xhi, p->d_xlo, p->d_d, p->d_r, p->d_ph, p->d_pl, p->d_norms, p->d_xpk, p->d_bpk,
                    p->d_err, p->d_V, p->d_tau, p->d_gpart, p->d_kry, p->d_cflags,
                    p->d_oz_xdig, p->d_oz_rdig, p->d_oz_bexp, p->d_colexp, p->d_rowexp};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    if (p->h_scal) (void)hipHostFree(p->h_scal);
    p->h_scal = nullptr;
    if (p->h_norms) (void)hipHostFree(p->h_norms);
    p->h_norms = nullptr;
}

rtproj_status upload_tables(rtproj_plan p)
{
    const HostTables &t = p->tab;
    const int64_t np = t.np, n1 = t.n1, n2 = t.n2, l = p->l;
    std::vector<int32_t> tauinv(n2);
    for (int64_t i = 0; i < n2; ++i) tauinv[t.tau[i]] = (int32_t)i;
    // selection lists, grouped by the k1-pair w = min(k1, n1 - k1) that owns k
    std::vector<std::vector<int32_t>> lists(n1 / 2 + 1);
    for (int64_t q = 0; q < l; ++q) {
        const int64_t j = t.J[q];
        int64_t k;
        int part;
        if (j == 0) { k = 0; part = 0; }
        else if (j == 1) { k = np / 2; part = 0; }
        else { k = j / 2; part = (int)(j % 2); }
        const int64_t k1 = k % n1;
        const int64_t w = std::min(k1, n1 - k1);
        lists[w].push_back((int32_t)k);
        lists[w].push_back(part);
        lists[w].push_back((int32_t)q);
    }
    std::vector<int32_t> off(n1 / 2 + 2, 0), sel;
    sel.reserve(3 * l);
    for (int64_t w = 0; w <= n1 / 2; ++w) {
        off[w] = (int32_t)(sel.size() / 3);
        sel.insert(sel.end(), lists[w].begin(), lists[w].end());
    }
    off[n1 / 2 + 1] = (int32_t)(sel.size() / 3);
    int e = 0;
    while ((int64_t(1) << e) < np) ++e;
    p->tl_bits = (e + 1) / 2;
    const int64_t tl = int64_t(1) << p->tl_bits;
    std::vector<double> tw1, tw2, twh, twl;
    twiddles(n1, n1 / 2, 1, tw1);
    twiddles(n2, n2 / 2, 1, tw2);
    twiddles(np, np / tl, tl, twh);
    twiddles(np, tl, 1, twl);
    RT_HIP(dalloc(&p->d_sign, np));
    RT_HIP(dalloc(&p->d_sigma, n1));
    RT_HIP(dalloc(&p->d_tauinv, n2));
    RT_HIP(dalloc(&p->d_sel_off, off.size()));
    RT_HIP(dalloc(&p->d_sel, sel.size()));
    RT_HIP(dalloc(&p->d_tw1, tw1.size()));
    RT_HIP(dalloc(&p->d_tw2, tw2.size()));
    RT_HIP(dalloc(&p->d_twh, twh.size()));
    RT_HIP(dalloc(&p->d_twl, twl.size()));
    RT_HIP(hipMemcpy(p->d_sign, t.sign.data(), np, hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(p->d_sigma, t.sigma.data(), n1 * 4, hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(p->d_tauinv, tauinv.data(), n2 * 4, hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(p->d_sel_off, off.data(), off.size() * 4, hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(p->d_sel, sel.data(), sel.size() * 4, hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(p->d_tw1, tw1.data(), tw1.size() * 8, hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(p->d_tw2, tw2.data(), tw2.size() * 8, hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(p->d_twh, twh.data(), twh.size() * 8, hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(p->d_twl, twl.data(), twl.size() * 8, hipMemcpyHostToDevice));
    // binary32 copies for the reduced-precision sketch
    std::vector<double> *srcs[] = {&tw1, &tw2, &twh, &twl};
    float **dsts[] = {&p->d_tw1f, &p->d_tw2f, &p->d_twhf, &p->d_twlf};
    for (int i = 0; i < 4; ++i) {
        std::vector<float> f(srcs[i]->begin(), srcs[i]->end());
        RT_HIP(dalloc(dsts[i], f.size()));
        RT_HIP(hipMemcpy(*dsts[i], f.data(), f.size() * 4, hipMemcpyHostToDevice));
    }
    return RTPROJ_OK;
}

// Newton-Schulz residual block sums: one per 16 x 16 tile of the fused
// products, one per 256 elements of the split ones' affine reduction.
int64_t ns_bsum_count(int64_t m) { return m <= RT_NS_FUSED_MAX_M ? rt::sq_mm_blocks(m) : (m * m + 255) / 256; }

rtproj_status alloc_state(rtproj_plan p)
{
    const int64_t m = p->m, n = p->n, l = p->l, np = p->tab.np;
    // sketch intermediate: at most ~512 MiB of row pairs at a time (measured
    // at m = 512, n = 65536: one 268 MB chunk 0.40 ms, four 64 MiB chunks
    // that stay in the Infinity Cache 0.44 ms, eight 32 MiB chunks 0.51 ms:
    // fewer, fuller launches beat cache residency)
    int64_t pairs = std::max<int64_t>(1, (int64_t(512) << 20) / (np * 16));
    p->rows_chunk = std::min<int64_t>(2 * pairs, (m + 1) / 2 * 2);
    RT_HIP(dalloc(&p->d_zbuf, (size_t)(p->rows_chunk / 2) * np * 2));
    RT_HIP(dalloc(&p->d_S, (size_t)m * l));
    RT_HIP(dalloc(&p->d_R, (size_t)m * m));
    RT_HIP(dalloc(&p->d_Y, (size_t)m * m));
    // W's rows are padded by 32 elements (128 or 256 bytes): with a
    // power-of-two n the unpadded rows would all fall on the same L2 sets,
    // and the Gram's row panels could not stay cached
    p->ldw = n + 32;
    RT_HIP(dalloc(&p->d_W, (size_t)m * p->ldw));
    const int gt = (int)((m + 127) / 128);
    const int tiles = gt * (gt + 1) / 2;
    p->syrk_splits = (int)std::max<int64_t>(1, std::min<int64_t>({64, (4 * p->cu_count + tiles - 1) / tiles, n / 256}));
    {
        // K splits of the Gram of P^-1 A: of the counts from half to twice
        // the one above, the one whose last round of lower 128 x 128 tile
        // blocks fills the compute units best (2048 x 262144: 15 splits,
        // 2040 blocks in 7.97 rounds; 8 splits left the fifth round a
        // quarter full)
        const int64_t sp0 = p->syrk_splits;
        const int64_t hi = std::max<int64_t>(1, std::min<int64_t>({64, 2 * sp0, n / 256}));
        const int64_t lo = std::max<int64_t>(1, std::min<int64_t>(sp0 / 2, hi));
        int64_t best = lo;
        double best_fill = -1.0;
        for (int64_t sp = lo; sp <= hi; ++sp) {
            const int64_t blocks = tiles * sp, rounds = (blocks + p->cu_count - 1) / p->cu_count;
            const double fill = (double)blocks / (double)(rounds * p->cu_count);
            if (fill > best_fill + 1e-9) { best_fill = fill; best = sp; }
        }
        p->wgram_splits = (int)best;
    }
    // split partials: room for twice the built-in split count (the
    // autotuner may pick more splits), at most 64
    p->part_cap = (int)std::min<int64_t>(64, std::max<int64_t>(1, std::min<int64_t>(2 * p->syrk_splits, n / 256)));
    p->part_cap = std::max({p->part_cap, p->syrk_splits, p->wgram_splits});
    RT_HIP(dalloc(&p->d_part, (size_t)p->part_cap * m * m));
    RT_HIP(dalloc(&p->d_G, (size_t)m * m));
    RT_HIP(dalloc(&p->d_L, (size_t)m * m));
    RT_HIP(dalloc(&p->d_Tp, (size_t)2 * m * m));
    RT_HIP(dalloc(&p->d_bsum, (size_t)ns_bsum_count(m)));
    const int64_t nblk = (m + NB - 1) / NB;
    RT_HIP(dalloc(&p->d_DinvR, (size_t)nblk * NB * NB));
    RT_HIP(dalloc(&p->d_DinvL, (size_t)nblk * NB * NB));
    RT_HIP(dalloc(&p->d_piv, (size_t)m));
    RT_HIP(dalloc(&p->d_sync, 4));
    int gcols = 0, gcols0 = 0;
    p->qr_blocks = rt::qrcp_max_blocks((int)l, (int)m, p->cu_count, p->lds_max, &gcols);
    p->qr_blocks0 = rt::qrcp_max_blocks((int)m, (int)m, p->cu_count, p->lds_max, &gcols0);
    if (p->qr_blocks <= 0 && p->qr_blocks0 <= 0 && m > rt::qrcp_wg_max_cols())
        return fail(RTPROJ_ERR_UNSUPPORTED, "pivoted QR: more than 16 columns per compute unit, or l too large, "
                                            "for this (m, l)");
    // register-resident form where the shapes allow it (rows <= 8192)
    int nc_, rpt_;
    int tt_;
    if (!rt::qrcp_reg_shape((int)l, (int)m, p->cu_count, &nc_, &rpt_, &p->qr_reg_l, &tt_)) p->qr_reg_l = 0;
    if (!rt::qrcp_reg_shape((int)m, (int)m, p->cu_count, &nc_, &rpt_, &p->qr_reg_m, &tt_)) p->qr_reg_m = 0;
    const int64_t gmax = std::max({(int64_t)p->qr_blocks, (int64_t)p->qr_blocks0, (int64_t)p->qr_reg_l,
                                   (int64_t)p->qr_reg_m});
    RT_HIP(dalloc(&p->d_slots, (size_t)4 * gmax));
    RT_HIP(dalloc(&p->d_vbuf, (size_t)2 * std::max({(int64_t)p->qr_blocks * l, (int64_t)p->qr_blocks0 * m,
                                                     (int64_t)p->qr_reg_l * l, (int64_t)p->qr_reg_m * m})));
    if (gcols || gcols0)
        RT_HIP(dalloc(&p->d_qrcols, (size_t)16 * std::max<int64_t>(gcols ? p->qr_blocks * l : 0,
                                                                     gcols0 ? p->qr_blocks0 * m : 0)));
    // two-stage pivoted QR: iterates of the Cholesky QR and R0
    RT_HIP(dalloc(&p->d_Yq, (size_t)m * l));
    RT_HIP(dalloc(&p->d_Yq2, (size_t)m * l));
    RT_HIP(dalloc(&p->d_R0, (size_t)m * m));
    {
        rt::QrcpWgArgs wa{};
        wa.M = p->d_R0; wa.ldm = m; wa.rows = (int)m; wa.cols = (int)m;
        wa.R = p->d_R; wa.piv = p->d_piv; wa.err = reinterpret_cast<int *>(p->d_sync + 2);
        RT_HIP(dalloc(&p->d_wgargs, 1));
        RT_HIP(hipMemcpy(p->d_wgargs, &wa, sizeof(wa), hipMemcpyHostToDevice));
    }
    RT_HIP(dalloc(&p->d_scal, 8));
    RT_HIP(hipHostMalloc((void **)&p->h_scal, 4 * sizeof(unsigned long long), hipHostMallocDefault));
    RT_HIP(hipHostMalloc((void **)&p->h_norms, 2 * RT_MAX_STEPS * sizeof(double), hipHostMallocDefault));
    RT_HIP(dalloc(&p->d_diag, 8));
    RT_HIP(dalloc(&p->d_err, 4));
    RT_HIP(dalloc(&p->d_rowscale, (size_t)m));
    RT_HIP(dalloc(&p->d_colexp, (size_t)n));
    RT_HIP(dalloc(&p->d_rowexp, (size_t)m));
    p->chol_blocks = rt::chol_coop_blocks((int)m, p->device);
    if (p->chol_blocks > 0) {
        const int64_t nflags = nblk + nblk * (nblk + 1) / 2;
        RT_HIP(dalloc(&p->d_cflags, (size_t)nflags));
        RT_HIP(rt::zero_u32(p->d_cflags, (int)nflags, p->stream));
        RT_HIP(hipStreamSynchronize(p->stream));  // cleared before any stream the caller sets uses them
    }
    // recursive-doubling inverses: R^{-T} (L = R^T, read as L(i, j) =
    // R[j m + i]) into d_Y with d_L as scratch; the inverses of Cholesky
    // factors in d_L (the Cholesky QR's first factor, and the Gram's) and
    // d_Y (the Cholesky QR's second factor), row-major, into d_Linv with d_G
    // as scratch
    RT_HIP(build_tri_inverse(m, p->d_R, 1, m, p->d_Y, p->d_L, p->rinv));
    RT_HIP(dalloc(&p->d_Linv, (size_t)m * m));
    RT_HIP(build_tri_inverse(m, p->d_L, m, 1, p->d_Linv, p->d_G, p->linv[0]));
    RT_HIP(build_tri_inverse(m, p->d_Y, m, 1, p->d_Linv, p->d_G, p->linv[1]));
    return RTPROJ_OK;
}

bool use_oz(rtproj_plan p, int64_t k)
{
    if (p->comp_method == RTPROJ_COMP_DOT2 || p->m > rt::OZ_KMAX) return false;
    return p->comp_method == RTPROJ_COMP_INT8 || k >= RT_OZ_KMIN;
}

ProjLayout proj_layout(int64_t m, int64_t n, int64_t k, int cu_count, bool oz)
{
    ProjLayout L;
    const int64_t rb = (m + 31) / 32, kb = (k + 31) / 32;  // row blocks x right-hand-side blocks of the A B pass
    L.ab_splits = (int)std::max<int64_t>(1, std::min<int64_t>(n / 256, (4 * cu_count + rb * kb - 1) / (rb * kb)));
    L.ab_sx_splits = rt::ab_sx_splits(m, n, k, cu_count);
    // the MFMA GEMM form: about four 64 x 64 tile blocks per compute unit, so
    // that resident blocks hide each other's load latency (one block per
    // unit leaves the two-chunk load ring exposed)
    const int64_t tiles = ((m + 63) / 64) * ((k + 63) / 64);
    L.ab_mma_splits = (int)std::max<int64_t>(1, std::min<int64_t>({64, n / 256, (4 * cu_count + tiles - 1) / tiles}));
    const int64_t kpad = (k + 63) / 64 * 64, mpad = (m + 63) / 64 * 64, npad = (n + 63) / 64 * 64;
    L.oz = oz;
    if (oz) {
        // the split count that the rounded chunk length really gives (every
        // split non-empty)
        const int s0 = rt::oz_splits(n, ((m + 63) / 64) * (kpad / 64), cu_count);
        const int64_t kc = rt::oz_kchunk(n, s0);
        L.oz_splits = (int)((n + kc - 1) / kc);
    }
    const int64_t psplits = std::max<int64_t>({(int64_t)L.ab_splits, (int64_t)L.ab_sx_splits, (int64_t)L.ab_mma_splits,
                                               (int64_t)L.oz_splits});
    // c, tmp, xhi, xlo, d (m k each), r (n k), ph, pl (split partials), bpk, norms, xpk
    const int64_t cnt[ProjLayout::NBUF] = {m * k, m * k, m * k, m * k, m * k, n * k, psplits * m * k,
                                           psplits * m * k, rt::ab_pack_size(n, k), 2 * RT_MAX_STEPS,
                                           rt::atx_pack_size(m, k),
                                           oz ? (rt::OZ_S * kpad * mpad + 7) / 8 : 1,
                                           oz ? (rt::OZ_S * kpad * npad + 7) / 8 : 1,
                                           oz ? kpad : 1};
    for (int i = 0; i < ProjLayout::NBUF; ++i) L.count[i] = std::max<int64_t>(1, cnt[i]);
    return L;
}

size_t ProjLayout::bytes() const
{
    size_t b = 0;
    for (int i = 0; i < NBUF; ++i) b += ((size_t)count[i] * sizeof(double) + 255) / 256 * 256;
    return b;
}

double **proj_buffers(rtproj_plan p, int i)
{
    double **bufs[ProjLayout::NBUF] = {&p->d_c, &p->d_tmp, &p->d_xhi, &p->d_xlo, &p->d_d, &p->d_r,
                                       &p->d_ph, &p->d_pl, &p->d_bpk, &p->d_norms, &p->d_xpk,
                                       &p->d_oz_xdig, &p->d_oz_rdig, &p->d_oz_bexp};
    return bufs[i];
}

rtproj_status ensure_k(rtproj_plan p, int64_t k)
{
    const bool oz = use_oz(p, std::max(k, p->kcap));
    if (k <= p->kcap && (!oz || p->oz_ready)) return RTPROJ_OK;
    k = std::max(k, p->kcap);
    for (int i = 0; i < ProjLayout::NBUF; ++i) {
        double **b = proj_buffers(p, i);
        if (*b) { (void)hipFree(*b); *b = nullptr; }
    }
    p->kcap = 0;
    p->oz_ready = false;
    const ProjLayout L = proj_layout(p->m, p->n, k, p->cu_count, oz);
    p->ab_splits = L.ab_splits;
    p->ab_sx_splits = L.ab_sx_splits;
    p->ab_mma_splits = L.ab_mma_splits;
    p->oz_splits = L.oz_splits;
    for (int i = 0; i < ProjLayout::NBUF; ++i) RT_HIP(dalloc(proj_buffers(p, i), (size_t)L.count[i]));
    p->kcap = k;
    p->oz_ready = oz;
    return RTPROJ_OK;
}

// Blocked right-looking Cholesky G = L L^T of the m x m matrix G (row-major,
// lower part read and overwritten by the trailing updates) into L; Dinv gets
// the inverses of L's diagonal blocks.  A failed pivot is flagged in d_err.
// One cooperative launch where the device allows it, else one launch per
// diagonal block, panel and trailing update.
rtproj_status cholesky(rtproj_plan p, double *G, double *L, double *Dinv)
{
    const int64_t m = p->m;
    const int64_t nblk = (m + NB - 1) / NB;
    RT_HIP(rt::set_matrix_f64(L, m, (int)m, (int)m, 0, p->stream));
    if (p->chol_blocks > 0) {
        // one cooperative launch; flags hold the call's epoch (never 0, the
        // value they were cleared to)
        if (++p->chol_epoch == 0) ++p->chol_epoch;
        rt::CholCoopArgs a{G, m, (int)m, L, m, Dinv, p->d_err, p->d_cflags, p->chol_epoch};
        RT_HIP(rt::chol_coop_f64(a, p->chol_blocks, p->stream));
        return RTPROJ_OK;
    }
    for (int64_t b = 0; b < nblk; ++b) {
        const int64_t r0 = b * NB, nbb = std::min<int64_t>(NB, m - r0);
        RT_HIP(rt::chol_diag_f64(G, m, (int)m, NB, (int)b, L, m, Dinv, p->d_err, p->stream));
        const int64_t rest = m - r0 - nbb;
        if (rest <= 0) continue;
        // panel: L21 = X21 L11^{-T}
        rt::GemmArgs g{};
        g.M = (int)rest; g.N = (int)nbb; g.K = (int)nbb;
        g.A = G + (r0 + nbb) * m + r0; g.a_i = m; g.a_k = 1;
        g.B = Dinv + b * NB * NB; g.b_k = 1; g.b_j = NB;
        g.C = L + (r0 + nbb) * m + r0; g.c_i = m; g.c_j = 1;
        g.alpha = 1.0; g.ksplit = 1;
        RT_HIP(rt::gemm_f64(g, p->stream));
        // trailing update: X22 -= L21 L21^T (lower tiles)
        rt::GemmArgs u{};
        u.M = (int)rest; u.N = (int)rest; u.K = (int)nbb;
        u.A = L + (r0 + nbb) * m + r0; u.a_i = m; u.a_k = 1;
        u.B = L + (r0 + nbb) * m + r0; u.b_k = 1; u.b_j = m;
        u.C = G + (r0 + nbb) * m + (r0 + nbb); u.c_i = m; u.c_j = 1;
        u.alpha = -1.0; u.beta = 1.0; u.c_lower = 1; u.ksplit = 1;
        RT_HIP(rt::gemm_f64(u, p->stream));
    }
    return RTPROJ_OK;
}

// G (m x m, row-major, both triangles) = A A^T for the row-major m x K
// matrix A: lower tiles on MFMA, split over K, fixed-order reduction.
// G = A A^T (m x m, both triangles) for row-major m x K A: lower tiles
// (tile 0: chosen from the shape; 64: 64 x 64) split over K (splits 0: the
// plan's default), then the fixed-order reduction of the splits.
hipError_t gram_f64_cfg(rtproj_plan p, const double *A, int64_t lda, int64_t K, double *G, int tile, int splits)
{
    const int64_t m = p->m;
    rt::GemmArgs g{};
    g.M = (int)m; g.N = (int)m; g.K = (int)K;
    g.A = A; g.a_i = lda; g.a_k = 1;
    g.B = A; g.b_k = 1; g.b_j = lda;
    g.C = p->d_part; g.c_i = m; g.c_j = 1; g.c_split = m * m;
    g.alpha = 1.0; g.c_lower = 1; g.tile = tile;
    const int64_t sp = splits > 0 ? splits : p->syrk_splits;
    g.ksplit = (int)std::max<int64_t>(1, std::min<int64_t>({sp, K / 256, (int64_t)p->part_cap}));
    hipError_t e = rt::gemm_f64(g, p->stream);
    if (e != hipSuccess) return e;
    return rt::reduce_splits_f64(p->d_part, m * m, g.ksplit, (int)m, (int)m, m, G, m, 1, p->stream);
}

rtproj_status gram_f64(rtproj_plan p, const double *A, int64_t lda, int64_t K, double *G)
{
    RT_HIP(gram_f64_cfg(p, A, lda, K, G, 0, 0));
    return RTPROJ_OK;
}

// One product of a Newton-Schulz step on row-major m x m matrices:
// out = scale (Am Bm) + diag I, with block sums of |out - I|^2 in bsum
// (U = 2I - X Yc, then Yn = Yc U).  Up to RT_NS_FUSED_MAX_M one launch with
// one wave per 16 x 16 tile over the whole K and the affine epilogue fused
// (small products are launch latency); above it, whose fused form would
// read about m^3 bytes from L2, 64 x 64 tiles with K split so that a product
// spans about one block per compute unit, then the affine reduction.
int ns_splits(rtproj_plan p)
{
    // about one block per compute unit, at least 4 splits (measured at
    // m = 512: 4 splits 0.57 ms per inverse, 8 splits 0.59, 2 splits 0.74)
    const int64_t m = p->m, tiles = ((m + 63) / 64) * ((m + 63) / 64);
    const int64_t want = std::max<int64_t>(4, (p->cu_count + tiles - 1) / tiles);
    return (int)std::max<int64_t>(1, std::min<int64_t>({want, m / 64, (int64_t)p->syrk_splits}));
}

rtproj_status ns_product(rtproj_plan p, const double *Am, const double *Bm, double *out, double scale, double diag,
                         double *bsum)
{
    const int64_t m = p->m;
    if (m <= RT_NS_FUSED_MAX_M) {
        RT_HIP(rt::sq_mm_f64((int)m, Am, Bm, out, scale, diag, bsum, p->stream));
        return RTPROJ_OK;
    }
    const int ks = ns_splits(p);
    rt::GemmArgs g{};
    g.M = (int)m; g.N = (int)m; g.K = (int)m;
    g.A = Am; g.a_i = m; g.a_k = 1;
    g.B = Bm; g.b_k = m; g.b_j = 1;
    g.C = p->d_part; g.c_i = m; g.c_j = 1; g.c_split = m * m;
    g.alpha = 1.0; g.ksplit = ks; g.small_tiles = 1;
    RT_HIP(rt::gemm_f64(g, p->stream));
    RT_HIP(rt::reduce_affine_f64(p->d_part, m * m, ks, (int)m, out, scale, diag, bsum, p->stream));
    return RTPROJ_OK;
}

// Y = X^{-1} (eq. inversion) for the SPD Gram X (d_G) by the Newton-Schulz
// iteration Y_{k+1} = Y_k (2I - X Y_k) from Y_0 = a I, a = 1 / |X|_inf: the
// spectrum of a X lies in (0, 1], the iterates are polynomials in X, and
// I - X Y_{k+1} = (I - X Y_k)^2, so the error squares at every step once
// below one.  Rounds of steps run on the stream; after each round the host
// reads e = |I - X Y_k|_F of the last U and sizes the next round so that
// e^(2^j) <= RT_NS_DONE (the step after such a U is the final one).  A
// residual that stops squaring between RT_NS_DONE and RT_NS_FLOOR is the
// rounding floor of an ill-conditioned X and is accepted; no convergence within RT_NS_MAX_IT
// steps (singular or indefinite X, NaN) is RTPROJ_ERR_RANK.  Y alternates
// between d_L and d_Tp's first half with U in its second half; rounds have
// an even number of steps, so Y ends in d_L.  d_scal slots: 0 |X|_inf,
// 1 max X_ii, 2..3 the same for Y (filled later), 4 e.
rtproj_status gram_inverse_ns(rtproj_plan p)
{
    const int64_t m = p->m;
    hipStream_t s = p->stream;
    unsigned long long *slots = reinterpret_cast<unsigned long long *>(p->d_scal);
    RT_HIP(rt::zero_u32(reinterpret_cast<unsigned *>(slots), 8, s));
    RT_HIP(rt::ns_norms_f64(p->d_G, (int)m, slots, s));
    double *Ya = p->d_L, *Yb = p->d_Tp, *U = p->d_Tp + m * m;
    RT_HIP(rt::ns_start_f64(p->d_G, (int)m, slots, Ya, s));
    const int nbs = (int)ns_bsum_count(m);
    int it = 0, round = RT_NS_FIRST;
    double e = INFINITY, eprev = INFINITY;
    rtproj_status st;
    for (;;) {
        for (int j = 0; j < round; ++j, ++it) {
            double *Yc = (it & 1) ? Yb : Ya, *Yn = (it & 1) ? Ya : Yb;
            if ((st = ns_product(p, p->d_G, Yc, U, -1.0, 2.0, p->d_bsum)) != RTPROJ_OK) return st;
            if ((st = ns_product(p, Yc, U, Yn, 1.0, 0.0, nullptr)) != RTPROJ_OK) return st;
        }
        RT_HIP(rt::sum_blocks_sqrt_f64(p->d_bsum, nbs, p->d_scal + 4, s));
        RT_HIP(hipMemcpyAsync(&e, p->d_scal + 4, 8, hipMemcpyDeviceToHost, s));
        RT_HIP(hipStreamSynchronize(s));
        p->info.inverse_iters = it;
        p->info.inverse_resid = e;
        if (!std::isfinite(e)) return fail(RTPROJ_ERR_RANK, "Newton-Schulz inverse of the Gram diverged");
        if (e <= RT_NS_DONE || (e < RT_NS_FLOOR && e > 0.5 * eprev)) return RTPROJ_OK;
        if (it >= RT_NS_MAX_IT)
            return fail(RTPROJ_ERR_RANK, "Newton-Schulz inverse of the Gram did not converge (singular Gram)");
        int j = 6;
        if (e < 0.5) {
            j = 1;
            while (std::pow(e, std::ldexp(1.0, j)) > RT_NS_DONE) ++j;
        }
        round = (j + 1) / 2 * 2;
        eprev = e;
    }
}

// Factors of M^{-1} = Pi^T R^{-1} Y R^{-T} Pi = T'^T Y T' with T' = R^{-T} Pi
// (d_Y holds R^{-T}): T'^T and T' by form_tp into d_Tp; Y stays in d_L.  Then
// max_i Y_ii into slot 3 for the conditioning estimate.
rtproj_status form_factors_ns(rtproj_plan p)
{
    const int64_t m = p->m;
    hipStream_t s = p->stream;
    RT_HIP(rt::form_tp_f64(p->d_Y, p->d_piv, (int)m, p->d_Tp, s));
    RT_HIP(rt::ns_norms_f64(p->d_L, (int)m, reinterpret_cast<unsigned long long *>(p->d_scal) + 2, s));
    return RTPROJ_OK;
}

// First stage of the two-stage pivoted QR: the factor R0 of S^T = Q0 R0 by
// shifted Cholesky QR (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa
// 2020) and one unshifted pass: with X = S^T,
//   R1^T R1 = X^T X + s I,  s = 11 (l m + m (m+1)) 2^-53 |X|_F^2,
//   Q1 = X R1^{-1},  R2^T R2 = Q1^T Q1,  R0 = R2 R1.
// The second stage needs R0 only, never Q0: R0^T R0 = R1^T Q1^T Q1 R1 is
// X^T X up to R1^T E R1 with |E| of order u (the shift cancels, Q1 being
// formed from X and not from its Gram), so R0^{-T} X^T X R0^{-1} is the
// identity up to about u cond(Q1)^2.  The published method's third pass,
// Q2 = Q1 R2^{-1}, R3^T R3 = Q2^T Q2, R0 = R3 R2 R1, makes Q0 orthonormal,
// which only matters here when Q1 is itself nearly rank deficient (X
// numerically rank deficient below the shift): then R2 resolves the
// smallest singular values of X only to about sqrt(u) |X| and the rank test
// would miss them.  So the third pass runs when diag(R2) spans more than
// 1 / RT_CQR_THIRD (read back after the second Cholesky).  Working with
// transposes: Y = Q^T = L^{-1} S and R0^T = L1 L2 (L3), lower, which is R0
// in column-major order, the layout the second stage reads.  Sets d_err
// when a Cholesky fails (then the direct method is used).
rtproj_status r0_factor(rtproj_plan p)
{
    const int64_t m = p->m, l = p->l;
    hipStream_t s = p->stream;
    const double shift = 11.0 * ((double)l * (double)m + (double)m * (double)(m + 1)) * std::ldexp(1.0, -53);
    double *Ls[3] = {p->d_L, p->d_Y, p->d_Tp};  // free until the preconditioner's own factors
    // iterates: S, then L1^{-1} S in d_Yq, then L2^{-1} L1^{-1} S in d_Yq2
    const double *Yin[3] = {p->d_S, p->d_Yq, p->d_Yq2};
    rtproj_status st;
    // the iterates' Grams (m x m from K = l) are short in K: with autotuning
    // the tile and split are measured on the first iterate (its Gram is then
    // formed again with the choice)
    std::vector<int> rcfg = {0, 0};
    if (p->autotune) {
        const std::string key = tune_key("r0g", m, l, 0);
        if (!tune_lookup(key, rcfg)) {
            std::vector<std::vector<int>> cands;
            for (int tile : {0, 64})
                for (int sp : {p->syrk_splits / 2, p->syrk_splits, 2 * p->syrk_splits})
                    if (sp >= 1 && sp <= p->part_cap && sp <= l / 256) cands.push_back({tile, sp});
            if (cands.empty()) cands.push_back({0, 0});
            int best = 0;
            st = tune_pick(p, (int)cands.size(),
                           [&](int c) { return gram_f64_cfg(p, Yin[0], l, l, p->d_G, cands[c][0], cands[c][1]); },
                           &best, nullptr);
            if (st != RTPROJ_OK) return st;
            rcfg = cands[best];
            tune_store(key, rcfg);
        }
    }
    int passes = 2;
    for (int it = 0; it < passes; ++it) {
        RT_HIP(gram_f64_cfg(p, Yin[it], l, l, p->d_G, rcfg[0], rcfg[1]));
        if (it == 0) RT_HIP(rt::shift_diag_f64(p->d_G, m, (int)m, shift, s));
        if ((st = cholesky(p, p->d_G, Ls[it], p->d_DinvL)) != RTPROJ_OK) return st;
        if (it == 1) {
            double d2[4];
            int cerr = 0;
            RT_HIP(rt::rdiag_ends_f64(Ls[1], m, (int)m, p->d_diag, s));
            RT_HIP(hipMemcpyAsync(d2, p->d_diag, 32, hipMemcpyDeviceToHost, s));
            RT_HIP(hipMemcpyAsync(&cerr, p->d_err, 4, hipMemcpyDeviceToHost, s));
            RT_HIP(hipStreamSynchronize(s));
            if (cerr) return RTPROJ_OK;  // the caller reads d_err and factors S^T directly
            if (!(d2[2] > RT_CQR_THIRD * d2[3])) passes = 3;
        }
        p->r0_passes = passes;
        if (it + 1 < passes) {
            // next iterate L^{-1} Y: the explicit inverse (its diagonal blocks
            // come from the Cholesky), then one triangular MFMA product
            RT_HIP(run_tri_inverse(p, p->linv[it], p->d_DinvL, p->d_Linv));
            rt::GemmArgs g{};
            g.M = (int)m; g.N = (int)l; g.K = (int)m;
            g.A = p->d_Linv; g.a_i = m; g.a_k = 1; g.a_lower = 1;
            g.B = Yin[it]; g.b_k = l; g.b_j = 1;
            g.C = const_cast<double *>(Yin[it + 1]); g.c_i = l; g.c_j = 1;
            g.alpha = 1.0; g.ksplit = 1;
            RT_HIP(rt::gemm_f64(g, s));
        }
    }
    // R0^T = L1 L2 (then times L3), products of lower-triangular factors
    for (int pass = 0; pass + 1 < passes; ++pass) {
        rt::GemmArgs g{};
        g.M = (int)m; g.N = (int)m; g.K = (int)m;
        g.A = pass == 0 ? Ls[0] : p->d_G; g.a_i = m; g.a_k = 1; g.a_lower = 1;
        g.B = Ls[pass + 1]; g.b_k = m; g.b_j = 1;
        g.C = pass + 2 == passes ? p->d_R0 : p->d_G; g.c_i = m; g.c_j = 1;
        g.alpha = 1.0; g.ksplit = 1;
        RT_HIP(rt::gemm_f64(g, s));
    }
    return RTPROJ_OK;
}

bool ld_ok(int64_t ld, int64_t need) { return ld >= need && ld > 0; }

// Refinement schedule (Remark 4.3).  The contraction of a step is modelled
// as rho = c_W u_W kappa + (the Gram's rounding), with kappa the rank
// estimate of the pivoted QR; the error of x after the first solve is about
// rho.  Calibrated on measured unrefined errors (the first correction):
//   - P^{-1}A in binary64: 16 u kappa (measured 0.3 to 1.3 times that);
//     in binary32: 2 u_32 kappa (measured at most a tenth of that);
//   - a binary32 Gram accumulated on MFMA in binary32 over K terms per
//     split: u_32 K / 32 (measured u_32 K / 117 at K = 256 and 32768), times
//     cond(P^{-1}A)^2 / 9 relative to a healthy preconditioner (cond ~ 3);
//     a bfloat16 Gram adds the rounding of its inputs, 4e-3 (measured 3.9e-3);
//     a split-bfloat16 Gram (hi + lo halves, three products) 2^-8 of that.
// A step with a plain binary64 residual takes the error to max(rho e, F)
// with the floor F = RT_FLOOR_C u kappa; a compensated step to rho e (its
// own floor is near u^2 kappa^2).  Plain steps cost a tenth of a compensated
// one (MFMA GEMMs from 32 right-hand sides on), so the schedule takes plain
// steps while they still lower the error, then compensated ones until the
// error is at most RT_REFINE_GOAL; when F itself is below the goal no
// compensated step is needed.
double refine_rho_model(double kappa_est, int precision, bool w32, double cond_w, double gram_k)
{
    const double k = std::max(1.0, std::isfinite(kappa_est) ? kappa_est : 1e16);
    const double wterm = w32 ? 2.0 * std::ldexp(1.0, -23) * k : 16.0 * std::ldexp(1.0, -52) * k;
    const double c2 = std::max(1.0, cond_w * cond_w / 9.0);
    double gram = 0.0;
    if (precision != RTPROJ_PREC_FP64) gram = std::ldexp(1.0, -24) * std::max(1.0, gram_k) / 32.0 * c2;
    if (precision == RTPROJ_PREC_MIXED_BF16) gram += 4e-3 * c2;
    if (precision == RTPROJ_PREC_MIXED_BF16X3) gram += 4e-3 / 256.0 * c2;
    return std::min(0.5, wterm + gram);
}

RefinePlan refine_schedule(double kappa_est, int precision, bool w32, double cond_w, double gram_k, int mode,
                           int max_steps)
{
    return refine_schedule_rho(refine_rho_model(kappa_est, precision, w32, cond_w, gram_k), kappa_est, mode,
                               max_steps);
}

RefinePlan refine_schedule_rho(double rho, double kappa_est, int mode, int max_steps)
{
    RefinePlan r;
    const double k = std::max(1.0, std::isfinite(kappa_est) ? kappa_est : 1e16);
    r.rho = std::min(0.5, rho);
    if (mode == RTPROJ_RESID_AUTO) mode = RTPROJ_RESID_FULL;
    r.comp_r = mode == RTPROJ_RESID_FULL;
    if (max_steps >= 0) {
        // explicit count: compensated steps (plain ones in the plain mode)
        if (mode == RTPROJ_RESID_PLAIN) r.plain = max_steps;
        else r.comp = max_steps;
        r.comp_final = mode == RTPROJ_RESID_FULL && max_steps > 0;
        return r;
    }
    const double floor64 = std::min(0.5, RT_FLOOR_C * std::ldexp(1.0, -52) * k);
    double e = r.rho;
    while (r.plain < 12 && e > RT_REFINE_GOAL && e > 1.5 * floor64) {
        e = std::max(e * r.rho, floor64);
        ++r.plain;
    }
    if (mode == RTPROJ_RESID_PLAIN || e <= RT_REFINE_GOAL) {
        // at least one step, whose correction measures the contraction for
        // the convergence check
        r.plain = std::max(r.plain, 1);
        r.comp_final = false;
        return r;
    }
    while (r.comp < 12 && e > RT_REFINE_GOAL) {
        e *= r.rho;
        ++r.comp;
    }
    r.comp_final = mode == RTPROJ_RESID_FULL;
    return r;
}

// Outcome of a refinement from its per-step (|d_j|^2, |x_j|^2) pairs.  The
// first correction |d_0| / |x_0| is the error of the unrefined x, about one
// contraction factor; successive corrections of steps of the same kind
// shrink by the contraction.  The error after the last step is estimated as
// the contraction estimate times the last relative correction when the
// steps contract (estimate <= RT_NC_RATIO), else as the last relative
// correction itself.
rtproj_status refine_verdict(const double *norms, int steps, int plain, double *rho_est, double *err_est)
{
    *rho_est = 0.0;
    *err_est = 0.0;
    if (steps <= 0) return RTPROJ_OK;
    double rho = 0.0, prev = 0.0, rel = 0.0;
    for (int j = 0; j < steps; ++j) {
        const double a = std::sqrt(norms[2 * j]), x = std::sqrt(norms[2 * j + 1]);
        if (!std::isfinite(a) || !std::isfinite(x)) {
            *rho_est = *err_est = INFINITY;
            return RTPROJ_ERR_NOCONV;
        }
        rel = x > 0.0 ? a / x : (a > 0.0 ? INFINITY : 0.0);
        if (j == 0) rho = rel;
        else if ((j < plain) == (j - 1 < plain) && prev > 0.0) rho = std::max(rho, a / prev);
        prev = a;
    }
    *rho_est = rho;
    *err_est = rho <= RT_NC_RATIO ? rho * rel : rel;
    return *err_est > RT_NC_TOL ? RTPROJ_ERR_NOCONV : RTPROJ_OK;
}

// Evaluates the pending convergence check of the last projection (the
// stream must have passed its copy of the norms to h_norms).
rtproj_status resolve_refine(rtproj_plan p)
{
    if (!p->nc_pending) return (rtproj_status)p->info.refine_status;
    p->nc_pending = false;
    double rho, err;
    const rtproj_status st = refine_verdict(p->h_norms, p->nc_steps, p->nc_plain, &rho, &err);
    p->info.refine_rho_est = rho;
    p->info.refine_err_est = err;
    p->info.refine_status = st;
    p->info.refine_last_ratio = p->nc_steps > 0
        ? std::sqrt(p->h_norms[2 * p->nc_steps - 2] / std::max(p->h_norms[2 * p->nc_steps - 1], 1e-300)) : 0.0;
    return st;
}

// Conditioning estimate of the Newton-Schulz route from the norm slots
// copied to h_scal (the stream must have passed that copy): X_ii <=
// lambda_max(X) and Y_ii <= 1 / lambda_min(X).
void resolve_cond(rtproj_plan p)
{
    if (!p->cond_pending) return;
    double dx, dy;
    std::memcpy(&dx, &p->h_scal[1], 8);
    std::memcpy(&dy, &p->h_scal[3], 8);
    p->info.gram_cond_est = (dx > 0 && dy > 0 && std::isfinite(dx * dy)) ? std::sqrt(dx * dy) : INFINITY;
    p->cond_pending = false;
}

// H = M^{-1} C = (A A^T)^{-1} C for an m x k column-major block C, applied
// in factored form so that only the well-conditioned Y is explicit (Sec. 4,
// steps 2-6): Newton-Schulz route H = T'^T (Y (T' C)), Cholesky route
// H = T'^T (T' C), with d_Tp holding T'^T (row-major) followed by T'.  MFMA
// GEMMs with the K = m contraction split over blocks and reduced in a fixed
// order, or (up to RT_SKINNY_KMAX right-hand sides) one launch per product
// with K split over the waves of each block.  H must not alias C.
rtproj_status apply_minv(rtproj_plan p, const double *C, int64_t ldc, double *H, int64_t ldh, int64_t k)
{
    const int64_t m = p->m;
    if (k <= RT_SKINNY_KMAX) {
        // one launch per product: blocks of 16 x 16 output tiles, K split
        // over the waves of a block
        const bool ns = p->inv_used == RTPROJ_INV_NEWTON_SCHULZ;
        const double *Tp = p->d_Tp + m * m, *TpT = p->d_Tp;  // T' and T'^T, row-major
        if (ns) {
            RT_HIP(rt::skinny_mm_f64((int)m, (int)k, (int)m, Tp, m, C, ldc, H, ldh, p->stream));
            RT_HIP(rt::skinny_mm_f64((int)m, (int)k, (int)m, p->d_L, m, H, ldh, p->d_tmp, m, p->stream));
        } else {
            RT_HIP(rt::skinny_mm_f64((int)m, (int)k, (int)m, Tp, m, C, ldc, p->d_tmp, m, p->stream));
        }
        RT_HIP(rt::skinny_mm_f64((int)m, (int)k, (int)m, TpT, m, p->d_tmp, m, H, ldh, p->stream));
        return RTPROJ_OK;
    }
    const int splits = (int)std::max<int64_t>(1, std::min<int64_t>(p->ab_splits, (m + 63) / 64));
    if (p->inv_used == RTPROJ_INV_NEWTON_SCHULZ) {
        // H = T' C;  d_tmp = Y H;  H = T'^T d_tmp
        const double *As[3] = {p->d_Tp + m * m, p->d_L, p->d_Tp};
        const double *Bs[3] = {C, H, p->d_tmp};
        const int64_t ldbs[3] = {ldc, ldh, m};
        double *outs[3] = {H, p->d_tmp, H};
        const int64_t ldos[3] = {ldh, m, ldh};
        for (int pass = 0; pass < 3; ++pass) {
            rt::GemmArgs g{};
            g.M = (int)m; g.N = (int)k; g.K = (int)m;
            g.A = As[pass]; g.a_i = m; g.a_k = 1;
            g.B = Bs[pass]; g.b_k = 1; g.b_j = ldbs[pass];
            g.C = p->d_ph; g.c_i = 1; g.c_j = m; g.c_split = m * k;
            g.alpha = 1.0; g.ksplit = splits;
            RT_HIP(rt::gemm_f64(g, p->stream));
            // partial s is column-major m x k, i.e. row-major k x m
            RT_HIP(rt::reduce_splits_f64(p->d_ph, m * k, splits, (int)k, (int)m, m, outs[pass], ldos[pass], 0,
                                         p->stream));
        }
        return RTPROJ_OK;
    }
    for (int pass = 0; pass < 2; ++pass) {
        rt::GemmArgs g{};
        g.M = (int)m; g.N = (int)k; g.K = (int)m;
        g.A = p->d_Tp + (pass == 0 ? m * m : 0); g.a_i = m; g.a_k = 1;
        g.B = pass == 0 ? C : p->d_tmp; g.b_k = 1; g.b_j = pass == 0 ? ldc : m;
        g.C = p->d_ph; g.c_i = 1; g.c_j = m; g.c_split = m * k;
        g.alpha = 1.0; g.ksplit = splits;
        RT_HIP(rt::gemm_f64(g, p->stream));
        // partial s is column-major m x k, i.e. row-major k x m
        double *out = pass == 0 ? p->d_tmp : H;
        const int64_t ldo = pass == 0 ? m : ldh;
        RT_HIP(rt::reduce_splits_f64(p->d_ph, m * k, splits, (int)k, (int)m, m, out, ldo, 0, p->stream));
    }
    return RTPROJ_OK;
}

// d_c (m x k, column-major) = A B in plain binary64: the MFMA GEMM (split
// over n, fixed-order reduction) from RT_MFMA_KMIN right-hand sides on, where
// the product has enough columns to be a contraction; below that one pass
// over A on the vector units (bound by reading A).
hipError_t ab_plain(rtproj_plan p, const double *B, int64_t ldb, int64_t k, hipStream_t s)
{
    const int64_t m = p->m, n = p->n;
    if (k < RT_MFMA_KMIN) {
        rt::ApplyArgs a{(int)m, (int)n, (int)k, p->A, p->lda};
        hipError_t e = rt::ab_sx_f64(a, B, ldb, p->d_bpk, p->ab_sx_splits, p->d_ph, s);
        return e != hipSuccess ? e
                               : rt::ab_reduce_f64(p->d_ph, p->d_pl, (int)m, (int)k, p->ab_sx_splits, 0, p->d_c, m, s);
    }
    rt::GemmArgs g{};
    g.M = (int)m; g.N = (int)k; g.K = (int)n;
    g.A = p->A; g.a_i = p->lda; g.a_k = 1;
    g.B = B; g.b_k = 1; g.b_j = ldb;
    g.C = p->d_ph; g.c_i = 1; g.c_j = m; g.c_split = m * k;
    g.alpha = 1.0; g.ksplit = p->ab_mma_splits;
    hipError_t e = rt::gemm_f64(g, s);
    return e != hipSuccess ? e
                           : rt::reduce_splits_f64(p->d_ph, m * k, p->ab_mma_splits, (int)k, (int)m, m, p->d_c, m, 0, s);
}

// d_r (n x k) = B - A^T x_hi in plain binary64 (refinement steps above the
// binary64 floor): B copied, then the MFMA GEMM with alpha = -1, beta = 1.
hipError_t resid_plain(rtproj_plan p, const double *B, int64_t ldb, int64_t k, hipStream_t s)
{
    const int64_t m = p->m, n = p->n;
    if (k < RT_MFMA_KMIN) {
        rt::ApplyArgs a{(int)m, (int)n, (int)k, p->A, p->lda};
        return rt::atx_f64(a, p->d_xhi, p->d_xlo, m, B, ldb, p->d_r, n, nullptr, 0, nullptr, 0, 0, s);
    }
    hipError_t e = rt::copy_cols_f64(B, ldb, p->d_r, n, (int)n, (int)k, nullptr, 0, s);
    if (e != hipSuccess) return e;
    rt::GemmArgs g{};
    g.M = (int)n; g.N = (int)k; g.K = (int)m;
    g.A = p->A; g.a_i = 1; g.a_k = p->lda;
    g.B = p->d_xhi; g.b_k = 1; g.b_j = m;
    g.C = p->d_r; g.c_i = 1; g.c_j = n;
    g.alpha = -1.0; g.beta = 1.0; g.ksplit = 1;
    return rt::gemm_f64(g, s);
}

// out (m x k, column-major, ld ldo) = Am B for a row-major m x m Am and a
// column-major m x k B: one launch per product up to RT_SKINNY_KMAX
// right-hand sides, else a split-K MFMA GEMM and its fixed-order reduction.
hipError_t small_mm(rtproj_plan p, const double *Am, const double *B, int64_t ldb, double *out, int64_t ldo, int64_t k)
{
    const int64_t m = p->m;
    if (k <= RT_SKINNY_KMAX) return rt::skinny_mm_f64((int)m, (int)k, (int)m, Am, m, B, ldb, out, ldo, p->stream);
    const int splits = (int)std::max<int64_t>(1, std::min<int64_t>(p->ab_splits, (m + 63) / 64));
    rt::GemmArgs g{};
    g.M = (int)m; g.N = (int)k; g.K = (int)m;
    g.A = Am; g.a_i = m; g.a_k = 1;
    g.B = B; g.b_k = 1; g.b_j = ldb;
    g.C = p->d_ph; g.c_i = 1; g.c_j = m; g.c_split = m * k;
    g.alpha = 1.0; g.ksplit = splits;
    hipError_t e = rt::gemm_f64(g, p->stream);
    return e != hipSuccess ? e : rt::reduce_splits_f64(p->d_ph, m * k, splits, (int)k, (int)m, m, out, ldo, 0, p->stream);
}

// out (n x k, ld n) = A^T V for a column-major m x k V (ld m), plain binary64:
// one pass over A on the vector units below RT_MFMA_KMIN right-hand sides,
// an MFMA GEMM from there.
hipError_t atx_out(rtproj_plan p, const double *V, double *out, int64_t k)
{
    const int64_t m = p->m, n = p->n;
    if (k < RT_MFMA_KMIN) {
        rt::ApplyArgs a{(int)m, (int)n, (int)k, p->A, p->lda};
        return rt::atx_f64(a, V, nullptr, m, nullptr, 0, nullptr, 0, out, n, nullptr, 0, 0, p->stream);
    }
    rt::GemmArgs g{};
    g.M = (int)n; g.N = (int)k; g.K = (int)m;
    g.A = p->A; g.a_i = 1; g.a_k = p->lda;
    g.B = V; g.b_k = 1; g.b_j = m;
    g.C = out; g.c_i = 1; g.c_j = n;
    g.alpha = 1.0; g.beta = 0.0; g.ksplit = 1;
    return rt::gemm_f64(g, p->stream);
}

// H = (A A^T)^{-1} C for the iterative variant: with P^{-1} = T' = R^{-T} Pi,
// (A A^T)^{-1} = T'^T (W W^T)^{-1} T' and W W^T v = T' A A^T T'^T v; conjugate
// gradients on W W^T from u = 0 for t = T' C, krylov_iters iterations, then
// H = T'^T u.  d_r (n x k) and d_c (m x k) serve as the passes' scratch, so C
// must not be d_c's contents needed afterwards (it is read first).
rtproj_status krylov_solve(rtproj_plan p, const double *C, int64_t ldc, double *H, int64_t ldh, int64_t k)
{
    const int64_t m = p->m;
    hipStream_t s = p->stream;
    if (k > p->kry_cap) {
        if (p->d_kry) (void)hipFree(p->d_kry);
        p->d_kry = nullptr;
        p->kry_cap = 0;
        RT_HIP(dalloc(&p->d_kry, (size_t)(5 * m * k + k)));
        p->kry_cap = k;
    }
    const int64_t mk = m * p->kry_cap;
    double *u = p->d_kry, *r = u + mk, *pp = r + mk, *q = pp + mk, *w = q + mk, *gamma = w + mk;
    const double *Tt = p->d_Tp, *T = p->d_Tp + m * m;  // T'^T and T', row-major
    RT_HIP(small_mm(p, T, C, ldc, w, m, k));
    RT_HIP(rt::cg_init_f64((int)m, (int)k, w, u, r, pp, gamma, s));
    for (int it = 0; it < p->krylov_iters; ++it) {
        RT_HIP(small_mm(p, Tt, pp, m, w, m, k));        // w = P^{-T} pp
        RT_HIP(atx_out(p, w, p->d_r, k));               // A^T w
        RT_HIP(ab_plain(p, p->d_r, p->n, k, s));        // d_c = A A^T w
        RT_HIP(small_mm(p, T, p->d_c, m, q, m, k));     // q = W W^T pp
        RT_HIP(rt::cg_step_f64((int)m, (int)k, u, r, pp, q, gamma, s));
    }
    RT_HIP(small_mm(p, Tt, u, m, H, ldh, k));
    return RTPROJ_OK;
}

// The solve with the normal matrix that every projection and refinement step
// needs: the explicit factored M^{-1} of the preconditioner, or conjugate
// gradients for the iterative variant.
rtproj_status solve_normal(rtproj_plan p, const double *C, int64_t ldc, double *H, int64_t ldh, int64_t k)
{
    if (p->method_used == RTPROJ_METHOD_KRYLOV) return krylov_solve(p, C, ldc, H, ldh, k);
    return apply_minv(p, C, ldc, H, ldh, k);
}

// Final row and null projections from x_hi in plain binary64: Y = A^T x,
// Z = B - A^T x.  Below RT_MFMA_KMIN right-hand sides one pass over A on the
// vector units; from there MFMA GEMMs: Z = B - A^T x (copy, then alpha = -1,
// beta = 1) and Y = B - Z, or Y = A^T x first when Z overwrites B.
hipError_t final_plain(rtproj_plan p, const double *B, int64_t ldb, int64_t k, double *Z, int64_t ldz, double *Y,
                       int64_t ldy, hipStream_t s)
{
    const int64_t m = p->m, n = p->n;
    if (k < RT_MFMA_KMIN) {
        rt::ApplyArgs a{(int)m, (int)n, (int)k, p->A, p->lda};
        return rt::atx_f64(a, p->d_xhi, p->d_xlo, m, B, ldb, nullptr, 0, Y, ldy, Z, ldz, 0, s);
    }
    rt::GemmArgs g{};
    g.M = (int)n; g.N = (int)k; g.K = (int)m;
    g.A = p->A; g.a_i = 1; g.a_k = p->lda;
    g.B = p->d_xhi; g.b_k = 1; g.b_j = m;
    g.ksplit = 1;
    hipError_t e;
    if (Z && !(Y && Z == B)) {
        // Z = B - A^T x (Z may be B itself), then Y = B - Z (Y may be B)
        e = Z == B ? hipSuccess : rt::copy_cols_f64(B, ldb, Z, ldz, (int)n, (int)k, nullptr, 0, s);
        if (e != hipSuccess) return e;
        g.C = Z; g.c_i = 1; g.c_j = ldz;
        g.alpha = -1.0; g.beta = 1.0;
        if ((e = rt::gemm_f64(g, s)) != hipSuccess) return e;
        return Y ? rt::sub_cols_f64(B, ldb, Z, ldz, Y, ldy, (int)n, (int)k, s) : hipSuccess;
    }
    // Y = A^T x, then (Z overwriting B) Z = B - Y
    g.C = Y; g.c_i = 1; g.c_j = ldy;
    g.alpha = 1.0; g.beta = 0.0;
    if ((e = rt::gemm_f64(g, s)) != hipSuccess) return e;
    return Z ? rt::sub_cols_f64(B, ldb, Y, ldy, Z, ldz, (int)n, (int)k, s) : hipSuccess;
}

// Final projections after a compensated last step.  That step left the
// residual r = b - A^T x_prev (compensated, rounded once) in d_r and its
// correction d in d_d, with x = x_prev + d; then z = b - A^T x = r - A^T d.
// The plain binary64 product A^T d errs by about u |A^T| |d|, and |d| is the
// error of x_prev, so z keeps the accuracy of the compensated residual
// without a second compensated pass over A.  Y = B - z.  d_r ends holding z.
hipError_t final_from_residual(rtproj_plan p, const double *B, int64_t ldb, int64_t k, double *Z, int64_t ldz,
                               double *Y, int64_t ldy, hipStream_t s)
{
    const int64_t m = p->m, n = p->n;
    hipError_t e;
    if (k < RT_MFMA_KMIN) {
        rt::ApplyArgs a{(int)m, (int)n, (int)k, p->A, p->lda};
        e = rt::atx_f64(a, p->d_d, nullptr, m, p->d_r, n, nullptr, 0, nullptr, 0, p->d_r, n, 0, s);
    } else {
        rt::GemmArgs g{};
        g.M = (int)n; g.N = (int)k; g.K = (int)m;
        g.A = p->A; g.a_i = 1; g.a_k = p->lda;
        g.B = p->d_d; g.b_k = 1; g.b_j = m;
        g.C = p->d_r; g.c_i = 1; g.c_j = n;
        g.alpha = -1.0; g.beta = 1.0; g.ksplit = 1;
        e = rt::gemm_f64(g, s);
    }
    if (e != hipSuccess) return e;
    return rt::finish_cols_f64(rt::FinishGroupArgs{p->d_r, n, B, ldb, Y, ldy, Z, ldz, (int)n, (int)k}, s);
}

// Exponents of A's columns and rows for the int8-MFMA products, computed once
// per preconditioned A (at its first compensated step).
hipError_t oz_ensure_exp(rtproj_plan p, hipStream_t s)
{
    if (p->oz_exp_valid) return hipSuccess;
    hipError_t e = rt::oz_exponents_f64(p->A, p->lda, (int)p->m, (int)p->n, p->d_colexp, p->d_rowexp, s);
    if (e == hipSuccess) p->oz_exp_valid = true;
    return e;
}

// d_r = B - A^T (x_hi + x_lo), exact digit products on the int8 matrix cores
// (K = m in one block per tile).
hipError_t oz_resid(rtproj_plan p, const double *B, int64_t ldb, int64_t k, hipStream_t s)
{
    const int64_t m = p->m, n = p->n, kpad = (k + 63) / 64 * 64, mpad = (m + 63) / 64 * 64;
    int *bexp = reinterpret_cast<int *>(p->d_oz_bexp);
    int8_t *xd = reinterpret_cast<int8_t *>(p->d_oz_xdig);
    hipError_t e = oz_ensure_exp(p, s);
    if (e == hipSuccess) e = rt::oz_digits_f64(p->d_xhi, p->d_xlo, m, (int)m, (int)k, mpad, (int)kpad, bexp, xd, s);
    if (e != hipSuccess) return e;
    rt::OzArgs g{};
    g.R = (int)n; g.K = (int)m; g.k = (int)k;
    g.A = p->A; g.lda = p->lda; g.rowexp = p->d_colexp;
    g.dig = xd; g.kpad = (int)kpad; g.Kpad = mpad; g.bexp = bexp; g.kchunk = mpad;
    g.B = B; g.ldb = ldb; g.Rout = p->d_r; g.ldr = n;
    return rt::oz_mm(g, 1, 1, s);
}

// d_c = A d_r, exact digit products on the int8 matrix cores, K = n split
// over blocks, double-binary64 partials summed by the compensated reduction.
hipError_t oz_ar(rtproj_plan p, int64_t k, hipStream_t s)
{
    const int64_t m = p->m, n = p->n, kpad = (k + 63) / 64 * 64, npad = (n + 63) / 64 * 64;
    int *bexp = reinterpret_cast<int *>(p->d_oz_bexp);
    int8_t *rd = reinterpret_cast<int8_t *>(p->d_oz_rdig);
    hipError_t e = oz_ensure_exp(p, s);
    if (e == hipSuccess) e = rt::oz_digits_f64(p->d_r, nullptr, n, (int)n, (int)k, npad, (int)kpad, bexp, rd, s);
    if (e != hipSuccess) return e;
    rt::OzArgs g{};
    g.R = (int)m; g.K = (int)n; g.k = (int)k;
    g.A = p->A; g.lda = p->lda; g.rowexp = p->d_rowexp;
    g.dig = rd; g.kpad = (int)kpad; g.Kpad = npad; g.bexp = bexp;
    g.kchunk = rt::oz_kchunk(n, p->oz_splits);
    g.ph = p->d_ph; g.pl = p->d_pl;
    if ((e = rt::oz_mm(g, 0, p->oz_splits, s)) != hipSuccess) return e;
    return rt::ab_reduce_f64(p->d_ph, p->d_pl, (int)m, (int)k, p->oz_splits, 1, p->d_c, m, s);
}

rtproj_status project(rtproj_plan p, const double *B, int64_t ldb, int64_t k, double *Z, int64_t ldz, double *Y,
                      int64_t ldy, double *X, int64_t ldx)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    if (k < 0) return fail(RTPROJ_ERR_INVALID_ARG, "k < 0");
    if (k == 0) return RTPROJ_OK;
    if (!B) return fail(RTPROJ_ERR_INVALID_ARG, "B is NULL");
    if (!ld_ok(ldb, p->n)) return fail(RTPROJ_ERR_INVALID_ARG, "ldb < n");
    if (Z && !ld_ok(ldz, p->n)) return fail(RTPROJ_ERR_INVALID_ARG, "ldz < n");
    if (Y && !ld_ok(ldy, p->n)) return fail(RTPROJ_ERR_INVALID_ARG, "ldy < n");
    if (X && !ld_ok(ldx, p->m)) return fail(RTPROJ_ERR_INVALID_ARG, "ldx < m");
    if ((Z == B && ldz != ldb) || (Y == B && ldy != ldb))
        return fail(RTPROJ_ERR_INVALID_ARG, "an output aliases B with a different leading dimension");
    if (Z && Z == Y) return fail(RTPROJ_ERR_INVALID_ARG, "Z and Y are the same buffer");
    if (!p->ready) return fail(RTPROJ_ERR_STATE, "project called before a successful rtproj_precondition");
    rtproj_status st = ensure_k(p, k);
    if (st != RTPROJ_OK) return st;
    const int64_t m = p->m, n = p->n;
    hipStream_t s = p->stream;
    rt::ApplyArgs a{(int)m, (int)n, (int)k, p->A, p->lda};
    // step 1: c = A b
    {
        StageScope sc(p, 7);
        RT_HIP(ab_plain(p, B, ldb, k, s));
    }
    if (p->method_used == RTPROJ_METHOD_CLASSICAL) {
        // eq. basic_identity directly: x = Pi R^{-1} Q^T c, then A^T x and
        // b - A^T x in plain binary64
        {
            StageScope sc(p, 8);
            RT_HIP(rt::qr_solve_f64((int)m, p->d_V, p->d_tau, p->d_R, p->d_piv, p->d_c, m, p->d_xhi, m, (int)k, s));
            RT_HIP(rt::set_matrix_f64(p->d_xlo, m, (int)k, (int)m, 0, s));
        }
        if (Z || Y) {
            StageScope sc(p, 15);
            RT_HIP(final_plain(p, B, ldb, k, Z, ldz, Y, ldy, s));
        }
        if (X) RT_HIP(rt::copy_cols_f64(p->d_xhi, m, X, ldx, (int)m, (int)k, nullptr, 0, s));
        p->info.refine_steps = p->info.refine_plain = p->info.refine_comp = 0;
        p->info.resid_mode = RTPROJ_RESID_PLAIN;
        p->info.refine_last_ratio = p->info.refine_rho_est = p->info.refine_err_est = p->info.refine_rho_model = 0.0;
        p->info.refine_status = RTPROJ_OK;
        p->nc_pending = false;
        p->nc_steps = 0;
        return RTPROJ_OK;
    }
    // steps 2-6: x = Pi^T R^{-1} Y R^{-T} Pi c
    {
        StageScope sc(p, 8);
        st = solve_normal(p, p->d_c, m, p->d_xhi, m, k);
        if (st != RTPROJ_OK) return st;
        RT_HIP(rt::set_matrix_f64(p->d_xlo, m, (int)k, (int)m, 0, s));
    }
    RefinePlan rp = refine_schedule(p->info.kappa_est, p->prec_used, p->w32, p->info.gram_cond_est,
                                    (double)p->n / std::max(1, p->gram_splits_used), p->resid_mode, p->refine_steps);
    if (p->method_used == RTPROJ_METHOD_KRYLOV) {
        // a solve ends within 2 (0.6)^iters of the exact correction (CG on W W^T
        // with cond(W) <= 4), plus the rounding of its passes, about 16 u kappa
        const double rin = std::min(0.5, 2.0 * std::pow(0.6, p->krylov_iters) +
                                              16.0 * std::ldexp(1.0, -52) * std::max(1.0, p->info.kappa_est));
        rp = refine_schedule_rho(rin, p->info.kappa_est, p->resid_mode, p->refine_steps);
    }
    p->info.refine_rho_model = rp.rho;
    const int nplain = rp.plain, nsteps = std::min(rp.plain + rp.comp, RT_MAX_STEPS);
    int steps = 0;
    double ratio = 0.0;
    bool last_dd_r = false;
    // compensated products on the int8 matrix cores when the plan's setting
    // and k allow it (the workspace was sized for it by ensure_k)
    const bool oz = p->oz_ready && use_oz(p, k) && p->method_used != RTPROJ_METHOD_KRYLOV;
    int comp_used = 0;
    for (int it = 0; it < nsteps; ++it) {
        // plain binary64 residuals while the error is above their floor,
        // compensated (Dot2) ones for the last steps
        const bool comp = it >= nplain;
        const bool dd_r = comp && rp.comp_r;
        last_dd_r = dd_r;
        if (comp) comp_used = oz ? RTPROJ_COMP_INT8 : RTPROJ_COMP_DOT2;
        {
            StageScope sc(p, dd_r ? 9 : 13);
            if (dd_r && oz) RT_HIP(oz_resid(p, B, ldb, k, s));
            else if (dd_r) RT_HIP(rt::atx_f64(a, p->d_xhi, p->d_xlo, m, B, ldb, p->d_r, n, nullptr, 0, nullptr, 0, 1, s,
                                              p->d_xpk));
            else RT_HIP(resid_plain(p, B, ldb, k, s));
        }
        {
            StageScope sc(p, comp ? 10 : 14);
            if (comp && oz) {
                RT_HIP(oz_ar(p, k, s));
            } else if (comp) {
                RT_HIP(rt::ab_partial_f64(a, p->d_r, n, p->ab_splits, p->d_ph, p->d_pl, 1, s));
                RT_HIP(rt::ab_reduce_f64(p->d_ph, p->d_pl, (int)m, (int)k, p->ab_splits, 1, p->d_c, m, s));
            } else {
                RT_HIP(ab_plain(p, p->d_r, n, k, s));
            }
        }
        {
            StageScope sc(p, 8);
            st = solve_normal(p, p->d_c, m, p->d_d, m, k);
            if (st != RTPROJ_OK) return st;
            RT_HIP(rt::dd_update_f64(p->d_xhi, p->d_xlo, p->d_d, (int)m, (int)k, p->d_norms + 2 * it, s));
        }
        ++steps;
        if (p->refine_rtol > 0.0) {
            double nrm[2];
            RT_HIP(hipMemcpyAsync(nrm, p->d_norms + 2 * it, 16, hipMemcpyDeviceToHost, s));
            RT_HIP(hipStreamSynchronize(s));
            ratio = nrm[1] > 0 ? std::sqrt(nrm[0] / nrm[1]) : 0.0;
            if (ratio <= p->refine_rtol) break;
        }
    }
    // step 7: b~ = A^T x, z = b - b~; after a compensated step from that
    // step's residual (the conjugate-gradient solves reuse d_r as scratch, so
    // that method evaluates the final pass compensated in full)
    if (Z || Y) {
        const bool comp_final = steps > 0 && rp.comp_final;
        const bool from_r = comp_final && last_dd_r && p->method_used != RTPROJ_METHOD_KRYLOV;
        StageScope sc(p, comp_final && !from_r ? 11 : 15);
        if (from_r) RT_HIP(final_from_residual(p, B, ldb, k, Z, ldz, Y, ldy, s));
        else if (comp_final)
            RT_HIP(rt::atx_f64(a, p->d_xhi, p->d_xlo, m, B, ldb, nullptr, 0, Y, ldy, Z, ldz, 1, s, p->d_xpk));
        else RT_HIP(final_plain(p, B, ldb, k, Z, ldz, Y, ldy, s));
    }
    if (X) RT_HIP(rt::copy_cols_f64(p->d_xhi, m, X, ldx, (int)m, (int)k, nullptr, 0, s));
    p->info.refine_steps = steps;
    p->info.comp_method = comp_used;
    p->info.refine_plain = std::min(steps, nplain);
    p->info.refine_comp = steps - p->info.refine_plain;
    p->info.resid_mode = p->resid_mode == RTPROJ_RESID_AUTO ? RTPROJ_RESID_FULL : p->resid_mode;
    p->info.refine_last_ratio = ratio;
    // the convergence check reads the steps' norms at the next wait
    p->nc_steps = steps;
    p->nc_plain = std::min(steps, nplain);
    p->nc_pending = false;
    p->info.refine_status = RTPROJ_OK;
    p->info.refine_rho_est = p->info.refine_err_est = 0.0;
    if (steps > 0) {
        RT_HIP(hipMemcpyAsync(p->h_norms, p->d_norms, (size_t)steps * 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        p->nc_pending = true;
    }
    if (p->refine_rtol > 0.0 && steps > 0) {
        RT_HIP(hipStreamSynchronize(s));
        const rtproj_status v = resolve_refine(p);
        if (v != RTPROJ_OK)
            return fail(v, "refinement did not converge: estimated error " + std::to_string(p->info.refine_err_est));
    }
    return RTPROJ_OK;
}

}  // namespace

extern "C" {

const char *rtproj_status_string(rtproj_status s)
{
    switch (s) {
    case RTPROJ_OK: return "ok";
    case RTPROJ_ERR_INVALID_ARG: return "invalid argument";
    case RTPROJ_ERR_ALLOC: return "device allocation failed";
    case RTPROJ_ERR_DEVICE: return "device error";
    case RTPROJ_ERR_STATE: return "plan not preconditioned";
    case RTPROJ_ERR_RANK: return "matrix numerically rank deficient";
    case RTPROJ_ERR_NOCONV: return "refinement did not converge";
    case RTPROJ_ERR_UNSUPPORTED: return "unsupported size or mode";
    }
    return "unknown status";
}

const char *rtproj_last_error(void) { return g_last_error.c_str(); }

rtproj_status rtproj_plan_create(int64_t m, int64_t n, int64_t l, uint64_t seed, rtproj_plan *out)
{
    if (!out) return fail(RTPROJ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (m < 1 || n < m || l < m || l > n)
        return fail(RTPROJ_ERR_INVALID_ARG, "sizes must satisfy 1 <= m <= l <= n");
    if (n > (int64_t(1) << 30) || m > 32768)
        return fail(RTPROJ_ERR_UNSUPPORTED, "n above 2^30 or m above 32768");
    rtproj_plan p = new (std::nothrow) rtproj_plan_s();
    if (!p) return fail(RTPROJ_ERR_ALLOC, "host allocation failed");
    p->m = m; p->n = n; p->l = l; p->seed = seed;
    hipError_t e = hipGetDevice(&p->device);
    hipDeviceProp_t prop;
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, p->device);
    if (e != hipSuccess) {
        delete p;
        return fail(RTPROJ_ERR_DEVICE, std::string("hipGetDeviceProperties: ") + hipGetErrorString(e));
    }
    p->cu_count = prop.multiProcessorCount;
    p->lds_max = prop.sharedMemPerBlock;
    // set-up of the static projection workspace on this device (once per device)
    if (resolve_static_workspace(p->device) != RTPROJ_OK) {
        const std::string msg = g_last_error;
        delete p;
        return fail(RTPROJ_ERR_DEVICE, msg);
    }
    draw_tables(seed, n, l, p->tab);
    rtproj_status st = upload_tables(p);
    if (st == RTPROJ_OK) st = alloc_state(p);
    if (st != RTPROJ_OK) {
        release(p);
        delete p;
        return st == RTPROJ_ERR_DEVICE ? fail(RTPROJ_ERR_ALLOC, g_last_error) : st;
    }
    p->info.m = m; p->info.n = n; p->info.l = l; p->info.np = p->tab.np;
    p->info.precision = p->precision;
    p->info.qrcp_blocks = p->qr_blocks;
    *out = p;
    return RTPROJ_OK;
}

rtproj_status rtproj_plan_destroy(rtproj_plan p)
{
    if (!p) return RTPROJ_OK;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    else (void)hipDeviceSynchronize();
    release(p);
    delete p;
    return RTPROJ_OK;
}

rtproj_status rtproj_plan_set_stream(rtproj_plan p, void *stream)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    p->stream = (hipStream_t)stream;
    return RTPROJ_OK;
}

rtproj_status rtproj_plan_set_precision(rtproj_plan p, int precision)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    if (precision != RTPROJ_PREC_FP64 && precision != RTPROJ_PREC_MIXED_FP32 && precision != RTPROJ_PREC_MIXED_BF16 &&
        precision != RTPROJ_PREC_MIXED_BF16X3)
        return fail(RTPROJ_ERR_INVALID_ARG, "unknown precision");
    p->precision = precision;
    return RTPROJ_OK;
}

rtproj_status rtproj_plan_set_w_bits(rtproj_plan p, int bits)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    if (bits != 0 && bits != 32 && bits != 64) return fail(RTPROJ_ERR_INVALID_ARG, "bits must be 0, 32 or 64");
    p->w_bits_req = bits;
    return RTPROJ_OK;
}

rtproj_status rtproj_plan_set_method(rtproj_plan p, int method)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    if (method != RTPROJ_METHOD_RANDOMIZED && method != RTPROJ_METHOD_CLASSICAL && method != RTPROJ_METHOD_KRYLOV)
        return fail(RTPROJ_ERR_INVALID_ARG, "unknown method");
    if (method == RTPROJ_METHOD_CLASSICAL && p->m > 4096)
        return fail(RTPROJ_ERR_UNSUPPORTED, "classical scheme: m above 4096");
    p->method = method;
    return RTPROJ_OK;
}

rtproj_status rtproj_plan_set_krylov(rtproj_plan p, int iters)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    if (iters < 1 || iters > 500) return fail(RTPROJ_ERR_INVALID_ARG, "iterations outside [1, 500]");
    p->krylov_iters = iters;
    return RTPROJ_OK;
}

rtproj_status rtproj_plan_set_sketch_matrix(rtproj_plan p, const double *G, int64_t ldg)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    if (G && ldg < p->l) return fail(RTPROJ_ERR_INVALID_ARG, "ldg < l");
    p->Gmat = G;
    p->ldg = G ? ldg : 0;
    return RTPROJ_OK;
}

rtproj_status rtproj_plan_set_residual(rtproj_plan p, int mode)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    if (mode < RTPROJ_RESID_AUTO || mode > RTPROJ_RESID_FULL) return fail(RTPROJ_ERR_INVALID_ARG, "unknown residual mode");
    p->resid_mode = mode;
    return RTPROJ_OK;
}

rtproj_status rtproj_plan_set_compensation(rtproj_plan p, int method)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    if (method < RTPROJ_COMP_AUTO || method > RTPROJ_COMP_INT8)
        return fail(RTPROJ_ERR_INVALID_ARG, "unknown compensation method");
    p->comp_method = method;
    return RTPROJ_OK;
}

rtproj_status rtproj_plan_set_qr(rtproj_plan p, int mode)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    if (mode < RTPROJ_QR_AUTO || mode > RTPROJ_QR_TWO_STAGE_WG) return fail(RTPROJ_ERR_INVALID_ARG, "unknown QR mode");
    if (mode == RTPROJ_QR_DIRECT && p->qr_blocks <= 0 && p->qr_reg_l <= 0)
        return fail(RTPROJ_ERR_UNSUPPORTED, "direct pivoted QR: the l x m sketch does not fit the cooperative kernel");
    if (mode == RTPROJ_QR_TWO_STAGE && p->qr_blocks0 <= 0 && p->qr_reg_m <= 0)
        return fail(RTPROJ_ERR_UNSUPPORTED, "two-stage pivoted QR: R0 does not fit the cooperative kernel");
    if (mode == RTPROJ_QR_TWO_STAGE_WG && (p->m > rt::qrcp_wg_max_rows() || p->m > rt::qrcp_wg_max_cols()))
        return fail(RTPROJ_ERR_UNSUPPORTED, "single-workgroup pivoted QR: m too large");
    p->qr_mode = mode;
    return RTPROJ_OK;
}

rtproj_status rtproj_plan_set_inverse(rtproj_plan p, int method)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    if (method < RTPROJ_INV_AUTO || method > RTPROJ_INV_CHOLESKY)
        return fail(RTPROJ_ERR_INVALID_ARG, "unknown inverse method");
    p->inv_method = method;
    return RTPROJ_OK;
}

rtproj_status rtproj_plan_set_refinement(rtproj_plan p, int max_steps, double rtol)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    if (max_steps < -1 || max_steps > 64 || !(rtol >= 0.0))
        return fail(RTPROJ_ERR_INVALID_ARG, "max_steps must be in [-1, 64] and rtol >= 0");
    p->refine_steps = max_steps;
    p->refine_rtol = rtol;
    return RTPROJ_OK;
}

}  // extern "C"

namespace {

// Cooperative pivoted QR of the rows x m matrix whose columns are the rows
// of M (ld ldm): the register-resident form when it applies (reg_blocks >
// 0), else the LDS / global-memory form with lds_blocks blocks.
hipError_t qrcp_any(rtproj_plan p, const double *M, int64_t ldm, int rows, rt::QrcpWork w, int reg_blocks,
                    int lds_blocks)
{
    const int m = (int)p->m;
    if (reg_blocks > 0) {
        w.cols = nullptr;
        p->info.qrcp_blocks = reg_blocks;
        return rt::qrcp_reg_f64(M, ldm, rows, m, p->d_R, p->d_piv, w, p->cu_count, p->stream);
    }
    int gc = 0;
    rt::qrcp_max_blocks(rows, m, p->cu_count, p->lds_max, &gc);
    w.cols = gc ? p->d_qrcols : nullptr;
    p->info.qrcp_blocks = lds_blocks;
    return rt::qrcp_f64(M, ldm, rows, m, p->d_R, p->d_piv, w, lds_blocks, p->lds_max, p->stream);
}

// The pivoted-QR method used when the caller leaves it to the plan.
int auto_qr_mode(rtproj_plan p)
{
    // the register-resident form on S^T when it applies; otherwise (sketches
    // taller than 8192 rows, or too many columns for one block per compute
    // unit) on the m x m factor R0 of the two-stage form
    if (p->qr_reg_l > 0) return RTPROJ_QR_DIRECT;
    if (p->qr_reg_m > 0) return RTPROJ_QR_TWO_STAGE;
    return p->qr_blocks > 0 ? RTPROJ_QR_DIRECT : RTPROJ_QR_TWO_STAGE;
}

// The classical scheme's set-up (the s_pre of Sec. 5): G = A A^T on MFMA
// (both triangles), then the Householder pivoted QR G Pi = Q R with the
// reflectors kept in d_V / d_tau.  The rank estimate is |R_11 / R_mm|
// (about cond(A)^2); only a zero or non-finite pivot is an error.
rtproj_status precondition_classical(rtproj_plan p, const double *A, int64_t lda)
{
    const int64_t m = p->m, n = p->n;
    hipStream_t s = p->stream;
    if (!p->d_V) RT_HIP(dalloc(&p->d_V, (size_t)m * m));
    if (!p->d_tau) RT_HIP(dalloc(&p->d_tau, (size_t)m));
    {
        StageScope sc(p, 4);
        rtproj_status st = gram_f64(p, A, lda, n, p->d_G);
        if (st != RTPROJ_OK) return st;
    }
    double diag[4];
    unsigned sync[4];
    {
        StageScope sc(p, 1);
        RT_HIP(rt::set_matrix_f64(p->d_R, m, (int)m, (int)m, 0, s));
        RT_HIP(rt::iota_f64piv(p->d_piv, (int)m, s));
        rt::QrcpWork w;
        w.counter = p->d_sync;
        w.flag = p->d_sync + 1;
        w.err = reinterpret_cast<int *>(p->d_sync + 2);
        w.slots = p->d_slots;
        w.vbuf = p->d_vbuf;
        w.V = p->d_V;
        w.tau = p->d_tau;
        if (p->qr_reg_m <= 0 && p->qr_blocks0 <= 0)
            return fail(RTPROJ_ERR_UNSUPPORTED, "classical scheme: the m x m QR does not fit the cooperative kernel");
        RT_HIP(qrcp_any(p, p->d_G, m, (int)m, w, p->qr_reg_m, p->qr_blocks0));
    }
    RT_HIP(rt::rdiag_ends_f64(p->d_R, m, (int)m, p->d_diag, s));
    RT_HIP(hipMemcpyAsync(diag, p->d_diag, 32, hipMemcpyDeviceToHost, s));
    RT_HIP(hipMemcpyAsync(sync, p->d_sync, 16, hipMemcpyDeviceToHost, s));
    RT_HIP(hipStreamSynchronize(s));
    if (sync[2] == 2) return fail(RTPROJ_ERR_RANK, "pivoted QR of A A^T: no finite pivot (A contains NaN or Inf)");
    if (sync[2] != 0) return fail(RTPROJ_ERR_DEVICE, "pivoted QR: cooperative barrier timed out");
    p->info.rdiag_min = diag[2];
    p->info.kappa_est = diag[2] > 0 ? diag[3] / diag[2] : INFINITY;
    if (!(diag[2] > 0.0) || !std::isfinite(diag[3]))
        return fail(RTPROJ_ERR_RANK, "pivoted QR of A A^T: zero pivot (rank deficient A)");
    p->info.qr_mode = RTPROJ_QR_DIRECT;
    p->info.sketch_bits = p->info.w_bits = 0;
    p->info.gram_bits = 64;
    p->info.inverse = 0;
    p->info.inverse_iters = 0;
    p->info.inverse_resid = 0.0;
    p->info.gram_cond_est = 0.0;
    p->cond_pending = false;
    return RTPROJ_OK;
}

// One pass of the preconditioner; sketch64 forces the binary64 sketch.
rtproj_status precondition_impl(rtproj_plan p, const double *A, int64_t lda, bool sketch64)
{
    p->oz_exp_valid = false;  // the int8-MFMA exponents describe the previous A
    const int64_t m = p->m, n = p->n, l = p->l;
    hipStream_t s = p->stream;
    // 1. sketch
    if (p->Gmat) {
        // S = A G with the caller's G, binary64 MFMA, K = n split over blocks
        StageScope sc(p, 0);
        const int64_t tiles = ((m + 63) / 64) * ((l + 63) / 64);
        const int splits = (int)std::max<int64_t>(1, std::min<int64_t>({32, n / 1024, (4 * p->cu_count + tiles - 1) / tiles}));
        if ((int64_t)splits * m * l > p->gpart_cap) {
            if (p->d_gpart) (void)hipFree(p->d_gpart);
            p->d_gpart = nullptr;
            p->gpart_cap = 0;
            RT_HIP(dalloc(&p->d_gpart, (size_t)splits * m * l));
            p->gpart_cap = (int64_t)splits * m * l;
        }
        rt::GemmArgs g{};
        g.M = (int)m; g.N = (int)l; g.K = (int)n;
        g.A = A; g.a_i = lda; g.a_k = 1;
        g.B = p->Gmat; g.b_k = p->ldg; g.b_j = 1;
        g.C = p->d_gpart; g.c_i = l; g.c_j = 1; g.c_split = m * l;
        g.alpha = 1.0; g.ksplit = splits;
        RT_HIP(rt::gemm_f64(g, s));
        RT_HIP(rt::reduce_splits_f64(p->d_gpart, m * l, splits, (int)m, (int)l, l, p->d_S, l, 0, s));
    } else {
        StageScope sc(p, 0);
        if (p->precision == RTPROJ_PREC_FP64 || sketch64)
            RT_HIP(rt::sketch_f64(p->sketch_tables(), A, lda, m, p->d_S, l, p->d_zbuf, p->rows_chunk, s));
        else  // complex binary32 fits twice the rows in the buffer sized for binary64 (fewer, fuller launches)
            RT_HIP(rt::sketch_f32(p->sketch_tables(), A, lda, m, p->d_S, l, p->d_zbuf, 2 * p->rows_chunk, s));
    }
    // 2. pivoted QR of S^T, directly or on the small factor R0 of S^T
    double diag[4];
    unsigned sync[4];
    int mode = p->qr_mode;
    if (mode == RTPROJ_QR_AUTO) mode = auto_qr_mode(p);
    {
        RT_HIP(rt::zero_u32(reinterpret_cast<unsigned *>(p->d_err), 1, s));
        if (mode != RTPROJ_QR_DIRECT) {
            StageScope sc(p, 12);
            rtproj_status st0 = r0_factor(p);
            if (st0 != RTPROJ_OK) return st0;
        }
        RT_HIP(rt::set_matrix_f64(p->d_R, m, (int)m, (int)m, 0, s));
        RT_HIP(rt::iota_f64piv(p->d_piv, (int)m, s));  // valid pivots even if the QR stops early
        rt::QrcpWork w;
        w.counter = p->d_sync;
        w.flag = p->d_sync + 1;
        w.err = reinterpret_cast<int *>(p->d_sync + 2);
        w.slots = p->d_slots;
        w.vbuf = p->d_vbuf;
        {
            StageScope sc(p, 1);
            if (mode == RTPROJ_QR_DIRECT) {
                RT_HIP(qrcp_any(p, p->d_S, l, (int)l, w, p->qr_reg_l, p->qr_blocks));
            } else if (mode == RTPROJ_QR_TWO_STAGE) {
                RT_HIP(qrcp_any(p, p->d_R0, m, (int)m, w, p->qr_reg_m, p->qr_blocks0));
            } else {
                RT_HIP(rt::zero_u32(p->d_sync, 4, s));
                RT_HIP(rt::qrcp_wg_f64(p->d_wgargs, 1, s));
            }
        }
        RT_HIP(rt::rdiag_ends_f64(p->d_R, m, (int)m, p->d_diag, s));
        RT_HIP(hipMemcpyAsync(diag, p->d_diag, 32, hipMemcpyDeviceToHost, s));
        RT_HIP(hipMemcpyAsync(sync, p->d_sync, 16, hipMemcpyDeviceToHost, s));
        int r0err = 0;
        RT_HIP(hipMemcpyAsync(&r0err, p->d_err, 4, hipMemcpyDeviceToHost, s));
        RT_HIP(hipStreamSynchronize(s));
        if (r0err == 3) return fail(RTPROJ_ERR_DEVICE, "cooperative Cholesky: a wait timed out");
        if (r0err && mode != RTPROJ_QR_DIRECT) {
            // the Cholesky QR broke down (S^T too ill-conditioned even for the
            // shifted first pass): factor S^T directly
            if (p->qr_blocks <= 0 && p->qr_reg_l <= 0)
                return fail(RTPROJ_ERR_RANK, "two-stage pivoted QR: Cholesky QR of the sketch failed");
            mode = RTPROJ_QR_DIRECT;
            RT_HIP(rt::set_matrix_f64(p->d_R, m, (int)m, (int)m, 0, s));
            RT_HIP(rt::iota_f64piv(p->d_piv, (int)m, s));
            {
                StageScope sc(p, 1);
                RT_HIP(qrcp_any(p, p->d_S, l, (int)l, w, p->qr_reg_l, p->qr_blocks));
            }
            RT_HIP(rt::rdiag_ends_f64(p->d_R, m, (int)m, p->d_diag, s));
            RT_HIP(hipMemcpyAsync(diag, p->d_diag, 32, hipMemcpyDeviceToHost, s));
            RT_HIP(hipMemcpyAsync(sync, p->d_sync, 16, hipMemcpyDeviceToHost, s));
        }
    }
    p->info.qr_mode = mode;
    RT_HIP(hipStreamSynchronize(s));
    if (sync[2] == 2) return fail(RTPROJ_ERR_RANK, "pivoted QR: no finite pivot (A contains NaN or Inf)");
    if (sync[2] != 0) return fail(RTPROJ_ERR_DEVICE, "pivoted QR: cooperative barrier timed out");
    p->info.rdiag_min = diag[2];
    p->info.kappa_est = diag[2] > 0 ? diag[3] / diag[2] : INFINITY;
    const bool lp = p->precision != RTPROJ_PREC_FP64;
    // a binary32 sketch whose rank estimate shows it too coarse for this A
    // (2^-24 kappa_est above RT_SKETCH32_MAX, or numerically rank deficient)
    // is redone in binary64 before anything is built on it
    if (lp && !sketch64 && !p->Gmat &&
        (!(std::ldexp(p->info.kappa_est, -24) <= RT_SKETCH32_MAX) ||
         !(diag[2] > (double)m * std::ldexp(1.0, -52) * diag[3]))) {
        p->resketch = true;
        return RTPROJ_OK;
    }
    if (!(diag[2] > (double)m * std::ldexp(1.0, -52) * diag[3]))
        return fail(RTPROJ_ERR_RANK, "pivoted QR of the sketch: |R_mm| <= m eps |R_11| (rank deficient A)");
    // 3. R^{-T} (lower): inverted 64 x 64 diagonal blocks, then recursive
    //    doubling over block pairs, X21 = -X22 L21 X11 (two grouped MFMA
    //    products per level, log2(m / 64) levels)
    rtproj_status st = RTPROJ_OK;
    {
        StageScope sc(p, 2);
        RT_HIP(rt::tri_diag_inv_f64(p->d_R, 1, m, (int)m, NB, p->d_DinvR, s));
        RT_HIP(run_tri_inverse(p, p->rinv, p->d_DinvR, p->d_Y));
    }
    if (p->method_used == RTPROJ_METHOD_KRYLOV) {
        // the iterative variant applies P^{-1} = R^{-T} Pi and its transpose
        // only: T' = R^{-T} Pi and T'^T into d_Tp; no W, Gram or inverse
        StageScope sc(p, 6);
        RT_HIP(rt::form_tp_f64(p->d_Y, p->d_piv, (int)m, p->d_Tp, s));
        p->w32 = false;
        p->inv_used = 0;
        p->info.inverse = 0;
        p->info.inverse_iters = 0;
        p->info.inverse_resid = 0.0;
        p->info.w_bits = p->info.gram_bits = 0;
        p->info.sketch_bits = (p->precision != RTPROJ_PREC_FP64 && !sketch64 && !p->Gmat) ? 32 : 64;
        p->info.gram_cond_est = 0.0;
        p->cond_pending = false;
        return RTPROJ_OK;
    }
    // 4. W = R^{-T} (Pi A), binary32 when the rank estimate allows it (or
    //    when forced by rtproj_plan_set_w_bits)
    p->w32 = lp && (p->w_bits_req == 32 || (p->w_bits_req == 0 && p->info.kappa_est <= RT_W32_KAPPA_MAX));
    // configurations of the two large contractions: built-in choices, or the
    // autotuner's (each candidate timed once per new shape, see rt_tune.hip)
    auto run_w = [&](int tile, int order, int tile_n) -> hipError_t {
        if (p->w32) {
            rt::GemmMxArgs g{};
            g.M = (int)m; g.N = (int)n; g.K = (int)m;
            g.A = p->d_Y; g.a_dbl = 1; g.a_i = m; g.a_k = 1; g.a_lower = 1;
            g.B = A; g.b_dbl = 1; g.b_k = lda; g.b_j = 1; g.b_gather = p->d_piv;
            g.C = p->d_W; g.c_dbl = 0; g.c_i = p->ldw; g.c_j = 1;
            g.alpha = 1.f; g.ksplit = 1; g.tile = tile;
            return rt::gemm_mx(g, rt::MX_F32, s);
        }
        // binary64 products; with a binary32 or bfloat16 Gram, which rounds
        // its inputs to binary32 first, stored as binary32 already
        rt::GemmArgs g{};
        g.M = (int)m; g.N = (int)n; g.K = (int)m;
        g.A = p->d_Y; g.a_i = m; g.a_k = 1; g.a_lower = 1;
        g.B = A; g.b_k = lda; g.b_j = 1; g.b_gather = p->d_piv;
        g.C = p->d_W; g.c_i = p->ldw; g.c_j = 1; g.c_f32 = lp ? 1 : 0;
        g.alpha = 1.0; g.ksplit = 1; g.tile = tile; g.tile_n = tile_n; g.order = order;
        return rt::gemm_f64(g, s);
    };
    const bool bf = p->precision == RTPROJ_PREC_MIXED_BF16;
    // the split-bfloat16 Gram needs W's rows 16-byte aligned (n % 4 == 0);
    // otherwise that precision takes the binary32 Gram
    bool x3 = false;
    auto run_gram = [&](int splits, int tile) -> hipError_t {
        hipError_t e;
        if (!lp) {
            rt::GemmArgs g{};
            g.M = (int)m; g.N = (int)m; g.K = (int)n;
            g.A = p->d_W; g.a_i = p->ldw; g.a_k = 1;
            g.B = p->d_W; g.b_k = 1; g.b_j = p->ldw;
            g.C = p->d_part; g.c_i = m; g.c_j = 1; g.c_split = m * m;
            g.alpha = 1.0; g.c_lower = 1; g.ksplit = splits; g.tile = tile;
            if ((e = rt::gemm_f64(g, s)) != hipSuccess) return e;
            return rt::reduce_splits_f64(p->d_part, m * m, splits > 1 ? splits : 1, (int)m, (int)m, m, p->d_G, m, 1, s);
        }
        const int wd = 0;  // W is binary32 in the mixed forms (either product)
        if (bf && (e = rt::row_pow2_scale(p->d_W, wd, p->ldw, (int)m, (int)n, p->d_rowscale, s)) != hipSuccess) return e;
        rt::GemmMxArgs g{};
        g.M = (int)m; g.N = (int)m; g.K = (int)n;
        g.A = p->d_W; g.a_dbl = wd; g.a_i = p->ldw; g.a_k = 1; g.a_scale = bf ? p->d_rowscale : nullptr;
        g.B = p->d_W; g.b_dbl = wd; g.b_k = 1; g.b_j = p->ldw; g.b_scale = bf ? p->d_rowscale : nullptr;
        g.C = p->d_part; g.c_dbl = 0; g.c_i = m; g.c_j = 1; g.c_split = m * m;
        g.alpha = 1.f; g.c_lower = 1; g.ksplit = splits; g.tile = tile;
        x3 = p->precision == RTPROJ_PREC_MIXED_BF16X3 && rt::gemm_mx_bf16x3_ok(g);
        if ((e = rt::gemm_mx(g, bf ? rt::MX_BF16 : (x3 ? rt::MX_BF16X3 : rt::MX_F32), s)) != hipSuccess) return e;
        return rt::reduce_f32_splits(reinterpret_cast<const float *>(p->d_part), m * m, splits > 1 ? splits : 1, (int)m,
                                     (int)m, m, bf ? p->d_rowscale : nullptr, bf ? p->d_rowscale : nullptr, p->d_G, m,
                                     1, s);
    };
    std::vector<int> wcfg = {0, 0, 0}, gcfg = {p->wgram_splits, 0};
    if (p->autotune) {
        const std::string wkey = tune_key(p->w32 ? "w32" : "w64", m, n, lda == n ? 0 : 1);
        if (!tune_lookup(wkey, wcfg)) {
            // (tile, order, tile_n): square and rectangular binary64 tiles in
            // both tile orders
            std::vector<std::vector<int>> cands =
                p->w32 ? std::vector<std::vector<int>>{{64, 0, 0}, {128, 0, 0}}
                       : std::vector<std::vector<int>>{{64, 1, 0},  {64, 2, 0},  {128, 1, 0},  {128, 2, 0},
                                                       {64, 1, 128}, {64, 2, 128}, {128, 1, 64}, {128, 2, 64}};
            int best = 0;
            st = tune_pick(p, (int)cands.size(), [&](int c) { return run_w(cands[c][0], cands[c][1], cands[c][2]); },
                           &best, nullptr);
            if (st != RTPROJ_OK) return st;
            wcfg = cands[best];
            tune_store(wkey, wcfg);
        }
        const bool x3req = p->precision == RTPROJ_PREC_MIXED_BF16X3;
        const std::string gkey = tune_key(!lp ? "g64" : (bf ? "g16" : (x3req ? "g3" : "g32")), m, n, 0);
        if (!tune_lookup(gkey, gcfg)) {
            // run W once with the chosen configuration so the Gram reads it
            RT_HIP(run_w(wcfg[0], wcfg[1], wcfg.size() > 2 ? wcfg[2] : 0));
            const int smax = (int)std::max<int64_t>(1, std::min<int64_t>(64, n / 256));
            // binary32 partials take half the room of binary64 ones
            const int cap = std::min(smax, lp ? 2 * p->part_cap : p->part_cap);
            std::vector<std::vector<int>> cands;
            for (int sp : {p->syrk_splits / 2, p->syrk_splits, 2 * p->syrk_splits, 4 * p->syrk_splits,
                           p->wgram_splits, 2 * p->wgram_splits}) {
                if (sp < 1 || sp > cap) continue;
                bool seen = false;
                for (const auto &c : cands) seen = seen || c[0] == sp;
                if (seen) continue;
                cands.push_back({sp, 0});
                if (!lp) cands.push_back({sp, 64});
                if (bf || x3req) cands.push_back({sp, 128});  // 128 x 128 instead of 256 x 128 tiles
            }
            if (cands.empty()) cands.push_back({p->wgram_splits, 0});
            int best = 0;
            st = tune_pick(p, (int)cands.size(), [&](int c) { return run_gram(cands[c][0], cands[c][1]); }, &best,
                           nullptr);
            if (st != RTPROJ_OK) return st;
            gcfg = cands[best];
            tune_store(gkey, gcfg);
        }
        gcfg[0] = std::min(gcfg[0], lp ? 2 * p->part_cap : p->part_cap);
    }
    {
        StageScope sc(p, 3);
        RT_HIP(run_w(wcfg[0], wcfg[1], wcfg.size() > 2 ? wcfg[2] : 0));
    }
    // 5. Gram X = W W^T (lower tiles, split over n, fixed-order reduction)
    {
        StageScope sc(p, 4);
        RT_HIP(run_gram(gcfg[0], gcfg[1]));
        p->gram_splits_used = std::max(1, gcfg[0]);
    }
    p->info.sketch_bits = (lp && !sketch64 && !p->Gmat) ? 32 : 64;
    p->info.w_bits = p->w32 ? 32 : 64;
    p->info.gram_bits = !lp ? 64 : (bf ? 16 : (x3 ? 17 : 32));
    // 6-7. Y = X^{-1} (eq. inversion) and the form of M^{-1} the projections apply
    p->inv_used = p->inv_method != RTPROJ_INV_AUTO ? p->inv_method
                  : (m <= RT_NS_MAX_M ? RTPROJ_INV_NEWTON_SCHULZ : RTPROJ_INV_CHOLESKY);
    p->info.inverse = p->inv_used;
    p->info.inverse_iters = 0;
    p->info.inverse_resid = 0.0;
    p->cond_pending = false;
    if (p->inv_used == RTPROJ_INV_NEWTON_SCHULZ) {
        {
            StageScope sc(p, 5);
            st = gram_inverse_ns(p);
        }
        if (st != RTPROJ_OK) return st;
        {
            StageScope sc(p, 6);
            st = form_factors_ns(p);
        }
        if (st != RTPROJ_OK) return st;
        RT_HIP(hipMemcpyAsync(p->h_scal, p->d_scal, 32, hipMemcpyDeviceToHost, s));
        p->cond_pending = true;
        // the mixed forms decide on a re-sketch from the estimate now; at
        // binary64 nothing before rtproj_plan_info needs it
        if (p->precision != RTPROJ_PREC_FP64) {
            RT_HIP(hipStreamSynchronize(s));
            resolve_cond(p);
        }
        return RTPROJ_OK;
    }
    // 6. Cholesky X = L L^T
    {
        StageScope sc(p, 5);
        RT_HIP(rt::zero_u32(reinterpret_cast<unsigned *>(p->d_err), 1, s));
        st = cholesky(p, p->d_G, p->d_L, p->d_DinvL);
    }
    if (st != RTPROJ_OK) return st;
    // 7. T = L^{-1} R^{-T}, T' = T Pi: the explicit L^{-1} (into d_Linv, its
    //    diagonal blocks from the Cholesky, d_G as scratch), then the product
    //    of the two lower-triangular factors into d_G
    {
        StageScope sc(p, 6);
        RT_HIP(run_tri_inverse(p, p->linv[0], p->d_DinvL, p->d_Linv));
        rt::GemmArgs g{};
        g.M = (int)m; g.N = (int)m; g.K = (int)m;
        g.A = p->d_Linv; g.a_i = m; g.a_k = 1; g.a_lower = 1;
        g.B = p->d_Y; g.b_k = m; g.b_j = 1;
        g.C = p->d_G; g.c_i = m; g.c_j = 1;
        g.alpha = 1.0; g.ksplit = 1;
        RT_HIP(rt::gemm_f64(g, s));
        RT_HIP(rt::form_tp_f64(p->d_G, p->d_piv, (int)m, p->d_Tp, s));
    }
    if (st != RTPROJ_OK) return st;
    int cerr = 0;
    double ldiag[4];
    RT_HIP(rt::rdiag_ends_f64(p->d_L, m, (int)m, p->d_diag, s));
    RT_HIP(hipMemcpyAsync(ldiag, p->d_diag, 32, hipMemcpyDeviceToHost, s));
    RT_HIP(hipMemcpyAsync(&cerr, p->d_err, 4, hipMemcpyDeviceToHost, s));
    RT_HIP(hipStreamSynchronize(s));
    if (cerr == 3) return fail(RTPROJ_ERR_DEVICE, "cooperative Cholesky: a wait timed out");
    if (cerr) return fail(RTPROJ_ERR_RANK, "Cholesky of the preconditioned Gram broke down");
    // max/min of diag(L) bounds cond(P^{-1}A) from below (about 3 for a
    // healthy sketch with l = 4m, Observation 3.2)
    p->info.gram_cond_est = ldiag[2] > 0 ? ldiag[3] / ldiag[2] : INFINITY;
    return RTPROJ_OK;
}

}  // namespace

extern "C" {

rtproj_status rtproj_precondition(rtproj_plan p, const double *A, int64_t lda)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    if (!A) return fail(RTPROJ_ERR_INVALID_ARG, "A is NULL");
    if (lda < p->n) return fail(RTPROJ_ERR_INVALID_ARG, "lda < n");
    p->ready = false;
    p->A = A;
    p->lda = lda;
    p->info.sketch_escalated = 0;
    p->resketch = false;
    p->prec_used = p->precision;
    p->info.precision = p->precision;
    p->method_used = p->method;
    p->info.method = p->method;
    if (p->method == RTPROJ_METHOD_CLASSICAL) {
        p->prec_used = p->info.precision = RTPROJ_PREC_FP64;
        const rtproj_status sc = precondition_classical(p, A, lda);
        if (sc != RTPROJ_OK) return sc;
        p->ready = true;
        return RTPROJ_OK;
    }
    rtproj_status st = precondition_impl(p, A, lda, false);
    // A binary32 sketch perturbs G by about 2^-24 kappa(A) relative to the
    // small singular directions; when the rank estimate shows that (right
    // after the pivoted QR), or the Gram shows a poorly conditioned P^{-1}A,
    // sketch again in binary64 (the identity holds for any G, only the
    // conditioning matters, Lemma 2.4).
    if (st == RTPROJ_OK && p->precision != RTPROJ_PREC_FP64 && !p->Gmat &&
        (p->resketch || p->info.gram_cond_est > RT_COND_ESCALATE)) {
        p->info.sketch_escalated = p->resketch ? 1 : 2;
        p->resketch = false;
        st = precondition_impl(p, A, lda, true);
    }
    if (st != RTPROJ_OK) return st;
    p->ready = true;
    return RTPROJ_OK;
}

rtproj_status rtproj_project_null(rtproj_plan p, const double *B, int64_t ldb, int64_t k, double *Z, int64_t ldz)
{
    if (k > 0 && !Z) return fail(RTPROJ_ERR_INVALID_ARG, "Z is NULL");
    return project(p, B, ldb, k, Z, ldz, nullptr, 0, nullptr, 0);
}

rtproj_status rtproj_project_row(rtproj_plan p, const double *B, int64_t ldb, int64_t k, double *Y, int64_t ldy)
{
    if (k > 0 && !Y) return fail(RTPROJ_ERR_INVALID_ARG, "Y is NULL");
    return project(p, B, ldb, k, nullptr, 0, Y, ldy, nullptr, 0);
}

rtproj_status rtproj_lstsq(rtproj_plan p, const double *B, int64_t ldb, int64_t k, double *X, int64_t ldx)
{
    if (k > 0 && !X) return fail(RTPROJ_ERR_INVALID_ARG, "X is NULL");
    return project(p, B, ldb, k, nullptr, 0, nullptr, 0, X, ldx);
}

rtproj_status rtproj_project_all(rtproj_plan p, const double *B, int64_t ldb, int64_t k, double *Z, int64_t ldz,
                                 double *Y, int64_t ldy, double *X, int64_t ldx)
{
    return project(p, B, ldb, k, Z, ldz, Y, ldy, X, ldx);
}

rtproj_status rtproj_plan_set_timing(rtproj_plan p, int enable)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    RT_HIP(hipStreamSynchronize(p->stream));
    collect_timing(p);
    p->timing = enable != 0;
    if (enable) {
        for (int i = 0; i < 16; ++i) { p->info.t_stage_ms[i] = 0.0; p->info.stage_calls[i] = 0; }
    }
    return RTPROJ_OK;
}

rtproj_status rtproj_plan_info(rtproj_plan p, rtproj_info *out)
{
    if (!p || !out) return fail(RTPROJ_ERR_INVALID_ARG, "null argument");
    RT_HIP(hipStreamSynchronize(p->stream));
    resolve_cond(p);
    resolve_refine(p);
    collect_timing(p);
    *out = p->info;
    return RTPROJ_OK;
}

rtproj_status rtproj_plan_status(rtproj_plan p)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    RT_HIP(hipStreamSynchronize(p->stream));
    const rtproj_status st = resolve_refine(p);
    if (st != RTPROJ_OK)
        return fail(st, "refinement did not converge: estimated relative error of x " +
                            std::to_string(p->info.refine_err_est) + ", contraction " +
                            std::to_string(p->info.refine_rho_est));
    return RTPROJ_OK;
}

rtproj_status rtproj_plan_export(rtproj_plan p, double *S, int64_t lds, double *R, int32_t *piv, double *Minv)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    if (!p->ready) return fail(RTPROJ_ERR_STATE, "plan not preconditioned");
    if (S && lds < p->l) return fail(RTPROJ_ERR_INVALID_ARG, "lds < l");
    const int64_t m = p->m;
    if (S)
        RT_HIP(hipMemcpy2DAsync(S, lds * 8, p->d_S, p->l * 8, p->l * 8, m, hipMemcpyDeviceToDevice, p->stream));
    if (R) RT_HIP(hipMemcpyAsync(R, p->d_R, m * m * 8, hipMemcpyDeviceToDevice, p->stream));
    if (piv) RT_HIP(hipMemcpyAsync(piv, p->d_piv, m * 4, hipMemcpyDeviceToDevice, p->stream));
    if (Minv) {
        // T'^T T' (Cholesky) or T'^T (Y T') with Y T' staged in d_G, whose
        // Gram is no longer needed (Newton-Schulz), from d_Tp = [T'^T; T']
        const bool ns = p->inv_used == RTPROJ_INV_NEWTON_SCHULZ;
        rt::GemmArgs g{};
        g.M = (int)m; g.N = (int)m; g.K = (int)m;
        g.a_i = m; g.a_k = 1; g.b_k = m; g.b_j = 1; g.c_i = m; g.c_j = 1;
        g.alpha = 1.0; g.ksplit = 1;
        if (ns) {
            g.A = p->d_L; g.B = p->d_Tp + m * m; g.C = p->d_G;
            RT_HIP(rt::gemm_f64(g, p->stream));
        }
        g.A = p->d_Tp; g.B = ns ? p->d_G : p->d_Tp + m * m; g.C = Minv;
        RT_HIP(rt::gemm_f64(g, p->stream));
    }
    RT_HIP(hipStreamSynchronize(p->stream));
    return RTPROJ_OK;
}

rtproj_status rtproj_sketch_tables(rtproj_plan p, int64_t *dims3, int8_t *sign, int32_t *sigma, int32_t *tau,
                                   int32_t *J)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    const HostTables &t = p->tab;
    if (dims3) { dims3[0] = t.np; dims3[1] = t.n1; dims3[2] = t.n2; }
    if (sign) std::memcpy(sign, t.sign.data(), t.sign.size());
    if (sigma) std::memcpy(sigma, t.sigma.data(), t.sigma.size() * 4);
    if (tau) std::memcpy(tau, t.tau.data(), t.tau.size() * 4);
    if (J) std::memcpy(J, t.J.data(), t.J.size() * 4);
    return RTPROJ_OK;
}

}  // extern "C"
