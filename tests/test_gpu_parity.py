"""GPU path vs the CPU oracle, through the C ABI (marker: gpu).

Tolerances
* sketch S: binary64 FFT; |dS_i| <= 64 u log2(np) |a_i| per row.
* tables (signs, permutations, subset): bit-exact.
* pivoted QR: pivots equal to the oracle's wherever the oracle's choice is not
  a near-tie (relative gap of the two largest trailing norms > 1e-8); R equal
  up to row signs on the agreeing prefix, within max(1e-9 |R_kk|, 1e-12 |R_11|).
* projection (the unique outputs z, A^T x, x): <= 1e-10 relative (z and the
  row projection relative to |b|, x relative to |x|), max over columns.
"""
import numpy as np
import pytest

import oracle
from paper_0912_1135_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def rt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0912_1135_amd as rt
    rt.lib()
    return rt


def dev():
    return torch.device("cuda", 0)


def run_gpu(rt, A, B, l, seed, steps=None):
    m, n = A.shape
    plan = rt.Plan(m, n, l, seed)
    if steps is not None:
        plan.set_refinement(steps, 0.0)
    At = torch.from_numpy(A).to(dev())
    Bt = torch.from_numpy(np.ascontiguousarray(B)).to(dev())
    plan.precondition(At)
    Z, Y, X = plan.project_all(Bt)
    torch.cuda.synchronize()
    out = Z.cpu().numpy(), Y.cpu().numpy(), X.cpu().numpy()
    return plan, out


def errors(B, Z, Y, X, Zr, Yr, Xr):
    nb = np.linalg.norm(B, axis=1)
    ez = np.max(np.linalg.norm(Z - Zr.T, axis=1) / nb)
    ey = np.max(np.linalg.norm(Y - Yr.T, axis=1) / nb)
    ex = np.max(np.linalg.norm(X - Xr.T, axis=1) / np.linalg.norm(Xr.T, axis=1))
    return ez, ey, ex


@pytest.mark.parametrize("m,n,l,kappa,k,seed", [
    (64, 4096, 256, 1e6, 1, 20091211),     # the 64 x 4096 FP64 workload
    (48, 3000, 192, 1e6, 3, 1),            # ragged n (padded to 4096)
    (100, 5000, 400, 1e8, 5, 2),           # m not a multiple of the 64-row blocks
    (130, 9000, 520, 1e10, 17, 3),         # k above one 16-column group
    (1, 50, 1, 1e0, 2, 4),                 # single row
    (12, 12, 12, 1e3, 2, 5),               # square: null space is {0}
    (33, 500, 33, 1e6, 4, 6),              # l = m
    (600, 8192, 4096, 1e6, 2, 7),          # tall sketch: register-resident QR, 8 rows per thread
    (600, 16384, 9000, 1e6, 2, 8),         # taller than the register form: QR columns in global memory
    (200, 6000, 800, 1e6, 40, 9),          # k >= 32: the plain A B pass on MFMA
    (96, 3000, 384, 1e6, 70, 12),          # k > 64: M^{-1} by split GEMMs, not the skinny products
])
def test_projection_matches_oracle(rt, m, n, l, kappa, k, seed):
    A = synth.make_problem(m, n, kappa, seed)
    B = synth.make_rhs(n, k, seed)
    plan, (Z, Y, X) = run_gpu(rt, A, B, l, seed)
    Zr, Yr, Xr, _ = oracle.project(A, B.T)
    ez, ey, ex = errors(B, Z, Y, X, Zr, Yr, Xr)
    assert ez <= TOL and ey <= TOL and ex <= TOL, (ez, ey, ex)
    plan.close()


@pytest.mark.parametrize("m,n,l,kappa,k,seed", [
    (70, 3001, 300, 1e8, 17, 10),   # odd n and row stride, A not 16-byte aligned
    (64, 4099, 256, 1e6, 9, 11),
])
def test_projection_with_strided_unaligned_a(rt, m, n, l, kappa, k, seed):
    # A and B as views into wider buffers: odd row strides and a start 8 bytes
    # past an allocation, so the passes over A take their unaligned paths
    A = synth.make_problem(m, n, kappa, seed)
    B = synth.make_rhs(n, k, seed)
    abuf = torch.zeros(m, n + 2 + (n + 1) % 2, dtype=torch.float64, device=dev())   # odd row stride
    abuf[:, 1:n + 1] = torch.from_numpy(A).to(dev())
    At = abuf[:, 1:n + 1]
    bbuf = torch.zeros(k, n + 5, dtype=torch.float64, device=dev())
    bbuf[:, 3:n + 3] = torch.from_numpy(np.ascontiguousarray(B)).to(dev())
    Bt = bbuf[:, 3:n + 3]
    assert At.stride(0) % 2 == 1 and At.data_ptr() % 16 == 8
    plan = rt.Plan(m, n, l, seed)
    plan.precondition(At)
    Z, Y, X = plan.project_all(Bt)
    torch.cuda.synchronize()
    Zr, Yr, Xr, _ = oracle.project(A, B.T)
    ez, ey, ex = errors(B, Z.cpu().numpy(), Y.cpu().numpy(), X.cpu().numpy(), Zr, Yr, Xr)
    assert ez <= TOL and ey <= TOL and ex <= TOL, (ez, ey, ex)
    plan.close()


def test_tables_match_oracle(rt):
    for (m, n, l, seed) in [(8, 100, 40, 3), (64, 4096, 256, 9), (16, 544, 64, 11)]:
        plan = rt.Plan(m, n, l, seed)
        got = plan.sketch_tables()
        ref = oracle.srft_tables(seed, n, l)
        for key in ["np", "n1", "n2"]:
            assert got[key] == ref[key]
        for key in ["sign", "sigma", "tau", "J"]:
            assert np.array_equal(got[key], ref[key]), key
        plan.close()


@pytest.mark.parametrize("m,n,l,seed", [(64, 4096, 256, 1), (37, 1000, 150, 2), (10, 33, 20, 3), (4, 4, 4, 4)])
def test_sketch_matches_oracle(rt, m, n, l, seed):
    if n < m:
        pytest.skip("invalid")
    A = synth.make_problem(m, n, 1e3, seed) if m <= n else None
    plan = rt.Plan(m, n, l, seed)
    plan.precondition(torch.from_numpy(A).to(dev()))
    S = plan.export()["S"].cpu().numpy()
    Sr = oracle.srft_sketch(A, seed, l)
    np_ = oracle.srft_dims(n)[0]
    tol = 64 * 2.0 ** -52 * np.log2(np_) * np.linalg.norm(A, axis=1)
    assert np.all(np.linalg.norm(S - Sr, axis=1) <= tol)
    plan.close()


@pytest.mark.parametrize("m,n,l,kappa,seed", [(64, 4096, 256, 1e6, 1), (96, 2000, 384, 1e4, 2), (200, 8192, 800, 1e8, 3),
                                               (600, 8192, 4096, 1e6, 7), (600, 16384, 9000, 1e6, 8),
                                               (1000, 4096, 4096, 1e6, 9)])
def test_qrcp_matches_oracle(rt, m, n, l, kappa, seed):
    A = synth.make_problem(m, n, kappa, seed)
    plan = rt.Plan(m, n, l, seed)
    plan.set_qr(rt.QR_DIRECT)  # Householder QRCP of S^T itself, as the oracle
    plan.precondition(torch.from_numpy(A).to(dev()))
    if l > 8192:
        assert plan.info()["qrcp_blocks"] == (m + 15) // 16  # global-memory column mode
    ex = plan.export()
    R, piv = ex["R"].cpu().numpy(), ex["piv"].cpu().numpy()
    Sr = oracle.srft_sketch(A, seed, l)
    Rr, pr = oracle.qrcp(Sr.T)
    assert sorted(piv.tolist()) == list(range(m))
    assert np.allclose(np.tril(R, -1), 0)
    # agreeing prefix of the pivot sequences
    agree = 0
    while agree < m and piv[agree] == pr[agree]:
        agree += 1
    if agree < m:
        # both chose from the same prefix: the GPU's pick must have a trailing
        # norm within 1e-8 of the largest one (a rounding-level near-tie)
        M = Sr.T
        chosen = pr[:agree]
        Q = np.linalg.qr(M[:, chosen])[0] if agree > 0 else np.zeros((l, 0))
        trail = lambda j: np.linalg.norm(M[:, j] - Q @ (Q.T @ M[:, j]))
        rest = [j for j in range(m) if j not in set(chosen.tolist())]
        best = max(trail(j) for j in rest)
        assert trail(piv[agree]) >= (1 - 1e-8) * best, (agree, trail(piv[agree]), best)
    # backward-stable factors of the same S^T: entries agree to a rounding-level
    # error relative to their row's diagonal or to |R_11| (graded rows)
    D = np.maximum(1e-9 * np.abs(np.diag(Rr))[:agree, None], 1e-12 * abs(Rr[0, 0]))
    assert np.all(np.abs(np.abs(R[:agree, :agree]) - np.abs(Rr[:agree, :agree])) <= D)
    assert agree >= min(m, 32)
    plan.close()


def test_lemma_2_4_on_gpu_preconditioner(rt):
    """cond(P^{-1}A) of the GPU's R and piv equals cond(V^T G) computed by the
    oracle's sketch of V^T (Lemma 2.4)."""
    import scipy.linalg as sl
    m, n, l, seed = 40, 2048, 160, 8
    A, U, s, V = synth.make_problem(m, n, 1e6, seed, with_factors=True)
    plan = rt.Plan(m, n, l, seed)
    plan.precondition(torch.from_numpy(A).to(dev()))
    ex = plan.export()
    R, piv = ex["R"].cpu().numpy(), ex["piv"].cpu().numpy()
    W = sl.solve_triangular(R.T, A[piv], lower=True)
    VG = oracle.srft_sketch(np.ascontiguousarray(V.T), seed, l)
    c1, c2 = np.linalg.cond(W), np.linalg.cond(VG)
    assert abs(c1 - c2) <= 1e-6 * c2 and c2 < 10
    plan.close()


def test_refinement_reduces_error(rt):
    m, n, l, k, seed = 128, 16384, 512, 4, 12
    A = synth.make_problem(m, n, 1e10, seed)
    B = synth.make_rhs(n, k, seed)
    Zr, Yr, Xr, _ = oracle.project(A, B.T)
    _, (Z0, Y0, X0) = run_gpu(rt, A, B, l, seed, steps=0)
    _, (Z3, Y3, X3) = run_gpu(rt, A, B, l, seed, steps=3)
    e0 = errors(B, Z0, Y0, X0, Zr, Yr, Xr)
    e3 = errors(B, Z3, Y3, X3, Zr, Yr, Xr)
    assert max(e3) <= TOL, e3
    assert e0[2] > 1e3 * e3[2]


def test_projector_invariants(rt):
    """Z Z = Z, Z^T = Z, A Z = 0 for the GPU projector assembled on the identity."""
    m, n, l, seed = 6, 64, 24, 3
    A = synth.make_problem(m, n, 1e4, seed)
    plan, (Z, Y, X) = run_gpu(rt, A, np.eye(n), l, seed)
    Zm = Z.T
    assert np.abs(Zm - Zm.T).max() <= 1e-14
    assert np.abs(Zm @ Zm - Zm).max() <= 1e-14
    assert np.abs(A @ Zm).max() <= 1e-14
    plan.close()


def test_seed_independence(rt):
    """Results do not depend on the sketch (eq. basic_precond is an identity)."""
    m, n, l, k = 50, 3000, 200, 2
    A = synth.make_problem(m, n, 1e8, 5)
    B = synth.make_rhs(n, k, 5)
    _, (Z1, Y1, X1) = run_gpu(rt, A, B, l, 1)
    _, (Z2, Y2, X2) = run_gpu(rt, A, B, l, 987654321)
    nb = np.linalg.norm(B, axis=1)
    assert np.max(np.linalg.norm(Z1 - Z2, axis=1) / nb) <= 2 * TOL


def test_error_codes(rt):
    with pytest.raises(rt.RtprojError) as e:
        rt.Plan(10, 5, 6, 0)
    assert e.value.status == 1
    with pytest.raises(rt.RtprojError):
        rt.Plan(10, 100, 5, 0)
    plan = rt.Plan(8, 100, 32, 0)
    B = torch.zeros((2, 100), dtype=torch.float64, device=dev())
    with pytest.raises(rt.RtprojError) as e:
        plan.project_null(B)
    assert e.value.status == 4
    # rank-deficient A: duplicated rows
    A = synth.make_problem(8, 100, 10.0, 1)
    A[3] = A[5]
    with pytest.raises(rt.RtprojError) as e:
        plan.precondition(torch.from_numpy(A).to(dev()))
    assert e.value.status == 5
    # k = 0 is a no-op
    A = synth.make_problem(8, 100, 10.0, 1)
    plan.precondition(torch.from_numpy(A).to(dev()))
    plan.project_null(torch.zeros((0, 100), dtype=torch.float64, device=dev()))
    plan.close()


def test_aliasing_z_equals_b(rt):
    m, n, l, k, seed = 20, 700, 80, 3, 4
    A = synth.make_problem(m, n, 1e4, seed)
    B = synth.make_rhs(n, k, seed)
    plan = rt.Plan(m, n, l, seed)
    plan.precondition(torch.from_numpy(A).to(dev()))
    Bt = torch.from_numpy(B).to(dev())
    Zs = plan.project_null(Bt.clone())
    plan.project_null(Bt, out=Bt)
    torch.cuda.synchronize()
    assert torch.equal(Zs, Bt)
    plan.close()


@pytest.mark.parametrize("prec,name", [(1, "fp32"), (2, "bf16"), (3, "bf16x3")])
@pytest.mark.parametrize("m,n,l,kappa,k,seed", [
    (64, 4096, 256, 1e3, 3, 31),      # P^{-1}A in binary32 (kappa_est small)
    (100, 5000, 400, 1e8, 4, 32),     # P^{-1}A stays binary64, reduced-precision Gram
    (130, 9000, 520, 1e10, 5, 33),
    (150, 6000, 600, 1e6, 36, 34),    # k >= 32: plain refinement steps and A B on MFMA
])
def test_mixed_precision_matches_oracle(rt, prec, name, m, n, l, kappa, k, seed):
    A = synth.make_problem(m, n, kappa, seed)
    B = synth.make_rhs(n, k, seed)
    plan = rt.Plan(m, n, l, seed)
    plan.set_precision(prec)
    plan.precondition(torch.from_numpy(A).to(dev()))
    Z, Y, X = plan.project_all(torch.from_numpy(B).to(dev()))
    torch.cuda.synchronize()
    info = plan.info()
    assert info["sketch_bits"] == (64 if info["sketch_escalated"] else 32)
    assert info["gram_cond_est"] < 10
    assert info["gram_bits"] == {1: 32, 2: 16, 3: 17}[prec]
    assert info["w_bits"] == (32 if info["kappa_est"] <= 1e5 else 64)
    Zr, Yr, Xr, _ = oracle.project(A, B.T)
    ez, ey, ex = errors(B, Z.cpu().numpy(), Y.cpu().numpy(), X.cpu().numpy(), Zr, Yr, Xr)
    assert ez <= TOL and ey <= TOL and ex <= TOL, (name, ez, ey, ex, info["refine_steps"])
    plan.close()


def test_fp32_sketch_matches_oracle(rt):
    m, n, l, seed = 40, 3000, 160, 9
    A = synth.make_problem(m, n, 1e3, seed)
    plan = rt.Plan(m, n, l, seed)
    plan.set_precision(1)
    plan.precondition(torch.from_numpy(A).to(dev()))
    S = plan.export()["S"].cpu().numpy()
    Sr = oracle.srft_sketch(A, seed, l)
    np_ = oracle.srft_dims(n)[0]
    tol = 64 * 2.0 ** -23 * np.log2(np_) * np.linalg.norm(A, axis=1)
    err = np.linalg.norm(S - Sr, axis=1)
    assert np.all(err <= tol)
    assert np.max(err / np.linalg.norm(A, axis=1)) > 1e-12  # really binary32
    plan.close()


@pytest.mark.parametrize("m,n,l,precision", [(37, 65436, 512, 0), (37, 65436, 512, 1), (9, 262137, 64, 0),
                                               (9, 262137, 64, 1), (300, 262144, 1024, 0), (300, 262144, 1024, 1),
                                               (1, 65537, 16, 1), (3, 131072, 24, 0), (3, 131072, 24, 1)])
def test_long_row_sketch_matches_oracle(rt, m, n, l, precision):
    """Transforms of 2^16 to 2^18 points, where both passes walk runs of row
    pairs with the next gathers in flight: odd m (a last pair with one row,
    down to a single row), n short of the padded length, a last group of row
    pairs shorter than the others, and a 512 x 256 grid (n1 != n2), in
    binary64 and binary32."""
    A = np.random.default_rng(4000 + m).standard_normal((m, n))
    plan = rt.Plan(m, n, l, 21)
    plan.set_precision(precision)
    plan.precondition(torch.from_numpy(A).to(dev()))
    assert plan.info()["sketch_bits"] == (64 if precision == 0 else 32)
    S = plan.export()["S"].cpu().numpy()
    Sr = oracle.srft_sketch(A, 21, l)
    np_ = oracle.srft_dims(n)[0]
    u = 2.0 ** -52 if precision == 0 else 2.0 ** -23
    tol = 64 * u * np.log2(np_) * np.linalg.norm(A, axis=1)
    assert np.all(np.linalg.norm(S - Sr, axis=1) <= tol)
    plan.close()


def test_bf16_gram_needs_refinement(rt):
    """Unrefined, the bfloat16 Gram leaves errors far above binary64 rounding;
    the refinement of Remark 4.3 brings them under the tolerance."""
    m, n, l, k, seed = 96, 6000, 384, 3, 40
    A = synth.make_problem(m, n, 1e6, seed)
    B = synth.make_rhs(n, k, seed)
    Zr, Yr, Xr, _ = oracle.project(A, B.T)
    plan = rt.Plan(m, n, l, seed)
    plan.set_precision(2)
    plan.precondition(torch.from_numpy(A).to(dev()))
    Bt = torch.from_numpy(B).to(dev())
    plan.set_refinement(0, 0.0)
    Z0, Y0, X0 = [t.cpu().numpy() for t in plan.project_all(Bt)]
    plan.set_refinement(-1, 0.0)
    Z1, Y1, X1 = [t.cpu().numpy() for t in plan.project_all(Bt)]
    e0 = errors(B, Z0, Y0, X0, Zr, Yr, Xr)
    e1 = errors(B, Z1, Y1, X1, Zr, Yr, Xr)
    assert e0[2] > 1e-6 and max(e1) <= TOL, (e0, e1)
    plan.close()


# ------------------------------------------------------------ two-stage QR

@pytest.mark.parametrize("mode", ["two_stage", "two_stage_wg"])
@pytest.mark.parametrize("m,n,l,kappa,seed", [(64, 4096, 256, 1e6, 1), (200, 8192, 800, 1e8, 3),
                                               (130, 9000, 520, 1e10, 4), (600, 8192, 4096, 1e6, 7)])
def test_two_stage_qrcp_is_backward_stable(rt, mode, m, n, l, kappa, seed):
    """R and piv of the two-stage pivoted QR: R^T R = Pi^T S S^T Pi up to a
    normwise rounding error c u |S|^2 (kappa-independent), the pivoting
    property |R_kk| >= |R[k:, j]| (j > k) within c u |S|, and a
    preconditioner as good as the direct one (Lemma 2.4)."""
    code = {"two_stage": rt.QR_TWO_STAGE, "two_stage_wg": rt.QR_TWO_STAGE_WG}[mode]
    A = synth.make_problem(m, n, kappa, seed)
    plan = rt.Plan(m, n, l, seed)
    plan.set_qr(code)
    plan.precondition(torch.from_numpy(A).to(dev()))
    assert plan.info()["qr_mode"] == code
    ex = plan.export()
    R, piv = ex["R"].cpu().numpy(), ex["piv"].cpu().numpy()
    assert sorted(piv.tolist()) == list(range(m))
    assert np.allclose(np.tril(R, -1), 0)
    Sr = oracle.srft_sketch(A, seed, l)
    nS = np.linalg.norm(Sr)
    u = 2.0 ** -53
    c = 8.0 * (l * m) ** 0.5 * m
    M = Sr[piv]                       # rows of S in pivot order = columns of S^T Pi
    assert np.max(np.abs(R.T @ R - M @ M.T)) <= c * u * nS ** 2
    for k in range(m - 1):
        tail = np.linalg.norm(R[k:, k + 1:], axis=0)
        assert np.all(tail <= abs(R[k, k]) * (1 + 1e-8) + c * u * nS), k
    W = np.linalg.solve(R.T, A[piv])  # P^{-1} A = R^{-T} Pi A
    sv = np.linalg.svd(W, compute_uv=False)
    assert sv[0] / sv[-1] < 10
    plan.close()


@pytest.mark.parametrize("precision", [0, 3])
def test_two_stage_rank_deficient_sketch_is_flagged(rt, precision):
    """A duplicated row makes S^T exactly rank deficient.  Two Cholesky QR
    passes resolve its smallest singular value only to about sqrt(u) |S|;
    the second factor's diagonal then spans far more than 1e5, the third
    pass runs, and the rank test reports RTPROJ_ERR_RANK as the direct QR
    does (the reduced precision first re-sketches in binary64)."""
    m, n, l, seed = 520, 3120, 2080, 1501
    A = synth.make_problem(m, n, 1e3, seed)
    A[-1] = A[0]
    plan = rt.Plan(m, n, l, seed)
    plan.set_qr(rt.QR_TWO_STAGE)
    plan.set_precision(precision)
    with pytest.raises(rt.RtprojError) as e:
        plan.precondition(torch.from_numpy(A).to(dev()))
    assert e.value.status == 5
    plan.close()


@pytest.mark.parametrize("mode", ["direct", "two_stage", "two_stage_wg"])
@pytest.mark.parametrize("m,n,l,kappa,k,seed", [(100, 5000, 400, 1e8, 5, 2), (130, 9000, 520, 1e10, 3, 3),
                                                 (1, 50, 1, 1e0, 2, 4), (12, 12, 12, 1e3, 2, 5)])
def test_projection_matches_oracle_all_qr_modes(rt, mode, m, n, l, kappa, k, seed):
    code = {"direct": rt.QR_DIRECT, "two_stage": rt.QR_TWO_STAGE, "two_stage_wg": rt.QR_TWO_STAGE_WG}[mode]
    A = synth.make_problem(m, n, kappa, seed)
    B = synth.make_rhs(n, k, seed)
    plan = rt.Plan(m, n, l, seed)
    plan.set_qr(code)
    At = torch.from_numpy(A).to(dev())
    Bt = torch.from_numpy(B).to(dev())
    plan.precondition(At)
    Z, Y, X = plan.project_all(Bt)
    Zr, Yr, Xr, _ = oracle.project(A, B.T)
    ez, ey, ex = errors(B, Z.cpu().numpy(), Y.cpu().numpy(), X.cpu().numpy(), Zr, Yr, Xr)
    assert ez <= TOL and ey <= TOL and ex <= TOL, (ez, ey, ex)
    plan.close()


# ------------------------------------------------------- inverse of the Gram

@pytest.mark.parametrize("method", ["newton_schulz", "cholesky"])
@pytest.mark.parametrize("m,n,l,kappa,k,seed", [
    (1, 50, 1, 1e0, 2, 41),            # 1 x 1 Gram
    (12, 12, 12, 1e3, 2, 42),          # square A, l = m
    (64, 4096, 68, 1e6, 3, 43),        # l = m + 4: a poorer preconditioner, more steps
    (33, 500, 33, 1e6, 2, 6),          # l = m: cond(X) near 3e3
    (300, 9000, 1200, 1e8, 4, 44),     # ragged 64-tiles, K split in two
    (600, 8192, 2400, 1e10, 5, 45),    # K split in four
])
def test_projection_matches_oracle_both_inverses(rt, method, m, n, l, kappa, k, seed):
    code = {"newton_schulz": rt.INV_NEWTON_SCHULZ, "cholesky": rt.INV_CHOLESKY}[method]
    A = synth.make_problem(m, n, kappa, seed)
    B = synth.make_rhs(n, k, seed)
    plan = rt.Plan(m, n, l, seed)
    plan.set_inverse(code)
    plan.precondition(torch.from_numpy(A).to(dev()))
    Z, Y, X = plan.project_all(torch.from_numpy(B).to(dev()))
    torch.cuda.synchronize()
    info = plan.info()
    assert info["inverse"] == code
    if code == rt.INV_NEWTON_SCHULZ:
        # rounds have an even number of steps; the last measured residual is
        # past the quadratic phase (or at the rounding floor)
        assert info["inverse_iters"] >= 2 and info["inverse_iters"] % 2 == 0
        assert info["inverse_resid"] <= 1e-4
    else:
        assert info["inverse_iters"] == 0
    assert 1.0 <= info["gram_cond_est"] < 100
    Zr, Yr, Xr, _ = oracle.project(A, B.T)
    ez, ey, ex = errors(B, Z.cpu().numpy(), Y.cpu().numpy(), X.cpu().numpy(), Zr, Yr, Xr)
    assert ez <= TOL and ey <= TOL and ex <= TOL, (method, ez, ey, ex, info["refine_steps"])
    plan.close()


@pytest.mark.parametrize("method", ["newton_schulz", "cholesky"])
def test_exported_minv_inverts_the_normal_matrix(rt, method):
    """M^{-1} = (P^*)^{-1} Y P^{-1} is (A A^T)^{-1} up to rounding for a well
    conditioned A (eq. basic_precond with Y = X^{-1}); both routes agree."""
    code = {"newton_schulz": rt.INV_NEWTON_SCHULZ, "cholesky": rt.INV_CHOLESKY}[method]
    m, n, l, seed = 200, 6000, 800, 46
    A = synth.make_problem(m, n, 1e2, seed)
    plan = rt.Plan(m, n, l, seed)
    plan.set_inverse(code)
    plan.precondition(torch.from_numpy(A).to(dev()))
    Mi = plan.export()["Minv"].cpu().numpy()
    N = A @ A.T
    E = Mi @ N - np.eye(m)
    assert np.linalg.norm(E, 2) <= 1e-10, np.linalg.norm(E, 2)
    assert np.max(np.abs(Mi - Mi.T)) <= 1e-8 * np.max(np.abs(Mi))
    plan.close()


@pytest.mark.parametrize("prec", [1, 2, 3])
@pytest.mark.parametrize("n", [20000, 20002])
def test_exported_minv_binary32_gram(rt, n, prec):
    """The binary32, bfloat16 and split-bfloat16 Grams (P^{-1}A)(P^{-1}A)^T on
    MFMA, seen through M^{-1}: n % 4 == 0 takes the 16-byte-load Gram kernels,
    n % 4 == 2 the general ones (the binary32 one for the split precision);
    m = 300 leaves ragged 128-row tiles.  The binary32 and split Grams of a
    well conditioned W give |M^{-1} A A^T - I| of order 1e-5 or below, the
    bfloat16 one of order 1e-3 (its inputs rounded to 8 bits); a wrong tile,
    split, half, scale or contraction order gives O(1)."""
    m, l, seed = 300, 1200, 47
    A = synth.make_problem(m, n, 10.0, seed)
    plan = rt.Plan(m, n, l, seed)
    plan.set_precision(prec)
    plan.set_inverse(rt.INV_CHOLESKY)
    plan.precondition(torch.from_numpy(A).to(dev()))
    info = plan.info()
    assert info["w_bits"] == 32
    assert info["gram_bits"] == {1: 32, 2: 16, 3: 17 if n % 4 == 0 else 32}[prec]
    Mi = plan.export()["Minv"].cpu().numpy()
    E = Mi @ (A @ A.T) - np.eye(m)
    print(f"n {n} precision {prec}: |M^-1 A A^T - I| = {np.linalg.norm(E, 2):.2e}")
    # measured 1.3e-6 (binary32), 1.4e-5 (split bfloat16) and 2.3e-3
    # (bfloat16, both kernels); a split Gram that lost its lo halves would
    # be near the bfloat16 figure
    assert np.linalg.norm(E, 2) <= (1e-2 if prec == 2 else 1e-4), np.linalg.norm(E, 2)
    plan.close()


def test_inverse_method_argument_checks(rt):
    plan = rt.Plan(8, 100, 32, 0)
    with pytest.raises(rt.RtprojError) as e:
        plan.set_inverse(3)
    assert e.value.status == 1
    plan.set_inverse(rt.INV_AUTO)
    A = synth.make_problem(8, 100, 10.0, 1)
    plan.precondition(torch.from_numpy(A).to(dev()))
    assert plan.info()["inverse"] == rt.INV_NEWTON_SCHULZ   # m <= 1024
    plan.close()
