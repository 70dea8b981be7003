"""Pins of the CPU oracle to facts outside itself (no GPU).

* projection/least squares: 80-digit mpmath brute force, textbook special
  cases, the closed form of the synthetic matrices, projector invariants
  ZZ = Z, Z^T = Z, AZ = 0 (Sec. 1, after eq. basic_identity);
* pivoted QR: LAPACK's dgeqp3 (scipy) and the pivoting inequalities;
* sketch: an explicit cosine/sine matrix instead of the FFT, orthogonality
  of the full transform, Lemma 2.4 (cond(P^{-1}A) = cond(V^* G));
* random tables: the published SplitMix64 vector and distributional checks
  that catch a wrong Fisher-Yates bound or a biased subset.
"""
import mpmath
import os

import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from paper_0912_1135_amd import synth

mpmath.mp.dps = 80


def mp_truth(A, b):
    """x = (A A^T)^{-1} A b, p = A^T x, z = b - p in 80-digit arithmetic."""
    m, n = A.shape
    Am = mpmath.matrix(A.tolist())
    bm = mpmath.matrix(b.tolist())
    x = mpmath.lu_solve(Am * Am.T, Am * bm)
    p = Am.T * x
    z = bm - p
    f = lambda v: np.array([float(v[i]) for i in range(v.rows)])
    return f(z), f(p), f(x)


@pytest.mark.parametrize("m,n,kappa,seed", [
    (1, 7, 1.0, 1), (2, 9, 1e3, 2), (3, 12, 1e6, 3), (4, 16, 1e8, 4),
    (5, 24, 1e10, 5), (4, 4, 1e4, 6), (6, 40, 1e10, 7),
])
def test_project_matches_mpmath(m, n, kappa, seed):
    A = synth.make_problem(m, n, kappa, seed)
    b = synth.make_rhs(n, 1, seed)[0]
    z, p, x, info = oracle.project(A, b)
    zt, pt, xt = mp_truth(A, b)
    nb = np.linalg.norm(b)
    assert np.linalg.norm(z - zt) <= 1e-15 * nb
    assert np.linalg.norm(p - pt) <= 1e-15 * nb
    assert np.linalg.norm(x - xt) <= 1e-15 * np.linalg.norm(xt)


@pytest.mark.parametrize("m,n,kappa,seed", [
    (1, 7, 1.0, 1), (3, 12, 1e6, 3), (5, 24, 1e10, 5), (4, 4, 1e4, 6), (6, 40, 1e10, 7),
])
def test_project_lapack_matches_mpmath(m, n, kappa, seed):
    A = synth.make_problem(m, n, kappa, seed)
    b = synth.make_rhs(n, 1, seed)[0]
    z, p, x, info = oracle.project_lapack(A, b)
    zt, pt, xt = mp_truth(A, b)
    nb = np.linalg.norm(b)
    assert np.linalg.norm(z - zt) <= 1e-15 * nb
    assert np.linalg.norm(p - pt) <= 1e-15 * nb
    assert np.linalg.norm(x - xt) <= 1e-15 * np.linalg.norm(xt)


@pytest.mark.parametrize("m,n,kappa,k", [(16, 600, 1e4, 3), (40, 2000, 1e8, 2), (64, 4096, 1e10, 2),
                                         (200, 3000, 1e12, 1)])
def test_project_lapack_agrees_with_householder_route(m, n, kappa, k):
    """Both routes refine in binary128 to the same fixed point, so they agree
    to the final rounding of binary64 (a few units in the last place)."""
    A = synth.make_problem(m, n, kappa, 100 + m)
    B = synth.make_rhs(n, k, 100 + m).T
    Z0, P0, X0, i0 = oracle.project(A, B)
    Z1, P1, X1, i1 = oracle.project_lapack(A, B)
    nb = np.linalg.norm(B, axis=0)
    assert np.max(np.linalg.norm(Z1 - Z0, axis=0) / nb) <= 4e-16
    assert np.max(np.linalg.norm(P1 - P0, axis=0) / nb) <= 4e-16
    assert np.max(np.linalg.norm(X1 - X0, axis=0) / np.linalg.norm(X0, axis=0)) <= 4e-16
    assert i1[1] <= 1e-20


def test_project_mpmath_svd_route():
    """Same truth through the SVD: p = V_A V_A^T b with V_A from mpmath's SVD."""
    A = synth.make_problem(3, 10, 1e5, 11)
    b = synth.make_rhs(10, 1, 11)[0]
    z, p, _, _ = oracle.project(A, b)
    mpmath.mp.dps = 60
    U, S, V = mpmath.svd_r(mpmath.matrix(A.tolist()))
    Vt = np.array([[float(V[i, j]) for j in range(V.cols)] for i in range(V.rows)])
    mpmath.mp.dps = 80
    pv = Vt.T @ (Vt @ b)
    assert np.linalg.norm(p - pv) <= 1e-14 * np.linalg.norm(b)
    assert np.linalg.norm(z - (b - pv)) <= 1e-14 * np.linalg.norm(b)


def test_project_single_row():
    """m = 1: z = b - a (a^T b)/|a|^2, x = a^T b/|a|^2."""
    rng = np.random.default_rng(3)
    a = rng.standard_normal(50)
    b = rng.standard_normal(50)
    z, p, x, _ = oracle.project(a[None, :], b)
    xe = a @ b / (a @ a)
    assert abs(x[0] - xe) <= 1e-15 * abs(xe)
    assert np.allclose(z, b - a * xe, atol=1e-14, rtol=0)


def test_project_orthonormal_rows():
    """A with orthonormal rows: p = A^T A b, x = A b."""
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((200, 20)))
    A = np.ascontiguousarray(Q.T)
    B = rng.standard_normal((200, 3))
    Z, P, X, _ = oracle.project(A, B)
    assert np.allclose(X, A @ B, atol=1e-14, rtol=0)
    assert np.allclose(P, A.T @ (A @ B), atol=1e-13, rtol=0)
    assert np.allclose(Z + P, B, atol=1e-14, rtol=0)


def test_project_square():
    """m = n: the null space is trivial, z = 0 and x = A^{-T} b."""
    A = synth.make_problem(8, 8, 1e3, 12)
    b = synth.make_rhs(8, 1, 12)[0]
    z, p, x, _ = oracle.project(A, b)
    assert np.linalg.norm(z) <= 1e-14 * np.linalg.norm(b)
    assert np.allclose(x, np.linalg.solve(A.T, b), rtol=1e-10, atol=0)


def test_project_closed_form():
    """For A = U S V^T: p = V V^T b and x = U S^{-1} V^T b, up to the rounding
    of the stored A (kept small by kappa = 100)."""
    A, U, s, V = synth.make_problem(16, 300, 1e2, 13, with_factors=True)
    B = synth.make_rhs(300, 4, 13).T
    Z, P, X, _ = oracle.project(A, B)
    assert np.allclose(P, V @ (V.T @ B), atol=2e-13, rtol=0)
    Xe = U @ ((V.T @ B) / s[:, None])
    assert np.allclose(X, Xe, rtol=0, atol=1e-11 * np.abs(Xe).max())


def test_projector_invariants():
    """Z Z = Z, Z^T = Z, A Z = 0 for the null-space projector built column by
    column from the oracle (Sec. 1, after eq. basic_identity)."""
    n = 30
    A = synth.make_problem(5, n, 1e6, 14)
    Zm, Pm, _, _ = oracle.project(A, np.eye(n))
    assert np.abs(Zm - Zm.T).max() <= 1e-15
    assert np.abs(Zm @ Zm - Zm).max() <= 1e-15
    assert np.abs(A @ Zm).max() <= 1e-15 * np.abs(A).max() * n
    # trace of the row projector is the rank m
    assert abs(np.trace(Pm) - 5) <= 1e-13


def test_project_matches_lapack_lstsq_moderate():
    A = synth.make_problem(12, 400, 1e4, 15)
    B = synth.make_rhs(400, 3, 15).T
    _, _, X, _ = oracle.project(A, B)
    Xl = np.linalg.lstsq(A.T, B, rcond=None)[0]
    assert np.allclose(X, Xl, rtol=1e-9, atol=0)


def test_project_refinement_reaches_extended_accuracy():
    """At kappa = 1e10 a plain double solve misses x by ~1e-7; the oracle must
    agree with 80-digit arithmetic to rounding."""
    A = synth.make_problem(6, 64, 1e10, 16)
    b = synth.make_rhs(64, 1, 16)[0]
    z0, p0, x0, info0 = oracle.project(A, b, maxit=0)
    z, p, x, info = oracle.project(A, b)
    _, _, xt = mp_truth(A, b)
    err0 = np.linalg.norm(x0 - xt) / np.linalg.norm(xt)
    err = np.linalg.norm(x - xt) / np.linalg.norm(xt)
    assert err <= 1e-15
    assert err0 > 1e3 * err  # the refinement is doing the work
    assert info[0] >= 2


# ---------------------------------------------------------------- pivoted QR

def graded(rows, cols, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((rows, cols)) * np.logspace(0, -6, cols)[rng.permutation(cols)]


@pytest.mark.parametrize("rows,cols,seed", [(40, 10, 1), (64, 64, 2), (100, 37, 3)])
def test_qrcp_matches_lapack(rows, cols, seed):
    M = graded(rows, cols, seed)
    R, piv = oracle.qrcp(M)
    Ql, Rl, pl = sl.qr(M, mode="economic", pivoting=True)
    assert np.array_equal(piv, pl)
    scale = np.abs(np.diag(Rl))[:, None]
    assert np.allclose(np.abs(R), np.abs(Rl), atol=1e-12 * scale, rtol=0)


def test_qrcp_reconstructs_and_pivots():
    M = graded(90, 30, 4)
    R, piv = oracle.qrcp(M)
    assert sorted(piv.tolist()) == list(range(30))
    assert np.allclose(np.tril(R, -1), 0)
    Q = sl.solve_triangular(R, M[:, piv].T, trans="T").T   # Q = M Pi^T R^{-1}
    assert np.allclose(Q.T @ Q, np.eye(30), atol=1e-10)
    for k in range(30):
        for j in range(k + 1, 30):
            assert abs(R[k, k]) >= np.linalg.norm(R[k:j + 1, j]) * (1 - 1e-12)


def test_qrcp_ties_take_lowest_index():
    M = np.zeros((6, 4))
    M[0, 1] = 2.0; M[1, 3] = 2.0; M[2, 0] = 1.0; M[3, 2] = 1.0
    R, piv = oracle.qrcp(M)
    assert piv.tolist() == [1, 3, 0, 2]


# ---------------------------------------------------------------- sketch

def test_splitmix64_published_vector():
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed1234567.txt")
    lines = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    seed = int(lines[0][1])
    want = [int(ln[0]) for ln in lines[1:]]
    assert oracle.splitmix64(seed, len(want)).tolist() == want


@pytest.mark.parametrize("n,l", [(5, 3), (8, 8), (13, 6), (16, 16), (33, 20), (64, 17)])
def test_srft_matches_explicit_matrix(n, l):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((3, n))
    S = oracle.srft_sketch(A, 99 + n, l)
    G = oracle.srft_matrix(n, 99 + n, l)
    assert np.allclose(S, A @ G, atol=1e-13, rtol=0)


@pytest.mark.parametrize("n", [16, 50, 1024, 3000])
def test_srft_full_transform_is_orthogonal(n):
    """With l = np the transform has orthonormal rows: S S^T = A A^T."""
    np_ = oracle.srft_dims(n)[0]
    A = np.random.default_rng(n).standard_normal((4, n))
    S = oracle.srft_sketch(A, 5, np_)
    assert np.allclose(S @ S.T, A @ A.T, atol=1e-11 * n, rtol=0)


def test_srft_tables_are_valid():
    for n, l in [(5, 3), (1000, 64), (4096, 256), (544, 64)]:
        t = oracle.srft_tables(7, n, l)
        assert set(np.unique(t["sign"]).tolist()) <= {-1, 1}
        assert sorted(t["sigma"].tolist()) == list(range(t["n1"]))
        assert sorted(t["tau"].tolist()) == list(range(t["n2"]))
        J = t["J"]
        assert len(J) == l and np.all(np.diff(J) > 0) and J[0] >= 0 and J[-1] < t["np"]
        pi = t["sigma"][np.arange(t["np"]) // t["n2"]].astype(np.int64) * t["n2"] + t["tau"][np.arange(t["np"]) % t["n2"]]
        assert sorted(pi.tolist()) == list(range(t["np"]))


def test_srft_tables_distribution():
    """Fisher-Yates (not Sattolo): fixed points occur with rate 1/n1; selection
    sampling includes each position with rate l/np; signs are fair."""
    n1_fixed = 0
    incl = np.zeros(64)
    signs = 0.0
    trials = 3000
    for s in range(trials):
        t = oracle.srft_tables(1000 + s, 64, 16)  # np = 64, n1 = n2 = 8
        n1_fixed += int(t["sigma"][0] == 0)
        incl[t["J"]] += 1
        signs += t["sign"].mean()
    assert abs(n1_fixed / trials - 1 / 8) < 0.03
    assert np.all(np.abs(incl / trials - 16 / 64) < 0.05)
    assert abs(signs / trials) < 0.02
    assert oracle.srft_tables(1, 64, 16)["J"].tolist() != oracle.srft_tables(2, 64, 16)["J"].tolist()


def _golden_splitmix():
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed1234567.txt")
    lines = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    return int(lines[0][1]), [int(ln[0]) for ln in lines[1:]]


@pytest.mark.parametrize("i", [0, 1, 5, 255, 1 << 20])
def test_instance_seed_matches_published_vector(i):
    """Member i of a batch seeded with `seed` draws its tables from the first
    SplitMix64 output of seed XOR i: with seed = 1234567 XOR i that generator
    starts at 1234567, whose first output is the published reference value."""
    seed, want = _golden_splitmix()
    assert oracle.instance_seed(seed ^ i, i) == want[0]


def test_lemma_2_4_oracle_preconditioner():
    """cond(P^{-1} A) = cond(V^T G) with P = Pi^T R^T from the oracle sketch and
    pivoted QR (Lemma 2.4); both sides small, as Observation 3.2 says for l = 4m."""
    m, n, l = 24, 2000, 96
    A, U, s, V = synth.make_problem(m, n, 1e6, 21, with_factors=True)
    S = oracle.srft_sketch(A, 77, l)
    R, piv = oracle.qrcp(S.T)
    W = sl.solve_triangular(R.T, A[piv], lower=True)
    VG = oracle.srft_sketch(np.ascontiguousarray(V.T), 77, l)
    c1, c2 = np.linalg.cond(W), np.linalg.cond(VG)
    assert abs(c1 - c2) <= 1e-6 * c2
    assert c2 < 10


# ------------------------------------------------------ the paper's matrices

@pytest.mark.parametrize("m,n,kappa", [(6, 30, 1e2), (8, 64, 1e8), (10, 50, 1e12), (16, 256, 1e6)])
def test_block_average_is_the_projection_of_the_paper_matrix(m, n, kappa):
    """The closed form (block averages of V b) against the oracle's refined
    Householder route, to the final rounding, including cond(A) = 1e12."""
    from oracle.paper_forms import block_average_projection
    A, rp, cp = synth.make_paper_matrix(m, n, kappa, 31 + m)
    B = synth.make_rhs(n, 2, 31 + m).T
    Z0, P0 = block_average_projection(m, cp, B)
    Z1, P1, X1, info = oracle.project(A, B)
    nb = np.linalg.norm(B, axis=0)
    assert np.max(np.linalg.norm(Z1 - Z0, axis=0) / nb) <= 1e-15
    assert np.max(np.linalg.norm(P1 - P0, axis=0) / nb) <= 1e-15
    sv = np.linalg.svd(A, compute_uv=False)
    assert abs(sv[0] / sv[-1] / kappa - 1) <= 1e-3 or kappa >= 1e12


def test_paper_matrix_has_the_stated_structure():
    """eq. pert_lap and eq. test_mat: the circulant's entries, cond = (16 + d)/d,
    and A a row and column permutation of n/m copies of B."""
    m, n, kappa = 12, 48, 1e6
    B = synth.circulant_b(m, kappa)
    d = 16 / (kappa - 1)
    assert B[0, 0] == 6 + d and B[0, 1] == -4 and B[0, 2] == 1 and B[0, m - 1] == -4 and B[0, m - 2] == 1
    sv = np.linalg.svd(B, compute_uv=False)
    assert abs(sv[0] / sv[-1] - (16 + d) / d) <= 1e-6 * kappa
    A, rp, cp = synth.make_paper_matrix(m, n, kappa, 5)
    assert sorted(rp.tolist()) == list(range(m)) and sorted(cp.tolist()) == list(range(n))
    assert np.array_equal(np.sort(A, axis=None), np.sort(np.tile(B, (1, n // m)), axis=None))
    G = synth.make_lfg_sketch(5000, 7, 3)
    assert G.min() >= -1 and G.max() < 1 and abs(G.mean()) < 0.02 and abs(G.std() - 3 ** -0.5) < 0.01
