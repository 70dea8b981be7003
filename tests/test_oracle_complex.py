"""Pins of the complex-valued oracle (oracle/complex_oracle.py) to facts
outside itself (no GPU): 50-digit mpmath brute force on tiny complex inputs,
the real oracle on real inputs, the closed forms of a single row and of
orthonormal rows, and the projector's invariants Z Z = Z, Z^* = Z, A Z = 0
(Sec. 1, after eq. basic_identity, with A^* the conjugate transpose).  Two
planted mistakes (a dropped conjugate, an unconjugated correction solve)
must each fail a pin."""
import os

import mpmath
import numpy as np
import pytest

import oracle
from oracle import complex_oracle
from paper_0912_1135_amd import synth


def cplx_problem(m, n, kappa, seed):
    """A = U diag(sigma) V^* with U, V complex orthonormal (QR of complex
    Gaussians), sigma log-spaced 1 -> 1/kappa (test input only)."""
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))[0]
    V = np.linalg.qr(rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m)))[0]
    s = synth.log_spaced(m, kappa)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return (U * s) @ V.conj().T, b


def mp_truth(A, b, dps=50):
    with mpmath.workdps(dps):
        Am = mpmath.matrix([[mpmath.mpc(v.real, v.imag) for v in row] for row in A])
        bm = mpmath.matrix([mpmath.mpc(v.real, v.imag) for v in b])
        Ah = Am.H
        x = mpmath.lu_solve(Am * Ah, Am * bm)
        p = Ah * x
        z = bm - p
        f = lambda v: np.array([complex(v[i]) for i in range(v.rows)])
        return f(z), f(p), f(x)


def pins_pass(project):
    for m, n, kappa, seed in [(1, 6, 1.0, 1), (3, 10, 1e4, 2), (4, 12, 1e6, 3)]:
        A, b = cplx_problem(m, n, kappa, seed)
        z, p, x, _ = project(A, b)
        zt, pt, xt = mp_truth(A, b)
        nb = np.linalg.norm(b)
        if not (np.linalg.norm(z - zt) <= 1e-15 * nb and np.linalg.norm(p - pt) <= 1e-15 * nb
                and np.linalg.norm(x - xt) <= 1e-14 * np.linalg.norm(xt)):
            return False
    return True


def test_complex_oracle_matches_mpmath():
    assert pins_pass(complex_oracle.project_complex)


def test_complex_oracle_equals_real_oracle_on_real_input():
    A = synth.make_problem(20, 600, 1e8, 4)
    B = synth.make_rhs(600, 2, 4).T
    Zc, Pc, Xc, _ = complex_oracle.project_complex(A.astype(complex), B.astype(complex))
    Zr, Pr, Xr, _ = oracle.project(A, B)
    assert np.max(np.abs(Zc.imag)) == 0 or np.max(np.abs(Zc.imag)) <= 1e-16 * np.max(np.abs(Zc))
    assert np.max(np.linalg.norm(Zc - Zr, axis=0) / np.linalg.norm(B, axis=0)) <= 2e-16
    assert np.max(np.linalg.norm(Xc - Xr, axis=0) / np.linalg.norm(Xr, axis=0)) <= 1e-15


def test_complex_single_row_closed_form():
    rng = np.random.default_rng(5)
    a = rng.standard_normal(30) + 1j * rng.standard_normal(30)
    b = rng.standard_normal(30) + 1j * rng.standard_normal(30)
    z, p, x, _ = complex_oracle.project_complex(a[None, :], b)
    xt = (a @ b) / np.vdot(a, a).real
    assert abs(x[0] - xt) <= 1e-15 * abs(xt)
    assert np.linalg.norm(z - (b - a.conj() * xt)) <= 1e-15 * np.linalg.norm(b)


def test_complex_orthonormal_rows_closed_form():
    rng = np.random.default_rng(6)
    Q = np.linalg.qr(rng.standard_normal((40, 7)) + 1j * rng.standard_normal((40, 7)))[0]
    A = Q.conj().T          # A A^* = I
    b = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    z, p, x, _ = complex_oracle.project_complex(A, b)
    assert np.linalg.norm(z - (b - A.conj().T @ (A @ b))) <= 1e-15 * np.linalg.norm(b)


def test_complex_projector_invariants():
    A, _ = cplx_problem(5, 16, 1e3, 7)
    Z, _, _, _ = complex_oracle.project_complex(A, np.eye(16, dtype=complex))
    assert np.abs(Z - Z.conj().T).max() <= 1e-15
    assert np.abs(Z @ Z - Z).max() <= 1e-15
    assert np.abs(A @ Z).max() <= 1e-14


MUTANTS = {
    "residual without conjugate": ("acc -= conjq(cq(A + 2 * (i * lda + t))) * x[i];",
                                   "acc -= cq(A + 2 * (i * lda + t)) * x[i];"),
    "R^* solve unconjugated": ("s -= conj(rji) * y[j];", "s -= rji * y[j];"),
    "row projection without conjugate": ("acc += conjq(cq(A + 2 * (i * lda + t))) * x[i];",
                                         "acc += cq(A + 2 * (i * lda + t)) * x[i];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_complex_mutant_is_caught(tmp_path, name):
    from tests.test_oracle_mutants import build_mutant
    lib = build_mutant(tmp_path, *MUTANTS[name])
    assert not pins_pass(lambda A, b: complex_oracle.project_complex(A, b, lib=lib))
