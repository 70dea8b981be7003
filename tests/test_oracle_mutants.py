"""The oracle's pins must catch plausible mistakes planted in the oracle.

Each case copies ``oracle/oracle.c``, applies one textual mutation (a dropped
term, a flipped sign, a wrong index or bound, a lost precision), compiles it
with gcc into a temporary library and checks that a pin from
``test_oracle.py`` rejects it.  CPU only.  (Flipping the sign convention of
the Householder beta is not a mistake: both signs give exact reflectors; and
a mistake confined to the starting guess x0 is repaired by the refinement,
whose fixed point depends only on the residual evaluation.)
"""
import os
import subprocess

import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from paper_0912_1135_amd import synth
from tests.test_oracle import graded, mp_truth

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

PROJECTION_MUTANTS = {
    "householder tau sign": ("t = (beta - alpha) / beta;", "t = (alpha - beta) / beta;"),
    "residual product rounded to double": ("acc -= (quad)A[i * lda + t] * x[i];",
                                           "acc -= (quad)(A[i * lda + t] * (double)x[i]);"),
    "R^T solve reads R row": ("s -= Rp[j * ri + i * rj] * y[j];", "s -= Rp[i * ri + j * rj] * y[j];"),
    "A r contraction index shifted": ("s += (quad)a[t] * r[t];", "s += (quad)a[t] * r[(t + 1) % n];"),
    "null projection sign": ("(double)((quad)b[t] - acc)", "(double)((quad)b[t] + acc)"),
    "correction dropped": ("x[i] += (quad)d[i];", "x[i] += (quad)(0.5 * d[i]);"),
    "z uses rounded x": ("acc += (quad)A[i * lda + t] * x[i];", "acc += (quad)(A[i * lda + t] * (double)x[i]);"),
}

# mistakes in the route that takes R from LAPACK (orc_project_r)
PROJECT_R_MUTANTS = {
    "R read transposed": ("R, ldr, 1, k, B, ldb, xq", "R, 1, ldr, k, B, ldb, xq"),
    "too few refinement steps": ("xq, Z, ldz, P, ldp, X, ldx, maxit, info);\n    free(xq);",
                                 "xq, Z, ldz, P, ldp, X, ldx, 1, info);\n    free(xq);"),
}

QRCP_MUTANTS = {
    "pivot ties to highest index": ("if (p < 0 || nrm[j] > nrm[p]) p = j;", "if (p < 0 || nrm[j] >= nrm[p]) p = j;"),
    "pivot by smallest norm": ("if (p < 0 || nrm[j] > nrm[p]) p = j;", "if (p < 0 || nrm[j] < nrm[p]) p = j;"),
    "norm from row 0": ("for (int64_t i = k; i < rows; ++i) s += c[i] * c[i];",
                        "for (int64_t i = 0; i < rows; ++i) s += c[i] * c[i];"),
    "reflector tau sign": ("c[i] -= w * v[i];", "c[i] += w * v[i];"),
}


def build_mutant(tmp_path, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, old
    mutated = src.replace(old, new, 1)
    c = tmp_path / "mut.c"
    c.write_text(mutated)
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", str(c), "-o", str(so), "-lquadmath",
                    "-lm"],
                   check=True)
    return oracle.bind(str(so))


def projection_pins_pass(lib):
    for m, n, kappa, seed in [(3, 12, 1e6, 3), (5, 24, 1e10, 5), (6, 40, 1e10, 7)]:
        A = synth.make_problem(m, n, kappa, seed)
        b = synth.make_rhs(n, 1, seed)[0]
        z, p, x, _ = oracle.project(A, b, lib=lib)
        zt, pt, xt = mp_truth(A, b)
        nb = np.linalg.norm(b)
        if not (np.linalg.norm(z - zt) <= 1e-15 * nb and np.linalg.norm(p - pt) <= 1e-15 * nb
                and np.linalg.norm(x - xt) <= 1e-15 * np.linalg.norm(xt)):
            return False
    return True


def project_r_pins_pass(lib):
    for m, n, kappa, seed in [(3, 12, 1e6, 3), (5, 24, 1e10, 5), (6, 40, 1e10, 7)]:
        A = synth.make_problem(m, n, kappa, seed)
        b = synth.make_rhs(n, 1, seed)[0]
        z, p, x, _ = oracle.project_lapack(A, b, lib=lib)
        zt, pt, xt = mp_truth(A, b)
        nb = np.linalg.norm(b)
        if not (np.linalg.norm(z - zt) <= 1e-15 * nb and np.linalg.norm(p - pt) <= 1e-15 * nb
                and np.linalg.norm(x - xt) <= 1e-15 * np.linalg.norm(xt)):
            return False
    return True


def qrcp_pins_pass(lib):
    for rows, cols, seed in [(40, 10, 1), (100, 37, 3)]:
        M = graded(rows, cols, seed)
        R, piv = oracle.qrcp(M, lib=lib)
        _, Rl, pl = sl.qr(M, mode="economic", pivoting=True)
        if not np.array_equal(piv, pl):
            return False
        if not np.allclose(np.abs(R), np.abs(Rl), atol=1e-12 * np.abs(np.diag(Rl))[:, None], rtol=0):
            return False
    M = np.zeros((6, 4))
    M[0, 1] = 2.0; M[1, 3] = 2.0; M[2, 0] = 1.0; M[3, 2] = 1.0
    return oracle.qrcp(M, lib=lib)[1].tolist() == [1, 3, 0, 2]


def test_unmutated_copy_passes(tmp_path):
    lib = build_mutant(tmp_path, "int orc_num_threads(void)", "int orc_num_threads(void)")
    assert projection_pins_pass(lib) and qrcp_pins_pass(lib) and project_r_pins_pass(lib)


@pytest.mark.parametrize("name", sorted(PROJECTION_MUTANTS))
def test_projection_mutant_is_caught(tmp_path, name):
    lib = build_mutant(tmp_path, *PROJECTION_MUTANTS[name])
    assert not projection_pins_pass(lib), name


@pytest.mark.parametrize("name", sorted(PROJECT_R_MUTANTS))
def test_project_r_mutant_is_caught(tmp_path, name):
    lib = build_mutant(tmp_path, *PROJECT_R_MUTANTS[name])
    assert not project_r_pins_pass(lib), name


@pytest.mark.parametrize("name", sorted(QRCP_MUTANTS))
def test_qrcp_mutant_is_caught(tmp_path, name):
    lib = build_mutant(tmp_path, *QRCP_MUTANTS[name])
    assert not qrcp_pins_pass(lib), name
