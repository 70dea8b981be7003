"""Compensated refinement products on the int8 matrix cores against the
Dot2 form and the oracle (marker: gpu).

The integer form evaluates r = b - A^T x and s = A r exactly on a digit grid
(13 signed 6-bit digits per operand on one power-of-two scale per row and per
right-hand side, digit pairs s + t <= 14 kept): both forms are accurate far
beyond binary64, so their refined projections agree to about the rounding of
the outputs, and both meet the oracle at 1e-10.  Cases cover sizes that are
not multiples of the 64-wide tiles, more than 64 right-hand sides, fewer
than 16 (the integer form forced), and all-zero columns of A (no scale).
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


def rel_err(B, Z, Zr):
    return float(np.max(np.linalg.norm(Z - Zr, axis=1) / np.linalg.norm(B, axis=1)))


def run(rt, A, B, l, seed, comp, steps):
    m, n = A.shape
    plan = rt.Plan(m, n, l, seed)
    plan.set_compensation(comp)
    plan.set_refinement(steps, 0.0)
    plan.precondition(torch.from_numpy(A).to(dev()))
    Z, Y, X = [t.cpu().numpy() for t in plan.project_all(torch.from_numpy(np.ascontiguousarray(B)).to(dev()))]
    plan.status()  # raises when the refinement did not converge
    info = plan.info()
    plan.close()
    return Z, Y, X, info["refine_status"], info


@pytest.mark.timeout(600)
@pytest.mark.parametrize("case", [
    # (m, n, l, kappa, k, seed, compensated steps)
    (256, 16384, 1024, 1e8, 32, 81, 2),     # tile multiples
    (200, 6000, 800, 1e10, 17, 82, 2),      # ragged m and n
    (130, 9000, 520, 1e6, 70, 83, 1),       # more than 64 right-hand sides, ragged
    (96, 4100, 384, 1e8, 3, 84, 2),         # fewer than 16 right-hand sides (integer form forced)
])
def test_int8_products_match_dot2_and_oracle(rt, case):
    m, n, l, kappa, k, seed, steps = case
    A = synth.make_problem(m, n, kappa, seed)
    B = synth.make_rhs(n, k, seed)
    Zr, Yr, Xr, _ = oracle.project(A, B.T)
    Zi, Yi, Xi, sti, infoi = run(rt, A, B, l, seed, rt.COMP_INT8, steps)
    Zd, Yd, Xd, std, infod = run(rt, A, B, l, seed, rt.COMP_DOT2, steps)
    ez_i, ey_i = rel_err(B, Zi, Zr.T), rel_err(B, Yi, Yr.T)
    ez_d = rel_err(B, Zd, Zr.T)
    ex_i = float(np.max(np.linalg.norm(Xi - Xr.T, axis=1) / np.linalg.norm(Xr.T, axis=1)))
    agree = rel_err(B, Zi, Zd)
    print(f"case {case}: int8 e_z {ez_i:.3g} e_p {ey_i:.3g} e_x {ex_i:.3g}; dot2 e_z {ez_d:.3g}; "
          f"int8 vs dot2 {agree:.3g}; comp {infoi['comp_method']}/{infod['comp_method']}")
    assert infoi["comp_method"] == rt.COMP_INT8 and infod["comp_method"] == rt.COMP_DOT2
    assert sti == 0 and std == 0
    assert max(ez_i, ey_i, ex_i) <= TOL and ez_d <= TOL
    assert agree <= 1e-12, agree


def test_int8_with_zero_columns(rt):
    """All-zero columns of A have no scale: their digits are zero and their
    residual entries are b itself."""
    m, n, l, k, seed = 128, 8192, 512, 24, 85
    A = synth.make_problem(m, n, 1e6, seed)
    A[:, [0, 77, 4095, n - 1]] = 0.0
    B = synth.make_rhs(n, k, seed)
    Zr, Yr, Xr, _ = oracle.project(A, B.T)
    Z, Y, X, st, info = run(rt, A, B, l, seed, rt.COMP_INT8, 2)
    assert info["comp_method"] == rt.COMP_INT8 and st == 0
    assert rel_err(B, Z, Zr.T) <= TOL and rel_err(B, Y, Yr.T) <= TOL
    assert np.array_equal(Z[:, [0, 77, 4095, n - 1]], B[:, [0, 77, 4095, n - 1]])


def test_automatic_form_follows_the_number_of_right_hand_sides(rt):
    m, n, l, seed = 96, 4096, 384, 86
    A = synth.make_problem(m, n, 1e8, seed)
    for k, want in ((4, rt.COMP_DOT2), (16, rt.COMP_INT8)):
        B = synth.make_rhs(n, k, seed)
        Z, Y, X, st, info = run(rt, A, B, l, seed, rt.COMP_AUTO, 1)
        assert info["comp_method"] == want, (k, info["comp_method"])
