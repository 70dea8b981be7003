"""Complex-valued A through the C ABI (rtproj_cplan_*) against the complex
oracle (marker: gpu): x = argmin |A^* x - b|, A^* x and b - A^* x with the
conjugate transpose, <= 1e-10 relative (z and the row projection relative to
|b|, x relative to |x|), max over right-hand sides."""
import numpy as np
import pytest

from oracle import complex_oracle
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


def errors(B, Z, Y, X, Zr, Yr, Xr):
    nb = np.linalg.norm(B, axis=1)
    return (np.max(np.linalg.norm(Z - Zr.T, axis=1) / nb), np.max(np.linalg.norm(Y - Yr.T, axis=1) / nb),
            np.max(np.linalg.norm(X - Xr.T, axis=1) / np.linalg.norm(Xr.T, axis=1)))


@pytest.mark.parametrize("m,n,l,kappa,k,seed,prec", [
    (40, 2000, 160, 1e4, 3, 101, 0),
    (64, 4096, 256, 1e8, 2, 102, 0),
    (130, 9000, 520, 1e6, 5, 103, 0),
    (100, 5000, 400, 1e6, 40, 104, 1),      # binary32 sketch and Gram; 40 right-hand sides
])
def test_complex_projection_matches_oracle(rt, m, n, l, kappa, k, seed, prec):
    A = synth.make_complex_problem(m, n, kappa, seed)
    B = synth.make_complex_rhs(n, k, seed)
    plan = rt.CPlan(m, n, l, seed)
    plan.real.set_precision(prec)
    plan.precondition(torch.from_numpy(A).to(dev()))
    Z, Y, X = [t.cpu().numpy() for t in plan.project_all(torch.from_numpy(B).to(dev()))]
    plan.real.status()
    Zr, Yr, Xr, _ = complex_oracle.project_complex(A, B.T)
    e = errors(B, Z, Y, X, Zr, Yr, Xr)
    assert max(e) <= TOL, e
    plan.close()


def test_complex_projector_is_hermitian_and_idempotent(rt):
    m, n = 6, 64
    A = synth.make_complex_problem(m, n, 1e3, 105)
    plan = rt.CPlan(m, n, 24, 105)
    plan.precondition(torch.from_numpy(A).to(dev()))
    Z, _, _ = plan.project_all(torch.eye(n, dtype=torch.complex128, device=dev()))
    Zm = Z.cpu().numpy().T     # column c of the projector = Z applied to e_c
    assert np.abs(Zm - Zm.conj().T).max() <= 1e-14
    assert np.abs(Zm @ Zm - Zm).max() <= 1e-14
    assert np.abs(A @ Zm).max() <= 1e-14
    plan.close()


def test_real_input_through_the_complex_plan(rt):
    """A real A given as complex agrees with the real plan's results."""
    m, n, l, k = 50, 3000, 200, 2
    A = synth.make_problem(m, n, 1e6, 106)
    B = synth.make_rhs(n, k, 106)
    cplan = rt.CPlan(m, n, l, 106)
    cplan.precondition(torch.from_numpy(A.astype(np.complex128)).to(dev()))
    Zc, Yc, Xc = [t.cpu().numpy() for t in cplan.project_all(torch.from_numpy(B.astype(np.complex128)).to(dev()))]
    plan = rt.Plan(m, n, l, 106)
    plan.precondition(torch.from_numpy(A).to(dev()))
    Zr, Yr, Xr = [t.cpu().numpy() for t in plan.project_all(torch.from_numpy(B).to(dev()))]
    nb = np.linalg.norm(B, axis=1)
    assert np.max(np.linalg.norm(Zc - Zr, axis=1) / nb) <= TOL
    assert np.max(np.abs(Zc.imag)) <= 1e-12 * np.max(np.abs(Zc))
    assert np.max(np.linalg.norm(Xc - Xr, axis=1) / np.linalg.norm(Xr, axis=1)) <= TOL
    cplan.close()
    plan.close()
