"""rtproj_project_all_noalloc against rtproj_project_all (marker: gpu).

The allocation-free entry point takes its workspace from the library's
static device array; its results must match the allocating entry point's
(same kernels; the split counts can differ with k, so the bar is the
projection tolerance, 1e-10 relative) and the oracle's, on two calls in a
row where the second has a smaller input (fewer right-hand sides, then a
smaller plan), so stale contents of the shared array must not leak in.
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


def rel(a, b, scale):
    return float(np.max(np.linalg.norm(a - b, axis=1) / scale))


def run_both(rt, plan, B):
    k = B.shape[0]
    Bt = torch.from_numpy(B).to(dev())
    Za, Ya, Xa = plan.project_all(Bt)
    Zn = torch.full_like(Bt, float("nan"))
    Yn = torch.full_like(Bt, float("nan"))
    Xn = torch.full((k, plan.m), float("nan"), dtype=torch.float64, device=dev())
    plan.project_all_noalloc(Bt, Zn, Yn, Xn)
    torch.cuda.synchronize()
    plan.status()
    return [t.cpu().numpy() for t in (Za, Ya, Xa, Zn, Yn, Xn)]


def test_noalloc_matches_allocating_entry_point(rt):
    cases = [(100, 5000, 400, 1e8, 7, 81), (100, 5000, 400, 1e8, 3, 81), (40, 2000, 160, 1e6, 2, 82)]
    plans = {}
    for (m, n, l, kappa, k, seed) in cases:
        A = synth.make_problem(m, n, kappa, seed)
        B = synth.make_rhs(n, k, seed)
        if (m, n) not in plans:
            plans[(m, n)] = rt.Plan(m, n, l, seed)
            plans[(m, n)].precondition(torch.from_numpy(A).to(dev()))
        plan = plans[(m, n)]
        Za, Ya, Xa, Zn, Yn, Xn = run_both(rt, plan, B)
        nb = np.linalg.norm(B, axis=1)
        assert np.all(np.isfinite(Zn)) and np.all(np.isfinite(Yn)) and np.all(np.isfinite(Xn))
        assert rel(Zn, Za, nb) <= TOL and rel(Yn, Ya, nb) <= TOL
        assert rel(Xn, Xa, np.linalg.norm(Xa, axis=1)) <= TOL
        Zr, Yr, Xr, _ = oracle.project(A, B.T)
        assert rel(Zn, Zr.T, nb) <= TOL and rel(Yn, Yr.T, nb) <= TOL
        assert rel(Xn, Xr.T, np.linalg.norm(Xr.T, axis=1)) <= TOL
    for p in plans.values():
        p.close()


def test_noalloc_rejects_a_workspace_above_its_limit(rt):
    m, n, l = 64, 262144, 256
    A = synth.make_problem(m, n, 1e3, 83)
    plan = rt.Plan(m, n, l, 83)
    plan.precondition(torch.from_numpy(A).to(dev()))
    k = 40  # r alone is n k doubles = 80 MiB
    B = torch.zeros((k, n), dtype=torch.float64, device=dev())
    Z = torch.empty_like(B)
    with pytest.raises(rt.RtprojError) as e:
        plan.project_all_noalloc(B, Z, None, None)
    assert e.value.status == 7
    plan.close()
