"""The autotuner of P^{-1}A and its Gram (marker: gpu): a tuning precondition
fills the process-wide table, the tuned plan matches the oracle, and the
table survives a save / load round trip."""
import os

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


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_autotuned_plan_matches_oracle(rt, prec, tmp_path):
    m, n, l, k, seed = 300, 12000, 1200, 3, 131 + prec
    A = synth.make_problem(m, n, 1e6, seed)
    B = synth.make_rhs(n, k, seed)
    before = rt.autotune_entries()
    plan = rt.Plan(m, n, l, seed)
    plan.set_precision(prec)
    plan.set_autotune(True)
    At = torch.from_numpy(A).to("cuda")
    plan.precondition(At)          # tunes this shape
    plan.precondition(At)          # uses the table
    Z, Y, X = [t.cpu().numpy() for t in plan.project_all(torch.from_numpy(B).to("cuda"))]
    plan.status()
    assert rt.autotune_entries() >= before + (2 if before == 0 else 0)
    Zr, Yr, Xr, _ = oracle.project(A, B.T)
    nb = np.linalg.norm(B, axis=1)
    assert np.max(np.linalg.norm(Z - Zr.T, axis=1) / nb) <= TOL
    assert np.max(np.linalg.norm(X - Xr.T, axis=1) / np.linalg.norm(Xr.T, axis=1)) <= TOL
    path = str(tmp_path / "tune.txt")
    rt.autotune_save(path)
    lines = [ln.split() for ln in open(path) if ln.strip()]
    assert len(lines) == rt.autotune_entries() and all(":" in ln[0] and len(ln) >= 2 for ln in lines)
    rt.autotune_load(path)
    assert rt.autotune_entries() == len(lines)
    bad = str(tmp_path / "bad.txt")
    open(bad, "w").write("not-a-key 1\n")
    with pytest.raises(rt.RtprojError):
        rt.autotune_load(bad)
    plan.close()


@pytest.mark.parametrize("cfg", ["64 1 0", "64 2 0", "64 2 128", "128 1 64"])
def test_forced_product_configuration_matches_oracle(rt, cfg, tmp_path):
    """P^{-1}A in a configuration set through a loaded table (tile, order,
    tile_n): the plain and XCD-grouped orders with square and rectangular
    tiles at 1024 rows."""
    m, n, l, k, seed = 1024, 8192, 4096, 3, 151
    A = synth.make_problem(m, n, 1e6, seed)
    B = synth.make_rhs(n, k, seed)
    path = str(tmp_path / "forced.txt")
    open(path, "w").write(f"w64:{m}x{n}x0 {cfg}\n")
    rt.autotune_load(path)
    plan = rt.Plan(m, n, l, seed)
    plan.set_autotune(True)
    plan.precondition(torch.from_numpy(A).to("cuda"))
    Z, Y, X = [t.cpu().numpy() for t in plan.project_all(torch.from_numpy(B).to("cuda"))]
    plan.status()
    Zr, Yr, Xr, _ = oracle.project(A, B.T)
    nb = np.linalg.norm(B, axis=1)
    assert np.max(np.linalg.norm(Z - Zr.T, axis=1) / nb) <= TOL
    assert np.max(np.linalg.norm(Y - Yr.T, axis=1) / nb) <= TOL
    assert np.max(np.linalg.norm(X - Xr.T, axis=1) / np.linalg.norm(Xr.T, axis=1)) <= TOL
    plan.close()
