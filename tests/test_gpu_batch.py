"""Batched path (grouped launches, optional HIP graph) vs the CPU oracle,
member by member, through the C ABI (marker: gpu).  Same tolerance as a
single plan: <= 1e-10 relative for z, the row projection and x."""
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


def members(count, seed, m_lo=8, m_hi=160, j_lo=4, j_hi=24, k_hi=9):
    shp = synth.make_batch_shapes(count, seed, m_lo=m_lo, m_hi=m_hi, j_lo=j_lo, j_hi=j_hi, k_lo=1, k_hi=k_hi)
    return shp


def check_member(A, B, Z, Y, X):
    Zr, Yr, Xr, _ = oracle.project(A, B.T)
    nb = np.linalg.norm(B, axis=1)
    ez = np.max(np.linalg.norm(Z - Zr.T, axis=1) / nb)
    ey = np.max(np.linalg.norm(Y - Yr.T, axis=1) / nb)
    ex = np.max(np.linalg.norm(X - Xr.T, axis=1) / np.linalg.norm(Xr.T, axis=1))
    return ez, ey, ex


@pytest.mark.parametrize("graph,k_hi", [(False, 9), (True, 9), (True, 40)])
def test_batch_matches_oracle(rt, graph, k_hi):
    shp = members(10, 71, k_hi=k_hi)
    As = [synth.make_problem(m, n, 1e6, 100 + i) for i, (m, n) in enumerate(zip(shp.m, shp.n))]
    Bs = [synth.make_rhs(n, k, 200 + i) for i, (n, k) in enumerate(zip(shp.n, shp.k))]
    bt = rt.Batch(shp.m, shp.n, shp.l, 5)
    bt.set_graph(graph)
    At = [torch.from_numpy(A).to(dev()) for A in As]
    Bt = [torch.from_numpy(B).to(dev()) for B in Bs]
    bt.precondition(At)
    Z, Y, X = bt.project_all(Bt)
    assert bt.status() == [0] * len(As)
    for i in range(len(As)):
        e = check_member(As[i], Bs[i], Z[i].cpu().numpy(), Y[i].cpu().numpy(), X[i].cpu().numpy())
        assert max(e) <= TOL, (i, shp.m[i], shp.n[i], e)
    bt.close()


def test_batch_graph_replay_sees_new_data(rt):
    """Two preconditions and projections with the same buffers: the second
    call replays the captured graphs and must see the new contents."""
    shp = members(6, 72, m_hi=96)
    bt = rt.Batch(shp.m, shp.n, shp.l, 9)
    bt.set_graph(True)
    At = [torch.empty((m, n), dtype=torch.float64, device=dev()) for m, n in zip(shp.m, shp.n)]
    Bt = [torch.empty((k, n), dtype=torch.float64, device=dev()) for n, k in zip(shp.n, shp.k)]
    Z = [torch.empty_like(B) for B in Bt]
    Y = [torch.empty_like(B) for B in Bt]
    X = [torch.empty((k, m), dtype=torch.float64, device=dev()) for m, k in zip(shp.m, shp.k)]
    for rep in range(3):
        As = [synth.make_problem(m, n, 1e4, 300 + 10 * rep + i) for i, (m, n) in enumerate(zip(shp.m, shp.n))]
        Bs = [synth.make_rhs(n, k, 400 + 10 * rep + i) for i, (n, k) in enumerate(zip(shp.n, shp.k))]
        for t, a in zip(At, As):
            t.copy_(torch.from_numpy(a))
        for t, b in zip(Bt, Bs):
            t.copy_(torch.from_numpy(b))
        torch.cuda.synchronize()
        bt.precondition(At)
        bt.project_all(Bt, Z, Y, X)
        torch.cuda.synchronize()
        assert bt.status() == [0] * len(As)
        for i in range(len(As)):
            e = check_member(As[i], Bs[i], Z[i].cpu().numpy(), Y[i].cpu().numpy(), X[i].cpu().numpy())
            assert max(e) <= TOL, (rep, i, e)
    bt.close()


def test_batch_status_flags_rank_deficient_member(rt):
    shp = members(4, 73, m_hi=64)
    As = [synth.make_problem(m, n, 1e3, 500 + i) for i, (m, n) in enumerate(zip(shp.m, shp.n))]
    As[2][-1] = As[2][0]  # duplicate row: rank m - 1
    bt = rt.Batch(shp.m, shp.n, shp.l, 3)
    bt.precondition([torch.from_numpy(A).to(dev()) for A in As])
    st = bt.status()
    assert st[2] == 5 and st[0] == st[1] == st[3] == 0, st
    bt.close()


def test_batch_member_equals_single_plan(rt):
    """A batch of one equals the same problem through a plan (both binary64,
    same sketch seed derivation, same refinement count)."""
    m, n, l, k, seed = 48, 3000, 192, 3, 11
    A = synth.make_problem(m, n, 1e6, 1)
    B = synth.make_rhs(n, k, 1)
    bt = rt.Batch([m], [n], [l], seed)
    bt.precondition([torch.from_numpy(A).to(dev())])
    Z, Y, X = bt.project_all([torch.from_numpy(B).to(dev())])
    e = check_member(A, B, Z[0].cpu().numpy(), Y[0].cpu().numpy(), X[0].cpu().numpy())
    assert max(e) <= TOL, e
    bt.close()


@pytest.mark.parametrize("k", [3, 40])
def test_batch_column_scaled_members_match_oracle(rt, k):
    """Interior-point shape: one base A, member t works on A diag(d_t) with
    d_t = 10^U(-6, 6), the scaling applied by every pass that reads A (no
    scaled copy); each member against the oracle on the scaled matrix formed
    on the host.  k = 40 takes the MFMA forms of the plain products (D b
    formed first, scaled GEMM outputs), k = 3 the vector forms."""
    m, n, l, steps = 40, 1500, 160, 4
    A = synth.make_problem(m, n, 1e4, 77)
    D = synth.make_scalings(n, steps, 77)
    Bs = [synth.make_rhs(n, k, 900 + t) for t in range(steps)]
    bt = rt.Batch([m] * steps, [n] * steps, [l] * steps, 13)
    bt.set_graph(True)
    At = torch.from_numpy(A).to(dev())
    Dt = [torch.from_numpy(np.ascontiguousarray(D[t])).to(dev()) for t in range(steps)]
    for rep in range(2):  # the second call replays the captured graphs
        bt.precondition([At] * steps, Dt)
        Z, Y, X = bt.project_all([torch.from_numpy(B).to(dev()) for B in Bs])
        assert bt.status() == [0] * steps
        for t in range(steps):
            e = check_member(A * D[t][None, :], Bs[t], Z[t].cpu().numpy(), Y[t].cpu().numpy(), X[t].cpu().numpy())
            assert max(e) <= TOL, (rep, t, e)
    bt.close()


def test_batch_member_tables_match_oracle(rt):
    """Member i's sketch tables are the oracle's tables for the instance seed
    of i (the first SplitMix64 output of seed XOR i), bit for bit."""
    seed = 20091214
    ms, ns = [8, 40, 17], [100, 2000, 544]
    ls = [4 * m for m in ms]
    bt = rt.Batch(ms, ns, ls, seed)
    for i in range(3):
        got = bt.member_tables(i)
        ref = oracle.srft_tables(oracle.instance_seed(seed, i), ns[i], ls[i])
        for key in ["np", "n1", "n2"]:
            assert got[key] == ref[key]
        for key in ["sign", "sigma", "tau", "J"]:
            assert np.array_equal(got[key], ref[key]), (i, key)
    bt.close()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_binary32_gram_matches_oracle(rt, graph):
    """Batches with the binary32 grouped Gram (rtproj_batch_set_precision):
    every member within 1e-10 of the oracle after the refinement."""
    shp = members(12, 20091215, m_hi=200)
    As = [synth.make_problem(m, n, 1e6, 300 + i) for i, (m, n) in enumerate(zip(shp.m, shp.n))]
    Bs = [synth.make_rhs(n, k, 400 + i) for i, (n, k) in enumerate(zip(shp.n, shp.k))]
    bt = rt.Batch(shp.m, shp.n, shp.l, 77)
    bt.set_precision(rt.PREC_MIXED_FP32)
    bt.set_graph(graph)
    At = [torch.from_numpy(A).to(dev()) for A in As]
    Bt = [torch.from_numpy(B).to(dev()) for B in Bs]
    for _ in range(2 if graph else 1):
        bt.precondition(At)
        Z, Y, X = bt.project_all(Bt)
    assert all(s == 0 for s in bt.status())
    assert bt.member_info(0)["gram_bits"] == 32
    for i in range(len(As)):
        e = check_member(As[i], Bs[i], Z[i].cpu().numpy(), Y[i].cpu().numpy(), X[i].cpu().numpy())
        assert max(e) <= TOL, (i, e)
    with pytest.raises(rt.RtprojError) as err:
        bt.set_precision(rt.PREC_MIXED_BF16)
    assert err.value.status == 7
    bt.close()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_split_bf16_gram_matches_oracle(rt, graph):
    """Batches with the grouped split-bfloat16 Gram of binary32 P^{-1}A
    (lower 256 x 128 tiles, members of uneven m: ragged tiles, tiles right of
    a member's column m, members with fewer K splits): every member within
    1e-10 of the oracle after the refinement, twice when replayed from the
    graph."""
    ms = [40, 130, 257, 300, 96]
    ns = [8 * m for m in ms]
    ls = [4 * m for m in ms]
    ks = [3, 1, 5, 2, 4]
    As = [synth.make_problem(m, n, 1e6, 310 + i) for i, (m, n) in enumerate(zip(ms, ns))]
    Bs = [synth.make_rhs(n, k, 410 + i) for i, (n, k) in enumerate(zip(ns, ks))]
    bt = rt.Batch(ms, ns, ls, 78)
    bt.set_precision(rt.PREC_MIXED_BF16X3)
    bt.set_graph(graph)
    At = [torch.from_numpy(A).to(dev()) for A in As]
    Bt = [torch.from_numpy(B).to(dev()) for B in Bs]
    for rep in range(2 if graph else 1):
        bt.precondition(At)
        Z, Y, X = bt.project_all(Bt)
        assert all(s == 0 for s in bt.status())
        assert all(bt.member_info(i)["gram_bits"] == 17 for i in range(len(ms)))
        for i in range(len(As)):
            e = check_member(As[i], Bs[i], Z[i].cpu().numpy(), Y[i].cpu().numpy(), X[i].cpu().numpy())
            assert max(e) <= TOL, (rep, i, e)
    bt.close()


def test_batch_split_bf16_gram_column_scaled_and_fallback(rt):
    """The interior-point shape with the split-bfloat16 Gram (P^{-1}A written
    in binary32 with its column scaling), and a batch with a member whose n
    is not a multiple of 4, which takes the binary32 Gram for all members."""
    m, n, l, steps = 64, 2048, 256, 3
    A = synth.make_problem(m, n, 1e4, 79)
    D = synth.make_scalings(n, steps, 79)
    Bs = [synth.make_rhs(n, 5, 950 + t) for t in range(steps)]
    bt = rt.Batch([m] * steps, [n] * steps, [l] * steps, 14)
    bt.set_precision(rt.PREC_MIXED_BF16X3)
    At = torch.from_numpy(A).to(dev())
    Dt = [torch.from_numpy(np.ascontiguousarray(D[t])).to(dev()) for t in range(steps)]
    bt.precondition([At] * steps, Dt)
    Z, Y, X = bt.project_all([torch.from_numpy(B).to(dev()) for B in Bs])
    assert bt.status() == [0] * steps
    assert bt.member_info(0)["gram_bits"] == 17
    for t in range(steps):
        e = check_member(A * D[t][None, :], Bs[t], Z[t].cpu().numpy(), Y[t].cpu().numpy(), X[t].cpu().numpy())
        assert max(e) <= TOL, (t, e)
    bt.close()
    ms, ns = [48, 64], [1000, 1002]
    As = [synth.make_problem(mm, nn, 1e5, 320 + i) for i, (mm, nn) in enumerate(zip(ms, ns))]
    Bs = [synth.make_rhs(nn, 2, 420 + i) for i, nn in enumerate(ns)]
    bt = rt.Batch(ms, ns, [4 * mm for mm in ms], 15)
    bt.set_precision(rt.PREC_MIXED_BF16X3)
    bt.precondition([torch.from_numpy(A).to(dev()) for A in As])
    Z, Y, X = bt.project_all([torch.from_numpy(B).to(dev()) for B in Bs])
    assert bt.status() == [0, 0]
    assert bt.member_info(1)["gram_bits"] == 32
    for i in range(2):
        e = check_member(As[i], Bs[i], Z[i].cpu().numpy(), Y[i].cpu().numpy(), X[i].cpu().numpy())
        assert max(e) <= TOL, (i, e)
    bt.close()


@pytest.mark.parametrize("prec", [0, 3])
def test_batch_long_rows_column_scaled(rt, prec):
    """Members long enough for the pipelined grouped sketch passes (2^16-point
    transforms, n short of the padded length, odd m), each on A diag(d_t).
    A wrong sketch would still refine to the right projection, so each
    member's Gram condition estimate (1.5-3 for a sound preconditioner) is
    checked too, and in binary64 its rank estimate against a single plan's
    on the scaled matrix with the member's seed (the same sketch)."""
    m, n, l, steps, seed = 37, 65436, 148, 3, 16
    A = synth.make_problem(m, n, 1e4, 81)
    # d_t = 10^U(-3, 3) keeps R's trailing diagonal accurate enough to compare
    # rank estimates; 10^U(-1, 1) keeps the binary32 sketch (no escalation)
    lo = 3.0 if prec == 0 else 1.0
    D = 10.0 ** np.random.default_rng(81).uniform(-lo, lo, size=(steps, n))
    Bs = [synth.make_rhs(n, 3, 960 + t) for t in range(steps)]
    bt = rt.Batch([m] * steps, [n] * steps, [l] * steps, seed)
    bt.set_precision(prec)
    bt.set_graph(True)
    At = torch.from_numpy(A).to(dev())
    Dt = [torch.from_numpy(np.ascontiguousarray(D[t])).to(dev()) for t in range(steps)]
    for rep in range(2):  # the second call replays the captured graphs
        bt.precondition([At] * steps, Dt)
        Z, Y, X = bt.project_all([torch.from_numpy(B).to(dev()) for B in Bs])
        assert bt.status() == [0] * steps
        for t in range(steps):
            info = bt.member_info(t)
            assert info["sketch_bits"] == (64 if prec == 0 else 32), (t, info["sketch_bits"])
            assert info["gram_cond_est"] <= 10.0, (rep, t, info["gram_cond_est"])
            e = check_member(A * D[t][None, :], Bs[t], Z[t].cpu().numpy(), Y[t].cpu().numpy(), X[t].cpu().numpy())
            assert max(e) <= TOL, (rep, t, e)
    if prec == 0:
        for t in range(steps):
            plan = rt.Plan(m, n, l, oracle.instance_seed(seed, t))
            plan.precondition(torch.from_numpy(A * D[t][None, :]).to(dev()))
            k_plan, k_member = plan.info()["kappa_est"], bt.member_info(t)["kappa_est"]
            assert abs(k_member - k_plan) <= 1e-4 * k_plan, (t, k_member, k_plan)
            plan.close()
    bt.close()


@pytest.mark.parametrize("prec", [1, 3])
def test_batch_binary32_sketch_escalates_for_an_ill_conditioned_member(rt, prec):
    """The reduced batch precisions sketch in binary32; a member with
    cond(A) = 1e10 makes that sketch too coarse (2^-24 kappa_est > 1), so the
    batch sketches every member again in binary64, and all of them still
    match the oracle.  Without such a member the sketch stays binary32."""
    ms, ns = [48, 64], [1024, 2048]
    for kappas, want_bits in (([1e5, 1e5], 32), ([1e5, 1e10], 64)):
        As = [synth.make_problem(m, n, kp, 330 + i) for i, (m, n, kp) in enumerate(zip(ms, ns, kappas))]
        Bs = [synth.make_rhs(n, 3, 430 + i) for i, n in enumerate(ns)]
        bt = rt.Batch(ms, ns, [4 * m for m in ms], 16)
        bt.set_precision(prec)
        bt.precondition([torch.from_numpy(A).to(dev()) for A in As])
        Z, Y, X = bt.project_all([torch.from_numpy(B).to(dev()) for B in Bs])
        assert bt.status() == [0, 0]
        for i in range(2):
            info = bt.member_info(i)
            assert info["sketch_bits"] == want_bits and info["sketch_escalated"] == (1 if want_bits == 64 else 0)
            e = check_member(As[i], Bs[i], Z[i].cpu().numpy(), Y[i].cpu().numpy(), X[i].cpu().numpy())
            assert max(e) <= TOL, (kappas, i, e)
        bt.close()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_grouped_pivoted_qr_matches_oracle(rt, graph):
    """Few large members: the pivoted QR of R0 runs as a group of blocks per
    member (each group with its own barrier; chosen over one workgroup per
    member for these sizes).  The second call replays the captured graphs, so
    the groups' arrival counters must start from zero again."""
    ms = [640, 300, 520]
    ns = [8 * m for m in ms]
    ls = [4 * m for m in ms]
    As = [synth.make_problem(m, n, 1e8, 1300 + i) for i, (m, n) in enumerate(zip(ms, ns))]
    Bs = [synth.make_rhs(n, 2, 1400 + i) for i, n in enumerate(ns)]
    bt = rt.Batch(ms, ns, ls, 23)
    bt.set_graph(graph)
    At = [torch.from_numpy(A).to(dev()) for A in As]
    Bt = [torch.from_numpy(B).to(dev()) for B in Bs]
    for rep in range(2):
        bt.precondition(At)
        assert bt.info()["qr_mode"] == rt.QR_TWO_STAGE
        Z, Y, X = bt.project_all(Bt)
        assert bt.status() == [0] * len(As)
        for i in range(len(As)):
            e = check_member(As[i], Bs[i], Z[i].cpu().numpy(), Y[i].cpu().numpy(), X[i].cpu().numpy())
            print(f"rep {rep} member {i} m {ms[i]}: e_z {e[0]:.3g} e_p {e[1]:.3g} e_x {e[2]:.3g}")
            assert max(e) <= TOL, (rep, i, e)
    bt.close()


def test_batch_grouped_pivoted_qr_flags_rank_deficient_member(rt):
    ms = [520, 600]
    ns = [6 * m for m in ms]
    ls = [4 * m for m in ms]
    As = [synth.make_problem(m, n, 1e3, 1500 + i) for i, (m, n) in enumerate(zip(ms, ns))]
    As[1][-1] = As[1][0]  # duplicate row: rank m - 1
    bt = rt.Batch(ms, ns, ls, 29)
    bt.precondition([torch.from_numpy(A).to(dev()) for A in As])
    assert bt.info()["qr_mode"] == rt.QR_TWO_STAGE
    st = bt.status()
    assert st[1] == 5 and st[0] == 0, st
    bt.close()
