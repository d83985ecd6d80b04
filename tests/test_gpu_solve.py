"""GPU solve parity against the FP64 oracle through the C ABI (pr_solve,
pr_dual_bound): lower bounds, certified dual values, one-step and few-step
iterate maps, node edge cases, and full-size workloads checked by properties
the oracle verifies at any size (weak duality certificate of the returned
primal/dual pair)."""
import math

import numpy as np
import pytest

import oracle
from workloads import make_instance, make_nodes, config_instance

pytestmark = pytest.mark.gpu


def _pr():
    import paper_2603_01306_amd as pr
    return pr


def _ctx(dev, inst):
    import torch
    pr = _pr()
    if inst.Xcm.dtype == np.uint16:
        X = torch.from_numpy(inst.Xcm.view(np.int16)).to(dev).view(torch.bfloat16)
    else:
        X = torch.from_numpy(inst.Xcm).to(dev)
    return pr.Context(X, torch.from_numpy(inst.y).to(dev), inst.loss)


@pytest.fixture(scope="module")
def c1(dev):
    inst = config_instance("ls_root_n500_p200_f64")
    ctx = _ctx(dev, inst)
    lam = float(np.linalg.eigvalsh(inst.X64() @ inst.X64().T).max())
    yield inst, ctx, lam
    ctx.close()


def test_c1_root_lower_bound_parity(c1):
    """Least-squares root relaxation, n=500, p=200, FP64, solved to 1e-8."""
    inst, ctx, lam = c1
    pr = _pr()
    L = 2.0 * lam
    res = ctx.solve(pr.Node(10, 1.0, 2.0), want_zeta=True, rel_gap_tol=1e-8, L=L)
    ref = oracle.solve(inst.Xcm, inst.y, 0, 1.0, 2.0, 10, L=L, tol=1e-11)
    print("gpu", {k: v for k, v in res.items() if k not in ("beta", "zeta")}, "oracle", ref["lb"], ref["iters"])
    assert res["status"] == pr.CONVERGED
    assert abs(res["lower_bound"] - ref["lb"]) <= 1e-8 * abs(res["primal"])
    # the bound is Psi of the returned zeta, recomputed by the oracle in FP64
    psi = oracle.dual(inst.Xcm, inst.y, res["zeta"].cpu().numpy(), 0, 1.0, 2.0, 10)
    assert abs(psi - res["lower_bound"]) <= 1e-12 * abs(psi)
    # and the returned beta attains the reported primal value
    phi = oracle.primal(inst.Xcm, inst.y, res["beta"].cpu().numpy(), 0, 1.0, 2.0, 10)
    assert abs(phi - res["primal"]) <= 1e-12 * abs(phi)
    assert (phi - psi) / abs(phi) <= 1e-8
    # pr_dual_bound agrees with both
    lb2, ph2 = ctx.dual_bound(pr.Node(10, 1.0, 2.0), zeta=res["zeta"], beta=res["beta"])
    assert abs(lb2 - psi) <= 1e-12 * abs(psi) and abs(ph2 - phi) <= 1e-12 * abs(phi)
    # same iteration sequence as the oracle: both restart on the same gap test
    assert abs(res["iters"] - ref["iters"]) <= max(3, ref["iters"] // 10) or ref["iters"] > res["iters"]


@pytest.mark.parametrize("steps", [1, 2, 5])
def test_c1_few_step_iterates_match(c1, steps):
    """With the same step constant, the first iterates of FISTA agree with the
    oracle's to FP64 round-off (beyond a few steps trajectories are only
    compared through their end values)."""
    inst, ctx, lam = c1
    pr = _pr()
    L = 2.0 * lam * 1.01
    node = pr.Node(10, 1.0, 2.0, J0=[3, 7, 11], J1=[0, 20])
    st = node.status(inst.p)
    res = ctx.solve(node, max_iter=steps, L=L, rel_gap_tol=0.0)
    ref = oracle.solve(inst.Xcm, inst.y, 0, 1.0, 2.0, 10, status=st, L=L, tol=0.0, max_iter=steps)
    assert res["iters"] == steps and res["status"] == pr.MAXITER
    assert abs(res["lower_bound"] - ref["lb"]) <= 1e-11 * abs(ref["lb"])
    assert abs(res["primal"] - ref["ub"]) <= 1e-11 * abs(ref["ub"])


@pytest.mark.parametrize("loss", [0, 1])
@pytest.mark.parametrize("node_seed", [0, 1, 2])
def test_small_nodes_lower_bound_parity(dev, loss, node_seed):
    inst = make_instance(n=1024, p=300, corr=0.7, k_true=8, snr=5.0, loss=loss, seed=11 + loss,
                         storage="f32")
    ctx = _ctx(dev, inst)
    pr = _pr()
    J0, J1 = make_nodes(inst.p, 1, seed=node_seed, max_j0=40, max_j1=6)[0]
    node = pr.Node(8, 0.3, 2.0, J0=J0, J1=J1)
    st = node.status(inst.p)
    lam = float(np.linalg.eigvalsh(inst.X64() @ inst.X64().T).max())
    L = (2.0 if loss == 0 else 0.25) * lam
    res = ctx.solve(node, want_zeta=True, rel_gap_tol=1e-7, L=L)
    ref = oracle.solve(inst.Xcm, inst.y, loss, 0.3, 2.0, 8, status=st, L=L, tol=1e-10)
    print(res["iters"], ref["iters"], res["lower_bound"], ref["lb"])
    assert res["status"] == pr.CONVERGED
    assert abs(res["lower_bound"] - ref["lb"]) <= 1e-6 * abs(ref["lb"])
    psi = oracle.dual(inst.Xcm, inst.y, res["zeta"].cpu().numpy(), loss, 0.3, 2.0, 8, status=st)
    assert abs(psi - res["lower_bound"]) <= 1e-11 * abs(psi)
    ctx.close()


@pytest.mark.parametrize("loss", [0, 1])
def test_default_step_on_mirrored_design(dev, loss):
    """Default L (from the context's ||X||_2^2) on X = [A, -A], whose top
    eigenvector is orthogonal to the all-ones direction: the solve converges
    to the oracle's bound, the oracle run with the exact eigenvalue."""
    import torch
    pr = _pr()
    inst = make_instance(n=600, p=60, corr=0.6, k_true=4, snr=5.0, loss=loss, seed=21, storage="f64")
    Xcm = np.ascontiguousarray(np.concatenate([inst.Xcm, -inst.Xcm], axis=0))
    ctx = pr.Context(torch.from_numpy(Xcm).to(dev), torch.from_numpy(inst.y).to(dev), loss)
    A = inst.X64()
    lam = 2.0 * float(np.linalg.eigvalsh(A @ A.T).max())
    node = pr.Node(5, 0.5, 2.0)
    res = ctx.solve(node, rel_gap_tol=1e-8, max_iter=20000)
    assert abs(res["L"] - 1.01 * (2.0 if loss == 0 else 0.25) * lam) <= 1e-9 * res["L"]
    ref = oracle.solve(Xcm, inst.y, loss, 0.5, 2.0, 5, L=1.01 * (2.0 if loss == 0 else 0.25) * lam, tol=1e-10)
    print(res["iters"], ref["iters"], res["lower_bound"], ref["lb"])
    assert res["status"] == pr.CONVERGED
    assert abs(res["lower_bound"] - ref["lb"]) <= 1e-7 * abs(ref["lb"])
    ctx.close()


@pytest.mark.parametrize("p,n,lam2", [(1000, 256, 0.5), (1500, 256, 0.75), (3000, 256, 1.5), (6000, 256, 3.0),
                                      (8192, 256, 4.0), (16000, 256, 8.0), (16384, 128, 8.0), (17000, 128, 20.0)])
@pytest.mark.parametrize("loss", [0, 1])
def test_node_step_tiers_match_oracle(dev, p, n, lam2, loss):
    """The per-node step keeps 2, 4, 8, 16 or 32 entries per thread in
    registers for p <= 1024, 2048, 4096, 8192, 16384 (the 16- and 32-entry
    tiers are the ones the full-size roots run) and switches to the strided
    kernel over HBM vectors beyond 16384 entries: first iterates and the
    converged bound agree with the oracle on each tier, p ragged against the
    workgroup and exactly at the tier limits."""
    inst = make_instance(n=n, p=p, corr=0.5, k_true=6, snr=5.0, loss=loss, seed=40 + loss, storage="f32")
    ctx = _ctx(dev, inst)
    pr = _pr()
    J0, J1 = make_nodes(inst.p, 1, seed=p, max_j0=60, max_j1=4)[0]
    node = pr.Node(6, lam2, 2.0, J0=J0, J1=J1)
    st = node.status(inst.p)
    lam = float(np.linalg.eigvalsh(inst.X64() @ inst.X64().T).max())
    L = (2.0 if loss == 0 else 0.25) * lam * 1.01
    few = ctx.solve(node, max_iter=3, L=L, rel_gap_tol=0.0)
    ref3 = oracle.solve(inst.Xcm, inst.y, loss, lam2, 2.0, 6, status=st, L=L, tol=0.0, max_iter=3)
    assert few["iters"] == 3
    assert abs(few["lower_bound"] - ref3["lb"]) <= 1e-11 * abs(ref3["ub"])
    assert abs(few["primal"] - ref3["ub"]) <= 1e-11 * abs(ref3["ub"])
    res = ctx.solve(node, want_zeta=True, rel_gap_tol=1e-7, L=L)
    ref = oracle.solve(inst.Xcm, inst.y, loss, lam2, 2.0, 6, status=st, L=L, tol=1e-8)
    print(p, loss, res["iters"], ref["iters"], res["lower_bound"], ref["lb"])
    assert res["status"] == pr.CONVERGED
    assert abs(res["lower_bound"] - ref["lb"]) <= 1e-6 * abs(ref["ub"])
    psi = oracle.dual(inst.Xcm, inst.y, res["zeta"].cpu().numpy(), loss, lam2, 2.0, 6, status=st)
    assert abs(psi - res["lower_bound"]) <= 1e-11 * abs(psi)
    ctx.close()


def test_node_edge_cases(c1):
    inst, ctx, lam = c1
    pr = _pr()
    # |J1| > k: infeasible, bound +inf, call succeeds
    res = ctx.solve(pr.Node(2, 1.0, 2.0, J1=[0, 1, 2]))
    assert res["status"] == pr.INFEASIBLE and res["lower_bound"] == math.inf
    # overlapping J0 / J1 and bad parameters are rejected
    with pytest.raises(pr.PrError):
        ctx.solve(pr.Node(5, 1.0, 2.0, J0=[4], J1=[4]))
    with pytest.raises(pr.PrError):
        ctx.solve(pr.Node(0, 1.0, 2.0))
    with pytest.raises(pr.PrError):
        ctx.solve(pr.Node(5, -1.0, 2.0))
    with pytest.raises(pr.PrError):
        ctx.solve(pr.Node(5, 1.0, 2.0, J0=[inst.p]))
    # leaf node (|J1| = k, everything else fixed to zero): restricted box ridge
    S = [0, 20, 40]
    node = pr.Node(3, 1.0, 100.0, J0=[j for j in range(inst.p) if j not in S], J1=S)
    res = ctx.solve(node, rel_gap_tol=1e-10, L=2.0 * lam)
    Xs = inst.X64()[S].T
    b = np.linalg.solve(Xs.T @ Xs + 1.0 * np.eye(3), Xs.T @ inst.y)
    closed = float(np.sum((inst.y - Xs @ b) ** 2) + 1.0 * b @ b)
    assert abs(res["lower_bound"] - closed) <= 1e-9 * closed


def test_cutoff_and_maxiter(c1):
    """Cutoff decisions and the iterate that takes them equal the oracle's
    (same step L); an iteration limit still reports a valid bound."""
    inst, ctx, lam = c1
    pr = _pr()
    lam = 2.0 * lam * 1.01                       # the step constant L of both runs
    ref = oracle.solve(inst.Xcm, inst.y, 0, 1.0, 2.0, 10, L=lam, tol=1e-10)
    for cutoff, want in ((ref["lb"] * 0.99, pr.CUTOFF_PRUNE), (ref["lb"] * 1.01, pr.CUTOFF_BRANCH),
                         (ref["lb"] * 0.5, pr.CUTOFF_PRUNE), (ref["ub"] * 1.5, pr.CUTOFF_BRANCH)):
        r = ctx.solve(pr.Node(10, 1.0, 2.0), cutoff=cutoff, L=lam, want_zeta=True, rel_gap_tol=1e-10)
        o = oracle.solve(inst.Xcm, inst.y, 0, 1.0, 2.0, 10, L=lam, tol=1e-10, cutoff=cutoff)
        assert r["status"] == o["status"] == want, (cutoff, r["status"], o["status"])
        assert r["iters"] == o["iters"]
        if want == pr.CUTOFF_PRUNE:
            assert r["lower_bound"] >= cutoff
            assert abs(r["lower_bound"] - o["lb"]) <= 1e-10 * abs(o["lb"])
            psi = oracle.dual(inst.Xcm, inst.y, r["zeta"].cpu().numpy(), 0, 1.0, 2.0, 10)
            assert abs(psi - r["lower_bound"]) <= 1e-12 * abs(psi)
        else:
            assert r["primal"] <= cutoff
            assert abs(r["primal"] - o["ub"]) <= 1e-10 * abs(o["ub"])
    r3 = ctx.solve(pr.Node(10, 1.0, 2.0), max_iter=3, rel_gap_tol=0.0, L=lam)
    o3 = oracle.solve(inst.Xcm, inst.y, 0, 1.0, 2.0, 10, L=lam, tol=0.0, max_iter=3)
    assert r3["status"] == pr.MAXITER and r3["iters"] == 3 and o3["iters"] == 3
    assert abs(r3["lower_bound"] - o3["lb"]) <= 1e-10 * abs(ref["ub"])
    assert r3["lower_bound"] <= ref["lb"] * (1 + 1e-12)   # still a valid bound


def test_warm_start_and_determinism(c1):
    import torch
    inst, ctx, lam = c1
    pr = _pr()
    a = ctx.solve(pr.Node(10, 1.0, 2.0), rel_gap_tol=1e-8)
    b = ctx.solve(pr.Node(10, 1.0, 2.0), rel_gap_tol=1e-8)
    assert a["lower_bound"] == b["lower_bound"] and a["iters"] == b["iters"]
    assert torch.equal(a["beta"], b["beta"])
    # warm start from the solution converges at once
    w = ctx.solve(pr.Node(10, 1.0, 2.0), beta0=a["beta"], rel_gap_tol=1e-6)
    assert w["iters"] <= 5 and w["status"] == pr.CONVERGED
    # child node warm-started from the parent (parent beta is off the child's
    # domain on J0): same bound as a cold start
    child = pr.Node(10, 1.0, 2.0, J0=[int(torch.argmax(a["beta"].abs()))])
    cw = ctx.solve(child, beta0=a["beta"], rel_gap_tol=1e-8)
    cc = ctx.solve(child, rel_gap_tol=1e-8)
    assert abs(cw["lower_bound"] - cc["lower_bound"]) <= 2e-8 * abs(cc["primal"])
    assert cc["lower_bound"] >= a["lower_bound"] - 1e-8 * abs(a["primal"])   # child >= parent


@pytest.mark.parametrize("method", ["fixed", "bt"])
def test_graph_length_does_not_change_the_solve(c1, method):
    """The host queues captured iterations by its prediction of the stop (long
    graphs, then a short tail graph): the solve is the same, bit for bit, for
    every graph length, and an iteration limit that falls inside a graph
    stops it exactly there."""
    import torch
    inst, ctx, lam = c1
    pr = _pr()
    kw = {} if method == "fixed" else {"method": pr.FISTA_BT_GAP}
    runs = [ctx.solve(pr.Node(10, 1.0, 2.0), rel_gap_tol=1e-9, check_every=ce, **kw) for ce in (2, 6, 8, 32, 64)]
    a = runs[0]
    assert a["status"] == pr.CONVERGED
    for r in runs[1:]:
        assert r["lower_bound"] == a["lower_bound"] and r["primal"] == a["primal"]
        assert (r["iters"], r["trials"], r["restarts"]) == (a["iters"], a["trials"], a["restarts"])
        assert torch.equal(r["beta"], a["beta"])
    for ce, cap in ((32, 37), (64, 9), (8, 41)):
        r = ctx.solve(pr.Node(10, 1.0, 2.0), rel_gap_tol=0.0, max_iter=cap, check_every=ce, **kw)
        assert r["status"] == pr.MAXITER and r["iters"] == cap


# ----------------------------------------------------------------- full size

@pytest.fixture(scope="module")
def c2(dev):
    inst = config_instance("ls_root_n16384_p8192_f32")
    ctx = _ctx(dev, inst)
    yield inst, ctx
    ctx.close()


def test_c2_full_size_certificate(c2):
    """n=16384, p=8192, FP32 X, FP64 gap, 1e-6: the oracle recomputes Psi of the
    returned zeta and Phi of the returned beta over the stored X in FP64; the
    pair certifies the bound to 1e-6 relative."""
    inst, ctx = c2
    pr = _pr()
    res = ctx.solve(pr.Node(20, 0.1, 2.0), want_zeta=True)
    print({k: v for k, v in res.items() if k not in ("beta", "zeta")})
    assert res["status"] == pr.CONVERGED
    psi = oracle.dual(inst.Xcm, inst.y, res["zeta"].cpu().numpy(), 0, 0.1, 2.0, 20)
    phi = oracle.primal(inst.Xcm, inst.y, res["beta"].cpu().numpy(), 0, 0.1, 2.0, 20)
    assert abs(psi - res["lower_bound"]) <= 1e-10 * abs(psi)
    assert abs(phi - res["primal"]) <= 1e-10 * abs(phi)
    assert 0.0 <= (phi - psi) / abs(phi) <= 1e-6


def test_c2_sampled_gemv_t(c2, dev):
    import torch
    inst, ctx = c2
    rng = np.random.default_rng(0)
    r = rng.standard_normal(inst.n)
    h = ctx.gemv_t(torch.from_numpy(r).to(dev)).cpu().numpy()
    cols = rng.choice(inst.p, 64, replace=False)
    for j in cols:
        ref = float(inst.Xcm[j].astype(np.float64) @ r)
        assert abs(h[j] - ref) <= 1e-12 * float(np.abs(inst.Xcm[j].astype(np.float64)) @ np.abs(r))


def test_c3_logistic_full_size_certificate(dev):
    """n=32768, p=16384 logistic, FP32 X, FP64 gap, 1e-6."""
    inst = config_instance("logistic_root_n32768_p16384_f32")
    ctx = _ctx(dev, inst)
    pr = _pr()
    res = ctx.solve(pr.Node(15, 0.1, 2.0), want_zeta=True)
    print({k: v for k, v in res.items() if k not in ("beta", "zeta")})
    assert res["status"] == pr.CONVERGED
    psi = oracle.dual(inst.Xcm, inst.y, res["zeta"].cpu().numpy(), 1, 0.1, 2.0, 15)
    phi = oracle.primal(inst.Xcm, inst.y, res["beta"].cpu().numpy(), 1, 0.1, 2.0, 15)
    assert abs(psi - res["lower_bound"]) <= 1e-10 * abs(psi)
    assert abs(phi - res["primal"]) <= 1e-10 * abs(phi)
    assert 0.0 <= (phi - psi) / abs(phi) <= 1e-6
    ctx.close()
