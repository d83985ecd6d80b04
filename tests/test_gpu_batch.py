"""Batched node relaxations (pr_solve_batch): both products of the iteration
are FP64 MFMA GEMMs over the stored design (BF16, FP32 or FP64; least squares
or logistic, the latter with two right-hand sides per node in the transposed
product), every stopped node is re-certified over the stored X.  Checked node
by node against the FP64 oracle on small instances (converged bounds and
few-step iterates), against the single-node GPU path, and at full size by the
oracle re-certifying the returned (beta, bound) pairs."""
import math

import numpy as np
import pytest

import oracle
from workloads import make_instance, make_nodes, config_instance

pytestmark = pytest.mark.gpu


def _pr():
    import paper_2603_01306_amd as pr
    return pr


def _ctx(dev, inst, max_batch):
    import torch
    pr = _pr()
    if inst.storage == "bf16":
        X = torch.from_numpy(inst.Xcm.view(np.int16)).to(dev).view(torch.bfloat16)
    else:
        X = torch.from_numpy(inst.Xcm).to(dev)
    c = pr.Context(X, torch.from_numpy(inst.y).to(dev), inst.loss, max_batch=max_batch)
    if max_batch > 1:
        c.set_debug(pr.DEBUG_FORCE_BATCH)   # the batched path even where one at a time would be cheaper
    return c


def _zeta(inst, beta):
    """Dual vector induced by beta: least squares 2 (y - X beta), logistic
    -grad F(X beta) = y / (1 + exp(y X beta))."""
    u = inst.X64().T @ beta
    if inst.loss == 0:
        return 2.0 * (inst.y - u)
    return inst.y / (1.0 + np.exp(inst.y * u))


@pytest.mark.parametrize("loss,storage", [(1, "bf16"), (1, "f32"), (1, "f64"), (0, "f32"), (0, "f64")])
def test_batch_loss_and_storage_match_oracle_per_node(dev, loss, storage):
    """Logistic nodes and FP32 / FP64 designs on the batched path: every node
    converges to the oracle's bound, and Phi(beta) and Psi(zeta(beta)) of the
    returned pair, recomputed by the oracle over the stored X, equal the
    reported values."""
    pr = _pr()
    inst = make_instance(n=1024, p=512, corr=0.8, k_true=8, snr=5.0, loss=loss, seed=40 + loss, storage=storage)
    ctx = _ctx(dev, inst, 16)
    raw = make_nodes(inst.p, 11, seed=4, max_j0=40, max_j1=6)
    nodes = [pr.Node(8, 0.2, 2.0, J0=a, J1=b) for a, b in raw]
    res, B = ctx.solve_batch(nodes, rel_gap_tol=1e-7, max_iter=20000)
    B = B.cpu().numpy()
    for i, (nd, r) in enumerate(zip(nodes, res)):
        st = nd.status(inst.p)
        ref = oracle.solve(inst.Xcm, inst.y, loss, 0.2, 2.0, 8, status=st, L=r["L"], tol=1e-10)
        print(i, r["iters"], ref["iters"], r["lower_bound"], ref["lb"], r["rel_gap"], flush=True)
        assert r["status"] == pr.CONVERGED and r["rel_gap"] <= 1e-7
        assert abs(r["lower_bound"] - ref["lb"]) <= 1.5e-7 * abs(r["primal"])
        assert r["lower_bound"] <= ref["ub"] * (1 + 1e-12)
        phi = oracle.primal(inst.Xcm, inst.y, B[i], loss, 0.2, 2.0, 8, status=st)
        psi = oracle.dual(inst.Xcm, inst.y, _zeta(inst, B[i]), loss, 0.2, 2.0, 8, status=st)
        assert abs(phi - r["primal"]) <= 1e-11 * abs(phi)
        assert abs(psi - r["lower_bound"]) <= 1e-10 * abs(phi)
    ctx.close()


@pytest.mark.parametrize("loss,storage", [(1, "f32"), (1, "bf16"), (0, "f64"), (0, "f32")])
@pytest.mark.parametrize("K", [1, 6, 40])
def test_batch_iterates_match_oracle(dev, loss, storage, K):
    """After exactly K iterations (iteration limit, no convergence) each
    node's returned iterate equals the oracle's x^K with the same step, to
    FP64 summation-order differences: the batched momentum, restart and (for
    logistic) gradient at the momentum point follow the method step by step."""
    pr = _pr()
    inst = make_instance(n=1024, p=512, corr=0.8, k_true=8, snr=5.0, loss=loss, seed=50 + loss, storage=storage)
    ctx = _ctx(dev, inst, 16)
    raw = make_nodes(inst.p, 7, seed=6, max_j0=40, max_j1=6)
    nodes = [pr.Node(8, 0.2, 2.0, J0=a, J1=b) for a, b in raw]
    res, B = ctx.solve_batch(nodes, rel_gap_tol=1e-15, max_iter=K, check_every=2)
    B = B.cpu().numpy()
    for i, (nd, r) in enumerate(zip(nodes, res)):
        st = nd.status(inst.p)
        ref = oracle.solve(inst.Xcm, inst.y, loss, 0.2, 2.0, 8, status=st, L=r["L"], tol=-1.0, max_iter=K)
        assert r["status"] == pr.MAXITER and r["iters"] == K == ref["iters"]
        # the oracle also tests the restart at its last iterate, the batch stops first
        assert ref["restarts"] - 1 <= r["restarts"] <= ref["restarts"]
        scale = max(1.0, float(np.max(np.abs(ref["beta"]))))
        err = float(np.max(np.abs(B[i] - ref["beta"])))
        print(K, i, r["restarts"], ref["restarts"], err, flush=True)
        assert err <= 1e-12 * scale
    ctx.close()


@pytest.fixture(scope="module")
def small(dev):
    inst = make_instance(n=1024, p=512, corr=0.8, k_true=8, snr=5.0, loss=0, seed=21, storage="bf16")
    ctx = _ctx(dev, inst, 16)
    yield inst, ctx
    ctx.close()


def test_batch_small_matches_oracle_per_node(small):
    inst, ctx = small
    pr = _pr()
    raw = make_nodes(inst.p, 11, seed=3, max_j0=40, max_j1=6)
    nodes = [pr.Node(8, 0.2, 2.0, J0=a, J1=b) for a, b in raw]
    nodes.append(pr.Node(3, 0.2, 2.0, J1=[1, 2, 3, 4]))    # infeasible: |J1| > k
    res, B = ctx.solve_batch(nodes, rel_gap_tol=1e-7)
    lam = float(np.linalg.eigvalsh(inst.X64() @ inst.X64().T).max())
    for i, (nd, r) in enumerate(zip(nodes, res)):
        if i == len(nodes) - 1:
            assert r["status"] == pr.INFEASIBLE and r["lower_bound"] == math.inf
            continue
        st = nd.status(inst.p)
        ref = oracle.solve(inst.Xcm, inst.y, 0, 0.2, 2.0, 8, status=st, L=2.02 * lam, tol=1e-10)
        print(i, r["iters"], ref["iters"], r["lower_bound"], ref["lb"], r["rel_gap"])
        assert r["status"] == pr.CONVERGED and r["rel_gap"] <= 1e-7
        assert abs(r["lower_bound"] - ref["lb"]) <= 1.5e-7 * abs(r["primal"])
        # the returned beta attains the reported primal value (oracle recomputation)
        # and the bound is valid: below the oracle's upper bound
        beta = B[i].cpu().numpy()
        phi = oracle.primal(inst.Xcm, inst.y, beta, 0, 0.2, 2.0, 8, status=st)
        assert abs(phi - r["primal"]) <= 1e-11 * abs(phi)
        assert r["lower_bound"] <= ref["ub"] * (1 + 1e-12)


def test_batch_agrees_with_single_node_path(small):
    inst, ctx = small
    pr = _pr()
    raw = make_nodes(inst.p, 6, seed=9, max_j0=30, max_j1=5)
    nodes = [pr.Node(8, 0.2, 2.0, J0=a, J1=b) for a, b in raw]
    res, _ = ctx.solve_batch(nodes, rel_gap_tol=1e-7)
    for nd, r in zip(nodes, res):
        s = ctx.solve(nd, rel_gap_tol=1e-7)
        assert abs(s["lower_bound"] - r["lower_bound"]) <= 2e-7 * abs(s["primal"])


def test_batch_warm_start_and_repeat(small):
    import torch
    inst, ctx = small
    pr = _pr()
    raw = make_nodes(inst.p, 4, seed=5, max_j0=20, max_j1=4)
    nodes = [pr.Node(8, 0.2, 2.0, J0=a, J1=b) for a, b in raw]
    r1, B1 = ctx.solve_batch(nodes, rel_gap_tol=1e-7)
    r2, _ = ctx.solve_batch(nodes, rel_gap_tol=1e-7)
    assert [a["lower_bound"] for a in r1] == [b["lower_bound"] for b in r2]   # deterministic
    rw, _ = ctx.solve_batch(nodes, B0=B1, rel_gap_tol=1e-7)
    for a, b in zip(r1, rw):
        assert b["iters"] <= max(5, a["iters"] // 4)
        assert abs(a["lower_bound"] - b["lower_bound"]) <= 2e-7 * abs(a["primal"])


@pytest.mark.parametrize("gram", [False, True])
@pytest.mark.parametrize("max_iter", [1, 7, 40])
def test_batch_iteration_limit_reports_certified_values(dev, gram, max_iter):
    """Nodes stopped by the iteration limit (the graph loop ends before they
    converge, so their iterate is taken from the working buffer of either
    parity) report Phi of the returned beta and Psi of zeta = 2 (y - X beta),
    both recomputed by the oracle over the stored X, and a bound no higher
    than the relaxation's optimum."""
    pr = _pr()
    inst = make_instance(n=1024, p=512, corr=0.8, k_true=8, snr=5.0, loss=0, seed=21, storage="bf16")
    ctx = _ctx(dev, inst, 16)
    if gram:
        ctx.enable_gram()
    raw = make_nodes(inst.p, 10, seed=8, max_j0=30, max_j1=5)
    nodes = [pr.Node(8, 0.2, 2.0, J0=a, J1=b) for a, b in raw]
    res, B = ctx.solve_batch(nodes, rel_gap_tol=1e-9, max_iter=max_iter, check_every=2)
    B = B.cpu().numpy()
    X64 = inst.X64()
    for q, (nd, r) in enumerate(zip(nodes, res)):
        st = nd.status(inst.p)
        assert r["status"] in (pr.MAXITER, pr.CONVERGED), r
        phi = oracle.primal(inst.Xcm, inst.y, B[q], 0, 0.2, 2.0, 8, status=st)
        zeta = 2.0 * (inst.y - X64.T @ B[q])
        psi = oracle.dual(inst.Xcm, inst.y, zeta, 0, 0.2, 2.0, 8, status=st)
        assert abs(phi - r["primal"]) <= 1e-10 * abs(phi), (q, phi, r)
        assert abs(psi - r["lower_bound"]) <= 1e-9 * abs(phi), (q, psi, r)
        ref = oracle.solve(inst.Xcm, inst.y, 0, 0.2, 2.0, 8, status=st, tol=1e-10)
        assert r["lower_bound"] <= ref["ub"] * (1 + 1e-12) and r["primal"] >= ref["lb"] * (1 - 1e-12)
    ctx.close()


def test_batch_full_size_256_nodes(dev):
    """256 nodes on the BF16 copy of the n=16384, p=8192 design; the oracle
    re-certifies 8 seeded nodes from the returned betas."""
    pr = _pr()
    inst = config_instance("ls_batch256_n16384_p8192_bf16")
    ctx = _ctx(dev, inst, 256)
    raw = make_nodes(inst.p, 256, seed=1, max_j0=64, max_j1=19)
    nodes = [pr.Node(20, 0.1, 2.0, J0=a, J1=b) for a, b in raw]
    res, B = ctx.solve_batch(nodes, max_iter=4000)
    ku, kp, nout = ctx.batch_union_size()
    print("iters", sorted(r["iters"] for r in res)[::32], "union", ku, kp, nout, flush=True)
    assert all(r["status"] == pr.CONVERGED and r["rel_gap"] <= 1e-6 for r in res)
    # the forward product ran compacted to the support union, and every node
    # finished in the batched iteration (no fallback to the single-node path,
    # which would take thousands of iterations)
    assert 0 < ku <= kp < inst.p
    assert max(r["iters"] for r in res) < 1000
    for i in np.random.default_rng(0).choice(256, 8, replace=False):
        st = nodes[i].status(inst.p)
        beta = B[i].cpu().numpy()
        phi = oracle.primal(inst.Xcm, inst.y, beta, 0, 0.1, 2.0, 20, status=st)
        assert abs(phi - res[i]["primal"]) <= 1e-10 * abs(phi)
        # the reported bound is Psi of the dual vector induced by the returned
        # iterate, zeta = 2 (y - X beta), recomputed over the stored X
        zeta = 2.0 * (inst.y - oracle.matvec(inst.Xcm, beta))
        psi = oracle.dual(inst.Xcm, inst.y, zeta, 0, 0.1, 2.0, 20, status=st)
        assert abs(psi - res[i]["lower_bound"]) <= 1e-10 * abs(psi), (i, psi, res[i])
        assert 0.0 <= (phi - psi) / abs(phi) <= 1e-6
    ctx.close()


@pytest.mark.parametrize("Mc,Nr,K,KS", [(128, 64, 32, 1), (256, 192, 1024, 2), (1024, 512, 4096, 4), (384, 128, 96, 3),
                                         (128, 64, 160, 5)])
def test_gemm_matches_float64_reference(dev, Mc, Nr, K, KS):
    """FP64 MFMA product over a BF16 A: within FP64 summation error of the
    exact product, |C - C_ref| <= 2 K 2^-53 (|B| |A|^T) per split."""
    import torch
    pr = _pr()
    g = torch.Generator().manual_seed(Mc + K)
    A = torch.randn(Mc, K, generator=g).to(torch.bfloat16)
    B = torch.randn(Nr, K, generator=g, dtype=torch.float64)
    C = pr.gemm(A.to(dev), B.to(dev), KS).cpu()
    Ad = A.double()
    kc = K // KS
    for z in range(KS):
        sl = slice(z * kc, (z + 1) * kc)
        ref = B[:, sl] @ Ad[:, sl].T     # (Nr, Mc)
        bound = 2.0 * kc * 2.0 ** -53 * (B[:, sl].abs() @ Ad[:, sl].abs().T) + 1e-300
        assert torch.all((C[z] - ref).abs() <= bound)


def test_gemm_rejects_bad_shapes(dev):
    import torch
    pr = _pr()
    A = torch.zeros(100, 64, dtype=torch.bfloat16, device=dev)
    B = torch.zeros(64, 64, dtype=torch.float64, device=dev)
    with pytest.raises(pr.PrError):
        pr.gemm(A, B)           # Mc not a multiple of 128
    A = torch.zeros(128, 64, dtype=torch.bfloat16, device=dev)
    with pytest.raises(pr.PrError):
        pr.gemm(A, B, KS=3)     # K not a multiple of 32 * KS


@pytest.mark.parametrize("loss,storage", [(0, "bf16"), (1, "f32"), (0, "f32")])
@pytest.mark.parametrize("K", [1, 6, 40])
def test_batch_backtracking_iterates_match_oracle(dev, loss, storage, K):
    """FISTA with backtracking and the gap restart on the batched path: after
    exactly K accepted iterations each node's iterate equals the oracle's
    x^K (same L0, growth and cap), with the same number of rejected trials."""
    pr = _pr()
    inst = make_instance(n=1024, p=512, corr=0.8, k_true=8, snr=5.0, loss=loss, seed=60 + loss, storage=storage)
    ctx = _ctx(dev, inst, 16)
    raw = make_nodes(inst.p, 7, seed=7, max_j0=40, max_j1=6)
    nodes = [pr.Node(8, 0.2, 2.0, J0=a, J1=b) for a, b in raw]
    Lmax = (2.0 if loss == 0 else 0.25) * 1.01 * ctx.norm2()
    res, B = ctx.solve_batch(nodes, rel_gap_tol=1e-15, max_iter=K, check_every=2, method=pr.FISTA_BT_GAP,
                             L=Lmax, L0=Lmax / 16.0, acfgm_c=2.0)
    B = B.cpu().numpy()
    for i, (nd, r) in enumerate(zip(nodes, res)):
        st = nd.status(inst.p)
        # a node may close its gap to rounding level (1e-15) before K; it is
        # then compared at the iterate where it stopped
        assert r["iters"] == K or (r["status"] == pr.CONVERGED and r["rel_gap"] <= 1e-14), r
        kk = r["iters"]
        ref = oracle.solve_bt(inst.Xcm, inst.y, loss, 0.2, 2.0, 8, status=st, L0=Lmax / 16.0, c=2.0, Lmax=Lmax,
                              tol=-1.0, max_iter=kk)
        scale = max(1.0, float(np.max(np.abs(ref["beta"]))))
        err = float(np.max(np.abs(B[i] - ref["beta"])))
        print(K, i, r["iters"], r["trials"], ref["rejected"], r["restarts"], ref["restarts"], err, flush=True)
        assert ref["iters"] == kk and (kk < K or r["status"] == pr.MAXITER)
        assert err <= 1e-12 * scale
        if kk < K:
            continue       # at a gap of 1e-15 the model test compares rounding noise: counts may differ
        assert r["trials"] == ref["rejected"]
        assert ref["restarts"] - 1 <= r["restarts"] <= ref["restarts"]
    ctx.close()


@pytest.mark.parametrize("loss,storage", [(0, "bf16"), (1, "f32")])
def test_batch_backtracking_converges_per_node(dev, loss, storage):
    """Batched FISTA with backtracking to 1e-7: every node's bound against the
    oracle's and its returned pair recertified by the oracle; fewer
    evaluations than the batched fixed step."""
    pr = _pr()
    inst = make_instance(n=1024, p=512, corr=0.8, k_true=8, snr=5.0, loss=loss, seed=40 + loss, storage=storage)
    ctx = _ctx(dev, inst, 16)
    raw = make_nodes(inst.p, 11, seed=4, max_j0=40, max_j1=6)
    nodes = [pr.Node(8, 0.2, 2.0, J0=a, J1=b) for a, b in raw]
    res, B = ctx.solve_batch(nodes, rel_gap_tol=1e-7, max_iter=20000, method=pr.FISTA_BT_GAP)
    fixed, _ = ctx.solve_batch(nodes, rel_gap_tol=1e-7, max_iter=20000, want_beta=False)
    B = B.cpu().numpy()
    for i, (nd, r) in enumerate(zip(nodes, res)):
        st = nd.status(inst.p)
        ref = oracle.solve(inst.Xcm, inst.y, loss, 0.2, 2.0, 8, status=st, tol=1e-10)
        assert r["status"] == pr.CONVERGED and r["rel_gap"] <= 1e-7
        assert abs(r["lower_bound"] - ref["lb"]) <= 1.5e-7 * abs(r["primal"])
        phi = oracle.primal(inst.Xcm, inst.y, B[i], loss, 0.2, 2.0, 8, status=st)
        psi = oracle.dual(inst.Xcm, inst.y, _zeta(inst, B[i]), loss, 0.2, 2.0, 8, status=st)
        assert abs(phi - r["primal"]) <= 1e-11 * abs(phi) and abs(psi - r["lower_bound"]) <= 1e-10 * abs(phi)
    ev_bt = sum(r["iters"] + r["trials"] for r in res)
    ev_fx = sum(r["iters"] for r in fixed)
    print("evaluations: backtracking", ev_bt, "fixed step", ev_fx, flush=True)
    assert ev_bt < ev_fx
    ctx.close()


@pytest.mark.parametrize("loss,storage", [(0, "bf16"), (1, "f32")])
def test_batch_cost_rule_and_tail_handoff(dev, loss, storage):
    """Without the test switch the batch may run a round one node at a time and
    hand its last nodes to the single-node path: every node still converges
    with the bound of the forced batched run, and its returned pair
    recertifies over the stored X."""
    pr = _pr()
    inst = make_instance(n=1024, p=512, corr=0.8, k_true=8, snr=5.0, loss=loss, seed=90 + loss, storage=storage)
    ctx = _ctx(dev, inst, 16)
    raw = make_nodes(inst.p, 12, seed=11, max_j0=40, max_j1=6)
    nodes = [pr.Node(8, 0.2, 2.0, J0=a, J1=b) for a, b in raw]
    forced, _ = ctx.solve_batch(nodes, rel_gap_tol=1e-7, method=pr.FISTA_BT_GAP)
    ctx.set_debug(0)
    for sub in (nodes, nodes[:1], nodes[:3]):
        res, B = ctx.solve_batch(sub, rel_gap_tol=1e-7, method=pr.FISTA_BT_GAP)
        B = B.cpu().numpy()
        for i, (nd, r, f) in enumerate(zip(sub, res, forced)):
            st = nd.status(inst.p)
            assert r["status"] == pr.CONVERGED and r["rel_gap"] <= 1e-7, r
            assert abs(r["lower_bound"] - f["lower_bound"]) <= 2e-7 * abs(f["primal"])
            phi = oracle.primal(inst.Xcm, inst.y, B[i], loss, 0.2, 2.0, 8, status=st)
            psi = oracle.dual(inst.Xcm, inst.y, _zeta(inst, B[i]), loss, 0.2, 2.0, 8, status=st)
            assert abs(phi - r["primal"]) <= 1e-11 * abs(phi) and psi <= r["lower_bound"] + 1e-10 * abs(phi)
    ctx.close()


def test_batch_full_size_logistic_fp32(dev):
    """64 logistic nodes on the FP32 n=32768, p=16384 design: every node
    converges on the batched path, and the oracle recomputes Phi and Psi at
    the returned pairs of 4 seeded nodes over the stored X."""
    pr = _pr()
    inst = config_instance("logistic_root_n32768_p16384_f32")
    ctx = _ctx(dev, inst, 64)
    raw = make_nodes(inst.p, 64, seed=2, max_j0=64, max_j1=14)
    nodes = [pr.Node(15, 0.1, 2.0, J0=a, J1=b) for a, b in raw]
    res, B = ctx.solve_batch(nodes, max_iter=6000)
    print("iters", sorted(r["iters"] for r in res)[::8], "union", ctx.batch_union_size(), flush=True)
    assert all(r["status"] == pr.CONVERGED and r["rel_gap"] <= 1e-6 for r in res)
    for i in np.random.default_rng(1).choice(64, 4, replace=False):
        st = nodes[i].status(inst.p)
        beta = B[i].cpu().numpy()
        phi = oracle.primal(inst.Xcm, inst.y, beta, 1, 0.1, 2.0, 15, status=st)
        psi = oracle.dual(inst.Xcm, inst.y, _zeta(inst, beta), 1, 0.1, 2.0, 15, status=st)
        assert abs(phi - res[i]["primal"]) <= 1e-10 * abs(phi)
        assert abs(psi - res[i]["lower_bound"]) <= 1e-10 * abs(phi)
        assert 0.0 <= (phi - psi) / abs(phi) <= 1e-6
    ctx.close()
