"""Branch and bound on the GPU (pr_bnb) and the batched dynamic termination
it relies on: the certified lower bound never exceeds the exact k-sparse
optimum found by enumeration, the incumbent's objective is exact and reaches
that optimum when the tree closes, and batched prune / branch decisions agree
with the single-node path."""
import math

import numpy as np
import pytest

import oracle
from oracle.ksparse import ksparse_bruteforce, ksparse_bruteforce_logistic
from workloads import make_instance

pytestmark = pytest.mark.gpu


def _ctx(inst, dev, max_batch):
    import torch
    import paper_2603_01306_amd as pr
    if inst.storage == "bf16":
        X = torch.from_numpy(inst.Xcm.view(np.int16)).to(dev).view(torch.bfloat16)
    else:
        X = torch.from_numpy(inst.Xcm).to(dev)
    c = pr.Context(X, torch.from_numpy(inst.y).to(dev), inst.loss, max_batch=max_batch)
    if max_batch > 1:
        c.set_debug(pr.DEBUG_FORCE_BATCH)   # the batched path even for rounds one at a time would win
    return c


def _objective(X, y, b, lam2):
    return float(np.sum((y - X @ b) ** 2) + lam2 * b @ b)


@pytest.mark.parametrize("seed,k,lam2,J0,J1", [(3, 4, 0.5, (), ()), (4, 3, 1.0, (2,), (7,)), (5, 5, 0.2, (), ())])
def test_bnb_matches_enumeration(dev, seed, k, lam2, J0, J1):
    import paper_2603_01306_amd as pr
    inst = make_instance(n=120, p=14, corr=0.5, k_true=4, snr=4.0, loss=0, seed=seed, storage="f64")
    X, y = inst.X64().T, inst.y
    ctx = _ctx(inst, dev, 8)
    res, beta = ctx.bnb(pr.Node(k, lam2, 2.0, J0=J0, J1=J1), rel_gap_tol=1e-7,
                        node_opts=dict(rel_gap_tol=1e-9, max_iter=200000))
    opt, S, _ = ksparse_bruteforce(X, y, k, lam2, 2.0, J0=J0, J1=J1)
    print(seed, res, opt, flush=True)
    assert res["status"] == pr.BNB_OPTIMAL
    assert res["lower_bound"] <= opt * (1 + 1e-9)
    assert res["upper_bound"] >= opt * (1 - 1e-9)
    assert res["upper_bound"] - opt <= 2e-7 * opt
    b = beta.cpu().numpy()
    assert np.count_nonzero(b) <= k and np.all(np.abs(b) <= 2.0) and np.all(b[list(J0)] == 0)
    assert abs(_objective(X, y, b, lam2) - res["upper_bound"]) <= 1e-10 * res["upper_bound"]
    ctx.close()


@pytest.mark.parametrize("seed,k,lam2,J0,J1", [(6, 3, 0.3, (), ()), (7, 2, 0.5, (1,), (4,))])
def test_bnb_logistic_matches_enumeration(dev, seed, k, lam2, J0, J1):
    """Logistic loss: the tree closes on the optimum of problem (1) found by
    enumerating every support (box-constrained logistic ridge per support);
    the incumbent is a feasible k-sparse point whose objective is the
    reported upper bound."""
    import paper_2603_01306_amd as pr
    inst = make_instance(n=120, p=12, corr=0.5, k_true=3, snr=4.0, loss=1, seed=seed, storage="f64")
    X, y = inst.X64().T, inst.y
    ctx = _ctx(inst, dev, 8)
    res, beta = ctx.bnb(pr.Node(k, lam2, 2.0, J0=J0, J1=J1), rel_gap_tol=1e-7,
                        node_opts=dict(rel_gap_tol=1e-9, max_iter=200000))
    opt, S, _ = ksparse_bruteforce_logistic(X, y, k, lam2, 2.0, J0=J0, J1=J1)
    print(seed, res, opt, S, flush=True)
    assert res["status"] == pr.BNB_OPTIMAL
    assert res["lower_bound"] <= opt * (1 + 1e-9)
    assert res["upper_bound"] >= opt * (1 - 1e-9)
    assert res["upper_bound"] - opt <= 2e-7 * opt
    b = beta.cpu().numpy()
    assert np.count_nonzero(b) <= k and np.all(np.abs(b) <= 2.0) and np.all(b[list(J0)] == 0)
    obj = float(np.sum(np.logaddexp(0.0, -y * (X @ b))) + lam2 * b @ b)
    assert abs(obj - res["upper_bound"]) <= 1e-10 * res["upper_bound"]
    ctx.close()


@pytest.mark.parametrize("loss,seed,k,lam2", [(0, 13, 3, 0.2), (0, 14, 4, 0.05), (1, 15, 3, 0.1)])
def test_bnb_with_a_binding_box_matches_enumeration(dev, loss, seed, k, lam2):
    """Box M = 0.3 binds at the optimum: the incumbent must be the box-constrained
    fit of its support (not a ridge fit clipped to the box), and leaves must
    offer their own problem as an incumbent, or the tree would close above the
    enumerated optimum."""
    import paper_2603_01306_amd as pr
    M = 0.3
    inst = make_instance(n=120, p=12, corr=0.5, k_true=3, snr=8.0, loss=loss, seed=seed, storage="f64")
    X, y = inst.X64().T, inst.y
    ctx = _ctx(inst, dev, 8)
    res, beta = ctx.bnb(pr.Node(k, lam2, M), rel_gap_tol=1e-7, node_opts=dict(rel_gap_tol=1e-9, max_iter=200000))
    if loss == 0:
        opt, S, bopt = ksparse_bruteforce(X, y, k, lam2, M)
    else:
        opt, S, bopt = ksparse_bruteforce_logistic(X, y, k, lam2, M)
    print(loss, seed, res, opt, S, bopt, flush=True)
    assert np.max(np.abs(bopt)) >= M * (1 - 1e-6)             # the box is active at the optimum
    assert res["status"] == pr.BNB_OPTIMAL
    assert res["lower_bound"] <= opt * (1 + 1e-9)
    assert abs(res["upper_bound"] - opt) <= 2e-7 * opt
    b = beta.cpu().numpy()
    assert np.count_nonzero(b) <= k and np.all(np.abs(b) <= M * (1 + 1e-12))
    if loss == 0:
        obj = _objective(X, y, b, lam2)
    else:
        obj = float(np.sum(np.logaddexp(0.0, -y * (X @ b))) + lam2 * b @ b)
    assert abs(obj - res["upper_bound"]) <= 1e-10 * res["upper_bound"]
    ctx.close()


def test_bnb_on_the_batched_path(dev):
    """BF16 design on the batched path: bounds ordered, incumbent objective
    exact, node accounting consistent."""
    import paper_2603_01306_amd as pr
    inst = make_instance(n=1024, p=512, corr=0.6, k_true=6, snr=5.0, loss=0, seed=9, storage="bf16")
    X, y = inst.X64().T, inst.y
    ctx = _ctx(inst, dev, 32)
    res, beta = ctx.bnb(pr.Node(6, 0.5, 2.0), rel_gap_tol=1e-4, max_nodes=400)
    print(res, flush=True)
    assert res["lower_bound"] <= res["upper_bound"] * (1 + 1e-12)
    b = beta.cpu().numpy()
    assert np.count_nonzero(b) <= 6
    assert abs(_objective(X, y, b, 0.5) - res["upper_bound"]) <= 1e-10 * res["upper_bound"]
    root = oracle.solve(inst.Xcm, inst.y, 0, 0.5, 2.0, 6, tol=1e-9)
    assert res["lower_bound"] >= root["lb"] * (1 - 1e-6)      # never below the root bound
    assert res["nodes_solved"] >= 1 and res["nodes_pruned"] + res["nodes_open"] <= 2 * res["nodes_solved"] + 1
    ctx.close()


@pytest.mark.parametrize("loss,storage,seed", [(0, "bf16", 10), (1, "f32", 11)])
def test_batched_cutoff_decisions_match_oracle(dev, loss, storage, seed):
    """Batched dynamic termination against the oracle's decisions: each node's
    relaxation value is at least 1% away from the cutoff, so prune (value above
    the cutoff) or branch (below) is the only correct outcome, and the oracle
    run with the same step reaches it at (nearly) the same iterate."""
    import paper_2603_01306_amd as pr
    inst = make_instance(n=1024, p=512, corr=0.6, k_true=6, snr=5.0, loss=loss, seed=seed, storage=storage)
    ctx = _ctx(inst, dev, 16)
    rng = np.random.default_rng(0)
    # fixed-zero sets of growing size spread the nodes' relaxation values
    nodes = [pr.Node(6, 0.5, 2.0, J0=rng.choice(512, 40 * q, replace=False)) for q in range(8)]
    free, _ = ctx.solve_batch(nodes, rel_gap_tol=1e-9)
    vals = np.sort([r["lower_bound"] for r in free])
    gaps = np.diff(vals) / vals[1:]
    i = int(np.argmax(gaps[1:6])) + 1                          # the widest gap between inner values
    cutoff = 0.5 * (vals[i] + vals[i + 1])
    assert min(abs(v - cutoff) for v in vals) >= 1e-3 * cutoff
    res, B = ctx.solve_batch(nodes, rel_gap_tol=1e-9, cutoff=cutoff)
    Bh = B.cpu().numpy()
    kinds = set()
    for q, (nd, r, f) in enumerate(zip(nodes, res, free)):
        st = nd.status(inst.p)
        ref = oracle.solve(inst.Xcm, inst.y, loss, 0.5, 2.0, 6, status=st, L=r["L"], tol=1e-9, cutoff=cutoff)
        assert r["status"] == ref["status"], (q, r, ref["status"])
        assert abs(r["iters"] - ref["iters"]) <= 2
        kinds.add(r["status"])
        if r["status"] == pr.CUTOFF_PRUNE:
            assert r["lower_bound"] >= cutoff and ref["lb"] >= cutoff
        else:
            assert r["status"] == pr.CUTOFF_BRANCH and r["primal"] <= cutoff
            phi = oracle.primal(inst.Xcm, inst.y, Bh[q], loss, 0.5, 2.0, 6, status=st)
            assert abs(phi - r["primal"]) <= 1e-11 * abs(phi)
    assert kinds == {pr.CUTOFF_PRUNE, pr.CUTOFF_BRANCH}
    ctx.close()


def test_logistic_bnb_on_the_batched_path(dev):
    """Logistic branch and bound on an FP32 design whose nodes run on the
    batched path (two right-hand sides per node in the transposed product):
    the same certified interval as the branch and bound whose nodes run one at
    a time, and an exact incumbent objective."""
    import paper_2603_01306_amd as pr
    inst = make_instance(n=1024, p=256, corr=0.5, k_true=4, snr=5.0, loss=1, seed=12, storage="f32")
    X, y = inst.X64().T, inst.y
    out = []
    for mb in (32, 1):
        ctx = _ctx(inst, dev, mb)
        res, beta = ctx.bnb(pr.Node(4, 0.5, 2.0), rel_gap_tol=1e-4, max_nodes=600)
        print(mb, res, flush=True)
        b = beta.cpu().numpy()
        assert np.count_nonzero(b) <= 4
        obj = float(np.sum(np.logaddexp(0.0, -y * (X @ b))) + 0.5 * b @ b)
        assert abs(obj - res["upper_bound"]) <= 1e-10 * res["upper_bound"]
        assert res["lower_bound"] <= res["upper_bound"] * (1 + 1e-12)
        out.append(res)
        ctx.close()
    a, b = out
    assert a["status"] == b["status"]
    assert a["lower_bound"] <= b["upper_bound"] * (1 + 1e-9) and b["lower_bound"] <= a["upper_bound"] * (1 + 1e-9)
    if a["status"] == pr.BNB_OPTIMAL:
        assert abs(a["upper_bound"] - b["upper_bound"]) <= 1e-4 * b["upper_bound"]
