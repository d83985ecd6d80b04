"""Least squares from the Gram matrix (pr_ctx_enable_gram): h = b - G x in
place of X x and X^T r.  The per-iterate (Phi, Psi) trace equals the
matrix-vector path's and the oracle's, bounds match the oracle, and the
reported bound is recomputed over the stored X."""
import numpy as np
import pytest

import oracle
from workloads import make_instance

pytestmark = pytest.mark.gpu


def _ctx(inst, dev, gram):
    import torch
    import paper_2603_01306_amd as pr
    if inst.storage == "bf16":
        X = torch.from_numpy(inst.Xcm.view(np.int16)).to(dev).view(torch.bfloat16)
    else:
        X = torch.from_numpy(inst.Xcm).to(dev)
    c = pr.Context(X, torch.from_numpy(inst.y).to(dev), 0)
    if gram:
        c.enable_gram()
    return c


@pytest.mark.parametrize("storage", ["f32", "bf16", "f64"])
def test_gram_trace_matches_oracle_and_matvec_path(dev, storage):
    import torch
    import paper_2603_01306_amd as pr
    inst = make_instance(n=1024, p=512, corr=0.7, k_true=8, snr=5.0, loss=0, seed=12, storage=storage)
    L = 2.02 * float(np.linalg.eigvalsh(inst.X64() @ inst.X64().T).max())
    node = pr.Node(8, 0.3, 2.0, J0=[1, 9], J1=[4])
    its = 60
    traces = []
    for gram in (False, True):
        c = _ctx(inst, dev, gram)
        tr = torch.full((2 * (its + 1),), float("nan"), dtype=torch.float64, device=dev)
        c.solve(node, rel_gap_tol=0.0, max_iter=its, L=L, trace=tr)
        traces.append(tr.cpu().numpy().reshape(-1, 2))
        c.close()
    ref = oracle.solve(inst.Xcm, inst.y, 0, 0.3, 2.0, 8, status=node.status(inst.p), L=L, tol=0.0,
                       max_iter=its, trace_cap=its + 1)
    ophi = ref["phi_trace"]
    fin = np.isfinite(ophi)
    for t in traces:
        assert np.array_equal(np.isfinite(t[:, 0]), fin)
        assert np.all(np.abs(t[fin, 0] - ophi[fin]) <= 1e-10 * np.abs(ophi[fin]))
        assert np.all(np.abs(t[:, 1] - (ophi - ref["trace"])) <= 1e-10 * abs(ophi[-1]))


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_gram_bound_is_certified_over_x(dev, storage):
    import torch
    import paper_2603_01306_amd as pr
    inst = make_instance(n=2048, p=1024, corr=0.8, k_true=10, snr=5.0, loss=0, seed=13, storage=storage)
    c = _ctx(inst, dev, True)
    node = pr.Node(10, 0.2, 2.0, J0=[0, 5, 77], J1=[100])
    r = c.solve(node, rel_gap_tol=1e-7, want_zeta=True)
    ref = oracle.solve(inst.Xcm, inst.y, 0, 0.2, 2.0, 10, status=node.status(inst.p), tol=1e-10)
    assert r["status"] == pr.CONVERGED and r["rel_gap"] <= 1e-7
    assert abs(r["lower_bound"] - ref["lb"]) <= 2e-7 * abs(ref["ub"])
    st = node.status(inst.p)
    zeta = r["zeta"].cpu().numpy()
    psi = oracle.dual(inst.Xcm, inst.y, zeta, 0, 0.2, 2.0, 10, status=st)
    assert abs(psi - r["lower_bound"]) <= 1e-11 * abs(psi)            # the reported bound is Psi(zeta) over X
    phi = oracle.primal(inst.Xcm, inst.y, r["beta"].cpu().numpy(), 0, 0.2, 2.0, 10, status=st)
    assert abs(phi - r["primal"]) <= 1e-11 * abs(phi)
    c.close()


def test_gram_rejects_unsupported_shapes(dev):
    import torch
    import paper_2603_01306_amd as pr
    inst = make_instance(n=300, p=200, corr=0.5, k_true=5, snr=5.0, loss=0, seed=1, storage="f64")
    c = _ctx(inst, dev, False)
    with pytest.raises(pr.PrError):
        c.enable_gram()                       # p not a multiple of 128
    c.close()


def _bctx(inst, dev, gram, m):
    import torch
    import paper_2603_01306_amd as pr
    X = torch.from_numpy(inst.Xcm.view(np.int16)).to(dev).view(torch.bfloat16)
    c = pr.Context(X, torch.from_numpy(inst.y).to(dev), 0, max_batch=m)
    c.set_debug(pr.DEBUG_FORCE_BATCH)
    if gram:
        c.enable_gram()
    return c


def test_batched_gram_bounds_match_matvec_batch_and_oracle(dev):
    """The batch in Gram mode (one product G X_it per iteration) certifies the
    same bounds as the batch over X and as the oracle, node by node."""
    import paper_2603_01306_amd as pr
    from workloads import make_nodes
    inst = make_instance(n=2048, p=512, corr=0.7, k_true=8, snr=5.0, loss=0, seed=21, storage="bf16")
    raw = make_nodes(inst.p, 12, seed=3, max_j0=20, max_j1=5)
    nodes = [pr.Node(8, 0.3, 2.0, J0=a, J1=b) for a, b in raw]
    res = {}
    for gram in (False, True):
        c = _bctx(inst, dev, gram, 16)
        r, B = c.solve_batch(nodes, rel_gap_tol=1e-7)
        res[gram] = (r, B.cpu().numpy())
        c.close()
    for q, nd in enumerate(nodes):
        rg, rm = res[True][0][q], res[False][0][q]
        assert rg["status"] == pr.CONVERGED and rg["rel_gap"] <= 1e-7, rg
        assert abs(rg["lower_bound"] - rm["lower_bound"]) <= 2e-7 * abs(rm["primal"])
        ref = oracle.solve(inst.Xcm, inst.y, 0, 0.3, 2.0, 8, status=nd.status(inst.p), tol=1e-10)
        assert rg["lower_bound"] <= ref["ub"] * (1 + 1e-12)
        assert abs(rg["lower_bound"] - ref["lb"]) <= 2e-7 * abs(ref["ub"])
        # the returned beta attains the reported primal value over the stored X
        phi = oracle.primal(inst.Xcm, inst.y, res[True][1][q], 0, 0.3, 2.0, 8, status=nd.status(inst.p))
        assert abs(phi - rg["primal"]) <= 1e-11 * abs(phi)


@pytest.mark.parametrize("check_every", [8, 32])
def test_batched_gram_union_compaction(dev, check_every):
    """After the first graph launch the batched Gram product runs over the
    union of the iterates' supports (plus the nonzeros that later fall outside
    it, added column by column).  Built after 8 iterations the union misses
    coordinates that enter later, which exercises that correction; after 32
    it has mostly settled.  Bounds agree with the batch over X and with the
    oracle."""
    import paper_2603_01306_amd as pr
    from workloads import make_nodes
    inst = make_instance(n=2048, p=2048, corr=0.7, k_true=8, snr=5.0, loss=0, seed=23, storage="bf16")
    raw = make_nodes(inst.p, 24, seed=5, max_j0=30, max_j1=4)
    nodes = [pr.Node(8, 0.3, 2.0, J0=a, J1=b) for a, b in raw]
    res = {}
    for gram in (False, True):
        c = _bctx(inst, dev, gram, 32)
        r, B = c.solve_batch(nodes, rel_gap_tol=1e-7, check_every=check_every)
        res[gram] = (r, B.cpu().numpy(), c.batch_union_size())
        c.close()
    ku, kp, nout = res[True][2]
    print("union", ku, kp, "of", inst.p, "outside", nout, "; batch over X:", res[False][2], flush=True)
    assert 0 < ku <= kp < inst.p
    if check_every == 8:
        assert nout > 0
    for q, nd in enumerate(nodes):
        rg, rm = res[True][0][q], res[False][0][q]
        assert rg["status"] == pr.CONVERGED and rg["rel_gap"] <= 1e-7, rg
        assert abs(rg["lower_bound"] - rm["lower_bound"]) <= 2e-7 * abs(rm["primal"])
        # the same iteration as the batch over X (a wrong product would stall
        # the node until the FP64 check sends it to the single-node path)
        assert abs(rg["iters"] - rm["iters"]) <= 3, (q, rg["iters"], rm["iters"])
        if q < 4:
            ref = oracle.solve(inst.Xcm, inst.y, 0, 0.3, 2.0, 8, status=nd.status(inst.p), tol=1e-10)
            assert abs(rg["lower_bound"] - ref["lb"]) <= 2e-7 * abs(ref["ub"])
            phi = oracle.primal(inst.Xcm, inst.y, res[True][1][q], 0, 0.3, 2.0, 8, status=nd.status(inst.p))
            assert abs(phi - rg["primal"]) <= 1e-11 * abs(phi)


def test_batched_gram_cutoff_decisions(dev):
    import paper_2603_01306_amd as pr
    inst = make_instance(n=1024, p=512, corr=0.6, k_true=6, snr=5.0, loss=0, seed=10, storage="bf16")
    c = _bctx(inst, dev, True, 16)
    rng = np.random.default_rng(0)
    nodes = [pr.Node(6, 0.5, 2.0, J0=rng.choice(512, 20, replace=False)) for _ in range(8)]
    free, _ = c.solve_batch(nodes, rel_gap_tol=1e-9)
    vals = sorted(r["lower_bound"] for r in free)
    cutoff = 0.5 * (vals[3] + vals[4])
    res, _ = c.solve_batch(nodes, rel_gap_tol=1e-9, cutoff=cutoff)
    for r, f in zip(res, free):
        assert r["status"] in (pr.CUTOFF_PRUNE, pr.CUTOFF_BRANCH, pr.CONVERGED)
        if r["status"] == pr.CUTOFF_PRUNE:
            assert r["lower_bound"] >= cutoff and f["lower_bound"] >= cutoff * (1 - 1e-9)
        if r["status"] == pr.CUTOFF_BRANCH:
            assert r["primal"] <= cutoff and f["lower_bound"] <= cutoff * (1 + 1e-9)
    c.close()


def test_gram_rejects_logistic(dev):
    import torch
    import paper_2603_01306_amd as pr
    inst = make_instance(n=256, p=128, corr=0.5, k_true=4, snr=5.0, loss=1, seed=2, storage="f64")
    c = pr.Context(torch.from_numpy(inst.Xcm).to(dev), torch.from_numpy(inst.y).to(dev), 1)
    with pytest.raises(pr.PrError):
        c.enable_gram()                       # the Gram identities hold for least squares only
    c.close()


def test_gram_cutoff_warm_start_and_iteration_limit(dev):
    """Single-node Gram mode: cutoff decisions agree with the matrix-vector
    path and are confirmed over X, a warm start reaches the same bound, and an
    iteration limit reports a valid (recomputed) bound."""
    import torch
    import paper_2603_01306_amd as pr
    inst = make_instance(n=1024, p=512, corr=0.7, k_true=8, snr=5.0, loss=0, seed=31, storage="f32")
    cg, cm = _ctx(inst, dev, True), _ctx(inst, dev, False)
    node = pr.Node(8, 0.3, 2.0, J0=[2, 40], J1=[7])
    free = cm.solve(node, rel_gap_tol=1e-9)
    lb = free["lower_bound"]
    for cutoff, want in ((lb * 0.99, pr.CUTOFF_PRUNE), (lb * 1.01, pr.CUTOFF_BRANCH)):
        rg = cg.solve(node, rel_gap_tol=1e-9, cutoff=cutoff)
        rm = cm.solve(node, rel_gap_tol=1e-9, cutoff=cutoff)
        assert rg["status"] == rm["status"] == want, (rg, rm)
        if want == pr.CUTOFF_PRUNE:
            assert rg["lower_bound"] >= cutoff
        else:
            assert rg["primal"] <= cutoff
    warm = cg.solve(node, beta0=free["beta"], rel_gap_tol=1e-8)
    assert warm["status"] == pr.CONVERGED and warm["iters"] < free["iters"]
    assert abs(warm["lower_bound"] - lb) <= 1e-8 * abs(free["primal"])
    short = cg.solve(node, rel_gap_tol=0.0, max_iter=5, want_zeta=True)
    assert short["status"] == pr.MAXITER and short["iters"] == 5
    st = node.status(inst.p)
    psi = oracle.dual(inst.Xcm, inst.y, short["zeta"].cpu().numpy(), 0, 0.3, 2.0, 8, status=st)
    assert abs(psi - short["lower_bound"]) <= 1e-11 * abs(psi) and psi <= lb * (1 + 1e-12)
    cg.close()
    cm.close()


def test_gram_unconfirmed_decision_reruns_on_matvec_path(dev):
    """A Gram-mode decision the recomputation over X does not confirm is redone
    on the matrix-vector path (forced here by the context's test switch).  The
    re-solve must use that path's own iteration graph: its bound is then the
    FP64 value over the stored X of the zeta it returns (the oracle
    recomputes it), and a Gram solve after the switch is cleared is again the
    plain Gram run."""
    import paper_2603_01306_amd as pr
    inst = make_instance(n=1024, p=512, corr=0.7, k_true=8, snr=5.0, loss=0, seed=33, storage="f32")
    c = _ctx(inst, dev, True)
    node = pr.Node(8, 0.3, 2.0, J0=[3, 77], J1=[5])
    st = node.status(inst.p)
    plain = c.solve(node, rel_gap_tol=1e-9, want_zeta=True)
    ref = oracle.solve(inst.Xcm, inst.y, 0, 0.3, 2.0, 8, status=st, L=plain["L"], tol=1e-11)
    c.set_debug(pr.DEBUG_GRAM_RECHECK)
    cases = [dict(rel_gap_tol=1e-9, want=pr.CONVERGED),
             dict(rel_gap_tol=1e-9, cutoff=ref["lb"] * 0.995, want=pr.CUTOFF_PRUNE),
             dict(rel_gap_tol=1e-9, cutoff=ref["lb"] * 1.005, want=pr.CUTOFF_BRANCH)]
    for cs in cases:
        want = cs.pop("want")
        r = c.solve(node, want_zeta=True, **cs)
        print(want, {k: v for k, v in r.items() if k not in ("beta", "zeta")}, flush=True)
        assert r["status"] == want
        psi = oracle.dual(inst.Xcm, inst.y, r["zeta"].cpu().numpy(), 0, 0.3, 2.0, 8, status=st)
        phi = oracle.primal(inst.Xcm, inst.y, r["beta"].cpu().numpy(), 0, 0.3, 2.0, 8, status=st)
        assert abs(psi - r["lower_bound"]) <= 1e-11 * abs(psi)
        assert abs(phi - r["primal"]) <= 1e-11 * abs(phi)
        assert r["lower_bound"] <= ref["ub"] * (1 + 1e-12)
        if want == pr.CONVERGED:
            assert abs(r["lower_bound"] - ref["lb"]) <= 1e-8 * abs(ref["ub"])
        elif want == pr.CUTOFF_PRUNE:
            assert r["lower_bound"] >= cs["cutoff"]
        else:
            assert r["primal"] <= cs["cutoff"]
    c.set_debug(0)
    again = c.solve(node, rel_gap_tol=1e-9, want_zeta=True)
    assert again["iters"] == plain["iters"] and again["lower_bound"] == plain["lower_bound"]
    c.close()
