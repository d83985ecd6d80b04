"""Pins of the oracle's duality-gap restart and its dynamic-termination
(cutoff) branch.  CPU only.

Restart (Section 3.3, "Restart in practice"): a restart is taken at the first
iterate whose gap is at most 1/eta of the gap at the start of the epoch, and
the algorithm then continues exactly as a fresh run started from that iterate
(t <- 1, momentum point <- iterate), i.e. the epoch is a new initialisation.

Cutoff (Section 5.3, dynamic termination): with an incumbent value c the node
is pruned as soon as the best dual value reaches c and branched as soon as the
best primal value falls to c.  The decision is checked against relaxation
values computed without the oracle: the box-constrained ridge fit of a leaf
node by bounded least squares (least squares) or L-BFGS-B (logistic), and the
relaxation solved directly in (beta, z) by SLSQP."""
import math

import numpy as np
import pytest
from scipy import optimize

import oracle
from oracle.ksparse import ksparse_bruteforce, logistic_box_ridge
from workloads import make_instance


def _inst(loss, seed, n=60, p=12):
    return make_instance(n=n, p=p, corr=0.6, k_true=3, snr=5.0, loss=loss, seed=seed, storage="f64")


def _L(inst, loss):
    return 1.01 * (2.0 if loss == 0 else 0.25) * oracle.power_norm2(inst.Xcm)


# --------------------------------------------------------------- restart

CASES = [(0, 1, math.e ** 3), (0, 2, math.e), (1, 3, math.e ** 3), (1, 4, math.e ** 2)]


@pytest.mark.parametrize("loss,seed,eta", CASES)
def test_restart_points_are_the_first_iterates_below_gap_ref_over_eta(loss, seed, eta):
    inst = _inst(loss, seed)
    st = oracle.status_vector(inst.p, J0=[5], J1=[2])
    L = _L(inst, loss)
    res = oracle.solve(inst.Xcm, inst.y, loss, 0.3, 2.0, 4, status=st, L=L, tol=1e-11, eta=eta,
                       trace_cap=100000, restart_cap=1000)
    gap = res["trace"]
    assert res["status"] == oracle.CONVERGED and res["restarts"] >= 3
    # the rule applied to the recorded gaps; the iterate that meets the
    # stopping test ends the run before any restart test
    want, ref = [], gap[0]
    for t in range(1, res["iters"]):
        if gap[t] <= ref / eta:
            want.append(t)
            ref = gap[t]
    assert list(res["restart_at"]) == want
    # between restarts the gap never fell below the epoch's threshold
    starts = [0] + want
    for a, b in zip(starts, starts[1:]):
        assert np.all(gap[a + 1:b] > gap[a] / eta)


@pytest.mark.parametrize("loss,seed,eta", CASES)
def test_epoch_after_a_restart_is_a_fresh_fista_run(loss, seed, eta):
    """Iterates r+1 .. r' of the restarted run (r, r' consecutive restarts)
    equal iterates 1 .. r'-r of plain FISTA started at x^r with t = 1 and the
    momentum point at x^r.  Keeping t, or keeping the momentum point, at the
    restart changes the first step after it and fails this equality."""
    inst = _inst(loss, seed)
    st = oracle.status_vector(inst.p, J0=[5], J1=[2])
    L = _L(inst, loss)
    kw = dict(status=st, L=L, eta=eta)
    full = oracle.solve(inst.Xcm, inst.y, loss, 0.3, 2.0, 4, tol=1e-11, trace_cap=100000, restart_cap=1000, **kw)
    rs = list(full["restart_at"]) + [full["iters"]]
    assert len(rs) >= 4
    for i, (r, r2) in enumerate(zip(rs[:3], rs[1:4])):
        # the run stopped at the restart iterate r has taken that restart
        head = oracle.solve(inst.Xcm, inst.y, loss, 0.3, 2.0, 4, tol=0.0, max_iter=r, **kw)
        assert head["iters"] == r and head["restarts"] == i + 1
        fresh = oracle.solve(inst.Xcm, inst.y, loss, 0.3, 2.0, 4, tol=0.0, max_iter=r2 - r, beta0=head["beta"],
                             trace_cap=100000, method=oracle.FISTA, **kw)
        assert fresh["iters"] == r2 - r
        assert np.array_equal(fresh["phi_trace"][1:], full["phi_trace"][r + 1:r2 + 1])
        assert np.array_equal(fresh["trace"][1:], full["trace"][r + 1:r2 + 1])


# --------------------------------------------------------------- cutoff

def _check_decision(inst, loss, lam2, M, k, st, L, v, rel):
    """Cutoffs rel below / above the relaxation value v: prune / branch, at
    the first iterate where the best dual (primal) value crosses the cutoff."""
    for c, want in ((v * (1 - rel), oracle.CUTOFF_PRUNE), (v * (1 + rel), oracle.CUTOFF_BRANCH)):
        # tol < 0: the gap test never stops the run (a box-bound leaf can reach
        # a gap of exactly 0), so only the cutoff decides
        r = oracle.solve(inst.Xcm, inst.y, loss, lam2, M, k, status=st, L=L, tol=-1.0, cutoff=c,
                         trace_cap=100000)
        assert r["status"] == want, (c, v, r["status"])
        phi, psi = r["phi_trace"], r["phi_trace"] - r["trace"]
        ub, lb = np.minimum.accumulate(phi), np.maximum.accumulate(psi)
        hit = (lb >= c) if want == oracle.CUTOFF_PRUNE else (ub <= c)
        assert r["iters"] == int(np.argmax(hit)) and hit[r["iters"]]
        if want == oracle.CUTOFF_PRUNE:
            assert c <= r["lb"] <= v * (1 + 1e-9)          # weak duality
            zeta_psi = oracle.dual(inst.Xcm, inst.y, r["zeta"], loss, lam2, M, k, status=st)
            assert zeta_psi == pytest.approx(r["lb"], rel=1e-12)
        else:
            assert v * (1 - 1e-9) <= r["ub"] <= c
            assert oracle.primal(inst.Xcm, inst.y, r["beta"], loss, lam2, M, k, status=st) <= c * (1 + 1e-12)


@pytest.mark.parametrize("loss", [0, 1])
@pytest.mark.parametrize("M", [2.0, 0.3])
def test_cutoff_on_leaf_nodes_against_box_ridge(loss, M):
    """Leaf node J1 = S (|S| = k), J0 = the rest: the relaxation is problem (1)
    restricted to S, whose value is the box-constrained ridge fit (with M = 0.3
    the box binds)."""
    inst = _inst(loss, 11 + loss)
    X = inst.X64().T
    S = [1, 4, 8]
    k, lam2 = 3, 0.4
    J0 = [j for j in range(inst.p) if j not in S]
    st = oracle.status_vector(inst.p, J0=J0, J1=S)
    if loss == 0:
        v, _, b = ksparse_bruteforce(X, inst.y, k, lam2, M, J0=J0, J1=S)
    else:
        v, b = logistic_box_ridge(X[:, S], inst.y, lam2, M)
    if M < 1:
        assert np.max(np.abs(b)) >= M * (1 - 1e-9)            # the box is active
    _check_decision(inst, loss, lam2, M, k, st, _L(inst, loss), v, 1e-3)


def test_cutoff_on_general_node_against_direct_relaxation_solve():
    """A node with free coordinates: the perspective relaxation solved in
    (beta, z) by SLSQP gives its value; cutoffs 1e-3 away decide prune / branch."""
    inst = make_instance(n=30, p=6, corr=0.5, k_true=2, snr=5.0, loss=0, seed=21, storage="f64")
    X = inst.X64().T
    p, k, M, lam2 = inst.p, 3, 2.0, 0.5
    J0, J1 = [4], [0]
    st = oracle.status_vector(p, J0=J0, J1=J1)

    def obj(w):
        b, z = w[:p], w[p:]
        return float(np.sum((inst.y - X @ b) ** 2) + lam2 * np.sum(b ** 2 / z))

    cons = [{"type": "ineq", "fun": lambda w: k - w[p:].sum()}]
    for j in range(p):
        cons.append({"type": "ineq", "fun": lambda w, j=j: M * w[p + j] - w[j]})
        cons.append({"type": "ineq", "fun": lambda w, j=j: M * w[p + j] + w[j]})
    bounds = []
    for j in range(p):
        bounds.append((0.0, 0.0) if j in J0 else (-M, M))
    for j in range(p):
        bounds.append((1.0, 1.0) if j in J1 else ((1e-9, 1e-9) if j in J0 else (1e-9, 1.0)))
    w0 = np.concatenate([np.zeros(p), [1.0 if j in J1 else (1e-9 if j in J0 else 0.5) for j in range(p)]])
    r = optimize.minimize(obj, w0, method="SLSQP", bounds=bounds, constraints=cons,
                          options={"ftol": 1e-15, "maxiter": 5000})
    assert r.success
    _check_decision(inst, 0, lam2, M, k, st, _L(inst, 0), r.fun, 1e-3)


def test_cutoff_far_from_the_value_decides_at_once():
    """Cutoff far above every primal value: branch at iterate 0 when that
    iterate is in the domain; far below every dual value: prune at iterate 0."""
    inst = _inst(0, 5)
    L = _L(inst, 0)
    r = oracle.solve(inst.Xcm, inst.y, 0, 0.3, 2.0, 4, L=L, cutoff=1e12)
    assert r["status"] == oracle.CUTOFF_BRANCH and r["iters"] == 0
    r = oracle.solve(inst.Xcm, inst.y, 0, 0.3, 2.0, 4, L=L, cutoff=-1e12)
    assert r["status"] == oracle.CUTOFF_PRUNE and r["iters"] == 0
