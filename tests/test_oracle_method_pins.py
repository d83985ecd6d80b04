"""Pins of the oracle's iteration variants used in the convergence study
(Section 5.2): proximal gradient, FISTA without restart, FISTA with
function-value restart, FISTA with the duality-gap restart.  Each is pinned to
textbook facts about the iteration it claims to be (Beck, First-Order Methods
in Optimization, 2017): the sufficient-decrease property and the O(1/k) bound
of proximal gradient (Lemma 10.4, Theorem 10.21), the O(1/k^2) bound of FISTA
(Theorem 10.34), and to the relaxation itself (every variant certifies the
same bound, below the brute-force k-sparse optimum).  CPU only."""
import itertools
import math

import numpy as np
import pytest

import oracle
from workloads import make_instance


@pytest.fixture(scope="module")
def small():
    inst = make_instance(n=60, p=16, corr=0.6, k_true=4, snr=3.0, loss=0, seed=5, storage="f64")
    X = inst.X64().T
    L = 2.0 * float(np.linalg.eigvalsh(X.T @ X).max())
    ref = oracle.solve(inst.Xcm, inst.y, 0, 0.5, 2.0, 4, L=L, tol=1e-13, max_iter=200000)
    return inst, X, L, ref


def _run(inst, L, method, iters):
    return oracle.solve(inst.Xcm, inst.y, 0, 0.5, 2.0, 4, L=L, tol=0.0, max_iter=iters, trace_cap=iters + 1,
                        method=method)


def test_pgd_sufficient_decrease_and_rate(small):
    inst, X, L, ref = small
    r = _run(inst, L, oracle.PGD, 400)
    phi = r["phi_trace"]
    assert np.all(np.diff(phi) <= 1e-10 * abs(phi[0]))                       # Lemma 10.4
    phistar, d0 = ref["ub"], np.linalg.norm(ref["beta"])                      # x0 = 0
    k = np.arange(1, phi.size)
    assert np.all(phi[1:] - phistar <= L * d0 ** 2 / (2 * k) + 1e-9 * abs(phistar))   # Theorem 10.21
    assert r["restarts"] == 0


def test_fista_without_restart_rate(small):
    inst, X, L, ref = small
    r = _run(inst, L, oracle.FISTA, 400)
    phi = r["phi_trace"]
    phistar, d0 = ref["ub"], np.linalg.norm(ref["beta"])
    k = np.arange(1, phi.size)
    assert np.all(phi[1:] - phistar <= 2 * L * d0 ** 2 / (k + 1) ** 2 + 1e-9 * abs(phistar))   # Theorem 10.34
    assert r["restarts"] == 0


def test_function_value_restart_fires_exactly_on_increases(small):
    inst, X, L, ref = small
    r = _run(inst, L, oracle.FISTA_FV, 400)
    phi = r["phi_trace"]
    assert r["restarts"] == int(np.sum(np.diff(phi) > 0))


def test_momentum_matters(small):
    """FISTA and PGD produce different iterates after the second step, and
    PGD's first step equals FISTA's (t = 1 gives zero momentum)."""
    inst, X, L, ref = small
    a = _run(inst, L, oracle.PGD, 3)["phi_trace"]
    b = _run(inst, L, oracle.FISTA, 3)["phi_trace"]
    assert a[1] == b[1]
    assert a[3] != b[3]


@pytest.mark.parametrize("method", [oracle.FISTA_GAP, oracle.FISTA, oracle.FISTA_FV, oracle.PGD])
def test_every_variant_certifies_the_same_bound(small, method):
    inst, X, L, ref = small
    r = oracle.solve(inst.Xcm, inst.y, 0, 0.5, 2.0, 4, L=L, tol=1e-8, max_iter=300000, method=method)
    assert r["status"] == oracle.CONVERGED
    assert abs(r["lb"] - ref["lb"]) <= 2e-8 * abs(ref["ub"])
    # the bound is below the k-sparse optimum found by enumerating supports
    best = math.inf
    for S in itertools.combinations(range(X.shape[1]), 4):
        XS = X[:, S]
        b = np.linalg.solve(XS.T @ XS + 0.5 * np.eye(4), XS.T @ inst.y)
        if np.max(np.abs(b)) <= 2.0:
            best = min(best, float(np.sum((inst.y - XS @ b) ** 2) + 0.5 * b @ b))
    assert r["lb"] <= best * (1 + 1e-12)


def test_gap_restart_needs_fewer_iterations(small):
    """The paper's claim in its convergence study: the duality-gap restart
    turns FISTA's sublinear rate into a linear one; at a tight tolerance it
    needs fewer iterations than PGD and than FISTA without restart."""
    inst, X, L, ref = small
    its = {m: oracle.solve(inst.Xcm, inst.y, 0, 0.5, 2.0, 4, L=L, tol=1e-10, max_iter=300000, method=m)["iters"]
           for m in (oracle.FISTA_GAP, oracle.FISTA, oracle.PGD)}
    assert its[oracle.FISTA_GAP] < its[oracle.FISTA] and its[oracle.FISTA_GAP] < its[oracle.PGD]
