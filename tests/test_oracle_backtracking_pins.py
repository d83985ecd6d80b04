"""Pins of the oracle's FISTA with backtracking (the "FISTA with line search"
the paper runs with its duality-gap restart, Section 5; the monotone
backtracking rule of Beck, First-Order Methods in Optimization, 2017,
Section 10.7): every accepted step satisfies the quadratic-model condition
recomputed here from the definition, the step constant is the smallest
c-multiple that does (the trial one factor below fails), the O(1/k^2) bound
of Theorem 10.34 with the backtracking constant, the fixed-step method as the
special case L0 = Lmax, and with the gap restart the line search restarting
from L0 while the certified bound stays the relaxation's.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from workloads import make_instance

LAM2, M, K = 0.5, 2.0, 4


def _inst(loss):
    if loss == 0:
        return make_instance(n=60, p=16, corr=0.6, k_true=4, snr=3.0, loss=0, seed=5, storage="f64")
    return make_instance(n=90, p=12, corr=0.5, k_true=3, snr=4.0, loss=1, seed=7, storage="f64")


def _f_and_grad(inst, loss):
    X, y = inst.X64().T, inst.y
    if loss == 0:
        return (lambda b: float(np.sum((y - X @ b) ** 2)),
                lambda b: -2.0 * X.T @ (y - X @ b))
    return (lambda b: float(np.sum(np.logaddexp(0.0, -y * (X @ b)))),
            lambda b: X.T @ (-y / (1.0 + np.exp(y * (X @ b)))))


def _lf(inst, loss):
    X = inst.X64().T
    return (2.0 if loss == 0 else 0.25) * float(np.linalg.eigvalsh(X.T @ X).max())


@pytest.mark.parametrize("loss", [0, 1])
def test_accepted_steps_satisfy_the_quadratic_model_and_are_minimal(loss):
    """FISTA with backtracking without restart, iterates x_1 .. x_12 from
    runs capped at k steps: x_{k+1} = prox(y_k - grad f(y_k) / L) with the
    reported L, f(x_{k+1}) <= f(y_k) + <grad f(y_k), x_{k+1} - y_k> +
    L/2 ||x_{k+1} - y_k||^2, and where L grew at this step the trial with
    L / c violates it."""
    inst = _inst(loss)
    f, df = _f_and_grad(inst, loss)
    Lf, c = _lf(inst, loss), 2.0
    L0, Lmax = Lf / 64.0, 8.0 * Lf
    kw = dict(L0=L0, c=c, Lmax=Lmax, restart=False, tol=-1.0)
    n_it = 12
    full = oracle.solve_bt(inst.Xcm, inst.y, loss, LAM2, M, K, max_iter=n_it, trace_cap=n_it + 1, **kw)
    Ls = full["L_trace"]
    xs = [np.zeros(inst.p)] + [oracle.solve_bt(inst.Xcm, inst.y, loss, LAM2, M, K, max_iter=i, **kw)["beta"]
                               for i in range(1, n_it + 1)]
    assert np.array_equal(xs[-1], full["beta"])
    t, grew = 1.0, 0
    yk = xs[0].copy()
    for k in range(n_it):
        L = Ls[k + 1]
        g = df(yk)
        xn = oracle.prox_g(yk - g / L, 2.0 * LAM2 / L, K, M)
        np.testing.assert_allclose(xn, xs[k + 1], rtol=0, atol=1e-12)
        d = xs[k + 1] - yk
        model = f(yk) + g @ d + 0.5 * L * d @ d
        assert f(xs[k + 1]) <= model + 1e-12 * abs(model)
        assert L >= Ls[k] and (L == Ls[k] or abs(L / Ls[k] - c ** round(math.log(L / Ls[k], c))) < 1e-12)
        if L > Ls[k]:
            grew += 1
            Lb = L / c
            xb = oracle.prox_g(yk - g / Lb, 2.0 * LAM2 / Lb, K, M)
            db = xb - yk
            assert f(xb) > f(yk) + g @ db + 0.5 * Lb * db @ db - 1e-12 * abs(f(yk))
        tn = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t * t))
        yk = xs[k + 1] + ((t - 1.0) / tn) * (xs[k + 1] - xs[k])
        t = tn
    assert grew >= 1 and full["rejected"] == round(math.log(Ls[-1] / L0, c))
    assert Ls[-1] <= c * Lf


@pytest.mark.parametrize("loss", [0, 1])
def test_backtracking_rate_bound(loss):
    """Theorem 10.34 with backtracking (L0 below the Lipschitz constant Lf):
    Phi(x_k) - Phi* <= 2 c Lf ||x_0 - x*||^2 / (k + 1)^2."""
    inst = _inst(loss)
    Lf, c = _lf(inst, loss), 2.0
    ref = oracle.solve(inst.Xcm, inst.y, loss, LAM2, M, K, L=Lf, tol=1e-13, max_iter=300000)
    r = oracle.solve_bt(inst.Xcm, inst.y, loss, LAM2, M, K, L0=Lf / 64.0, c=c, Lmax=8.0 * Lf, restart=False,
                        tol=-1.0, max_iter=300, trace_cap=301)
    phi = r["phi_trace"]
    phistar, d0 = ref["ub"], np.linalg.norm(ref["beta"])
    k = np.arange(1, phi.size)
    assert np.all(phi[1:] - phistar <= 2.0 * c * Lf * d0 ** 2 / (k + 1) ** 2 + 1e-9 * abs(phistar))
    assert r["rejected"] >= 1 and r["L"] <= c * Lf


@pytest.mark.parametrize("loss", [0, 1])
def test_start_at_the_cap_is_the_fixed_step_method(loss):
    """L0 = Lmax leaves nothing to search: the iterates, traces and restarts
    of the fixed-step FISTA with the gap restart, exactly."""
    inst = _inst(loss)
    Lf = _lf(inst, loss)
    a = oracle.solve(inst.Xcm, inst.y, loss, LAM2, M, K, L=Lf, tol=1e-10, max_iter=5000, trace_cap=5001)
    b = oracle.solve_bt(inst.Xcm, inst.y, loss, LAM2, M, K, L0=Lf, Lmax=Lf, tol=1e-10, max_iter=5000,
                        trace_cap=5001)
    assert a["iters"] == b["iters"] and a["restarts"] == b["restarts"] and b["rejected"] == 0
    assert np.array_equal(a["phi_trace"], b["phi_trace"]) and np.array_equal(a["trace"], b["trace"])
    assert np.array_equal(a["beta"], b["beta"]) and a["lb"] == b["lb"]


@pytest.mark.parametrize("loss", [0, 1])
def test_gap_restart_restarts_the_line_search_and_certifies_the_bound(loss):
    """With the gap restart: restarts happen at the first accepted iterate
    whose gap is at most the epoch's starting gap / eta; the step constant
    only decreases right after a restart, and then to L0 c^j; the converged
    bound equals the fixed-step method's and is below the k-sparse optimum
    found by enumerating supports."""
    inst = _inst(loss)
    Lf, c, eta = _lf(inst, loss), 2.0, math.exp(3.0)
    L0 = Lf / 16.0
    r = oracle.solve_bt(inst.Xcm, inst.y, loss, LAM2, M, K, L0=L0, c=c, Lmax=Lf, tol=1e-9, eta=eta,
                        max_iter=20000, trace_cap=20001)
    assert r["status"] == oracle.CONVERGED and r["restarts"] >= 2
    gap, Ls = r["trace"], r["L_trace"]
    gref, restarts_at = gap[0], []
    for k in range(1, gap.size):
        if gap[k] <= gref / eta and k < gap.size - 1:
            restarts_at.append(k)
            gref = gap[k]
    assert len(restarts_at) == r["restarts"]
    for k in range(1, Ls.size - 1):
        if Ls[k + 1] < Ls[k]:
            assert k in restarts_at
        if k in restarts_at:
            j = math.log(Ls[k + 1] / L0, c)
            assert abs(j - round(j)) < 1e-9 and round(j) >= 0
    assert any(Ls[k + 1] < Ls[k] for k in restarts_at)          # the search restarted below the last L
    ref = oracle.solve(inst.Xcm, inst.y, loss, LAM2, M, K, L=Lf, tol=1e-9, max_iter=100000)
    assert abs(r["lb"] - ref["lb"]) <= 2e-8 * abs(ref["ub"])
    from oracle import ksparse
    X = inst.X64().T
    brute = ksparse.ksparse_bruteforce if loss == 0 else ksparse.ksparse_bruteforce_logistic
    best = brute(X, inst.y, K, LAM2, M)[0]
    assert r["lb"] <= best * (1 + 1e-9)
