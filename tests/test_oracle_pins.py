"""Pins of the FP64 oracle to facts that do not come from the oracle itself:
values printed in the paper, closed forms, generic solvers (scipy LP / NLP),
the definition of g_N evaluated by an independent water-filling argument, and
brute force on tiny instances.  CPU only."""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy import optimize

import oracle
from workloads import make_instance

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_worked_examples.json")


def _node(rng, p, k):
    st = np.zeros(p, np.int8)
    idx = rng.permutation(p)
    n0 = int(rng.integers(0, p // 2 + 1))
    n1 = int(rng.integers(0, min(k, p - n0) + 1))
    st[idx[:n0]] = oracle.ZERO
    st[idx[n0:n0 + n1]] = oracle.ONE
    return st


# --------------------------------------------------------------- g_N

def test_worked_examples_from_paper():
    gold = json.load(open(GOLDEN))
    for ex in gold["majorization_examples"]:
        val = oracle.g(ex["beta"], ex["k"])
        assert val == pytest.approx(ex["g"], abs=1e-15), ex["cite"]
        assert val == pytest.approx(0.5 * sum(w * w for w in ex["omega"]), abs=1e-15)


def test_figure2_boundary_and_transition_values():
    f2 = json.load(open(GOLDEN))["figure2_root_node"]
    M, k = f2["M"], f2["k"]
    for t in np.linspace(0.0, 1.0, 11):
        b = np.array([t * M, (1.0 - t) * M])
        assert oracle.g(b, k) == pytest.approx(f2["g_on_boundary"], abs=1e-15)
        assert oracle.in_dom(b, k, M)
        assert not oracle.in_dom(b * (1 + 1e-6), k, M)
    for a2 in np.linspace(-M, M, 9):
        assert oracle.gstar([M, a2], k, M) == pytest.approx(f2["gstar_on_transition"], abs=1e-15)
    # quadratic inside (max|a| <= M), linear outside
    assert oracle.gstar([0.3, -0.7], k, M) == pytest.approx(0.5 * 0.49, abs=1e-15)
    assert oracle.gstar([3.0, 0.2], k, M) == pytest.approx(M * 3.0 - 0.5 * M * M, abs=1e-15)


def _g_waterfill(beta, k, st):
    """g_N from its definition (Section 2.4): inf over z of 0.5 sum beta_j^2/z_j
    with z_J0 = 0, z_J1 = 1, z_Jf in [|beta_j|/M, 1], sum z <= k.  Lagrangian
    stationarity gives z_j = clip(|beta_j| / sqrt(2 mu), lo_j, 1); mu is found by
    bisection so that the budget holds (mu = 0 if it is slack)."""
    b = np.abs(np.asarray(beta, float))
    free = st == oracle.FREE
    one = st == oracle.ONE
    kb = k - one.sum()
    bf = b[free]
    if np.any(b[st == oracle.ZERO] > 0) or kb < 0:
        return math.inf
    if bf.size == 0 or np.all(bf == 0):
        return 0.5 * np.sum(b[one] ** 2)
    if bf.size <= kb:
        return 0.5 * np.sum(b[one] ** 2) + 0.5 * np.sum(bf ** 2)

    M = np.inf if not np.isfinite(_g_waterfill.M) else _g_waterfill.M

    def z_of(mu):
        return np.minimum(np.maximum(bf / math.sqrt(2 * mu), bf / M), 1.0)

    lo, hi = 1e-300, 1e300
    if z_of(lo).sum() <= kb:
        z = z_of(lo)
    else:
        for _ in range(3000):
            mid = math.sqrt(lo * hi)
            if z_of(mid).sum() > kb:
                lo = mid
            else:
                hi = mid
            if hi / lo < 1 + 1e-15:
                break
        z = z_of(hi)
    nz = bf > 0
    return 0.5 * np.sum(b[one] ** 2) + 0.5 * np.sum(bf[nz] ** 2 / z[nz])


@pytest.mark.parametrize("seed", range(40))
def test_algorithm1_matches_definition_by_waterfilling(seed):
    rng = np.random.default_rng(seed)
    p = int(rng.integers(2, 30))
    k = int(rng.integers(1, p + 1))
    st = _node(rng, p, k) if seed % 2 else np.zeros(p, np.int8)
    M = [5.0, 1.0, 0.6][seed % 3]
    beta = rng.standard_normal(p)
    beta[st == oracle.ZERO] = 0.0
    kb = k - np.sum(st == oracle.ONE)
    free = st == oracle.FREE
    # scale into dom: ||beta_free||_1 <= M kbar, |beta| <= M
    if kb == 0:
        beta[free] = 0.0
    else:
        s = max(1.0, np.abs(beta[free]).sum() / (M * kb * 0.9)) if free.any() else 1.0
        beta[free] /= s
    beta = np.clip(beta, -M, M)
    assert oracle.in_dom(beta, k, M, st)
    _g_waterfill.M = M
    assert oracle.g(beta, k, st) == pytest.approx(_g_waterfill(beta, k, st), rel=1e-10, abs=1e-14)


@pytest.mark.parametrize("seed", range(6))
def test_algorithm1_matches_generic_nlp_solver(seed):
    """Solve the defining convex program of g_N with SLSQP on tiny p."""
    rng = np.random.default_rng(100 + seed)
    p, k, M = 4, 2, 2.0
    beta = rng.uniform(-1, 1, p)
    beta *= min(1.0, 0.9 * M * k / np.abs(beta).sum())
    lo = np.abs(beta) / M

    def obj(z):
        return 0.5 * np.sum(beta ** 2 / z)

    res = optimize.minimize(obj, np.full(p, k / p), method="SLSQP",
                            bounds=[(max(l, 1e-9), 1.0) for l in lo],
                            constraints=[{"type": "ineq", "fun": lambda z: k - z.sum()}],
                            options={"ftol": 1e-14, "maxiter": 1000})
    assert oracle.g(beta, k) == pytest.approx(res.fun, rel=1e-6)


def test_root_kbar1_is_half_l1_squared():
    rng = np.random.default_rng(0)
    for _ in range(20):
        b = rng.standard_normal(9)
        b *= 0.8 / np.abs(b).sum()
        assert oracle.g(b, 1) == pytest.approx(0.5 * np.abs(b).sum() ** 2, rel=1e-14)


def test_kbar_ge_pbar_is_ridge():
    rng = np.random.default_rng(1)
    b = rng.uniform(-1, 1, 7)
    assert oracle.g(b, 7) == pytest.approx(0.5 * np.sum(b ** 2), rel=1e-15)
    assert oracle.g(b, 12) == pytest.approx(0.5 * np.sum(b ** 2), rel=1e-15)


# --------------------------------------------------------------- g_N*

@pytest.mark.parametrize("seed", range(12))
def test_conjugate_matches_linear_program(seed):
    """g_N*(alpha) = max over the z-polytope of sum z_j H_M(alpha_j) (sup over
    beta for fixed z is z_j H_M(alpha_j) per coordinate); solve that LP with
    scipy and compare with the closed form."""
    rng = np.random.default_rng(seed)
    p = int(rng.integers(2, 25))
    k = int(rng.integers(1, p + 1))
    st = _node(rng, p, k)
    M = [0.5, 1.0, 3.0][seed % 3]
    a = rng.standard_normal(p) * 2
    h = np.array([oracle.huber(x, M) for x in a])
    bounds = [(0, 0) if s == oracle.ZERO else ((1, 1) if s == oracle.ONE else (0, 1)) for s in st]
    lp = optimize.linprog(-h, A_ub=np.ones((1, p)), b_ub=[k], bounds=bounds, method="highs")
    assert oracle.gstar(a, k, M, st) == pytest.approx(-lp.fun, rel=1e-12, abs=1e-12)


def test_huber_and_its_prox_against_scalar_minimisation():
    for M in (0.5, 2.0):
        assert oracle.huber(M, M) == pytest.approx(0.5 * M * M)
        assert oracle.huber(3 * M, M) == pytest.approx(3 * M * M - 0.5 * M * M)
        for u in np.linspace(-5, 5, 21):
            for c in (0.0, 0.3, 4.0):
                r = optimize.minimize_scalar(lambda a: 0.5 * (a - u) ** 2 + c * oracle.huber(a, M),
                                             bounds=(-10, 10), method="bounded",
                                             options={"xatol": 1e-12})
                x = oracle.prox_huber(u, c, M)
                f = lambda a: 0.5 * (a - u) ** 2 + c * oracle.huber(a, M)
                assert f(x) <= f(r.x) + 1e-13     # the closed form is the minimiser
                assert x == pytest.approx(r.x, abs=1e-6)


# --------------------------------------------------------------- prox

def _prox_case(seed):
    rng = np.random.default_rng(seed)
    p = int(rng.integers(1, 40))
    k = int(rng.integers(1, 10))
    st = _node(rng, p, k) if seed % 2 else np.zeros(p, np.int8)
    M = [0.7, 2.0][seed % 2]
    rho = 10 ** rng.uniform(-3, 1)
    v = rng.standard_normal(p) * 2
    return v, rho, k, M, st


@pytest.mark.parametrize("seed", range(40))
def test_prox_fenchel_young_equality(seed):
    """x = prox_{rho g}(v) iff a = (v - x)/rho in dg(x) iff g(x) + g*(a) = a^T x."""
    v, rho, k, M, st = _prox_case(seed)
    x = oracle.prox_g(v, rho, k, M, st)
    a = (v - x) / rho
    a[st == oracle.ZERO] = 0.0          # g* ignores J0 coordinates
    x[st == oracle.ZERO] = 0.0
    assert oracle.in_dom(x, k, M, st)
    lhs = oracle.g(x, k, st) + oracle.gstar(a, k, M, st)
    assert lhs == pytest.approx(float(a @ x), rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("seed", range(8))
def test_prox_matches_generic_minimisation(seed):
    """prox by minimising 0.5||x - v||^2 + rho g(x) over (x, z) jointly with SLSQP."""
    rng = np.random.default_rng(200 + seed)
    p, k, M, rho = 4, 2, 1.5, 0.4
    v = rng.standard_normal(p) * 1.5

    def obj(w):
        x, z = w[:p], w[p:]
        return 0.5 * np.sum((x - v) ** 2) + rho * 0.5 * np.sum(x ** 2 / z)

    cons = [{"type": "ineq", "fun": lambda w: k - w[p:].sum()}]
    for j in range(p):
        cons.append({"type": "ineq", "fun": lambda w, j=j: M * w[p + j] - w[j]})
        cons.append({"type": "ineq", "fun": lambda w, j=j: M * w[p + j] + w[j]})
    w0 = np.concatenate([np.zeros(p), np.full(p, k / p)])
    r = optimize.minimize(obj, w0, method="SLSQP", bounds=[(-M, M)] * p + [(1e-10, 1)] * p,
                          constraints=cons, options={"ftol": 1e-15, "maxiter": 2000})
    x = oracle.prox_g(v, rho, k, M)
    assert np.allclose(x, r.x[:p], atol=2e-5)


def test_prox_structural_special_cases():
    rng = np.random.default_rng(3)
    v = rng.standard_normal(12) * 3
    rho, M = 0.25, 1.0
    # kbar >= pbar: ridge shrink then box on every coordinate
    x = oracle.prox_g(v, rho, 12, M)
    assert np.allclose(x, np.sign(v) * np.minimum(np.abs(v) / (1 + rho), M), atol=1e-13)
    # J0 -> 0, J1 -> ridge/box
    st = np.zeros(12, np.int8)
    st[[0, 1]] = oracle.ZERO
    st[[2]] = oracle.ONE
    x = oracle.prox_g(v, rho, 4, M, st)
    assert np.all(np.abs(x[:2]) < 1e-14)
    assert x[2] == pytest.approx(np.sign(v[2]) * min(abs(v[2]) / (1 + rho), M), abs=1e-13)


# --------------------------------------------------------------- losses

@pytest.mark.parametrize("kind", [oracle.LSQ, oracle.LOGISTIC])
def test_loss_gradient_and_conjugate(kind):
    rng = np.random.default_rng(kind)
    n = 30
    u = rng.standard_normal(n) * 2
    y = rng.standard_normal(n) if kind == oracle.LSQ else np.where(rng.random(n) < 0.5, -1.0, 1.0)
    g = oracle.loss_grad(kind, u, y)
    eps = 1e-6
    for i in range(0, n, 7):
        e = np.zeros(n)
        e[i] = eps
        fd = (oracle.loss(kind, u + e, y) - oracle.loss(kind, u - e, y)) / (2 * eps)
        assert fd == pytest.approx(g[i], rel=1e-6, abs=1e-8)
    # Fenchel-Young at zeta = -grad F(u): -F*(-zeta) = F(u) + u^T zeta
    zeta = -g
    assert oracle.neg_conj(kind, zeta, y) == pytest.approx(oracle.loss(kind, u, y) + float(u @ zeta), rel=1e-12)
    if kind == oracle.LOGISTIC:
        # conjugate of one coordinate by direct scalar maximisation
        zi, yi = zeta[0], y[0]
        r = optimize.minimize_scalar(lambda t: -(-zi * t - math.log1p(math.exp(-yi * t))),
                                     bounds=(-60, 60), method="bounded", options={"xatol": 1e-12})
        a = yi * zi
        ent = -a * math.log(a) - (1 - a) * math.log(1 - a)
        assert ent == pytest.approx(r.fun, abs=1e-9)   # -F_i*(-zeta_i) = entropy
        assert oracle.neg_conj(kind, np.array([2.0]), np.array([1.0])) == -math.inf


# --------------------------------------------------------------- products

def test_matvec_and_power_iteration_against_numpy():
    inst = make_instance(n=64, p=20, corr=0.5, k_true=4, snr=5.0, loss=0, seed=1, storage="f32")
    X = inst.X64().T   # (n, p)
    b = np.arange(20) / 7.0
    r = np.linspace(-1, 1, 64)
    assert np.allclose(oracle.matvec(inst.Xcm, b), X @ b, rtol=1e-13, atol=1e-12)
    assert np.allclose(oracle.rmatvec(inst.Xcm, r), X.T @ r, rtol=1e-13, atol=1e-12)
    lam = np.linalg.eigvalsh(X.T @ X).max()
    assert oracle.power_norm2(inst.Xcm) == pytest.approx(lam, rel=1e-9)


# --------------------------------------------------------------- dual / solver

def _tiny(loss, seed=0, n=40, p=8):
    return make_instance(n=n, p=p, corr=0.5, k_true=3, snr=5.0, loss=loss, seed=seed, storage="f64")


@pytest.mark.parametrize("loss", [0, 1])
def test_weak_duality_random_pairs(loss):
    inst = _tiny(loss)
    rng = np.random.default_rng(7)
    k, M, lam2 = 3, 2.0, 0.5
    for _ in range(30):
        beta = oracle.prox_g(rng.standard_normal(inst.p) * 3, 0.7, k, M)
        if loss == 0:
            zeta = rng.standard_normal(inst.n) * 3
        else:
            zeta = inst.y * rng.uniform(0, 1, inst.n)
        phi = oracle.primal(inst.Xcm, inst.y, beta, loss, lam2, M, k)
        psi = oracle.dual(inst.Xcm, inst.y, zeta, loss, lam2, M, k)
        assert phi >= psi


@pytest.mark.parametrize("loss", [0, 1])
def test_root_bound_below_bruteforce_sparse_optimum(loss):
    """Root lower bound <= min over all supports |S| = k of the box-constrained
    ridge (LS) / ridge-logistic fit on S (problem (1) enumerated), p = 10."""
    inst = _tiny(loss, seed=4, n=40, p=10)
    k, M, lam2 = 3, 2.0, 0.5
    res = oracle.solve(inst.Xcm, inst.y, loss, lam2, M, k, tol=1e-10)
    assert res["status"] == oracle.CONVERGED
    X = inst.X64().T
    best = math.inf
    for S in itertools.combinations(range(inst.p), k):
        XS = X[:, S]
        if loss == 0:
            A = np.vstack([XS, math.sqrt(lam2) * np.eye(k)])
            b = np.concatenate([inst.y, np.zeros(k)])
            fit = optimize.lsq_linear(A, b, bounds=(-M, M), tol=1e-12)
            val = float(np.sum((A @ fit.x - b) ** 2))
        else:
            f = lambda w: float(np.sum(np.logaddexp(0.0, -inst.y * (XS @ w))) + lam2 * w @ w)
            val = optimize.minimize(f, np.zeros(k), method="L-BFGS-B", bounds=[(-M, M)] * k,
                                    options={"ftol": 1e-14, "gtol": 1e-10}).fun
        best = min(best, val)
    assert res["lb"] <= best + 1e-9 * abs(best)
    assert res["ub"] - res["lb"] <= 1e-10 * abs(res["ub"])   # strong duality reached


def test_relaxation_matches_generic_conic_solve():
    """The perspective relaxation (problem perspective_relaxation) solved
    directly in (beta, z) by SLSQP equals the oracle's bound."""
    inst = _tiny(0, seed=2, n=25, p=5)
    k, M, lam2 = 2, 2.0, 0.5
    X = inst.X64().T
    p = inst.p

    def obj(w):
        b, z = w[:p], w[p:]
        return float(np.sum((inst.y - X @ b) ** 2) + lam2 * np.sum(b ** 2 / z))

    cons = [{"type": "ineq", "fun": lambda w: k - w[p:].sum()}]
    for j in range(p):
        cons.append({"type": "ineq", "fun": lambda w, j=j: M * w[p + j] - w[j]})
        cons.append({"type": "ineq", "fun": lambda w, j=j: M * w[p + j] + w[j]})
    w0 = np.concatenate([np.zeros(p), np.full(p, k / p)])
    r = optimize.minimize(obj, w0, method="SLSQP", bounds=[(-M, M)] * p + [(1e-9, 1)] * p,
                          constraints=cons, options={"ftol": 1e-15, "maxiter": 3000})
    res = oracle.solve(inst.Xcm, inst.y, 0, lam2, M, k, tol=1e-12)
    assert res["lb"] == pytest.approx(r.fun, rel=1e-6)


def test_leaf_node_is_restricted_ridge():
    inst = _tiny(0, seed=5, n=40, p=10)
    S = [1, 4, 7]
    st = np.full(inst.p, oracle.ZERO, np.int8)
    st[S] = oracle.ONE
    res = oracle.solve(inst.Xcm, inst.y, 0, 0.5, 50.0, 3, status=st, tol=1e-12)
    XS = inst.X64()[S].T
    b = np.linalg.solve(XS.T @ XS + 0.5 * np.eye(3), XS.T @ inst.y)
    closed = float(np.sum((inst.y - XS @ b) ** 2) + 0.5 * b @ b)
    assert res["lb"] == pytest.approx(closed, rel=1e-10)


def test_child_bound_not_below_parent():
    inst = _tiny(0, seed=6, n=40, p=10)
    root = oracle.solve(inst.Xcm, inst.y, 0, 0.5, 2.0, 3, tol=1e-11)
    j = int(np.argmax(np.abs(root["beta"])))
    for s in (oracle.ZERO, oracle.ONE):
        st = np.zeros(inst.p, np.int8)
        st[j] = s
        child = oracle.solve(inst.Xcm, inst.y, 0, 0.5, 2.0, 3, status=st, tol=1e-11)
        assert child["lb"] >= root["lb"] - 1e-9 * abs(root["lb"])


def test_infeasible_node():
    inst = _tiny(0)
    st = np.zeros(inst.p, np.int8)
    st[:4] = oracle.ONE
    res = oracle.solve(inst.Xcm, inst.y, 0, 0.5, 2.0, 3, status=st)
    assert res["status"] == oracle.INFEASIBLE and res["lb"] == math.inf


def test_restart_epochs_contract_by_eta():
    """Gap restart (Section 3.3): an epoch ends exactly when the gap has fallen
    by eta, so the number of restarts is at most log_eta(gap0 / gap_final)."""
    inst = make_instance(n=200, p=80, corr=0.5, k_true=5, snr=5.0, loss=0, seed=9, storage="f64")
    eta = math.e ** 2
    res = oracle.solve(inst.Xcm, inst.y, 0, 0.5, 2.0, 5, tol=1e-9, eta=eta, trace_cap=100000)
    tr = res["trace"]
    assert res["status"] == oracle.CONVERGED and res["restarts"] >= 1
    bound = math.ceil(math.log(tr[0] / tr[-1]) / math.log(eta))
    assert res["restarts"] <= bound


def test_power_norm2_on_mirrored_integer_design():
    """X = [B, -B] with integer entries: X 1 = 0 exactly, so a constant start
    would see only the zero eigenvalue; ||X||_2^2 = 2 ||B||_2^2 by a dense
    symmetric eigensolver."""
    inst = make_instance(n=300, p=40, corr=0.5, k_true=1, snr=5.0, loss=0, seed=9, storage="f64")
    B = np.round(inst.Xcm * 4.0)
    Xcm = np.ascontiguousarray(np.concatenate([B, -B], axis=0))
    assert np.all(oracle.matvec(Xcm, np.ones(80)) == 0.0)
    lam = 2.0 * np.linalg.eigvalsh(B @ B.T).max()
    assert oracle.power_norm2(Xcm) == pytest.approx(lam, rel=1e-9)
