"""Pins of the oracle's AC-FGM iteration and of its LASSO solvers.  CPU only.

AC-FGM (Section 3.3, rate table; Section 5.2 convergence study): the rate
bound Phi(x_t) - Phi* <= 15 c L d0^2 / (2 t (t+1) b (1-b)) of the table, with
L the smoothness constant of f = F(X .) from a dense eigensolver, Phi* and
the solution from a direct SLSQP solve of the relaxation in (beta, z); the
first-step line search ending at L1 = L0 c^j with Lhat_1 <= L1 <= c L; every
local estimate Lhat_t <= L; with the duality-gap restart the same bound as
FISTA's.

LASSO (Section 5.2, the restart beyond perspective relaxations): soft
thresholding and the l1-ball projection against generic minimisation, the
conjugates through Fenchel-Young, the l1-regularised solve against
scikit-learn's coordinate descent, the l1-ball solve against the l1-penalised
solution of the same l1 norm (Lagrange duality), and weak duality."""
import math

import numpy as np
import pytest
from scipy import optimize

import oracle
from workloads import make_instance


def _direct_relaxation(inst, k, M, lam2, loss):
    """Perspective relaxation solved in (beta, z) by SLSQP (root node)."""
    X = inst.X64().T
    p = inst.p
    y = inst.y

    def obj(w):
        b, z = w[:p], w[p:]
        u = X @ b
        F = float(np.sum((y - u) ** 2)) if loss == 0 else float(np.sum(np.logaddexp(0.0, -y * u)))
        return F + lam2 * float(np.sum(b ** 2 / z))

    cons = [{"type": "ineq", "fun": lambda w: k - w[p:].sum()}]
    for j in range(p):
        cons.append({"type": "ineq", "fun": lambda w, j=j: M * w[p + j] - w[j]})
        cons.append({"type": "ineq", "fun": lambda w, j=j: M * w[p + j] + w[j]})
    w0 = np.concatenate([np.zeros(p), np.full(p, k / p)])
    r = optimize.minimize(obj, w0, method="SLSQP", bounds=[(-M, M)] * p + [(1e-9, 1)] * p,
                          constraints=cons, options={"ftol": 1e-15, "maxiter": 5000})
    return r.fun, r.x[:p]


@pytest.mark.parametrize("loss,seed", [(0, 2), (0, 5), (1, 3)])
def test_acfgm_rate_bound_of_the_table(loss, seed):
    inst = make_instance(n=25, p=5, corr=0.5, k_true=2, snr=5.0, loss=loss, seed=seed, storage="f64")
    k, M, lam2, c, b = 2, 2.0, 0.5, 2.0, 0.1
    lam_max = float(np.linalg.eigvalsh(inst.X64() @ inst.X64().T).max())
    L = (2.0 if loss == 0 else 0.25) * lam_max
    phi_star, x_star = _direct_relaxation(inst, k, M, lam2, loss)
    fista = oracle.solve(inst.Xcm, inst.y, loss, lam2, M, k, tol=1e-12)
    assert fista["lb"] == pytest.approx(phi_star, rel=1e-6)
    d0 = float(np.linalg.norm(x_star))                        # start at 0
    r = oracle.solve_acfgm(inst.Xcm, inst.y, loss, lam2, M, k, L0=L / 50.0, c=c, b=b, restart=False,
                           tol=-1.0, max_iter=400, trace_cap=1000)
    step, phi = r["step"], r["phi_trace"]
    acc = np.flatnonzero(step > 0)
    assert acc.size > 300
    for i in acc:
        t = step[i]
        bound = 15.0 * c * L * d0 ** 2 / (2.0 * t * (t + 1.0) * b * (1.0 - b))
        assert phi[i] - phi_star <= bound * (1 + 1e-6) + 1e-9 * abs(phi_star), (t, phi[i] - phi_star, bound)
    # the bound is not vacuous at the end: the iterate is close to optimal
    assert phi[acc[-1]] - phi_star <= 1e-3 * abs(phi_star)
    assert np.all(r["trace"][1:] >= -1e-9 * abs(phi_star))   # weak duality at every evaluation


@pytest.mark.parametrize("loss", [0, 1])
def test_acfgm_first_step_line_search_and_local_estimates(loss):
    inst = make_instance(n=60, p=12, corr=0.6, k_true=3, snr=5.0, loss=loss, seed=7, storage="f64")
    lam_max = float(np.linalg.eigvalsh(inst.X64() @ inst.X64().T).max())
    L = (2.0 if loss == 0 else 0.25) * lam_max
    c, L0 = 3.0, L / 500.0
    r = oracle.solve_acfgm(inst.Xcm, inst.y, loss, 0.3, 2.0, 4, L0=L0, c=c, restart=False, tol=-1.0,
                           max_iter=60, trace_cap=100)
    step, lhat = r["step"], r["lhat"]
    j = r["rejected"]
    assert j >= 1 and np.all(step[1:j + 1] == -1) and step[j + 1] == 1
    assert r["L1"] == pytest.approx(L0 * c ** j, rel=1e-15)
    assert lhat[j + 1] <= r["L1"] <= c * L                     # the accepted trial passes its test
    assert np.all(lhat[1:j + 1] > L0 * c ** np.arange(j))       # each rejected one failed it
    assert np.all(lhat[1:] <= L * (1 + 1e-12))                  # local estimates never exceed L
    assert np.all(np.diff(step[j + 1:]) == 1)                   # then one step per evaluation


@pytest.mark.parametrize("loss", [0, 1])
def test_acfgm_with_gap_restart_reaches_the_fista_bound(loss):
    inst = make_instance(n=60, p=12, corr=0.6, k_true=3, snr=5.0, loss=loss, seed=8, storage="f64")
    st = oracle.status_vector(inst.p, J0=[3], J1=[0])
    L = (2.0 if loss == 0 else 0.25) * oracle.power_norm2(inst.Xcm) * 1.01
    ref = oracle.solve(inst.Xcm, inst.y, loss, 0.3, 2.0, 4, status=st, L=L, tol=1e-11)
    eta = math.e
    r = oracle.solve_acfgm(inst.Xcm, inst.y, loss, 0.3, 2.0, 4, status=st, L0=L / 16, eta=eta, tol=1e-9,
                           trace_cap=100000)
    assert r["status"] == oracle.CONVERGED and r["restarts"] >= 2
    assert abs(r["lb"] - ref["lb"]) <= 1e-9 * abs(ref["ub"])
    assert oracle.dual(inst.Xcm, inst.y, r["zeta"], loss, 0.3, 2.0, 4, status=st) == pytest.approx(r["lb"], rel=1e-13)
    # an accepted iterate whose gap fell to 1/eta of the epoch's reference
    # starts a new epoch (the next evaluation is a first-step trial, t = 1);
    # any other accepted iterate is followed by the next step of its epoch
    gap, step = r["trace"], r["step"]
    ref_gap, starts = gap[0], 0
    for i in range(1, r["iters"]):
        if step[i] < 0:
            assert abs(step[i + 1]) == 1                    # a rejected trial is retried
            continue
        if gap[i] <= ref_gap / eta:
            assert abs(step[i + 1]) == 1, (i, step[i], step[i + 1])
            ref_gap = gap[i]
            starts += 1
        else:
            assert step[i + 1] == step[i] + 1, (i, step[i], step[i + 1])
    assert starts == r["restarts"]


# --------------------------------------------------------------- LASSO

def test_soft_threshold_against_scalar_minimisation():
    rng = np.random.default_rng(1)
    v = rng.standard_normal(40) * 2
    t, lam = 0.7, 1.3
    x = oracle.lasso_prox(oracle.L1_REG, v, t, lam)
    for j in range(40):
        r = optimize.minimize_scalar(lambda a: 0.5 * (a - v[j]) ** 2 + t * lam * abs(a), bracket=(-10, 10),
                                     tol=1e-14)
        assert x[j] == pytest.approx(r.x, abs=1e-7)


@pytest.mark.parametrize("seed", range(6))
def test_l1_ball_projection_against_generic_qp(seed):
    rng = np.random.default_rng(10 + seed)
    p = 8
    v = rng.standard_normal(p) * 2
    rad = [0.5, 1.0, 3.0, 100.0, 2.0, 0.1][seed]
    x = oracle.lasso_prox(oracle.L1_BALL, v, 0.37, rad)          # t plays no role for a projection
    # min 0.5 ||a - b - v||^2 over a, b >= 0 with sum(a + b) <= rad
    obj = lambda w: 0.5 * float(np.sum((w[:p] - w[p:] - v) ** 2))
    cons = [{"type": "ineq", "fun": lambda w: rad - w.sum()}]
    r = optimize.minimize(obj, np.zeros(2 * p), method="SLSQP", bounds=[(0, None)] * (2 * p), constraints=cons,
                          options={"ftol": 1e-15, "maxiter": 1000})
    np.testing.assert_allclose(x, r.x[:p] - r.x[p:], atol=1e-6)
    assert np.sum(np.abs(x)) <= rad * (1 + 1e-12)
    if np.sum(np.abs(v)) <= rad:
        assert np.array_equal(x, v)


@pytest.mark.parametrize("kind", [0, 1])
def test_lasso_prox_fenchel_young(kind):
    rng = np.random.default_rng(20 + kind)
    for _ in range(20):
        p = int(rng.integers(1, 30))
        v = rng.standard_normal(p) * 3
        t, lam = 10 ** rng.uniform(-2, 1), 10 ** rng.uniform(-1, 1)
        x = oracle.lasso_prox(kind, v, t, lam)
        a = (v - x) / t                   # a in dG(x)
        lhs = oracle.lasso_G(kind, x, lam) + oracle.lasso_Gstar(kind, a, lam * (1 + 1e-12))
        assert lhs == pytest.approx(float(a @ x), rel=1e-10, abs=1e-12)


def _lasso_inst(seed=3, n=80, p=30):
    return make_instance(n=n, p=p, corr=0.6, k_true=5, snr=5.0, loss=0, seed=seed, storage="f64")


def test_l1_regularised_solve_against_sklearn():
    from sklearn.linear_model import Lasso
    inst = _lasso_inst()
    X = inst.X64().T
    lam = 0.2 * 2.0 * float(np.max(np.abs(X.T @ inst.y)))       # 20% of the smallest lam giving beta = 0
    r = oracle.lasso_solve(inst.Xcm, inst.y, oracle.L1_REG, lam, tol=1e-12)
    assert r["status"] == oracle.CONVERGED
    # scikit-learn minimises (1 / 2n) ||y - X w||^2 + alpha ||w||_1
    sk = Lasso(alpha=lam / (2 * inst.n), fit_intercept=False, tol=1e-14, max_iter=1000000).fit(X, inst.y)
    np.testing.assert_allclose(r["beta"], sk.coef_, atol=1e-6)
    obj = float(np.sum((inst.y - X @ sk.coef_) ** 2) + lam * np.sum(np.abs(sk.coef_)))
    assert r["ub"] == pytest.approx(obj, rel=1e-9)
    assert 0 < np.count_nonzero(np.abs(r["beta"]) > 1e-9) < inst.p
    # KKT: |2 X^T (y - X b)|_j <= lam, with equality and matching sign on the support
    g = 2.0 * X.T @ (inst.y - X @ r["beta"])
    sup = np.abs(r["beta"]) > 1e-8
    assert np.all(np.abs(g) <= lam * (1 + 1e-6))
    np.testing.assert_allclose(g[sup], lam * np.sign(r["beta"][sup]), rtol=1e-6)


def test_l1_ball_solve_equals_penalised_solution_of_the_same_norm():
    inst = _lasso_inst(seed=4)
    X = inst.X64().T
    lam = 0.1 * 2.0 * float(np.max(np.abs(X.T @ inst.y)))
    pen = oracle.lasso_solve(inst.Xcm, inst.y, oracle.L1_REG, lam, tol=1e-13)
    rad = float(np.sum(np.abs(pen["beta"])))
    ball = oracle.lasso_solve(inst.Xcm, inst.y, oracle.L1_BALL, rad, tol=1e-12)
    assert ball["status"] == oracle.CONVERGED
    np.testing.assert_allclose(ball["beta"], pen["beta"], atol=1e-5)
    F_pen = float(np.sum((inst.y - X @ pen["beta"]) ** 2))
    assert ball["ub"] == pytest.approx(F_pen, rel=1e-8)


@pytest.mark.parametrize("kind", [0, 1])
def test_lasso_weak_duality_and_zero_gap(kind):
    inst = _lasso_inst(seed=5)
    X = inst.X64().T
    lam = 0.15 * 2.0 * float(np.max(np.abs(X.T @ inst.y))) if kind == 0 else 3.0
    rng = np.random.default_rng(0)
    for _ in range(20):
        b = oracle.lasso_prox(kind, rng.standard_normal(inst.p), 1.0, lam)
        zeta = rng.standard_normal(inst.n) * 5
        phi = float(np.sum((inst.y - X @ b) ** 2)) + oracle.lasso_G(kind, b, lam)
        psi, _ = oracle.lasso_dual(inst.Xcm, inst.y, kind, lam, zeta)
        assert psi <= phi
    r = oracle.lasso_solve(inst.Xcm, inst.y, kind, lam, tol=1e-12)
    assert r["status"] == oracle.CONVERGED and 0 <= r["rel_gap"] <= 1e-12
    psi, s = oracle.lasso_dual(inst.Xcm, inst.y, kind, lam, r["zeta"])
    assert psi == pytest.approx(r["lb"], rel=1e-12) and s == pytest.approx(1.0, abs=1e-12)
