"""Pins of the brute-force k-sparse reference: with k = p it is the box-
constrained ridge problem on all coordinates, whose unconstrained solution
has a closed form when the box is inactive; with a tight box every active
coefficient sits on the box.  The logistic enumeration's per-support
minimiser satisfies the projected first-order conditions, agrees with the
relaxation at a leaf node (an independent method: FISTA with the gap restart,
where the relaxation is the restricted problem), and bounds the root
relaxation from above.  CPU only."""
import numpy as np

import math

import oracle
from oracle.ksparse import ksparse_bruteforce, ksparse_bruteforce_logistic, logistic_box_ridge


def test_full_support_equals_ridge_closed_form():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(40, 5))
    y = X @ np.array([0.5, -0.3, 0.2, 0.0, 0.1]) + 0.1 * rng.normal(size=40)
    val, S, b = ksparse_bruteforce(X, y, 5, 0.7, 10.0)
    ridge = np.linalg.solve(X.T @ X + 0.7 * np.eye(5), X.T @ y)
    assert S == [0, 1, 2, 3, 4]
    assert np.allclose(b, ridge, atol=1e-10)
    assert abs(val - (np.sum((y - X @ ridge) ** 2) + 0.7 * ridge @ ridge)) <= 1e-10 * val


def test_single_coordinate_matches_scalar_minimisation():
    rng = np.random.default_rng(1)
    X = rng.normal(size=(30, 4))
    y = 3.0 * X[:, 2] + 0.01 * rng.normal(size=30)
    val, S, b = ksparse_bruteforce(X, y, 1, 0.1, 1.0)      # box active: |b| <= 1 < 3
    assert S == [2] and abs(b[0] - 1.0) <= 1e-12
    for j in range(4):                                       # brute force over the scalar too
        for t in np.linspace(-1, 1, 2001):
            assert val <= np.sum((y - t * X[:, j]) ** 2) + 0.1 * t * t + 1e-9


def test_fixings_are_respected():
    rng = np.random.default_rng(2)
    X = rng.normal(size=(30, 6))
    y = X[:, 0] + X[:, 1] + 0.1 * rng.normal(size=30)
    val0, S0, _ = ksparse_bruteforce(X, y, 2, 0.1, 5.0)
    val1, S1, _ = ksparse_bruteforce(X, y, 2, 0.1, 5.0, J0=[0])
    val2, S2, _ = ksparse_bruteforce(X, y, 2, 0.1, 5.0, J1=[5])
    assert S0 == [0, 1] and 0 not in S1 and 5 in S2
    assert val1 >= val0 and val2 >= val0


def _logistic_instance(seed, n=80, p=7):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, p))
    y = np.where(X[:, 0] - X[:, 3] + 0.5 * rng.normal(size=n) >= 0, 1.0, -1.0)
    return X, y


def test_logistic_box_ridge_first_order_conditions():
    X, y = _logistic_instance(3)
    for M in (0.3, 2.0, math.inf):
        val, b = logistic_box_ridge(X[:, [0, 3, 5]], y, 0.2, M)
        z = y * (X[:, [0, 3, 5]] @ b)
        g = X[:, [0, 3, 5]].T @ (-y / (1.0 + np.exp(z))) + 0.4 * b
        for bj, gj in zip(b, g):
            if math.isfinite(M) and abs(abs(bj) - M) <= 1e-9:
                assert gj * np.sign(bj) <= 1e-8            # at the box: the gradient points outward
            else:
                assert abs(gj) <= 1e-7                      # interior: stationary
        assert abs(val - (np.sum(np.log1p(np.exp(-z))) + 0.2 * b @ b)) <= 1e-12 * val


def test_logistic_enumeration_agrees_with_leaf_relaxation_and_bounds_root():
    X, y = _logistic_instance(4)
    Xcm = np.ascontiguousarray(X.T)
    k, lam2, M = 2, 0.3, 1.5
    opt, S, b = ksparse_bruteforce_logistic(X, y, k, lam2, M)
    p = X.shape[1]
    st = np.full(p, oracle.ZERO, np.int8)
    st[S] = oracle.ONE
    leaf = oracle.solve(Xcm, y, 1, lam2, M, k, status=st, tol=1e-12, max_iter=200000)
    assert abs(leaf["ub"] - opt) <= 1e-9 * opt and abs(leaf["lb"] - opt) <= 1e-9 * opt
    root = oracle.solve(Xcm, y, 1, lam2, M, k, tol=1e-11, max_iter=200000)
    assert root["lb"] <= opt * (1 + 1e-12)
    # every other support is no better
    for j0 in range(p):
        v1, _, _ = ksparse_bruteforce_logistic(X, y, k, lam2, M, J0=[j0])
        assert v1 >= opt * (1 - 1e-12)
