"""Exact optimum of the k-sparse problem (1) by enumeration of supports, for
tiny p: least-squares loss (bounded linear least squares per support) and
logistic loss (box-constrained smooth convex minimisation per support).

TEST INFRASTRUCTURE ONLY (tests/ may use it; the product never does).

Problem (1): min ||y - X b||^2 + lambda2 ||b||^2  s.t.  ||b||_0 <= k,
|b_j| <= M, b_j = 0 on J0, b_j != 0 allowed on J1 (J1 coordinates are counted
in the support).  Every support of size k that contains J1 and avoids J0 is
enumerated (smaller supports are covered: coefficients may be zero) and the
box-constrained ridge problem on it is solved exactly as a bounded linear
least-squares problem, [X_S; sqrt(lambda2) I] b ~ [y; 0], by scipy's BVLS.
"""
import itertools
import math

import numpy as np
from scipy.optimize import lsq_linear, minimize


def ksparse_bruteforce(X, y, k, lambda2, M, J0=(), J1=()):
    """(optimal value, support, b) of problem (1); X is (n, p) float64."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n, p = X.shape
    J0, J1 = set(int(j) for j in J0), sorted(int(j) for j in J1)
    if len(J1) > k:
        return math.inf, None, None
    rest = [j for j in range(p) if j not in J0 and j not in J1]
    size = min(k - len(J1), len(rest))
    best = (math.inf, None, None)
    for extra in itertools.combinations(rest, size):
        S = sorted(J1 + list(extra))
        if not S:
            val = float(y @ y)
            if val < best[0]:
                best = (val, S, np.zeros(0))
            continue
        A = np.vstack([X[:, S], math.sqrt(lambda2) * np.eye(len(S))])
        rhs = np.concatenate([y, np.zeros(len(S))])
        r = lsq_linear(A, rhs, bounds=(-M, M), method="bvls", tol=1e-14)
        b = r.x
        val = float(np.sum((y - X[:, S] @ b) ** 2) + lambda2 * b @ b)
        if val < best[0]:
            best = (val, S, b)
    return best


def logistic_box_ridge(XS, y, lambda2, M):
    """(value, b) of min sum_i log(1 + exp(-y_i x_i^T b)) + lambda2 ||b||^2
    over |b_j| <= M, by L-BFGS-B with the exact gradient; the objective is
    strongly convex, so the minimiser is unique."""
    XS = np.asarray(XS, dtype=np.float64)
    m = XS.shape[1]
    if m == 0:
        return float(np.sum(np.logaddexp(0.0, np.zeros_like(y)))), np.zeros(0)

    def fg(b):
        z = y * (XS @ b)
        val = float(np.sum(np.logaddexp(0.0, -z)) + lambda2 * b @ b)
        s = -y / (1.0 + np.exp(z))          # d/du log(1 + exp(-y u)) at u = x^T b
        return val, XS.T @ s + 2.0 * lambda2 * b

    bounds = None if not math.isfinite(M) else [(-M, M)] * m
    r = minimize(fg, np.zeros(m), jac=True, method="L-BFGS-B", bounds=bounds,
                 options={"maxiter": 20000, "ftol": 1e-16, "gtol": 1e-12, "maxcor": 30})
    return fg(r.x)[0], r.x


def ksparse_bruteforce_logistic(X, y, k, lambda2, M, J0=(), J1=()):
    """(optimal value, support, b) of problem (1) with the logistic loss
    sum_i log(1 + exp(-y_i x_i^T b)), y in {-1, +1}; X is (n, p) float64."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n, p = X.shape
    J0, J1 = set(int(j) for j in J0), sorted(int(j) for j in J1)
    if len(J1) > k:
        return math.inf, None, None
    rest = [j for j in range(p) if j not in J0 and j not in J1]
    size = min(k - len(J1), len(rest))
    best = (math.inf, None, None)
    for extra in itertools.combinations(rest, size):
        S = sorted(J1 + list(extra))
        val, b = logistic_box_ridge(X[:, S], y, lambda2, M)
        if val < best[0]:
            best = (val, S, b)
    return best
