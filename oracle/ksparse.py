"""Exact optimum of the k-sparse problem (1) with least-squares loss by
enumeration, for tiny p.

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
from scipy.optimize import lsq_linear


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
