"""Pins of the brute-force k-sparse reference: with k = p it is the box-
constrained ridge problem on all coordinates, whose unconstrained solution
has a closed form when the box is inactive; with a tight box every active
coefficient sits on the box.  CPU only."""
import numpy as np

from oracle.ksparse import ksparse_bruteforce


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
