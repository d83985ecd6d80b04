"""Pins of the FP64 MLP oracle (learned warm start) to facts outside it:
central finite differences of its own loss for the gradient, networks whose
output has a closed form, the closed form of Adam's first step, and feature
values worked out by hand.  CPU only."""
import numpy as np
import pytest

from oracle import mlp


def _rand(seed, rows=7):
    rng = np.random.default_rng(seed)
    P = mlp.init_params(seed)
    P[mlp.OFF_B1:mlp.OFF_W2] = rng.normal(0, 0.3, mlp.H)     # nonzero biases exercise every term
    P[mlp.OFF_B2:mlp.OFF_W3] = rng.normal(0, 0.3, mlp.H)
    P[mlp.OFF_B3] = 0.2
    F = rng.normal(0, 1, (rows, mlp.NF))
    T = rng.normal(0, 1, rows)
    return P, F, T


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    P, F, T = _rand(seed)
    _, g = mlp.loss_grad(P, F, T)
    rng = np.random.default_rng(100 + seed)
    # every bias and output weight, and a sample of the hidden weights
    idx = list(range(mlp.OFF_B1, mlp.OFF_W2)) + list(range(mlp.OFF_B2, mlp.NPARAM))
    idx += list(rng.choice(mlp.OFF_B1, 40, replace=False)) + list(mlp.OFF_W2 + rng.choice(4096, 80, replace=False))
    eps = 1e-6
    for i in idx:
        a, b = P.copy(), P.copy()
        a[i] += eps
        b[i] -= eps
        fd = (mlp.loss_grad(a, F, T)[0] - mlp.loss_grad(b, F, T)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), i


def test_forward_closed_form_identity_network():
    """W1 = [e0; -e0; 0], W2 = I on the first two units, w3 = (1, -1, 0...):
    relu(f0) - relu(-f0) = f0, so the network returns feature 0 exactly."""
    W1 = np.zeros((mlp.H, mlp.NF))
    W1[0, 0], W1[1, 0] = 1.0, -1.0
    W2 = np.zeros((mlp.H, mlp.H))
    W2[0, 0] = W2[1, 1] = 1.0
    w3 = np.zeros(mlp.H)
    w3[0], w3[1] = 1.0, -1.0
    P = mlp.pack(W1, np.zeros(mlp.H), W2, np.zeros(mlp.H), w3, 0.25)
    F = np.random.default_rng(3).normal(0, 2, (50, mlp.NF))
    assert np.array_equal(mlp.forward(P, F), F[:, 0] + 0.25)


def test_loss_and_gradient_of_constant_network():
    """All weights zero: out = b3 everywhere, loss = mean (b3 - t)^2 and the
    only nonzero gradient entry is d/db3 = 2 mean (b3 - t)."""
    P = np.zeros(mlp.NPARAM)
    P[mlp.OFF_B3] = 0.5
    T = np.array([1.0, -2.0, 0.5, 3.0])
    F = np.ones((4, mlp.NF))
    loss, g = mlp.loss_grad(P, F, T)
    assert loss == pytest.approx(np.mean((0.5 - T) ** 2), rel=1e-15)
    assert g[mlp.OFF_B3] == pytest.approx(2 * np.mean(0.5 - T), rel=1e-15)
    assert np.count_nonzero(g[:mlp.OFF_B3]) == 0


def test_adam_first_step_closed_form():
    """After one step from zero moments the bias-corrected moments are g and
    g^2, so the update is -lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0, 5.0])
    p0 = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    p1, m, v = mlp.adam(p0, g, np.zeros(5), np.zeros(5), 1, lr=0.01, eps=1e-8)
    assert np.allclose(p1, p0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_converges_on_quadratic():
    target = np.array([1.0, -3.0, 0.5])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 3001):
        p, m, v = mlp.adam(p, 2 * (p - target), m, v, t, lr=0.05)
    assert np.allclose(p, target, atol=1e-3)


def test_features_hand_example():
    beta = np.array([0.0, 2.0, -1.0, 0.0, 1.5])
    h = np.array([4.0, -8.0, 2.0, 0.0, 1.0])
    st = np.array([1, 0, 2, 0, 0])         # j0 fixed to zero, j2 fixed to one
    F = mlp.features(beta, h, st, 0.1, 4)
    assert np.array_equal(F[:, 0], beta)
    assert np.array_equal(F[:, 1], [0.5, -1.0, 0.25, 0.0, 0.125])
    assert np.array_equal(F[:, 2], np.array([3, 0, 2, 3, 1]) / 5)   # larger magnitudes
    assert np.array_equal(F[:, 3], [-1, 0, 1, 0, 0])
    assert np.all(F[:, 4] == 0.1)
    assert np.all(F[:, 5] == 1 / 4) and np.all(F[:, 6] == 1 / 4)
    assert np.all(F[:, 7] == 3 / 4)        # kbar = min(4 - 1, 3 free)


def test_features_zero_gradient_and_kbar_limited_by_free():
    F = mlp.features(np.zeros(4), np.zeros(4), np.array([1, 1, 0, 2]), 1.0, 5)
    assert np.all(F[:, 1] == 0) and np.all(F[:, 2] == 0)
    assert np.all(F[:, 7] == 1 / 5)        # kbar = min(5 - 1, 1 free)


def test_feature_rank_matches_brute_force():
    rng = np.random.default_rng(7)
    beta = rng.normal(size=60) * (rng.random(60) < 0.3)
    beta[5] = beta[9] = 0.7                # ties share a rank
    F = mlp.features(beta, rng.normal(size=60), np.zeros(60, int), 0.1, 5)
    brute = [sum(abs(b) > abs(a) for b in beta) / 60 for a in beta]
    assert np.array_equal(F[:, 2], brute)
